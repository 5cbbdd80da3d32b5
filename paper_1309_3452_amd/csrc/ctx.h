// Host-side context behind the opaque dirac_ctx handle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

struct dirac_ctx {
    // lattice
    int ndim = 3;
    int64_t nx = 1, ny = 1, nz = 1;
    int dtype = 2;
    double dt = 0.0, rx = 0.0, ry = 0.0, rz = 0.0;
    unsigned flags = 0;
    int zh = 0;               // z-slab mode: halo planes per side (arrays hold nz + 2 zh planes)
    bool zbc = false;         // zero values outside the lattice instead of periodic wrap
    std::string err;

    // state: two caller-owned buffer sets; cur says which holds the state
    void *buf[2][8] = {};
    bool bound = false;
    int cur = 0;

    // caller-owned scratch (reductions, coefficient tables, gradient partials)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;

    // mass and V(z) profile, or per-site theta
    double m = 0.0;
    std::vector<double> v_int, v_half;
    std::vector<double> w_int, w_half;    // Im V(z) (absorbing layers), empty if none
    bool tab_dirty = true;
    std::vector<double> tab_host64;
    std::vector<float> tab_host32;
    void *theta[8] = {};
    bool site_mode = false;

    // gauge links (vector potential), caller-owned; links_on when bound
    void *links[24] = {};
    bool links_on = false;

    // kernel choice
    int kernel = 0, tile_y = 0, zchunk = 0;

    // batched lattices
    bool is_batch = false;
    int64_t count = 0;
    std::vector<int64_t> bnx, bny;
    std::vector<double> bdt;      // per-lattice time step (r_x = r_y = dt, unit spacing)
    std::vector<void *> bstate, bpartner, btheta;
    size_t batch_scratch_need = 0;
    int tune_choice = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_n = -1;
    int graph_mode = -1;
    int graph_cur = -1;
    int64_t graph_flips = 0;      // ping-pong launches in the captured graph
    hipStream_t graph_stream = nullptr;
};
