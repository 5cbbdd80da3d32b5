// Difference terms S_X of the update equations, from values already loaded.
// 3D: Eqs. ss1-ss4 (Sect. 2); 2D: Eqs. scheme2Deq-scheme4thline (Sect. 3).
// Centred differences over one cell; "i ry" terms are the y derivatives.
#pragma once

#include "device.h"

namespace dirac {

template <typename C> struct St3 { C s0, s1, s2, s3; };
template <typename C> struct St2 { C s0, s1; };

// a u + b v + i c w for real a, b, c: one z, one x and one y difference.
template <typename C, typename R>
__device__ __forceinline__ C sterm3(R a, C u, R b, C v, R c, C w) {
    return mk2(fmx(a, u.x, fmx(b, v.x, -(c * w.y))), fmx(a, u.y, fmx(b, v.y, c * w.x)));
}
// b v + i c w: one x and one y difference (2D rows).
template <typename C, typename R> __device__ __forceinline__ C sterm2(R b, C v, R c, C w) {
    return mk2(fmx(b, v.x, -(c * w.y)), fmx(b, v.y, c * w.x));
}

// A0, A1, B0, B1 rows from C0, C1, D0, D1 (Eqs. ss1, ss2):
//   S_A0 =  rz(C0 - C0[k-1]) + rx(D0 - D0[i-1]) - i ry(D1 - D1[j-1])
//   S_A1 =  rz(C1 - C1[k-1]) + rx(D1[i+1] - D1) - i ry(D0[j+1] - D0)
//   S_B0 = -rz(D0[k+1] - D0) + rx(C0[i+1] - C0) + i ry(C1 - C1[j-1])
//   S_B1 = -rz(D1[k+1] - D1) + rx(C1 - C1[i-1]) + i ry(C0[j+1] - C0)
template <typename C, typename R>
__device__ __forceinline__ St3<C> stencil_ab(R rx, R ry, R rz,
                                             C c0, C c0zm, C c0xp, C c0yp,
                                             C c1, C c1zm, C c1ym, C c1xm,
                                             C d0, C d0xm, C d0yp, C d0zp,
                                             C d1, C d1ym, C d1xp, C d1zp) {
    St3<C> s;
    s.s0 = sterm3(rz, csub(c0, c0zm), rx, csub(d0, d0xm), -ry, csub(d1, d1ym));
    s.s1 = sterm3(rz, csub(c1, c1zm), rx, csub(d1xp, d1), -ry, csub(d0yp, d0));
    s.s2 = sterm3(-rz, csub(d0zp, d0), rx, csub(c0xp, c0), ry, csub(c1, c1ym));
    s.s3 = sterm3(-rz, csub(d1zp, d1), rx, csub(c1, c1xm), ry, csub(c0yp, c0));
    return s;
}

// C0, C1, D0, D1 rows from A0, A1, B0, B1 (Eqs. ss3, ss4):
//   S_C0 =  rz(A0[k+1] - A0) + rx(B0 - B0[i-1]) - i ry(B1 - B1[j-1])
//   S_C1 =  rz(A1[k+1] - A1) + rx(B1[i+1] - B1) - i ry(B0[j+1] - B0)
//   S_D0 = -rz(B0 - B0[k-1]) + rx(A0[i+1] - A0) + i ry(A1 - A1[j-1])
//   S_D1 = -rz(B1 - B1[k-1]) + rx(A1 - A1[i-1]) + i ry(A0[j+1] - A0)
template <typename C, typename R>
__device__ __forceinline__ St3<C> stencil_cd(R rx, R ry, R rz,
                                             C a0, C a0zp, C a0xp, C a0yp,
                                             C a1, C a1zp, C a1xm, C a1ym,
                                             C b0, C b0zm, C b0xm, C b0yp,
                                             C b1, C b1zm, C b1xp, C b1ym) {
    St3<C> s;
    s.s0 = sterm3(rz, csub(a0zp, a0), rx, csub(b0, b0xm), -ry, csub(b1, b1ym));
    s.s1 = sterm3(rz, csub(a1zp, a1), rx, csub(b1xp, b1), -ry, csub(b0yp, b0));
    s.s2 = sterm3(-rz, csub(b0, b0zm), rx, csub(a0xp, a0), ry, csub(a1, a1ym));
    s.s3 = sterm3(-rz, csub(b1, b1zm), rx, csub(a1, a1xm), ry, csub(a0yp, a0));
    return s;
}

// (2+1)D: u rows from v (Eqs. scheme2Deq, scheme3rdline):
//   S_u0 = rx(v0 - v0[i-1]) - i ry(v1 - v1[j-1])
//   S_u1 = rx(v1[i+1] - v1) - i ry(v0[j+1] - v0)
template <typename C, typename R>
__device__ __forceinline__ St2<C> stencil_u(R rx, R ry, C v0, C v0xm, C v0yp, C v1, C v1ym, C v1xp) {
    St2<C> s;
    s.s0 = sterm2(rx, csub(v0, v0xm), -ry, csub(v1, v1ym));
    s.s1 = sterm2(rx, csub(v1xp, v1), -ry, csub(v0yp, v0));
    return s;
}

// v rows from u (Eqs. scheme2ndline, scheme4thline):
//   S_v0 = rx(u0[i+1] - u0) + i ry(u1 - u1[j-1])
//   S_v1 = rx(u1 - u1[i-1]) + i ry(u0[j+1] - u0)
template <typename C, typename R>
__device__ __forceinline__ St2<C> stencil_v(R rx, R ry, C u0, C u0xp, C u0yp, C u1, C u1ym, C u1xm) {
    St2<C> s;
    s.s0 = sterm2(rx, csub(u0xp, u0), ry, csub(u1, u1ym));
    s.s1 = sterm2(rx, csub(u1, u1xm), ry, csub(u0yp, u0));
    return s;
}

}  // namespace dirac
