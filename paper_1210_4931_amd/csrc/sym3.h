// Symmetric 3x3 blocks of the T, Q, U noise precision (Sect. 3: the pixel-space quantities
// of the polarized problem are 3x3 blocks per pixel), stored packed as (a, b, c, d, e, f) =
// [[a, b, c], [b, d, e], [c, e, f]], and the messenger pixel update of Eq. (3) with them.
#pragma once

#include <hip/hip_runtime.h>

namespace mfwf {

struct Sym3 {
    double a, b, c, d, e, f;  // [[a, b, c], [b, d, e], [c, e, f]]
};

__device__ __forceinline__ Sym3 load_sym3(const double *__restrict__ M6, long p) {
    const double *q = M6 + 6 * p;
    return Sym3{q[0], q[1], q[2], q[3], q[4], q[5]};
}

__device__ __forceinline__ void sym3_mv(const Sym3 &M, const double x[3], double y[3]) {
    y[0] = M.a * x[0] + M.b * x[1] + M.c * x[2];
    y[1] = M.b * x[0] + M.d * x[1] + M.e * x[2];
    y[2] = M.c * x[0] + M.e * x[1] + M.f * x[2];
}

// x = M^{-1} y with every product-sum an explicit fma (no contraction left to the compiler)
__device__ __forceinline__ void sym3_solve_fma(const Sym3 &M, const double y[3], double x[3]) {
    const double A = fma(M.d, M.f, -(M.e * M.e)), B = fma(M.c, M.e, -(M.b * M.f));
    const double C = fma(M.b, M.e, -(M.c * M.d)), D = fma(M.a, M.f, -(M.c * M.c));
    const double E = fma(M.b, M.c, -(M.a * M.e)), F = fma(M.a, M.d, -(M.b * M.b));
    const double det = fma(M.a, A, fma(M.b, B, M.c * C));
    x[0] = fma(A, y[0], fma(B, y[1], C * y[2])) / det;
    x[1] = fma(B, y[0], fma(D, y[1], E * y[2])) / det;
    x[2] = fma(C, y[0], fma(E, y[1], F * y[2])) / det;
}

// Eq. (3) at one pixel of the T, Q, U problem:
//   t = [1 + (lam - 1) tau M]^{-1} [lam tau rho + (1 - tau M) s],
// lt = lam tau, l1t = (lam - 1) tau.  Every product-sum is an explicit fma, so that each
// kernel that forms t (the separate pixel kernel, the chained ring step) rounds it alike.
__device__ __forceinline__ void pol_messenger_pixel(const Sym3 &M, const double s[3],
                                                    const double rho[3], double lam, double lt,
                                                    double l1t, double tau, double t[3]) {
    const double Ms0 = fma(M.a, s[0], fma(M.b, s[1], M.c * s[2]));
    const double Ms1 = fma(M.b, s[0], fma(M.d, s[1], M.e * s[2]));
    const double Ms2 = fma(M.c, s[0], fma(M.e, s[1], M.f * s[2]));
    const double r[3] = {fma(-tau, Ms0, fma(lt, rho[0], s[0])), fma(-tau, Ms1, fma(lt, rho[1], s[1])),
                         fma(-tau, Ms2, fma(lt, rho[2], s[2]))};
    if (lam != 1.0) {
        const Sym3 A{fma(l1t, M.a, 1.0), l1t * M.b, l1t * M.c, fma(l1t, M.d, 1.0), l1t * M.e,
                     fma(l1t, M.f, 1.0)};
        sym3_solve_fma(A, r, t);
    } else {
        t[0] = r[0];
        t[1] = r[1];
        t[2] = r[2];
    }
}

}  // namespace mfwf
