// Device helpers shared by the step and adjoint kernels.
#pragma once
#include "step.h"

namespace chns {

struct U3 {
    const double *a[3];
};
struct W3 {
    double *a[3];
};

inline U3 mk_u3(const double *const u[3]) { return U3{{u[0], u[1], u[2]}}; }
inline W3 mk_w3(double *const u[3]) { return W3{{u[0], u[1], u[2]}}; }

__device__ inline double dpsi(double p) { return p * p * p - p; }
__device__ inline double pullback(double p) { return fabs(p) <= 1.0 ? p : copysign(1.0, p); }
// derivative of the pull-back (1 inside (-1, 1), 0 outside)
__device__ inline double dpullback(double p) { return fabs(p) < 1.0 ? 1.0 : 0.0; }

#define CELL_LOOP(N) \
    for (int c = (int)(blockIdx.x * blockDim.x + threadIdx.x); c < (int)(N); c += (int)(gridDim.x * blockDim.x))

template <int DIM>
__device__ inline void cc(const Geo &g, int c, int &i, int &j, int &k) {
    if (DIM == 2)
        cell_coords2(g, c, i, j, k);
    else
        cell_coords(g, c, i, j, k);
}

// Mass flux m_b = A_b(alpha phi + beta) u_b + J_b / Pe on the face f of axis
// b (index ib of f along b), zero on wall faces.
template <int DIM>
__device__ inline double mflux(const Geo &g, const StepConst &k, const double *__restrict__ phi,
                               const double *__restrict__ mu, const double *__restrict__ ub, int b, int f, int ib) {
    if (f < 0) return 0.0;                       // unstored upper wall face
    if (!g.per[b] && ib == 0) return 0.0;        // stored wall face
    const int lo = nb_lo(g, f, ib, b);
    const double rl = k.alpha * phi[f] + k.beta, rlo = k.alpha * phi[lo] + k.beta;
    return (0.5 * (rl + rlo)) * ub[f] - (k.alpha / (k.Cn * k.Pe)) * ((mu[f] - mu[lo]) * k.ih);
}

__device__ inline int wrap_next(int ib, int n) { return ib + 1 < n ? ib + 1 : 0; }
__device__ inline int wrap_prev(int ib, int n) { return ib > 0 ? ib - 1 : n - 1; }


}  // namespace chns
