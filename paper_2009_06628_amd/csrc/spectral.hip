// Direct (spectral) solve of the Cahn-Hilliard system; see spectral.h.
#include <rocblas/rocblas.h>

#include <cmath>
#include <algorithm>
#include <utility>
#include <vector>

#include "spectral.h"

namespace chns {

void spectral_carve(Bump &B, const Geo &g, int dim, Spectral &S) {
    S.carved = 1;
    S.on = 0;
    S.dim = dim;
    S.blas = nullptr;
    for (int a = 0; a < 3; ++a) {
        S.n[a] = a < dim ? (int)g.n[a] : 1;
        S.per[a] = a < dim ? g.per[a] : 1;
        S.Q[a] = S.lam[a] = nullptr;
        if (a < dim && g.n[a] > kSpectralMaxN) S.carved = 0;
    }
    if (!S.carved) return;
    for (int a = 0; a < dim; ++a) {
        S.Q[a] = B.take<double>((size_t)S.n[a] * S.n[a]);
        S.lam[a] = B.take<double>((size_t)S.n[a]);
    }
}

// Eigenbasis of the 1D cell-centred second difference with spacing h on n
// cells.  Walled (Neumann: the flux through the wall faces is zero): column
// k = sqrt((k ? 2 : 1) / n) cos(pi k (j + 1/2) / n), eigenvalue
// -(4 / h^2) sin^2(pi k / (2 n)).  Periodic: the constant, then
// sqrt(2 / n) cos(2 pi k j / n) and sqrt(2 / n) sin(2 pi k j / n) for
// 0 < k < n / 2 (eigenvalue -(4 / h^2) sin^2(pi k / n) for both), then
// (-1)^j / sqrt(n) when n is even.  Angles are reduced exactly in integers
// before the trigonometric call.
void spectral_axis(int n, int per, double h, std::vector<double> &Q, std::vector<double> &lam) {
    const double pi = std::acos(-1.0), ih2 = 1.0 / (h * h);
    Q.assign((size_t)n * n, 0.0);
    lam.assign((size_t)n, 0.0);
    if (!per) {
        for (int k = 0; k < n; ++k) {
            const double s = std::sqrt((k ? 2.0 : 1.0) / n);
            for (int j = 0; j < n; ++j) {
                const long long m = ((long long)k * (2 * j + 1)) % (4LL * n);   // angle pi m / (2 n)
                Q[j + (size_t)n * k] = s * std::cos(pi * (double)m / (2.0 * n));
            }
            const double sn = std::sin(pi * k / (2.0 * n));
            lam[k] = -4.0 * ih2 * sn * sn;
        }
        return;
    }
    const double s0 = std::sqrt(1.0 / n), s1 = std::sqrt(2.0 / n);
    for (int j = 0; j < n; ++j) Q[j] = s0;
    lam[0] = 0.0;
    int col = 1;
    for (int k = 1; 2 * k < n; ++k, col += 2) {
        for (int j = 0; j < n; ++j) {
            const long long m = ((long long)k * j) % n;   // angle 2 pi m / n
            const double ang = 2.0 * pi * (double)m / n;
            Q[j + (size_t)n * col] = s1 * std::cos(ang);
            Q[j + (size_t)n * (col + 1)] = s1 * std::sin(ang);
        }
        const double sn = std::sin(pi * k / n);
        lam[col] = lam[col + 1] = -4.0 * ih2 * sn * sn;
    }
    if (n % 2 == 0) {
        for (int j = 0; j < n; ++j) Q[j + (size_t)n * col] = (j & 1) ? -s0 : s0;
        lam[col] = -4.0 * ih2;
    }
}

int spectral_init(Spectral &S, double h, std::string &err) {
    S.on = 0;
    if (!S.carved) return 0;
    std::vector<double> Q, lam;
    for (int a = 0; a < S.dim; ++a) {
        spectral_axis(S.n[a], S.per[a], h, Q, lam);
        hipError_t e = hipMemcpy(S.Q[a], Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(S.lam[a], lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            err = std::string("spectral basis upload: ") + hipGetErrorString(e);
            return 1;
        }
    }
    rocblas_handle hb = nullptr;
    const rocblas_status st = rocblas_create_handle(&hb);
    if (st != rocblas_status_success) {
        err = std::string("rocblas_create_handle: ") + rocblas_status_to_string(st);
        return 1;
    }
    S.blas = hb;
    S.on = 1;
    return 0;
}

void spectral_release(Spectral &S) {
    if (S.blas) (void)rocblas_destroy_handle((rocblas_handle)S.blas);
    S.blas = nullptr;
    S.on = 0;
}

// t /= 1 - a lam + b lam^2, lam = lam_x(i) + lam_y(j) + lam_z(k)
__global__ void __launch_bounds__(kBlock) k_spectral_scale(Geo g, const double *__restrict__ lx,
                                                           const double *__restrict__ ly,
                                                           const double *__restrict__ lz, double a, double b,
                                                           double *__restrict__ t) {
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int c = xcd_block() * (int)blockDim.x + (int)threadIdx.x; c < (int)g.N; c += stride) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        const double lam = lx[i] + ly[j] + (lz ? lz[k] : 0.0);
        t[c] = t[c] / (1.0 - a * lam + b * lam * lam);
    }
}

#define BLASCHK(call)                                                    \
    do {                                                                 \
        const rocblas_status st_ = (call);                               \
        if (st_ != rocblas_status_success) {                             \
            err = std::string("rocBLAS: ") + rocblas_status_to_string(st_); \
            return hipErrorLaunchFailure;                                \
        }                                                                \
    } while (0)

hipError_t spectral_solve(Spectral &S, double a, double b, const double *r, double *x, double *t0, double *t1,
                          hipStream_t st, std::string &err) {
    rocblas_handle hb = (rocblas_handle)S.blas;
    const int nx = S.n[0], ny = S.n[1], nz = S.dim == 3 ? S.n[2] : 1;
    const rocblas_stride sxy = (rocblas_stride)nx * ny;
    const double one = 1.0, zero = 0.0;
    const rocblas_operation N = rocblas_operation_none, T = rocblas_operation_transpose;
    // the field is column-major nx x (ny nz) (x fastest); each axis
    // transform multiplies by that axis' basis
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_prof) {
        const double N3 = (double)nx * ny * nz;
        prof_slot(K_CH_SPECTRAL, 8.0 * N3 * 2.0 * (2 * S.dim + 1), &e0, &e1);
        (void)hipEventRecord(e0, st);
    }
    BLASCHK(rocblas_set_stream(hb, st));
    // forward: x, then y (slab by slab), then z
    BLASCHK(rocblas_dgemm(hb, T, N, nx, ny * nz, nx, &one, S.Q[0], nx, r, nx, &zero, t0, nx));
    BLASCHK(rocblas_dgemm_strided_batched(hb, N, N, nx, ny, ny, &one, t0, nx, sxy, S.Q[1], ny, 0, &zero, t1, nx,
                                          sxy, nz));
    double *cur = t1, *oth = t0;
    if (S.dim == 3) {
        BLASCHK(rocblas_dgemm(hb, N, N, nx * ny, nz, nz, &one, cur, nx * ny, S.Q[2], nz, &zero, oth, nx * ny));
        std::swap(cur, oth);
    }
    Geo g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.per[0] = g.per[1] = g.per[2] = 1;
    g.N = (long long)nx * ny * nz;
    hipLaunchKernelGGL(k_spectral_scale, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, (const double *)S.lam[0],
                       (const double *)S.lam[1], (const double *)(S.dim == 3 ? S.lam[2] : nullptr), a, b, cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // inverse: z, y, x
    if (S.dim == 3) {
        BLASCHK(rocblas_dgemm(hb, N, T, nx * ny, nz, nz, &one, cur, nx * ny, S.Q[2], nz, &zero, oth, nx * ny));
        std::swap(cur, oth);
    }
    BLASCHK(rocblas_dgemm_strided_batched(hb, N, T, nx, ny, ny, &one, cur, nx, sxy, S.Q[1], ny, 0, &zero, oth, nx,
                                          sxy, nz));
    std::swap(cur, oth);
    BLASCHK(rocblas_dgemm(hb, N, N, nx, ny * nz, nx, &one, S.Q[0], nx, cur, nx, &zero, x, nx));
    if (e1) (void)hipEventRecord(e1, st);
    return hipGetLastError();
}

// t_p /= 1 - a_p lam + b_p lam^2, lam = (lam_x(i) + lam_y(j)) / h_p^2;
// blockIdx.y = problem of the group
__global__ void __launch_bounds__(kBlock) k_spectral_scale_batch(int nx, int ny, const double *__restrict__ lx,
                                                                 const double *__restrict__ ly,
                                                                 const double *__restrict__ abh,
                                                                 double *const *__restrict__ t) {
    const int p = (int)blockIdx.y;
    const double a = abh[3 * p], b = abh[3 * p + 1], ih2 = abh[3 * p + 2];
    double *tp = t[p];
    const int n = nx * ny, stride = (int)(gridDim.x * blockDim.x);
    for (int c = (int)(blockIdx.x * blockDim.x + threadIdx.x); c < n; c += stride) {
        const int j = c / nx, i = c - j * nx;
        const double lam = ih2 * (lx[i] + ly[j]);
        tp[c] = tp[c] / (1.0 - a * lam + b * lam * lam);
    }
}

hipError_t spectral_batch_solve(void *blas, const std::vector<SpecGroup> &groups, hipStream_t st, std::string &err) {
    rocblas_handle hb = (rocblas_handle)blas;
    const double one = 1.0, zero = 0.0;
    const rocblas_operation N = rocblas_operation_none, T = rocblas_operation_transpose;
    BLASCHK(rocblas_set_stream(hb, st));
    for (const SpecGroup &G : groups) {
        const int nx = G.nx, ny = G.ny, m = G.m;
        // column-major nx x ny per problem (x fastest): t0 = Qx^T r, t1 = t0 Qy
        BLASCHK(rocblas_dgemm_batched(hb, T, N, nx, ny, nx, &one, G.Qx, nx, G.r, nx, &zero, G.t0, nx, m));
        BLASCHK(rocblas_dgemm_batched(hb, N, N, nx, ny, ny, &one, (const double *const *)G.t0, nx, G.Qy, ny, &zero,
                                      G.t1, nx, m));
        const int bx = std::min((nx * ny + kBlock - 1) / kBlock, 64);
        hipLaunchKernelGGL(k_spectral_scale_batch, dim3(bx, m), dim3(kBlock), 0, st, nx, ny, (const double *)G.lam[0],
                           (const double *)G.lam[1], (const double *)G.abh, (double *const *)G.t1);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // back: t0 = t1 Qy^T, x = Qx t0
        BLASCHK(rocblas_dgemm_batched(hb, N, T, nx, ny, ny, &one, (const double *const *)G.t1, nx, G.Qy, ny, &zero,
                                      G.t0, nx, m));
        BLASCHK(rocblas_dgemm_batched(hb, N, N, nx, ny, nx, &one, G.Qx, nx, (const double *const *)G.t0, nx, &zero,
                                      G.x, nx, m));
    }
    return hipGetLastError();
}

}  // namespace chns
