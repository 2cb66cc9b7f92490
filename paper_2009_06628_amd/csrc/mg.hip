// Matrix-free multigrid-preconditioned conjugate gradients on the uniform
// grid (gfx950).  The elliptic solver is not fixed by the paper (its coupled
// system goes to Krylov solvers with ASM / algebraic multigrid
// preconditioners); this is a geometric cell-centred multigrid:
//   * operator       (A x)_c = s_c x_c + sum_b cs_b(c)(x_c - x_{c-e_b})
//                                       + cs_b(c+e_b)(x_c - x_{c+e_b}),
//   * smoother       red-black Gauss-Seidel, pre (red, black), post (black,
//                    red): the V-cycle is a symmetric positive definite
//                    preconditioner;
//   * transfers      cell-centred bilinear / trilinear prolongation P and
//                    full-weighting restriction R = P^T / 2^d;
//   * coarse levels  re-discretised: s averaged over children, face
//                    coefficients averaged over the fine faces of a coarse
//                    face and divided by 4 (spacing doubles);
//   * coarsest       explicit inverse (Gauss-Jordan, one workgroup), with a
//                    rank-one shift tau 1 1^T for the singular pressure
//                    operator;
//   * reductions     deterministic: fixed grid-stride partition, wave
//                    shuffles, fixed-order final sum by the last block.
// PCG scalars stay on the device; every iteration kernel returns at once
// when the device-side "done" flag is set, so the host launches iterations
// in chunks and checks the flag once per chunk.
#include "solvers.h"

namespace chns {

// ---------------------------------------------------------------------------
// stencil helpers
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ inline void op_at(const Level<T> &L, const T *__restrict__ x, long long c, int i, int j, int k,
                             double &Ax, double &diag, double &offsum) {
    // Ax = (A x)_c, diag = A_cc, offsum = sum of cs * x_nb (for Gauss-Seidel)
    const Geo &g = L.g;
    const double xc = (double)x[c];
    double d = (double)L.s[c];
    double off = 0.0;
    const int ia[3] = {i, j, k};
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        long long lo = nb_lo(g, c, ia[b], b);
        long long hi = nb_hi(g, c, ia[b], b);
        if (lo >= 0) {
            double w = (double)L.cs[b][c];
            d += w;
            off += w * (double)x[lo];
        }
        if (hi >= 0) {
            double w = (double)L.cs[b][hi];
            d += w;
            off += w * (double)x[hi];
        }
    }
    diag = d;
    offsum = off;
    Ax = d * xc - off;
}

// ---------------------------------------------------------------------------
// V-cycle kernels
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_rbgs(Level<T> L, const T *__restrict__ b, T *__restrict__ x,
                                                 int color, int zero_init, const int *__restrict__ done) {
    if (*done) return;
    const Geo g = L.g;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        const int col = (i + j + k) & 1;
        if (zero_init) {
            if (col != color) {
                x[c] = (T)0;
                continue;
            }
            double d = (double)L.s[c];
            const int ia[3] = {i, j, k};
#pragma unroll
            for (int bb = 0; bb < DIM; ++bb) {
                if (nb_lo(g, c, ia[bb], bb) >= 0) d += (double)L.cs[bb][c];
                long long hi = nb_hi(g, c, ia[bb], bb);
                if (hi >= 0) d += (double)L.cs[bb][hi];
            }
            x[c] = (T)((double)b[c] / d);
            continue;
        }
        if (col != color) continue;
        double Ax, d, off;
        op_at<T, DIM>(L, x, c, i, j, k, Ax, d, off);
        x[c] = (T)(((double)b[c] + off) / d);
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_residual(Level<T> L, const T *__restrict__ b, const T *__restrict__ x,
                                                     T *__restrict__ r, const int *__restrict__ done) {
    if (*done) return;
    const Geo g = L.g;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        double Ax, d, off;
        op_at<T, DIM>(L, x, c, i, j, k, Ax, d, off);
        r[c] = (T)((double)b[c] - Ax);
    }
}

// Per-axis weights of the cell-centred linear prolongation: fine cell f
// takes 3/4 of its parent f/2 and 1/4 of the coarse neighbour on its side
// (f even: parent - 1, f odd: parent + 1); past a walled boundary the
// neighbour is replaced by the parent (weight 1).
__device__ inline void prolong_axis(int f, int nc, int per, int &c0, double &w0, int &c1, double &w1) {
    const int p = f >> 1;
    int q = (f & 1) ? p + 1 : p - 1;
    c0 = p;
    if (q < 0 || q >= nc) {
        if (per) {
            q = (q + nc) % nc;
        } else {
            w0 = 1.0;
            c1 = p;
            w1 = 0.0;
            return;
        }
    }
    w0 = 0.75;
    c1 = q;
    w1 = 0.25;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_prolong_add(Geo gf, Geo gc, const T *__restrict__ xc, T *__restrict__ xf,
                                                        const int *__restrict__ done) {
    if (*done) return;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < gf.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(gf, c, i, j, k);
        int ci[3][2];
        double wi[3][2];
        const int fi[3] = {i, j, k};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a < DIM) {
                prolong_axis(fi[a], gc.n[a], gc.per[a], ci[a][0], wi[a][0], ci[a][1], wi[a][1]);
            } else {
                ci[a][0] = ci[a][1] = 0;
                wi[a][0] = 1.0;
                wi[a][1] = 0.0;
            }
        }
        double v = 0.0;
#pragma unroll
        for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const double w = wi[0][dx] * wi[1][dy] * wi[2][dz];
                    const long long idx = ci[0][dx] + (long long)gc.n[0] * (ci[1][dy] + (long long)gc.n[1] * ci[2][dz]);
                    v += w * (double)xc[idx];
                }
        xf[c] = (T)((double)xf[c] + v);
    }
}

// R = P^T / 2^d: coarse cell I gathers the fine cells whose prolongation
// stencil contains I (children 2I, 2I+1 and the outer neighbours 2I-1, 2I+2).
__device__ inline int restrict_axis(int I, int nc, int nf, int per, int *fidx, double *w) {
    int m = 0;
    for (int f = 2 * I - 1; f <= 2 * I + 2; ++f) {
        int ff = f;
        if (ff < 0 || ff >= nf) {
            if (!per) continue;
            ff = (ff + nf) % nf;
        }
        int c0, c1;
        double w0, w1;
        prolong_axis(ff, nc, per, c0, w0, c1, w1);
        double wt = 0.0;
        if (c0 == I) wt += w0;
        if (c1 == I) wt += w1;
        if (wt != 0.0) {
            fidx[m] = ff;
            w[m] = wt;
            ++m;
        }
    }
    return m;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_restrict(Geo gf, Geo gc, const T *__restrict__ rf, T *__restrict__ bc,
                                                     const int *__restrict__ done) {
    if (*done) return;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < gc.N;
         c += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        cell_coords(gc, c, I, J, K);
        int fx[4], fy[4], fz[4];
        double wx[4], wy[4], wz[4];
        const int mx = restrict_axis(I, gc.n[0], gf.n[0], gc.per[0], fx, wx);
        const int my = restrict_axis(J, gc.n[1], gf.n[1], gc.per[1], fy, wy);
        int mz = 1;
        fz[0] = 0;
        wz[0] = 1.0;
        if (DIM == 3) mz = restrict_axis(K, gc.n[2], gf.n[2], gc.per[2], fz, wz);
        double v = 0.0;
        for (int a = 0; a < mz; ++a)
            for (int bq = 0; bq < my; ++bq) {
                const long long row = (long long)gf.n[0] * (fy[bq] + (long long)gf.n[1] * fz[a]);
                const double wyz = wy[bq] * wz[a];
                for (int e = 0; e < mx; ++e) v += wx[e] * wyz * (double)rf[row + fx[e]];
            }
        bc[c] = (T)(v * (DIM == 3 ? 0.125 : 0.25));
    }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_coarse_solve(int n, const double *__restrict__ Ainv, const T *__restrict__ b,
                                                       T *__restrict__ x, const int *__restrict__ done) {
    if (*done) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v = 0.0;
        const double *row = Ainv + (long long)i * n;
        for (int j = 0; j < n; ++j) v += row[j] * (double)b[j];
        x[i] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_coarsen(Level<T> F, Level<T> C) {
    const Geo gf = F.g, gc = C.g;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < gc.N;
         c += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        cell_coords(gc, c, I, J, K);
        const int I3[3] = {I, J, K};
        double s = 0.0;
        double cs[3] = {0.0, 0.0, 0.0};
        for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int d3[3] = {dx, dy, dz};
                    const long long f = (2 * I + dx) + (long long)gf.n[0] * ((2 * J + dy) + (long long)gf.n[1] * (2 * K + dz));
                    s += (double)F.s[f];
#pragma unroll
                    for (int b = 0; b < DIM; ++b)
                        if (d3[b] == 0) cs[b] += (double)F.cs[b][f];   // fine faces on the coarse lower b-face
                }
        (void)I3;
        const double nchild = (DIM == 3) ? 8.0 : 4.0;
        C.s[c] = (T)(s / nchild);
#pragma unroll
        for (int b = 0; b < DIM; ++b) C.cs[b][c] = (T)(cs[b] / (nchild * 0.5) * 0.25);
    }
}

// Assemble the coarsest operator densely into aug = [A | I] and invert it
// by Gauss-Jordan elimination (SPD: no pivoting), one workgroup.
template <typename T, int DIM>
__global__ void __launch_bounds__(1024) k_dense_inverse(Level<T> L, int singular, double *__restrict__ aug,
                                                        double *__restrict__ Ainv) {
    const Geo g = L.g;
    const int n = (int)g.N;
    const int w = 2 * n;
    __shared__ double f[kMaxCoarse];
    __shared__ double red[1024 / kWave];
    __shared__ double sh_piv, sh_tau;
    for (long long e = threadIdx.x; e < (long long)n * w; e += blockDim.x) aug[e] = 0.0;
    __syncthreads();
    double dsum = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        const int ia[3] = {i, j, k};
        double d = (double)L.s[c];
        for (int b = 0; b < DIM; ++b) {
            long long lo = nb_lo(g, c, ia[b], b);
            long long hi = nb_hi(g, c, ia[b], b);
            if (lo >= 0) {
                double cw = (double)L.cs[b][c];
                d += cw;
                aug[(long long)c * w + lo] -= cw;
            }
            if (hi >= 0) {
                double cw = (double)L.cs[b][hi];
                d += cw;
                aug[(long long)c * w + hi] -= cw;
            }
        }
        aug[(long long)c * w + c] += d;
        aug[(long long)c * w + n + c] = 1.0;
        dsum += d;
    }
    double tot = block_sum(dsum, red);
    if (threadIdx.x == 0) sh_tau = singular ? (tot / n) / n : 0.0;
    __syncthreads();
    if (singular) {
        const double tau = sh_tau;
        for (long long e = threadIdx.x; e < (long long)n * n; e += blockDim.x) aug[(e / n) * w + (e % n)] += tau;
    }
    for (int kk = 0; kk < n; ++kk) {
        __syncthreads();
        if (threadIdx.x == 0) sh_piv = 1.0 / aug[(long long)kk * w + kk];
        for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = aug[(long long)i * w + kk];
        __syncthreads();
        const double pinv = sh_piv;
        for (int jj = threadIdx.x; jj < w; jj += blockDim.x) aug[(long long)kk * w + jj] *= pinv;
        __syncthreads();
        for (long long e = threadIdx.x; e < (long long)n * w; e += blockDim.x) {
            const int i = (int)(e / w), jj = (int)(e % w);
            if (i != kk) aug[e] -= f[i] * aug[(long long)kk * w + jj];
        }
    }
    __syncthreads();
    for (long long e = threadIdx.x; e < (long long)n * n; e += blockDim.x)
        Ainv[e] = aug[(e / n) * w + n + (e % n)];
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------

// Lap(x) at c for the CH operator (unit-spacing coefficients cs = 1/h^2 in
// every direction, walled axes Neumann).  x given by a functor.
template <int DIM, typename F>
__device__ inline double lap_at(const Geo &g, long long c, int i, int j, int k, double ih2, F val) {
    const int ia[3] = {i, j, k};
    const double xc = val(c);
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        long long lo = nb_lo(g, c, ia[b], b);
        long long hi = nb_hi(g, c, ia[b], b);
        if (lo >= 0) acc += val(lo) - xc;
        if (hi >= 0) acc += val(hi) - xc;
    }
    return acc * ih2;
}

// first: p_new = z, otherwise p_new = z + beta p_old; then q = A p_new
// (slot operator), partial p.q; the last block sets alpha = rz / pq.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_apply_slot(Level<T> L, const T *__restrict__ z, const T *__restrict__ pold,
                                                           T *__restrict__ pnew, T *__restrict__ q, Scal *sc,
                                                           double *part, unsigned int *counter) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    const double beta = sc->beta;
    const double zm = sc->zmean;
    const Geo g = L.g;
    double acc = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        const int ia[3] = {i, j, k};
        const double pc = ((double)z[c] - zm) + (beta != 0.0 ? beta * (double)pold[c] : 0.0);
        double d = (double)L.s[c];
        double off = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            long long lo = nb_lo(g, c, ia[b], b);
            long long hi = nb_hi(g, c, ia[b], b);
            if (lo >= 0) {
                double w = (double)L.cs[b][c];
                d += w;
                off += w * (((double)z[lo] - zm) + (beta != 0.0 ? beta * (double)pold[lo] : 0.0));
            }
            if (hi >= 0) {
                double w = (double)L.cs[b][hi];
                d += w;
                off += w * (((double)z[hi] - zm) + (beta != 0.0 ? beta * (double)pold[hi] : 0.0));
            }
        }
        const double qc = d * pc - off;
        pnew[c] = (T)pc;
        q[c] = (T)qc;
        acc += pc * qc;
    }
    double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(counter)) {
        double tot = sum_partials(part, gridDim.x, lds);
        if (threadIdx.x == 0) {
            sc->pq = tot;
            sc->alpha = (tot != 0.0) ? sc->rz / tot : 0.0;
            *counter = 0;
        }
    }
}

// CH operator, first half: p_new = z + beta p_old, t = L p_new.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_ch_lap(Geo g, double ih2, const T *__restrict__ z, const T *__restrict__ pold,
                                                       T *__restrict__ pnew, T *__restrict__ t, const Scal *sc) {
    if (sc->done) return;
    const double beta = sc->beta;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        auto val = [&](long long e) { return (double)z[e] + (beta != 0.0 ? beta * (double)pold[e] : 0.0); };
        pnew[c] = (T)val(c);
        t[c] = (T)lap_at<DIM>(g, c, i, j, k, ih2, val);
    }
}

// CH operator, second half: q = p - a t + b L t; partial p.q, alpha.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_ch_apply(Geo g, double ih2, double ca, double cb, const T *__restrict__ p,
                                                         const T *__restrict__ t, T *__restrict__ q, Scal *sc,
                                                         double *part, unsigned int *counter) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    double acc = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        auto val = [&](long long e) { return (double)t[e]; };
        const double pc = (double)p[c];
        const double qc = pc - ca * (double)t[c] + cb * lap_at<DIM>(g, c, i, j, k, ih2, val);
        q[c] = (T)qc;
        acc += pc * qc;
    }
    double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(counter)) {
        double tot = sum_partials(part, gridDim.x, lds);
        if (threadIdx.x == 0) {
            sc->pq = tot;
            sc->alpha = (tot != 0.0) ? sc->rz / tot : 0.0;
            *counter = 0;
        }
    }
}

// x += alpha p, r -= alpha q, partial r.r; the last block tests convergence.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_update(long long N, const T *__restrict__ p, const T *__restrict__ q,
                                                       T *__restrict__ x, T *__restrict__ r, Scal *sc, double *part,
                                                       unsigned int *counter) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    const double alpha = sc->alpha;
    double acc = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        x[c] = (T)((double)x[c] + alpha * (double)p[c]);
        const double rc = (double)r[c] - alpha * (double)q[c];
        r[c] = (T)rc;
        acc += rc * rc;
    }
    double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(counter)) {
        double tot = sum_partials(part, gridDim.x, lds);
        if (threadIdx.x == 0) {
            sc->rr = tot;
            sc->iter += 1;
            if (!isfinite(tot)) {
                sc->nonfinite = 1;
                sc->done = 1;
            } else if (tot <= sc->rtol2 * sc->bb) {
                sc->done = 1;
            } else if (sc->iter >= sc->max_iter) {
                sc->unconverged = 1;
                sc->done = 1;
            }
            *counter = 0;
        }
    }
}

// rz_new = r.(z - zmean); beta = rz_new / rz (0 on the first call); rz = rz_new.
// For a singular (pure Neumann / periodic) operator the preconditioned vector
// is projected onto the range: zmean = mean(z), otherwise zmean = 0.  The
// V-cycle amplifies the constant mode, and without the projection rounding
// noise in that mode destroys the conjugacy of the search directions.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_rz(long long N, const T *__restrict__ r, const T *__restrict__ z, Scal *sc,
                                                   double *part0, double *part1, double *part2, unsigned int *counter,
                                                   int first, int singular) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    double arz = 0.0, az = 0.0, ar = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        const double rc = (double)r[c], zc = (double)z[c];
        arz += rc * zc;
        az += zc;
        ar += rc;
    }
    double s0 = block_sum(arz, lds);
    double s1 = singular ? block_sum(az, lds) : 0.0;
    double s2 = singular ? block_sum(ar, lds) : 0.0;
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = s0;
        part1[blockIdx.x] = s1;
        part2[blockIdx.x] = s2;
    }
    if (last_block(counter)) {
        double trz = sum_partials(part0, gridDim.x, lds);
        double tz = singular ? sum_partials(part1, gridDim.x, lds) : 0.0;
        double tr = singular ? sum_partials(part2, gridDim.x, lds) : 0.0;
        if (threadIdx.x == 0) {
            const double zm = singular ? tz / (double)N : 0.0;
            const double rz = trz - zm * tr;
            sc->zmean = zm;
            sc->beta = (first || sc->rz == 0.0) ? 0.0 : rz / sc->rz;
            sc->rz = rz;
            if (!isfinite(rz)) {
                sc->nonfinite = 1;
                sc->done = 1;
            }
            *counter = 0;
        }
    }
}

// r = b - A x (slot operator), partials b.b and r.r; initialises the scalars.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_init_slot(Level<T> L, const T *__restrict__ b, const T *__restrict__ x,
                                                          T *__restrict__ r, Scal *sc, double *part0, double *part1,
                                                          unsigned int *counter, double rtol, int max_iter) {
    __shared__ double lds[kBlock / kWave];
    const Geo g = L.g;
    double bb = 0.0, rr = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        double Ax, d, off;
        op_at<T, DIM>(L, x, c, i, j, k, Ax, d, off);
        const double bc = (double)b[c];
        const double rc = bc - Ax;
        r[c] = (T)rc;
        bb += bc * bc;
        rr += rc * rc;
    }
    double s0 = block_sum(bb, lds);
    double s1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = s0;
        part1[blockIdx.x] = s1;
    }
    if (last_block(counter)) {
        double tb = sum_partials(part0, gridDim.x, lds);
        double tr = sum_partials(part1, gridDim.x, lds);
        if (threadIdx.x == 0) {
            sc->bb = tb > tr ? tb : tr;
            sc->rr = tr;
            sc->rtol2 = rtol * rtol;
            sc->iter = 0;
            sc->max_iter = max_iter;
            sc->unconverged = 0;
            sc->nonfinite = 0;
            sc->beta = 0.0;
            sc->rz = 0.0;
            sc->zmean = 0.0;
            sc->done = 0;
            if (!isfinite(tr) || !isfinite(tb)) {
                sc->nonfinite = 1;
                sc->done = 1;
            } else if (tr <= sc->rtol2 * sc->bb) {
                sc->done = 1;
            }
            *counter = 0;
        }
    }
}

// CH init: t = L x computed first by k_ch_lap_plain; r = b - (x - a t + b L t).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_ch_lap_plain(Geo g, double ih2, const T *__restrict__ x, T *__restrict__ t) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        auto val = [&](long long e) { return (double)x[e]; };
        t[c] = (T)lap_at<DIM>(g, c, i, j, k, ih2, val);
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_init_ch(Geo g, double ih2, double ca, double cb, const T *__restrict__ b,
                                                        const T *__restrict__ x, const T *__restrict__ t, T *__restrict__ r,
                                                        Scal *sc, double *part0, double *part1, unsigned int *counter,
                                                        double rtol, int max_iter) {
    __shared__ double lds[kBlock / kWave];
    double bb = 0.0, rr = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        auto val = [&](long long e) { return (double)t[e]; };
        const double Mx = (double)x[c] - ca * (double)t[c] + cb * lap_at<DIM>(g, c, i, j, k, ih2, val);
        const double bc = (double)b[c];
        const double rc = bc - Mx;
        r[c] = (T)rc;
        bb += bc * bc;
        rr += rc * rc;
    }
    double s0 = block_sum(bb, lds);
    double s1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = s0;
        part1[blockIdx.x] = s1;
    }
    if (last_block(counter)) {
        double tb = sum_partials(part0, gridDim.x, lds);
        double tr = sum_partials(part1, gridDim.x, lds);
        if (threadIdx.x == 0) {
            sc->bb = tb > tr ? tb : tr;
            sc->rr = tr;
            sc->rtol2 = rtol * rtol;
            sc->iter = 0;
            sc->max_iter = max_iter;
            sc->unconverged = 0;
            sc->nonfinite = 0;
            sc->beta = 0.0;
            sc->rz = 0.0;
            sc->zmean = 0.0;
            sc->done = 0;
            if (!isfinite(tr) || !isfinite(tb)) {
                sc->nonfinite = 1;
                sc->done = 1;
            } else if (tr <= sc->rtol2 * sc->bb) {
                sc->done = 1;
            }
            *counter = 0;
        }
    }
}

// mean removal: partial sums, then subtract (two kernels, deterministic)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum(long long N, const T *__restrict__ x, double *part, unsigned int *counter,
                                                double *out) {
    __shared__ double lds[kBlock / kWave];
    double acc = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x)
        acc += (double)x[c];
    double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    if (last_block(counter)) {
        double tot = sum_partials(part, gridDim.x, lds);
        if (threadIdx.x == 0) {
            *out = tot;
            *counter = 0;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_mean(long long N, T *__restrict__ x, const double *__restrict__ sum) {
    const double m = *sum / (double)N;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x)
        x[c] = (T)((double)x[c] - m);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_slot_apply(Level<T> L, const T *__restrict__ x, T *__restrict__ y) {
    const Geo g = L.g;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < g.N;
         c += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        double Ax, d, off;
        op_at<T, DIM>(L, x, c, i, j, k, Ax, d, off);
        y[c] = (T)Ax;
    }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)

template <typename T, int DIM>
static void mg_setup_d(Slot<T> &S, hipStream_t st) {
    constexpr double W = sizeof(T);
    for (int l = 0; l + 1 < S.nlev; ++l)
        LAUNCH(K_MG_SETUP, W * (1 + DIM) * (S.lev[l].g.N + S.lev[l + 1].g.N), (k_coarsen<T, DIM>), S.lev[l + 1].g.N, st,
               S.lev[l], S.lev[l + 1]);
    const Level<T> &C = S.lev[S.nlev - 1];
    TLAUNCH(K_MG_SETUP, 8.0 * 3.0 * C.g.N * C.g.N, (k_dense_inverse<T, DIM>), dim3(1), dim3(1024), st, C, S.singular,
            (double *)S.aug, (double *)S.Ainv);
}

template <typename T>
void mg_setup(Slot<T> &S, int dim, hipStream_t st) {
    if (dim == 2)
        mg_setup_d<T, 2>(S, st);
    else
        mg_setup_d<T, 3>(S, st);
}

template <typename T, int DIM>
static void vcycle_d(Slot<T> &S, const T *b0, T *x0, const int *done, hipStream_t st) {
    constexpr double W = sizeof(T);
    const int L = S.nlev;
    for (int l = 0; l < L - 1; ++l) {
        Level<T> &lv = S.lev[l];
        const T *b = l == 0 ? b0 : lv.b;
        T *x = l == 0 ? x0 : lv.x;
        const long long N = lv.g.N;
        LAUNCH(K_SMOOTH, W * (3 + DIM) * N, (k_rbgs<T, DIM>), N, st, lv, b, x, 0, 1, done);
        LAUNCH(K_SMOOTH, W * (3.5 + DIM) * N, (k_rbgs<T, DIM>), N, st, lv, b, x, 1, 0, done);
        LAUNCH(K_RESIDUAL, W * (4 + DIM) * N, (k_residual<T, DIM>), N, st, lv, b, (const T *)x, lv.r, done);
        LAUNCH(K_RESTRICT, W * (N + S.lev[l + 1].g.N), (k_restrict<T, DIM>), S.lev[l + 1].g.N, st, lv.g, S.lev[l + 1].g,
               (const T *)lv.r, S.lev[l + 1].b, done);
    }
    {
        Level<T> &lc = S.lev[L - 1];
        const T *b = L == 1 ? b0 : lc.b;
        T *x = L == 1 ? x0 : lc.x;
        TLAUNCH(K_COARSE_SOLVE, 8.0 * lc.g.N * lc.g.N + W * 2.0 * lc.g.N, (k_coarse_solve<T>), dim3(1), dim3(1024), st,
                (int)lc.g.N, (const double *)S.Ainv, b, x, done);
    }
    for (int l = L - 2; l >= 0; --l) {
        Level<T> &lv = S.lev[l];
        const T *b = l == 0 ? b0 : lv.b;
        T *x = l == 0 ? x0 : lv.x;
        const long long N = lv.g.N;
        LAUNCH(K_PROLONG, W * (2 * N + S.lev[l + 1].g.N), (k_prolong_add<T, DIM>), N, st, lv.g, S.lev[l + 1].g,
               (const T *)S.lev[l + 1].x, x, done);
        LAUNCH(K_SMOOTH, W * (3.5 + DIM) * N, (k_rbgs<T, DIM>), N, st, lv, b, x, 1, 0, done);
        LAUNCH(K_SMOOTH, W * (3.5 + DIM) * N, (k_rbgs<T, DIM>), N, st, lv, b, x, 0, 0, done);
    }
}

template <typename T>
void mg_vcycle(Slot<T> &S, int dim, const T *b0, T *x0, const int *done, hipStream_t st) {
    if (dim == 2)
        vcycle_d<T, 2>(S, b0, x0, done, st);
    else
        vcycle_d<T, 3>(S, b0, x0, done, st);
}

template <typename T, int DIM>
static void precond_d(Slot<T> &S, OpKind kind, const T *r, T *z, T *tmp, const int *done, hipStream_t st) {
    if (kind == OP_CH) {
        // M ~ (I - c L)^2 with c = sqrt(b): two V-cycles of the slot operator
        vcycle_d<T, DIM>(S, r, tmp, done, st);
        vcycle_d<T, DIM>(S, tmp, z, done, st);
    } else {
        vcycle_d<T, DIM>(S, r, z, done, st);
    }
}

template <typename T, int DIM>
static hipError_t pcg_d(Slot<T> &S, OpKind kind, ChOp ch, const T *b, T *x, double rtol, int max_iter, int predict,
                        Red &red, PcgVecs<T> &v, hipStream_t st, SolveOut *out) {
    constexpr double W = sizeof(T);
    const Level<T> &L0 = S.lev[0];
    const Geo g = L0.g;
    const long long N = g.N;
    Scal *sc = red.scal;
    const int *done = &sc->done;
    if (kind == OP_SLOT) {
        LAUNCH(K_PCG_INIT, W * (4 + DIM) * N, (k_pcg_init_slot<T, DIM>), N, st, L0, b, (const T *)x, v.r, sc, red.part0,
               red.part1, red.counter, rtol, max_iter);
    } else {
        LAUNCH(K_PCG_INIT, W * 2 * N, (k_ch_lap_plain<T, DIM>), N, st, g, ch.ih2, (const T *)x, v.t);
        LAUNCH(K_PCG_INIT, W * 4 * N, (k_pcg_init_ch<T, DIM>), N, st, g, ch.ih2, ch.a, ch.b, b, (const T *)x,
               (const T *)v.t, v.r, sc, red.part0, red.part1, red.counter, rtol, max_iter);
    }
    precond_d<T, DIM>(S, kind, v.r, v.z, v.t, done, st);
    LAUNCH(K_PCG_DOT, W * 2 * N, (k_pcg_rz<T>), N, st, N, (const T *)v.r, (const T *)v.z, sc, red.part0, red.part1,
           red.part2, red.counter, 1, S.singular);
    int launched = 0;
    int chunk = predict < 1 ? 1 : predict;
    Scal hs;
    for (;;) {
        if (chunk > max_iter - launched) chunk = max_iter - launched;
        for (int it = 0; it < chunk; ++it) {
            const int k = launched + it;
            T *pnew = (k & 1) ? v.p1 : v.p0;
            T *pold = (k & 1) ? v.p0 : v.p1;
            if (kind == OP_SLOT) {
                LAUNCH(K_PCG_APPLY, W * (5 + DIM) * N, (k_pcg_apply_slot<T, DIM>), N, st, L0, (const T *)v.z,
                       (const T *)pold, pnew, v.q, sc, red.part0, red.counter);
            } else {
                LAUNCH(K_PCG_APPLY, W * 4 * N, (k_pcg_ch_lap<T, DIM>), N, st, g, ch.ih2, (const T *)v.z, (const T *)pold,
                       pnew, v.t, (const Scal *)sc);
                LAUNCH(K_PCG_APPLY, W * 3 * N, (k_pcg_ch_apply<T, DIM>), N, st, g, ch.ih2, ch.a, ch.b, (const T *)pnew,
                       (const T *)v.t, v.q, sc, red.part0, red.counter);
            }
            LAUNCH(K_PCG_UPDATE, W * 6 * N, (k_pcg_update<T>), N, st, N, (const T *)pnew, (const T *)v.q, x, v.r, sc,
                   red.part0, red.counter);
            precond_d<T, DIM>(S, kind, v.r, v.z, v.t, done, st);
            LAUNCH(K_PCG_DOT, W * 2 * N, (k_pcg_rz<T>), N, st, N, (const T *)v.r, (const T *)v.z, sc, red.part0, red.part1,
                   red.part2, red.counter, 0, S.singular);
        }
        launched += chunk;
        hipError_t e = hipMemcpyAsync(&hs, sc, sizeof(Scal), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (hs.done || launched >= max_iter) break;
        chunk = 2;
    }
    if (out) {
        out->iters = hs.iter;
        out->rel_res = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : 0.0;
        out->unconverged = hs.unconverged || !hs.done;
        out->nonfinite = hs.nonfinite;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_solve(Slot<T> &S, int dim, OpKind kind, ChOp ch, const T *b, T *x, double rtol, int max_iter,
                     int predict, Red &red, PcgVecs<T> &v, hipStream_t st, SolveOut *out) {
    if (dim == 2) return pcg_d<T, 2>(S, kind, ch, b, x, rtol, max_iter, predict, red, v, st, out);
    return pcg_d<T, 3>(S, kind, ch, b, x, rtol, max_iter, predict, red, v, st, out);
}

template <typename T>
void remove_mean(const Geo &g, T *x, Red &red, hipStream_t st) {
    constexpr double W = sizeof(T);
    (void)W;
    LAUNCH(K_MEAN, sizeof(T) * g.N, (k_sum<T>), g.N, st, g.N, (const T *)x, red.part0, red.counter, &red.scal->sum0);
    LAUNCH(K_MEAN, 2.0 * sizeof(T) * g.N, (k_sub_mean<T>), g.N, st, g.N, x, (const double *)&red.scal->sum0);
}

template <typename T>
void slot_apply(Slot<T> &S, int dim, const T *x, T *y, hipStream_t st) {
    if (dim == 2)
        LAUNCH(K_PCG_APPLY, 0, (k_slot_apply<T, 2>), S.lev[0].g.N, st, S.lev[0], x, y);
    else
        LAUNCH(K_PCG_APPLY, 0, (k_slot_apply<T, 3>), S.lev[0].g.N, st, S.lev[0], x, y);
}

template void mg_setup<double>(Slot<double> &, int, hipStream_t);
template void mg_vcycle<double>(Slot<double> &, int, const double *, double *, const int *, hipStream_t);
template hipError_t pcg_solve<double>(Slot<double> &, int, OpKind, ChOp, const double *, double *, double, int, int,
                                      Red &, PcgVecs<double> &, hipStream_t, SolveOut *);
template void remove_mean<double>(const Geo &, double *, Red &, hipStream_t);
template void slot_apply<double>(Slot<double> &, int, const double *, double *, hipStream_t);

}  // namespace chns
