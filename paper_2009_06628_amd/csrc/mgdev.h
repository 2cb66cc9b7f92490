// Device building blocks of the multigrid: per-cell operator, smoother and
// transfer bodies, the workgroup-level V-cycle and hierarchy set-up, and the
// Laplacian of the CH operator.  Shared by the grid-wide kernels (one pass
// per launch), the single-workgroup coarse-level kernels and the batched
// workgroup-per-problem step.
#pragma once
#include <algorithm>

#include "common.h"

namespace chns {

// ---------------------------------------------------------------------------
// per-cell building blocks (shared by the grid-wide and single-block kernels)
// ---------------------------------------------------------------------------
template <int DIM>
__device__ inline void coords_of(const Geo &g, int c, int ia[3]) {
    if (DIM == 2)
        cell_coords2(g, c, ia[0], ia[1], ia[2]);
    else
        cell_coords(g, c, ia[0], ia[1], ia[2]);
}

// Neighbour stencils are branch-free: a missing neighbour (outside a walled
// axis) is replaced by the cell itself with weight 0, so every load of a
// stencil is unconditional and can be issued together (adding 0 leaves the
// sums unchanged).

// a * b + c, rounded once.  The stencil sums of the multigrid spell their
// fused multiply-adds out: left to contraction, a sum that starts with two
// products is fused on one or the other depending on the surrounding code,
// and the grid-wide, marching, tile and LDS forms of a pass must round alike
// (they are compared bit for bit).
__device__ inline float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// (A x)_c
template <typename T, int DIM>
__device__ inline T apply_at(const Level<T> &L, const T *__restrict__ x, int c, const int ia[3]) {
    using R = T;
    const Geo &g = L.g;
    const R xc = (R)x[c];
    R acc = (R)L.s[c] * xc;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b);
        const int hi = nb_hi(g, c, ia[b], b);
        const int l = lo >= 0 ? lo : c, h = hi >= 0 ? hi : c;
        const R xl = (R)x[l], xh = (R)x[h];
        const R wl = (R)L.cs[b][c], wh = (R)L.cs[b][h];
        acc = fmar(lo >= 0 ? wl : (R)0, xc - xl, acc);
        acc = fmar(hi >= 0 ? wh : (R)0, xc - xh, acc);
    }
    return acc;
}

// sum_b cs * x_nb over the neighbours (x given by a functor)
template <typename T, int DIM, typename F>
__device__ inline T offsum_at(const Level<T> &L, int c, const int ia[3], F xv) {
    using R = T;
    const Geo &g = L.g;
    R acc = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b);
        const int hi = nb_hi(g, c, ia[b], b);
        const int l = lo >= 0 ? lo : c, h = hi >= 0 ? hi : c;
        const R vl = xv(l), vh = xv(h);
        const R wl = (R)L.cs[b][c], wh = (R)L.cs[b][h];
        acc = fmar(lo >= 0 ? wl : (R)0, vl, acc);
        acc = fmar(hi >= 0 ? wh : (R)0, vh, acc);
    }
    return acc;
}

template <typename T, int DIM>
__device__ inline void invd_cell(const Level<T> &L, int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    R d = (R)L.s[c];
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        if (nb_lo(L.g, c, ia[b], b) >= 0) d += (R)L.cs[b][c];
        const int hi = nb_hi(L.g, c, ia[b], b);
        if (hi >= 0) d += (R)L.cs[b][hi];
    }
    L.invd[c] = (T)((R)1 / d);
}

// zero-guess pre-smoothing: red x = b / d, black from those red values
template <typename T, typename TB, int DIM>
__device__ inline void presmooth_cell(const Level<T> &L, const TB *__restrict__ b, T *__restrict__ x, int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    const int col = (ia[0] + ia[1] + ia[2]) & 1;
    if (col == 0) {
        x[c] = (T)((R)b[c] * (R)L.invd[c]);
    } else {
        auto red = [&](int e) { return (R)b[e] * (R)L.invd[e]; };
        x[c] = (T)(((R)b[c] + offsum_at<T, DIM>(L, c, ia, red)) * (R)L.invd[c]);
    }
}

template <typename T, typename TB, int DIM>
__device__ inline void residual_cell(const Level<T> &L, const TB *__restrict__ b, const T *__restrict__ x,
                                     int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    L.r[c] = (T)((R)b[c] - apply_at<T, DIM>(L, x, c, ia));
}

// One (z, y) row of the prolongation: v + wyz (w0 a + w1 b)
template <typename R>
__device__ inline R pro_row(R v, R wyz, R w0, R a, R w1, R b) {
    return fmar(wyz, fmar(w0, a, w1 * b), v);
}

// cell-centred linear prolongation along one axis: fine f takes 3/4 of its
// parent f/2 and 1/4 of the coarse neighbour on its side; past a wall the
// neighbour is the parent itself (weight 1 in total)
template <typename R>
__device__ inline void pro_axis(int f, int nc, int per, int &c0, int &c1, R &w0, R &w1) {
    const int p = f >> 1;
    int q = (f & 1) ? p + 1 : p - 1;
    c0 = p;
    if (q < 0 || q >= nc) {
        if (per) {
            q = q < 0 ? nc - 1 : 0;
        } else {
            c1 = p;
            w0 = (R)1;
            w1 = (R)0;
            return;
        }
    }
    c1 = q;
    w0 = (R)0.75;
    w1 = (R)0.25;
}

template <typename T, int DIM>
__device__ inline T prolong_at(const Geo &gf, const Geo &gc, const T *__restrict__ xc, const int fi[3]) {
    using R = T;
    int c0[3], c1[3];
    R w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
            pro_axis<R>(fi[a], gc.n[a], gc.per[a], c0[a], c1[a], w0[a], w1[a]);
        } else {
            c0[a] = c1[a] = 0;
            w0[a] = 1.0;
            w1[a] = 0.0;
        }
    }
    const int nx = gc.n[0], nxy = (int)gc.n[0] * gc.n[1];
    R v = 0.0;
#pragma unroll
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz) {
        const int kz = (dz ? c1[2] : c0[2]) * nxy;
        const R wz = dz ? w1[2] : w0[2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int ky = kz + (dy ? c1[1] : c0[1]) * nx;
            const R wyz = wz * (dy ? w1[1] : w0[1]);
            v = pro_row(v, wyz, w0[0], (R)xc[ky + c0[0]], w1[0], (R)xc[ky + c1[0]]);
        }
    }
    return v;
}

// full weighting along one axis: the four fine cells 2I-1 .. 2I+2 with
// weights (1,3,3,1)/8; at a wall the missing outer cell's weight moves to the
// adjacent child (4,3,1)/8 -- exactly the transpose of pro_axis / 2.  Always
// four taps (an absent one gets weight 0 and a valid index) so that the
// loads of a fully unrolled stencil issue together.
template <typename R>
__device__ inline void res_axis(int I, int nc, int nf, int per, int f[4], R w[4]) {
    const bool lo = (I > 0) || per, hi = (I < nc - 1) || per;
    f[0] = I > 0 ? 2 * I - 1 : (per ? nf - 1 : 0);
    w[0] = lo ? (R)0.125 : (R)0;
    f[1] = 2 * I;
    w[1] = lo ? (R)0.375 : (R)0.5;
    f[2] = 2 * I + 1;
    w[2] = hi ? (R)0.375 : (R)0.5;
    f[3] = I < nc - 1 ? 2 * I + 2 : (per ? 0 : nf - 1);
    w[3] = hi ? (R)0.125 : (R)0;
}

template <typename T, int DIM>
__device__ inline void restrict_cell(const Geo &gf, const Geo &gc, const T *__restrict__ rf, T *__restrict__ bc,
                                     int c) {
    using R = T;
    int I[3];
    coords_of<DIM>(gc, c, I);
    int fx[4], fy[4], fz[4];
    R wx[4], wy[4], wz[4];
    res_axis<R>(I[0], gc.n[0], gf.n[0], gc.per[0], fx, wx);
    res_axis<R>(I[1], gc.n[1], gf.n[1], gc.per[1], fy, wy);
    if (DIM == 3) res_axis<R>(I[2], gc.n[2], gf.n[2], gc.per[2], fz, wz);
    const int nx = gf.n[0], nxy = (int)gf.n[0] * gf.n[1];
    R v = 0.0;
#pragma unroll
    for (int a = 0; a < (DIM == 3 ? 4 : 1); ++a) {
        const int kz = DIM == 3 ? fz[a] * nxy : 0;
        const R wza = DIM == 3 ? wz[a] : 1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = kz + fy[q] * nx;
            R s = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) s = fmar(wx[e], (R)rf[row + fx[e]], s);
            v = fmar(wy[q] * wza, s, v);
        }
    }
    bc[c] = (T)v;
}

// fused prolongation + black sweep: writes tmp = {red: x + P e, black:
// GS update from those red values}; x is left untouched
template <typename T, typename TB, int DIM>
__device__ inline void prolong_black_cell(const Level<T> &L, const Geo &gc, const T *__restrict__ xc,
                                          const TB *__restrict__ b, const T *__restrict__ x, T *__restrict__ tmp,
                                          int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    const int col = (ia[0] + ia[1] + ia[2]) & 1;
    if (col == 0) {
        tmp[c] = (T)((R)x[c] + prolong_at<T, DIM>(L.g, gc, xc, ia));
    } else {
        auto red = [&](int e) {
            int ie[3];
            coords_of<DIM>(L.g, e, ie);
            return (R)x[e] + prolong_at<T, DIM>(L.g, gc, xc, ie);
        };
        tmp[c] = (T)(((R)b[c] + offsum_at<T, DIM>(L, c, ia, red)) * (R)L.invd[c]);
    }
}

// red sweep from tmp: x = {red: GS update from black tmp values, black: tmp}
template <typename T, typename TB, int DIM>
__device__ inline void red_from_tmp_cell(const Level<T> &L, const TB *__restrict__ b, const T *__restrict__ tmp,
                                         T *__restrict__ x, int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    const int col = (ia[0] + ia[1] + ia[2]) & 1;
    if (col == 1) {
        x[c] = tmp[c];
    } else {
        auto blk = [&](int e) { return (R)tmp[e]; };
        x[c] = (T)(((R)b[c] + offsum_at<T, DIM>(L, c, ia, blk)) * (R)L.invd[c]);
    }
}

// in-place Gauss-Seidel update of one colour (neighbours have the other colour)
template <typename T, typename TB, int DIM>
__device__ inline void gs_color_cell(const Level<T> &L, const TB *__restrict__ b, T *__restrict__ x, int color, int c) {
    using R = T;
    int ia[3];
    coords_of<DIM>(L.g, c, ia);
    if (((ia[0] + ia[1] + ia[2]) & 1) != color) return;
    auto xv = [&](int e) { return (R)x[e]; };
    x[c] = (T)(((R)b[c] + offsum_at<T, DIM>(L, c, ia, xv)) * (R)L.invd[c]);
}

template <typename T, int DIM>
__device__ inline void coarsen_cell(const Level<T> &F, const Level<T> &C, int c) {
    int I[3];
    coords_of<DIM>(C.g, c, I);
    const Geo &gf = F.g;
    double s = 0.0;
    double cs[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int d3[3] = {dx, dy, dz};
                const int f =
                    (2 * I[0] + dx) + (int)gf.n[0] * ((2 * I[1] + dy) + (int)gf.n[1] * (2 * I[2] + dz));
                s += (double)F.s[f];
#pragma unroll
                for (int b = 0; b < DIM; ++b)
                    if (d3[b] == 0) cs[b] += (double)F.cs[b][f];   // fine faces on the coarse lower b-face
            }
    constexpr double nchild = (DIM == 3) ? 8.0 : 4.0;
    C.s[c] = (T)(s / nchild);
    // a face on a wall holds 0: every other pass masks it, and the LDS
    // V-cycle relies on it to index walled axes as periodic ones
#pragma unroll
    for (int b = 0; b < DIM; ++b)
        C.cs[b][c] = (C.g.per[b] || I[b] > 0) ? (T)(cs[b] / (nchild * 0.5) * 0.25) : (T)0;
}


// ---------------------------------------------------------------------------
// single-workgroup kernels for the small levels
// ---------------------------------------------------------------------------
#define BLOCK_LOOP(N) for (int c = (int)threadIdx.x; c < (int)(N); c += (int)blockDim.x)

// Red-black sweeps on each side of the cycle on the levels of at most
// kSmallSweepCells cells, the part run by one workgroup (one sweep on the
// larger levels).  With one sweep there, the coarse levels of a high-
// contrast system (density ratio 1000) leave most of the error: a CPU
// emulation of the bubble's pressure system at 256 x 512 needs 30 CG
// iterations with one sweep, 18 with two and 15 with three on these
// levels, which cost LDS passes but no launches (measured on the device:
// 30 / 19 / 17 iterations, 2.67 / 2.25 / 2.17 ms per bubble step).  The
// pre-sweeps run red then black, the post-sweeps black then red, so the
// cycle stays symmetric.
#ifndef CHNS_SMALL_SWEEPS
#define CHNS_SMALL_SWEEPS 3
#endif
constexpr int kSmallSweeps = CHNS_SMALL_SWEEPS;
constexpr int kSmallSweepCells = 2048;

// x = Ainv b on the coarsest level (FP64 matrix, block-wide)
template <typename T, typename TB>
__device__ inline void coarse_solve_block(int n, const double *__restrict__ Ainv, const TB *__restrict__ b,
                                          T *__restrict__ x) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v = 0.0;
        const double *row = Ainv + i * n;
        for (int j = 0; j < n; ++j) v += row[j] * (double)b[j];
        x[i] = (T)v;
    }
}

template <typename T, typename TB, int DIM>
__device__ inline void block_down(const Slot<T> &S, int l, const TB *__restrict__ b, T *__restrict__ x) {
    const Level<T> &lv = S.lev[l];
    BLOCK_LOOP(lv.g.N) presmooth_cell<T, TB, DIM>(lv, b, x, c);
    __syncthreads();
    if (lv.g.N <= kSmallSweepCells)
        for (int sw = 1; sw < kSmallSweeps; ++sw) {
            BLOCK_LOOP(lv.g.N) gs_color_cell<T, TB, DIM>(lv, b, x, 0, c);
            __syncthreads();
            BLOCK_LOOP(lv.g.N) gs_color_cell<T, TB, DIM>(lv, b, x, 1, c);
            __syncthreads();
        }
    BLOCK_LOOP(lv.g.N) residual_cell<T, TB, DIM>(lv, b, x, c);
    __syncthreads();
    BLOCK_LOOP(S.lev[l + 1].g.N) restrict_cell<T, DIM>(lv.g, S.lev[l + 1].g, lv.r, S.lev[l + 1].b, c);
    __syncthreads();
}

template <typename T, typename TB, int DIM>
__device__ inline void block_up(const Slot<T> &S, int l, const TB *__restrict__ b, T *__restrict__ x) {
    const Level<T> &lv = S.lev[l];
    BLOCK_LOOP(lv.g.N) prolong_black_cell<T, TB, DIM>(lv, S.lev[l + 1].g, S.lev[l + 1].x, b, x, lv.r, c);
    __syncthreads();
    BLOCK_LOOP(lv.g.N) red_from_tmp_cell<T, TB, DIM>(lv, b, lv.r, x, c);
    __syncthreads();
    if (lv.g.N <= kSmallSweepCells)
        for (int sw = 1; sw < kSmallSweeps; ++sw) {
            BLOCK_LOOP(lv.g.N) gs_color_cell<T, TB, DIM>(lv, b, x, 1, c);
            __syncthreads();
            BLOCK_LOOP(lv.g.N) gs_color_cell<T, TB, DIM>(lv, b, x, 0, c);
            __syncthreads();
        }
}

// V-cycle over levels [l0, nlev) in one workgroup.  b0 / x0 are the
// right-hand side / result of level l0 (they replace its own arrays; b0 may
// be stored in another precision).  Ends with a workgroup barrier.
template <typename T, typename TB, int DIM>
__device__ inline void vcycle_block_dev(const Slot<T> &S, int l0, const TB *__restrict__ b0, T *__restrict__ x0) {
    const int L = S.nlev;
    if (l0 == L - 1) {
        coarse_solve_block<T, TB>((int)S.lev[L - 1].g.N, S.Ainv, b0, x0);
        __syncthreads();
        return;
    }
    block_down<T, TB, DIM>(S, l0, b0, x0);
    for (int l = l0 + 1; l < L - 1; ++l) block_down<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x);
    coarse_solve_block<T, T>((int)S.lev[L - 1].g.N, S.Ainv, S.lev[L - 1].b, S.lev[L - 1].x);
    __syncthreads();
    for (int l = L - 2; l > l0; --l) block_up<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x);
    block_up<T, TB, DIM>(S, l0, b0, x0);
}

// ---------------------------------------------------------------------------
// LDS-resident V-cycle of the small levels
// ---------------------------------------------------------------------------
// The storage of levels [l0, nlev) of a slot is one contiguous range of the
// workspace (per level s, cs, invd, r, x, b, then the coarsest inverse).  A
// one-workgroup launch may land on an XCD whose L2 holds none of it, so the
// global-memory form pays several dependent memory round trips in every
// sweep.  Here the workgroup copies the whole range into LDS in one round of
// independent 16-byte loads, runs every sweep out of LDS with the same
// per-cell code, and writes back x of level l0.
constexpr int kLdsCopyUnroll = 10;                  // 16-byte loads in flight per thread

// The LDS kernel always runs kSBThreads threads; a compile-time stride keeps
// the loops from reading the workgroup size from the dispatch arguments.
#define LDS_LOOP(N) for (int c = (int)threadIdx.x; c < (int)(N); c += kSBThreads)


// Copy the segments: every load of a round is issued before its stores.
// Indices past the end are clamped to the last word, which is then stored
// again with its own value, so no load or store is conditional.
__device__ inline void copy_to_lds(uint4 *dst_words, const uint4 *src_words, const LdsCopy &cp) {
    // src is device memory: global loads (a pointer read from a table would
    // otherwise be generic, and the loaded words went through scratch)
    using Word = unsigned int __attribute__((ext_vector_type(4)));
    using GWord = const __attribute__((address_space(1))) Word;
    GWord *src = (GWord *)src_words;
    Word *dst = (Word *)dst_words;
    const int n = cp.total;
    for (int base = 0; base < n; base += kLdsCopyUnroll * kSBThreads) {
        Word v[kLdsCopyUnroll];
        int w[kLdsCopyUnroll];
#pragma unroll
        for (int k = 0; k < kLdsCopyUnroll; ++k) {
            int i = base + k * kSBThreads + (int)threadIdx.x;
            i = i < n ? i : n - 1;
            int sh = cp.shift[0];
#pragma unroll
            for (int j = 1; j < kLdsCopySegs; ++j) sh = i >= cp.cend[j - 1] ? cp.shift[j] : sh;
            w[k] = i + sh;
            v[k] = src[w[k]];
        }
#pragma unroll
        for (int k = 0; k < kLdsCopyUnroll; ++k) dst[w[k]] = v[k];
    }
}

// Copy plan of the LDS V-cycle of levels [lsb, nlev): the byte intervals
// read before they are written (s, cs, invd of each level, b of level lsb,
// the coarsest inverse), merged across the smallest gaps down to
// kLdsCopySegs segments, in whole 16-byte words of the range (arrays start
// on 256-byte boundaries; a rounded-up end stays inside the workspace).
template <typename T>
inline LdsCopy lds_copy_plan(const Slot<T> &S, int lsb) {
    const char *base = (const char *)S.lev[lsb].s;
    long long a[2 * kMaxLev + 2], e[2 * kMaxLev + 2];
    int n = 0;
    auto add = [&](const void *p, size_t bytes) {
        a[n] = (const char *)p - base;
        e[n] = a[n] + (long long)bytes;
        ++n;
    };
    for (int l = lsb; l < S.nlev; ++l) {
        const Level<T> &L = S.lev[l];
        add(L.s, (size_t)((const char *)(L.invd + L.g.N) - (const char *)L.s));   // s, cs[], invd
        if (l == lsb) add(L.b, sizeof(T) * (size_t)L.g.N);
    }
    add(S.Ainv, sizeof(double) * (size_t)S.ncoarse * S.ncoarse);
    // sort by start (a handful of entries)
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && a[j] < a[j - 1]; --j) {
            std::swap(a[j], a[j - 1]);
            std::swap(e[j], e[j - 1]);
        }
    while (n > kLdsCopySegs) {
        int best = 0;
        for (int i = 1; i + 1 < n; ++i)
            if (a[i + 1] - e[i] < a[best + 1] - e[best]) best = i;
        e[best] = std::max(e[best], e[best + 1]);
        for (int i = best + 1; i + 1 < n; ++i) {
            a[i] = a[i + 1];
            e[i] = e[i + 1];
        }
        --n;
    }
    LdsCopy cp;
    int done = 0;
    for (int i = 0; i < kLdsCopySegs; ++i) {
        if (i < n) {
            const int w0 = (int)(a[i] / 16), w1 = (int)((e[i] + 15) / 16);
            cp.shift[i] = w0 - done;
            done += w1 - w0;
            cp.cend[i] = done;
        } else {
            cp.shift[i] = cp.shift[n - 1];
            cp.cend[i] = done;
        }
    }
    cp.total = done;
    return cp;
}

// LDS bytes of the V-cycle of levels [lsb, nlev) of S in one workgroup (its
// storage from lev[lsb].s to the end of the coarsest inverse, in whole
// 16-byte words), or 0 where that kernel does not apply: lsb == 0, more
// than kLdsVcycleBytes, or a level with more than one red-black pair per
// thread.
template <typename T>
inline size_t lds_vcycle_bytes(const Slot<T> &S, int lsb) {
    if (lsb <= 0 || S.lev[lsb].g.N > 2 * kSBThreads) return 0;
    const size_t range =
        (size_t)((const char *)(S.Ainv + (size_t)S.ncoarse * S.ncoarse) - (const char *)S.lev[lsb].s);
    const size_t range16 = (range + 15) & ~(size_t)15;
    return range16 <= (size_t)kLdsVcycleBytes ? range16 : 0;
}

// The LDS image of a workspace pointer p of the copied range starting at base.
template <typename T>
__device__ inline T *lds_image(char *lds, const char *base, const T *p) {
    return (T *)(lds + (unsigned)((const char *)p - base));
}

template <typename T, int DIM>
__device__ inline Level<T> lds_level(const Level<T> &G, char *lds, const char *base) {
    Level<T> L;
    L.g = G.g;
    L.s = lds_image(lds, base, G.s);
#pragma unroll
    for (int b = 0; b < 3; ++b) L.cs[b] = b < DIM ? lds_image(lds, base, G.cs[b]) : L.s;
    L.invd = lds_image(lds, base, G.invd);
    L.r = lds_image(lds, base, G.r);
    L.x = lds_image(lds, base, G.x);
    L.b = lds_image(lds, base, G.b);
    return L;
}

// x = Ainv b on the coarsest level (FP64 inverse, all operands in LDS): G
// lanes per row (G a power of two, at most a wave, G n <= kSBThreads where
// n allows), lane q summing columns q, q + G, ... in order, then a butterfly
// sum over the G lanes.  The lanes of a group (aligned within a wave) run
// the same rows, so every shuffle pairs two active lanes of one group.
template <typename T>
__device__ inline void coarse_solve_lds(int n, const double *Ainv, const T *b, T *x) {
    int G = 1;
    while (G < kWave && 2 * G * n <= kSBThreads) G *= 2;
    const int q = (int)threadIdx.x & (G - 1);
    for (int i = (int)threadIdx.x / G; i < n; i += kSBThreads / G) {
        const double *row = Ainv + i * n;
        double v = 0.0;
        for (int j = q; j < n; j += G) v += row[j] * (double)b[j];
        for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if (q == 0) x[i] = (T)v;
    }
}

// V-cycle over levels [l0, nlev), l0 >= 1, on the LDS image of their
// storage, with the arithmetic of vcycle_block_dev per cell:
//   pre-smoothing  red x = b / d and black GS from its red neighbours' b / d
//                  in one pass, then kSmallSweeps - 1 more red | black sweeps
//   post-smoothing red x += P e, then kSmallSweeps x (black GS | red GS)
//                  (black x is overwritten by its GS update, so only red
//                  cells take the prolonged correction)
// Thread k takes the k-th red and the k-th black cell of a level (x extent
// even), a pair in one row: row = y + ny z = k / (nx / 2), red at
// x = 2 (k mod nx / 2) + ((y + z) & 1), black at x ^ 1.  The host runs this
// kernel only when every level has at most 2 kSBThreads cells, so each
// thread owns at most one pair per level and keeps it in registers for all
// passes of a side of the cycle: its neighbour indices, b, 1 / diag and the
// coefficients of its faces.  A pass then issues only the reads of the
// neighbours' x and one write per cell, where recomputing the indices (an
// integer division) and re-reading the coefficients took most of the issue
// slots of a pass (bubble 256 x 512: 2.09 -> 1.90 ms per step, with
// bit-identical results).
// Faces on walls hold 0 on these levels (coarsen_cell), so every axis is
// indexed as periodic: the wrapped neighbour of a cell on a wall enters with
// weight 0, where the masked stencils add 0 for the missing neighbour.
template <typename T, int DIM>
struct LdsPair {
    int c[2];              // red, black
    int nb[2][2 * DIM];    // wrapped neighbours: x low, x high, y low, y high (, z low, z high)
    int ia[3];             // coordinates of the red cell
    T b[2], invd[2];
    T cw[2][2 * DIM];      // coefficients of the faces towards nb, in the same order
};

template <typename T, int DIM>
__device__ inline void load_lds_pair(const Level<T> &lv, int k, LdsPair<T, DIM> &P) {
    const int nx = (int)lv.g.n[0], ny = (int)lv.g.n[1], nz = DIM == 3 ? (int)lv.g.n[2] : 1;
    const int nxy = nx * ny;
    const int row = k / (nx >> 1);   // y + ny z
    const int z = DIM == 3 ? row / ny : 0;
    const int y = row - z * ny;
    const int xr = 2 * (k - row * (nx >> 1)) + ((y + z) & 1);
    P.ia[0] = xr;
    P.ia[1] = y;
    P.ia[2] = z;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int x = q ? xr ^ 1 : xr;
        const int c = x + nx * row;
        int *nb = P.nb[q];
        P.c[q] = c;
        nb[0] = x > 0 ? c - 1 : c + nx - 1;
        nb[1] = x < nx - 1 ? c + 1 : c + 1 - nx;
        nb[2] = y > 0 ? c - nx : c + nx * (ny - 1);
        nb[3] = y < ny - 1 ? c + nx : c - nx * (ny - 1);
        if (DIM == 3) {
            nb[2 * DIM - 2] = z > 0 ? c - nxy : c + nxy * (nz - 1);
            nb[2 * DIM - 1] = z < nz - 1 ? c + nxy : c - nxy * (nz - 1);
        }
        P.b[q] = lv.b[c];
        P.invd[q] = lv.invd[c];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            P.cw[q][2 * a] = lv.cs[a][c];
            P.cw[q][2 * a + 1] = lv.cs[a][nb[2 * a + 1]];
        }
    }
}

// sum over the faces of cell Q of the pair of cs * v(neighbour)
template <int Q, typename T, int DIM, typename V>
__device__ inline T pair_offsum(const LdsPair<T, DIM> &P, V v) {
    T acc = 0.0;
#pragma unroll
    for (int i = 0; i < 2 * DIM; ++i) acc = fmar(P.cw[Q][i], v(P.nb[Q][i]), acc);
    return acc;
}

// Gauss-Seidel update of cell Q of the pair from its neighbours' current x
template <int Q, typename T, int DIM>
__device__ inline void pair_gs(const LdsPair<T, DIM> &P, T *x) {
    x[P.c[Q]] = (P.b[Q] + pair_offsum<Q>(P, [&](int e) { return x[e]; })) * P.invd[Q];
}

// residual b - A x at cell Q of the pair
template <int Q, typename T, int DIM>
__device__ inline T pair_residual(const LdsPair<T, DIM> &P, const T *s, const T *x) {
    const T xc = x[P.c[Q]];
    T acc = s[P.c[Q]] * xc;
#pragma unroll
    for (int i = 0; i < 2 * DIM; ++i) acc = fmar(P.cw[Q][i], xc - x[P.nb[Q][i]], acc);
    return P.b[Q] - acc;
}

template <typename T, int DIM>
__device__ __forceinline__ void vcycle_lds_dev(const Slot<T> &S, int l0, char *lds, const char *base) {
    const int L = S.nlev;
    const int tid = (int)threadIdx.x;
    LdsPair<T, DIM> own;   // pair tid of the current level, if the level has one
    auto load_own = [&](const Level<T> &lv) {
        if (tid < (int)lv.g.N / 2) load_lds_pair(lv, tid, own);
    };
    auto each_pair = [&](const Level<T> &lv, auto body) {
        if (tid < (int)lv.g.N / 2) body(own);
    };
    using P_t = LdsPair<T, DIM>;
    for (int l = l0; l < L - 1; ++l) {
        const Level<T> lv = lds_level<T, DIM>(S.lev[l], lds, base);
        const Level<T> lc = lds_level<T, DIM>(S.lev[l + 1], lds, base);
        load_own(lv);
        // zero-guess smoothing: red x = b / d, black GS from those values
        each_pair(lv, [&](const P_t &P) {
            lv.x[P.c[0]] = P.b[0] * P.invd[0];
            lv.x[P.c[1]] = (P.b[1] + pair_offsum<1>(P, [&](int e) { return lv.b[e] * lv.invd[e]; })) * P.invd[1];
        });
        __syncthreads();
        for (int sw = 1; sw < kSmallSweeps; ++sw) {
            each_pair(lv, [&](const P_t &P) { pair_gs<0>(P, lv.x); });
            __syncthreads();
            each_pair(lv, [&](const P_t &P) { pair_gs<1>(P, lv.x); });
            __syncthreads();
        }
        each_pair(lv, [&](const P_t &P) {
            lv.r[P.c[0]] = pair_residual<0>(P, lv.s, lv.x);
            lv.r[P.c[1]] = pair_residual<1>(P, lv.s, lv.x);
        });
        __syncthreads();
        LDS_LOOP(lc.g.N) restrict_cell<T, DIM>(lv.g, lc.g, lv.r, lc.b, c);
        __syncthreads();
    }
    {
        const Level<T> lc = lds_level<T, DIM>(S.lev[L - 1], lds, base);
        coarse_solve_lds<T>((int)lc.g.N, lds_image(lds, base, S.Ainv), lc.b, lc.x);
        __syncthreads();
    }
    for (int l = L - 2; l >= l0; --l) {
        const Level<T> lv = lds_level<T, DIM>(S.lev[l], lds, base);
        const Level<T> lc = lds_level<T, DIM>(S.lev[l + 1], lds, base);
        load_own(lv);
        each_pair(lv, [&](const P_t &P) {
            lv.x[P.c[0]] = lv.x[P.c[0]] + prolong_at<T, DIM>(lv.g, lc.g, lc.x, P.ia);
        });
        __syncthreads();
        for (int sw = 0; sw < kSmallSweeps; ++sw) {
            each_pair(lv, [&](const P_t &P) { pair_gs<1>(P, lv.x); });
            __syncthreads();
            each_pair(lv, [&](const P_t &P) { pair_gs<0>(P, lv.x); });
            __syncthreads();
        }
    }
}

// In-place Gauss-Jordan inversion of the n x n SPD matrix held in A (no
// pivoting), block-wide; f is a scratch row of n doubles.
__device__ inline void gauss_jordan_inplace(double *A, int n, double *f, double *piv) {
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        if (threadIdx.x == 0) *piv = 1.0 / A[k * n + k];
        for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = A[i * n + k];
        __syncthreads();
        const double p = *piv;
        for (int j = threadIdx.x; j < n; j += blockDim.x) A[k * n + j] = (j == k) ? p : A[k * n + j] * p;
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int i = e / n, j = e % n;
            if (i == k) continue;
            const double fi = f[i];
            A[e] = (j == k) ? -fi * p : A[e] - fi * A[k * n + j];
        }
    }
    __syncthreads();
}

// Gauss-Jordan inversion as above with one barrier per pivot: pivot step k
// reads the whole matrix from src and writes the next one to dst (the same
// arithmetic per entry, in the same order), then the two swap.  src and dst
// are n x n arrays; returns the one holding the inverse.  Block-wide; ends
// with a workgroup barrier.  (n = 32: 19 us against 27 us for the in-place
// form, which waits on three barriers and a one-thread step per pivot; one
// wave alone with wavefront fences took 101 us.)
__device__ inline double *gauss_jordan_pingpong(double *src, double *dst, int n, double *rp) {
    // Each thread steps its entries' (i, j) by the stride instead of dividing
    // e by n per pivot, and the thread that writes the next pivot entry also
    // stores its reciprocal (rp, two slots by pivot parity), so the other
    // threads read 1 / a_kk instead of each dividing (the same division of
    // the same value: results unchanged; whole set-up kernel with n = 32:
    // 34.7 -> 30.8 us, with n = 64 in 3D: 129 -> 108 us).
    const int nn = n * n, bd = (int)blockDim.x, tid = (int)threadIdx.x;
    const int di = bd / n, dj = bd - di * n;
    const int i0 = tid / n, j0 = tid - i0 * n;
    if (tid == 0) rp[0] = 1.0 / src[0];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double p = rp[k & 1];
        const int kn = k + 1;
        int i = i0, j = j0;
        for (int e = tid; e < nn; e += bd) {
            const double akj = j == k ? p : src[k * n + j] * p;   // the scaled pivot row
            const double v = i == k ? akj : (j == k ? -src[i * n + k] * p : src[e] - src[i * n + k] * akj);
            dst[e] = v;
            if (i == kn && j == kn) rp[kn & 1] = 1.0 / v;
            i += di;
            j += dj;
            if (j >= n) {
                j -= n;
                ++i;
            }
        }
        __syncthreads();
        double *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// LDS of the set-up: room for CAP doubles of the coarsest matrix (which is
// in LDS when it has at most kLdsInverse cells; with room for a second copy
// the inverse takes one barrier per pivot), a scratch row, reduction slots
// and the pivot.  SetupLds is the size kernels with other LDS use;
// SetupLdsPP (64 KB more) is for the set-up kernels alone.
template <int CAP>
struct SetupLdsT {
    double A[CAP];
    double f[kMaxCoarse];
    double red[kSBThreads / kWave];
    double piv;
};
using SetupLds = SetupLdsT<kLdsInverse * kLdsInverse>;
using SetupLdsPP = SetupLdsT<2 * kLdsInverse * kLdsInverse>;

// Set-up of the small levels in one workgroup: coarsen from level
// max(l0,1) - 1 downwards, inverse diagonals, then the coarsest inverse
// (in LDS when it has at most kLdsInverse cells, else in S.aug).  Ends with
// a workgroup barrier.
template <typename T, int DIM, int CAP>
__device__ inline void setup_block_dev(const Slot<T> &S, int l0, SetupLdsT<CAP> &sh) {
    double *A = sh.A, *f = sh.f, *red = sh.red;
    double &piv = sh.piv;
    const int L = S.nlev;
    if (l0 == 0) {
        BLOCK_LOOP(S.lev[0].g.N) invd_cell<T, DIM>(S.lev[0], c);
        __syncthreads();
    }
    for (int l = (l0 > 1 ? l0 : 1); l < L; ++l) {
        BLOCK_LOOP(S.lev[l].g.N) coarsen_cell<T, DIM>(S.lev[l - 1], S.lev[l], c);
        __syncthreads();
        BLOCK_LOOP(S.lev[l].g.N) invd_cell<T, DIM>(S.lev[l], c);
        __syncthreads();
    }
    // dense coarsest operator
    const Level<T> &C = S.lev[L - 1];
    const int n = (int)C.g.N;
    double *M = n <= kLdsInverse ? A : S.aug;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = 0.0;
    __syncthreads();
    double dsum = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        int ia[3];
        coords_of<DIM>(C.g, c, ia);
        double d = (double)C.s[c];
        for (int b = 0; b < DIM; ++b) {
            const int lo = nb_lo(C.g, c, ia[b], b);
            const int hi = nb_hi(C.g, c, ia[b], b);
            if (lo >= 0) {
                const double w = (double)C.cs[b][c];
                d += w;
                M[c * n + lo] -= w;
            }
            if (hi >= 0) {
                const double w = (double)C.cs[b][hi];
                d += w;
                M[c * n + hi] -= w;
            }
        }
        M[c * n + c] += d;
        dsum += d;
    }
    const double tot = block_sum_all(dsum, red);
    if (S.singular) {
        const double tau = (tot / n) / n;
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] += tau;
    }
    // in LDS with room for a second copy: one barrier per pivot
    if (M == A && 2 * n * n <= CAP)
        M = gauss_jordan_pingpong(A, A + n * n, n, f);
    else
        gauss_jordan_inplace(M, n, f, &piv);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) S.Ainv[e] = M[e];
    __syncthreads();
}


// Lap(x) at c for the CH operator (walled axes Neumann), x given by a functor
// (branch-free like apply_at)
template <int DIM, typename F>
__device__ inline double lap_at(const Geo &g, int c, const int ia[3], double ih2, F val) {
    const double xc = val(c);
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const int lo = nb_lo(g, c, ia[b], b);
        const int hi = nb_hi(g, c, ia[b], b);
        const double vl = val(lo >= 0 ? lo : c), vh = val(hi >= 0 ? hi : c);
        acc += lo >= 0 ? vl - xc : 0.0;
        acc += hi >= 0 ? vh - xc : 0.0;
    }
    return acc * ih2;
}

}  // namespace chns
