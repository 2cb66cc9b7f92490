// Device bodies of the 2D multigrid tile passes (gfx950).
#pragma once
#include "mgdev.h"

namespace chns {

// ---------------------------------------------------------------------------
// 2D tile passes of the grid levels: one for the way down, one for the way
// up (shared by the single-grid kernels and the tiled batched form)
// ---------------------------------------------------------------------------
// A workgroup owns kTFX x kTFY fine cells (kTFX/2 x kTFY/2 coarse cells) and
// stages the level on the tile plus a halo in LDS.  Cells outside a walled
// axis are zero with zero coupling, which is what the branch-free per-cell
// stencils add for a missing neighbour; periodic axes wrap.  Halo values are
// recomputed by every tile that needs them, with the arithmetic of the
// per-cell passes in the same order, so the results are those of the
// separate passes.  Levels here have even extents (only the coarsest may
// not), so colours do not change across a periodic seam.
#ifndef CHNS_TILE2_X
#define CHNS_TILE2_X 32
#endif
#ifndef CHNS_TILE2_Y
#define CHNS_TILE2_Y 16
#endif
#ifndef CHNS_TILE2_THREADS
#define CHNS_TILE2_THREADS 512
#endif
#ifndef CHNS_TILE2_BATCH_THREADS
#define CHNS_TILE2_BATCH_THREADS 256
#endif
constexpr int kTFX = CHNS_TILE2_X, kTFY = CHNS_TILE2_Y;   // fine cells per tile (even)
// Threads per tile: a single grid has few tiles per CU, so more threads per
// tile shorten each phase; the batched form has many tiles per CU and
// prefers more workgroups of fewer threads (measured).
constexpr int kTileThreads = CHNS_TILE2_THREADS;              // single-grid kernels
constexpr int kTileThreadsBatch = CHNS_TILE2_BATCH_THREADS;   // batched form
static_assert(kTFX % 2 == 0 && kTFY % 2 == 0, "tile extents must be even");

// Local x of the m-th cell of colour col in local row ly of a region that
// starts at local x 1 and has an even width, for a tile whose local (0, 0)
// has global parity par: the colour of a cell is the parity of its global
// x + y.
__device__ inline int tile_color_x(int m, int ly, int par, int col) {
    return 1 + 2 * m + ((ly + par + col + 1) & 1);
}

// Local index -> global coordinate along one axis: wrapped on a periodic
// axis; v tells whether the cell exists.
__device__ inline int tile_coord(int g, int n, int per, bool &v) {
    v = per || (g >= 0 && g < n);
    return per ? ((g % n) + n) % n : g;
}

// Right-hand side of a tile pass, staged in the hierarchy's precision T.
// As stored:
template <typename TB>
struct RhsStored {
    const TB *b;
    template <typename T>
    __device__ T at(int g) const {
        return (T)b[g];
    }
};
// The residual r - alpha q of a CG iteration whose store is still pending
// (the next operator apply stores it): the value the update stores in the
// CG precision TR, as read by the hierarchy through its right-hand side
// type TB.
__device__ inline double cg_residual(double r, double q, double alpha) { return fma(-alpha, q, r); }
template <typename TR, typename TB>
struct RhsPending {
    const TR *r, *q;
    double alpha;
    template <typename T>
    __device__ T at(int g) const {
        return (T)(TB)(TR)cg_residual((double)r[g], (double)q[g], alpha);
    }
};

// Sums of three per-thread values over a workgroup of NT threads, valid in
// thread 0 (fixed order: waves by shuffles, then the waves in order).
template <int NT>
__device__ inline void tile_sum3(double &a, double &b, double &c) {
    __shared__ double ws[3][NT / kWave];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = (int)threadIdx.x & (kWave - 1), w = (int)threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) {
        ws[0][w] = a;
        ws[1][w] = b;
        ws[2][w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / kWave; ++k) {
            a += ws[0][k];
            b += ws[1][k];
            c += ws[2][k];
        }
}

// Epilogue of the way up: nothing, or the partials of r.z, sum z and sum r
// over the tile's cells for the CG iteration that consumes z (r as stored,
// or pending as in RhsPending).
struct NoDots {
    __device__ void add(int, double) {}
    template <int NT>
    __device__ void finish() {}
};
template <typename TR>
struct RzDots {
    const TR *r, *q;
    double alpha;
    int pending;
    double *p0, *p1, *p2;
    int slot;
    double arz = 0.0, az = 0.0, ar = 0.0;
    __device__ void add(int g, double z) {
        const double rc =
            pending ? (double)(TR)cg_residual((double)r[g], (double)q[g], alpha) : (double)r[g];
        arz += rc * z;
        az += z;
        ar += rc;
    }
    template <int NT>
    __device__ void finish() {
        tile_sum3<NT>(arz, az, ar);
        if (threadIdx.x == 0) {
            p0[slot] = arz;
            p1[slot] = az;
            p2[slot] = ar;
        }
    }
};

// Way down: zero-guess pre-smoothing (red x = b / d, black GS from those),
// residual r = b - A x, restriction of r to the coarse right-hand side bc.
// Writes the smoothed x of the tile to xs (the level's residual array, which
// no longer holds a residual: the way up reads x from there while it writes
// the level's x) and bc on the tile's coarse cells.
template <typename T, int NT, typename BS>
__device__ inline void down_tile2(const Level<T> &L, const Geo &gc, const BS &b, T *__restrict__ xs,
                                  T *__restrict__ bc, int tx, int ty, int skip) {
    using R = T;
    constexpr int H = 3, WX = kTFX + 2 * H, WY = kTFY + 2 * H, NL = WX * WY;
    constexpr int KL = (NL + NT - 1) / NT;   // staged cells per thread
    __shared__ T sB[NL], sI[NL], sS[NL], sC0[NL], sC1[NL], sX[NL], sR[NL];
    const int nx = (int)L.g.n[0], ny = (int)L.g.n[1];
    const int px = L.g.per[0], py = L.g.per[1];
    const int gx0 = tx * kTFX - H, gy0 = ty * kTFY - H;
    // Stage: every load of the thread is issued before the first LDS store
    // (indices past the region are clamped to its last cell, which is then
    // stored again with the same values).
    T lb[KL], li[KL], ls[KL], l0[KL], l1[KL];
    bool lv[KL], m0[KL], m1[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int i0 = (int)threadIdx.x + k * NT, i = i0 < NL ? i0 : NL - 1;
        const int ly = i / WX, lx = i - ly * WX;
        bool vx, vy;
        const int gx = tile_coord(gx0 + lx, nx, px, vx), gy = tile_coord(gy0 + ly, ny, py, vy);
        const bool v = vx && vy;
        const int g = v ? gx + nx * gy : 0;
        lb[k] = b.template at<T>(g);
        li[k] = L.invd[g];
        ls[k] = L.s[g];
        l0[k] = L.cs[0][g];
        l1[k] = L.cs[1][g];
        lv[k] = v;
        m0[k] = v && (px || gx > 0);   // a wall face couples nothing
        m1[k] = v && (py || gy > 0);
    }
    if (skip) return;   // tested once the staging loads are in flight
    // masks applied as factors 0 / 1 (the values come from valid addresses and
    // are finite), so that no load turns into a branch of its own
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int i0 = (int)threadIdx.x + k * NT, i = i0 < NL ? i0 : NL - 1;
        const T fv = lv[k] ? (T)1 : (T)0;
        sB[i] = lb[k] * fv;
        sI[i] = li[k] * fv;
        sS[i] = ls[k] * fv;
        sC0[i] = l0[k] * (m0[k] ? (T)1 : (T)0);
        sC1[i] = l1[k] * (m1[k] ? (T)1 : (T)0);
    }
    __syncthreads();
    // x on the tile and 2 halo cells (local [1, WX-1) x [1, WY-1), rows of
    // even width): the k-th red and the k-th black cell in one thread, so no
    // wave runs both colours' branches
    const int par = (gx0 + gy0) & 1;
    constexpr int XP = (WX - 2) / 2;   // cells of one colour per row
    for (int k = (int)threadIdx.x; k < XP * (WY - 2); k += NT) {
        const int row = k / XP, m = k - row * XP, ly = 1 + row;
        const int ir = ly * WX + tile_color_x(m, ly, par, 0);
        const int i = ly * WX + tile_color_x(m, ly, par, 1);
        sX[ir] = (T)((R)sB[ir] * (R)sI[ir]);
        auto red = [&](int j) { return (R)sB[j] * (R)sI[j]; };
        R acc = 0.0;
        acc += (R)sC0[i] * red(i - 1);
        acc += (R)sC0[i + 1] * red(i + 1);
        acc += (R)sC1[i] * red(i - WX);
        acc += (R)sC1[i + WX] * red(i + WX);
        sX[i] = (T)(((R)sB[i] + acc) * (R)sI[i]);
    }
    __syncthreads();
    // residual on the tile and 1 halo cell (local [2, WX-2) x [2, WY-2))
    constexpr int RW = WX - 4;
    for (int j = (int)threadIdx.x; j < RW * (WY - 4); j += NT) {
        const int ry = j / RW, i = (ry + 2) * WX + (j - ry * RW) + 2;
        const R xc = (R)sX[i];
        R acc = (R)sS[i] * xc;
        acc += (R)sC0[i] * (xc - (R)sX[i - 1]);
        acc += (R)sC0[i + 1] * (xc - (R)sX[i + 1]);
        acc += (R)sC1[i] * (xc - (R)sX[i - WX]);
        acc += (R)sC1[i + WX] * (xc - (R)sX[i + WX]);
        sR[i] = (T)((R)sB[i] - acc);
    }
    __syncthreads();
    // restriction (taps 2I-1 .. 2I+2 per axis; an absent tap has weight 0)
    constexpr int CX = kTFX / 2, CY = kTFY / 2;
    const int ncx = (int)gc.n[0], ncy = (int)gc.n[1];
    for (int j = (int)threadIdx.x; j < CX * CY; j += NT) {
        const int cy = j / CX, cx = j - cy * CX;
        const int I = tx * CX + cx, J = ty * CY + cy;
        if (I >= ncx || J >= ncy) continue;
        int fx[4], fy[4];
        R wx[4], wy[4];
        res_axis<R>(I, ncx, nx, gc.per[0], fx, wx);
        res_axis<R>(J, ncy, ny, gc.per[1], fy, wy);
        R v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = (2 * cy + H - 1 + q) * WX + 2 * cx + H - 1;
            R s = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) s += wx[e] * (R)sR[row + e];
            v += (wy[q] * (R)1.0) * s;
        }
        bc[I + ncx * J] = (T)v;
    }
    // x of the tile's own cells
    for (int j = (int)threadIdx.x; j < kTFX * kTFY; j += NT) {
        const int ly = j / kTFX, lx = j - ly * kTFX;
        const int gx = tx * kTFX + lx, gy = ty * kTFY + ly;
        if (gx < nx && gy < ny) xs[gx + nx * gy] = sX[(ly + H) * WX + lx + H];
    }
}

// Way up: red x += P e, black GS, red GS (the post-smoothing), with e the
// coarse correction xc and the pre-smoothed x read from xs.  Writes x on the
// tile (never read here, so tiles do not race on their halos).
template <typename T, int NT, typename BS, typename DOTS = NoDots>
__device__ inline void up_tile2(const Level<T> &L, const Geo &gc, const T *__restrict__ xc, const BS &b,
                                const T *__restrict__ xs, T *__restrict__ x, int tx, int ty, int skip,
                                DOTS dots = DOTS()) {
    using R = T;
    constexpr int H = 2, WX = kTFX + 2 * H, WY = kTFY + 2 * H, NL = WX * WY;
    constexpr int KL = (NL + NT - 1) / NT;
    __shared__ T sB[NL], sI[NL], sC0[NL], sC1[NL], sX[NL];
    const int nx = (int)L.g.n[0], ny = (int)L.g.n[1];
    const int px = L.g.per[0], py = L.g.per[1];
    const int gx0 = tx * kTFX - H, gy0 = ty * kTFY - H;
    // Stage as on the way down; the prolongation is evaluated for every
    // staged cell (at coordinate 0 for cells that do not exist) and kept for
    // the red cells only.
    T lb[KL], li[KL], l0[KL], l1[KL], lx_[KL];
    bool lv[KL], m0[KL], m1[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int i0 = (int)threadIdx.x + k * NT, i = i0 < NL ? i0 : NL - 1;
        const int ly = i / WX, lx = i - ly * WX;
        bool vx, vy;
        const int gx = tile_coord(gx0 + lx, nx, px, vx), gy = tile_coord(gy0 + ly, ny, py, vy);
        const bool v = vx && vy;
        const int g = v ? gx + nx * gy : 0;
        lb[k] = b.template at<T>(g);
        li[k] = L.invd[g];
        l0[k] = L.cs[0][g];
        l1[k] = L.cs[1][g];
        const int ia[3] = {v ? gx : 0, v ? gy : 0, 0};
        const R pe = prolong_at<T, 2>(L.g, gc, xc, ia);
        const T red = (v && ((gx0 + lx + gy0 + ly) & 1) == 0) ? (T)1 : (T)0;
        lx_[k] = (T)((R)xs[g] + pe) * red;
        lv[k] = v;
        m0[k] = v && (px || gx > 0);
        m1[k] = v && (py || gy > 0);
    }
    if (skip) return;
#pragma unroll
    for (int k = 0; k < KL; ++k) {
        const int i0 = (int)threadIdx.x + k * NT, i = i0 < NL ? i0 : NL - 1;
        const T fv = lv[k] ? (T)1 : (T)0;
        sB[i] = lb[k] * fv;
        sI[i] = li[k] * fv;
        sC0[i] = l0[k] * (m0[k] ? (T)1 : (T)0);
        sC1[i] = l1[k] * (m1[k] ? (T)1 : (T)0);
        sX[i] = lx_[k];
    }
    __syncthreads();
    auto gs = [&](int i) {
        R acc = 0.0;
        acc += (R)sC0[i] * (R)sX[i - 1];
        acc += (R)sC0[i + 1] * (R)sX[i + 1];
        acc += (R)sC1[i] * (R)sX[i - WX];
        acc += (R)sC1[i + WX] * (R)sX[i + WX];
        return (T)(((R)sB[i] + acc) * (R)sI[i]);
    };
    // black on the tile and 1 halo cell (local [1, WX-1) x [1, WY-1); reads
    // red cells only)
    const int par = (gx0 + gy0) & 1;
    constexpr int XP = (WX - 2) / 2;
    for (int k = (int)threadIdx.x; k < XP * (WY - 2); k += NT) {
        const int row = k / XP, m = k - row * XP, ly = 1 + row;
        const int i = ly * WX + tile_color_x(m, ly, par, 1);
        sX[i] = gs(i);
    }
    __syncthreads();
    // red on the tile (reads black cells only); both colours written out
    for (int j = (int)threadIdx.x; j < kTFX * kTFY; j += NT) {
        const int ly = j / kTFX, lx = j - ly * kTFX;
        const int gx = tx * kTFX + lx, gy = ty * kTFY + ly;
        if (gx >= nx || gy >= ny) continue;
        const int i = (ly + H) * WX + lx + H;
        const T v = ((gx + gy) & 1) == 0 ? gs(i) : sX[i];
        x[gx + nx * gy] = v;
        dots.add(gx + nx * gy, (double)v);
    }
    dots.template finish<NT>();
}

}  // namespace chns
