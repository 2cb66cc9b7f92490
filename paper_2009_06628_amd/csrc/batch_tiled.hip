// Tiled form of the batched ensemble (gfx950): every sweep of the step is one
// launch over the cells of ALL problems.  The cells of each level of each
// problem are cut into tiles of tile_cells cells; one 256-thread workgroup
// takes one tile (numbered so that each XCD owns a contiguous range of
// tiles).  Problems therefore share the whole chip whatever their size,
// instead of one workgroup per problem.  Each problem keeps its own solver
// scalars (Scal): reductions write one partial per tile, and a one-workgroup-
// per-problem kernel sums a problem's partials in tile order (deterministic).
// A problem whose solve has converged skips every later sweep of that solve.
// The levels of a problem that have at most kSBCells cells run in one
// workgroup per problem (the same V-cycle and set-up code as the persistent
// form).  Per-cell arithmetic is shared with the single-grid kernels.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "mgdev.h"
#include "plan.h"
#include "stepdev.h"
#include "tile2d.h"

namespace chns {

// solves of one step
enum TSolve { TS_CH = 0, TS_MOM0 = 1, TS_MOM1 = 2, TS_MOM2 = 3, TS_P = 4 };

template <typename TP>
__device__ inline const Slot<TP> &tslot(const BatchProb<TP> &P, int s) {
    return s == TS_CH ? P.chs : (s == TS_P ? P.pres : P.mom);
}
template <typename TP>
__device__ inline const double *tb_of(const BatchProb<TP> &P, int s) {
    return s == TS_CH ? P.rch : P.rhs;
}
template <typename TP>
__device__ inline double *tx_of(const BatchProb<TP> &P, int s, const BatchState &st) {
    return s == TS_CH ? P.phihat : (s == TS_P ? st.p + P.off : P.ustar[s - TS_MOM0]);
}

// The tile of this workgroup (uniform); false for padding.
__device__ inline bool tile_of(const BTile *__restrict__ tiles, int ntiles, BTile &t) {
    const int i = xcd_block();
    if (i >= ntiles) return false;
    t = tiles[i];
    return t.prob >= 0;
}

#define TILE_LOOP(t) for (int c = (t).c0 + (int)threadIdx.x; c < (t).c1; c += (int)blockDim.x)

// ---------------------------------------------------------------------------
// step phases (FP64), over the level-0 tiles
// ---------------------------------------------------------------------------
// (one kernel per phase, so that the light phases are not held to the
// register count of the momentum set-up: 97 VGPRs for all of them in one)
template <typename TP, int DIM, int PHASE>
__global__ void __launch_bounds__(kTileBlock) k_t_phase(const BatchProb<TP> *__restrict__ probs,
                                                        const BTile *__restrict__ tiles, int ntiles, BatchState st,
                                                        int a) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    const Geo &g = P.g;
    const StepConst &k = P.k;
    double *phi = st.phi + P.off, *mu = st.mu + P.off, *pr = st.p + P.off;
    const U3 uc{{st.u[0] + P.off, st.u[1] + P.off, DIM == 3 ? st.u[2] + P.off : nullptr}};
    const W3 uw{{st.u[0] + P.off, st.u[1] + P.off, DIM == 3 ? st.u[2] + P.off : nullptr}};
    const U3 usc{{P.ustar[0], P.ustar[1], P.ustar[2]}};
    const W3 opcs{{P.op.cs[0], P.op.cs[1], P.op.cs[2]}};
    if constexpr (PHASE == 0) {
        TILE_LOOP(t) ch_rhs_cell<DIM>(g, k, phi, uc, P.rch, P.phihat, c);
    } else if constexpr (PHASE == 1) {
        TILE_LOOP(t) mu_cell<DIM>(g, k, phi, P.phihat, mu, c);
    } else if constexpr (PHASE == 2) {
        TILE_LOOP(t) phi_update_cell<DIM>(g, k, phi, uc, mu, P.phi_new, c);
    } else if constexpr (PHASE == 3) {
        TILE_LOOP(t) mom_setup_cell<DIM>(g, k, a, phi, P.phi_new, mu, uc, P.op.s, opcs, P.rhs, P.ustar[a], 0, c);
    } else if constexpr (PHASE == 4) {
        TILE_LOOP(t) p_setup_cell<DIM>(g, k, P.phi_new, usc, P.op.s, opcs, P.rhs, kPCoef | kPRhs, c);
    } else {
        TILE_LOOP(t) project_cell<DIM>(g, k, P.phi_new, usc, pr, phi, uw, c);
    }
}

// mean removal of the pressure right-hand side (which = 0) or the pressure
// (which = 1): tile partials, then every tile subtracts its problem's mean
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_sum(const BatchProb<TP> *__restrict__ probs,
                                                      const BTile *__restrict__ tiles, int ntiles, BatchState st,
                                                      int which, double *__restrict__ part) {
    __shared__ double lds[kTileBlock / kWave];
    BTile t;
    const bool ok = tile_of(tiles, ntiles, t);
    double acc = 0.0;
    if (ok) {
        const BatchProb<TP> &P = probs[t.prob];
        const double *x = which ? st.p + P.off : P.rhs;
        TILE_LOOP(t) acc += x[c];
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[xcd_block()] = s;
}

template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_sub_mean(const BatchProb<TP> *__restrict__ probs,
                                                           const BTile *__restrict__ tiles, int ntiles, BatchState st,
                                                           int which, const double *__restrict__ part) {
    __shared__ double lds[kTileBlock / kWave];
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    double v = 0.0;
    for (int i = P.t0 + (int)threadIdx.x; i < P.t1; i += (int)blockDim.x) v += part[i];
    const double m = block_sum_all(v, lds) / (double)P.g.N;
    double *x = which ? st.p + P.off : P.rhs;
    TILE_LOOP(t) x[c] -= m;
}

// ---------------------------------------------------------------------------
// multigrid set-up of the variable hierarchy (after the level-0 coefficients
// were written into P.op)
// ---------------------------------------------------------------------------
// op 0: level-0 coefficients in the hierarchy's precision (l = 0) or the
// coarsened coefficients of level l >= 1; op 1: inverse diagonals of level l
// (a separate launch: it reads the upper neighbour's coefficients, which
// other workgroups write in op 0)
template <typename TP, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_setup_level(const BatchProb<TP> *__restrict__ probs,
                                                              const BTile *__restrict__ tiles, int ntiles, int l,
                                                              int op) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    const Slot<TP> &S = P.mom;
    if (op == 0) {
        if (l == 0) {
            if (sizeof(TP) < sizeof(double)) {
                const Level<TP> &L0 = S.lev[0];
                TILE_LOOP(t) {
                    L0.s[c] = (TP)P.op.s[c];
#pragma unroll
                    for (int b = 0; b < DIM; ++b) L0.cs[b][c] = (TP)P.op.cs[b][c];
                }
            }
        } else if (l < P.lsb) {
            TILE_LOOP(t) coarsen_cell<TP, DIM>(S.lev[l - 1], S.lev[l], c);
        }
        return;
    }
    if (l >= P.lsb) return;   // the single-workgroup set-up does these levels
    TILE_LOOP(t) invd_cell<TP, DIM>(S.lev[l], c);
}

// The small levels and the coarsest inverse, one workgroup per problem.
// singular: the pressure hierarchy (same arrays as the momentum one).
template <typename TP, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_t_setup_small(const BatchProb<TP> *__restrict__ probs, int singular) {
    __shared__ SetupLdsPP sh;
    const BatchProb<TP> &P = probs[blockIdx.x];
    setup_block_dev<TP, DIM>(singular ? P.pres : P.mom, P.lsb, sh);
}

// ---------------------------------------------------------------------------
// V-cycle sweeps on the levels above lsb.  Level 0 reads its right-hand side
// from the CG residual r (bsel 0, FP64), the scratch w (bsel 1, TP) or the
// residual rounded to TP (bsel 2, the value the sweeps would round r to) and
// writes z (xsel 0) or w (xsel 1); coarser levels use their own b, x.
// ---------------------------------------------------------------------------
template <typename TP, typename TB>
__device__ inline const TB *level_b(const BatchProb<TP> &P, const Slot<TP> &S, int l, int bsel) {
    if (l) return (const TB *)(const void *)S.lev[l].b;
    if (bsel == 2) return (const TB *)(const void *)P.rp;
    return bsel ? (const TB *)(const void *)P.w : (const TB *)(const void *)P.r;
}
template <typename TP>
__device__ inline TP *level_x(const BatchProb<TP> &P, const Slot<TP> &S, int l, int xsel) {
    return l ? S.lev[l].x : (xsel ? P.w : P.z);
}

// op: 0 presmooth, 1 residual, 4 prolong-add, 5 black GS, 6 red GS (3D; the
// 2D V-cycle runs the fused tile passes)
template <typename TP, typename TB, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_sweep(const BatchProb<TP> *__restrict__ probs,
                                                        const BTile *__restrict__ tiles, int ntiles, int s, int l,
                                                        int bsel, int xsel, int op) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    if (P.sc->done || l >= P.lsb) return;
    const Slot<TP> &S = tslot(P, s);
    const Level<TP> &L = S.lev[l];
    const TB *b = level_b<TP, TB>(P, S, l, bsel);
    TP *x = level_x(P, S, l, xsel);
    switch (op) {
        case 0: TILE_LOOP(t) presmooth_cell<TP, TB, DIM>(L, b, x, c); break;
        case 1: TILE_LOOP(t) residual_cell<TP, TB, DIM>(L, b, x, c); break;
        case 4:
            TILE_LOOP(t) {
                int ia[3];
                coords_of<DIM>(L.g, c, ia);
                x[c] = (TP)(x[c] + prolong_at<TP, DIM>(L.g, S.lev[l + 1].g, S.lev[l + 1].x, ia));
            }
            break;
        default: TILE_LOOP(t) gs_color_cell<TP, TB, DIM>(L, b, x, op == 5 ? 1 : 0, c); break;
    }
}

// 2D: the fused way down / way up of level l over the kTFX x kTFY tiles of
// every problem whose level l lies above its single-workgroup levels (the
// tile list holds only those); same bodies as the single-grid kernels.  The
// level's residual array carries the smoothed x from the way down to the
// way up.
template <typename TP, typename TB>
__global__ void __launch_bounds__(kTileThreadsBatch) k_t_down2(const BatchProb<TP> *__restrict__ probs,
                                                          const BTile *__restrict__ tiles, int ntiles, int s, int l,
                                                          int bsel) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    const Slot<TP> &S = tslot(P, s);
    down_tile2<TP, kTileThreadsBatch>(S.lev[l], S.lev[l + 1].g, RhsStored<TB>{level_b<TP, TB>(P, S, l, bsel)},
                                      S.lev[l].r, S.lev[l + 1].b, t.c0, t.c1, P.sc->done);
}

template <typename TP, typename TB>
__global__ void __launch_bounds__(kTileThreadsBatch) k_t_up2(const BatchProb<TP> *__restrict__ probs,
                                                        const BTile *__restrict__ tiles, int ntiles, int s, int l,
                                                        int bsel, int xsel) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    const Slot<TP> &S = tslot(P, s);
    up_tile2<TP, kTileThreadsBatch>(S.lev[l], S.lev[l + 1].g, (const TP *)S.lev[l + 1].x,
                                    RhsStored<TB>{level_b<TP, TB>(P, S, l, bsel)}, (const TP *)S.lev[l].r,
                                    level_x(P, S, l, xsel), t.c0, t.c1, P.sc->done);
}

// restriction of level l's residual into level l + 1 (tiles of level l + 1)
template <typename TP, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_restrict(const BatchProb<TP> *__restrict__ probs,
                                                           const BTile *__restrict__ tiles, int ntiles, int s, int l) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    if (P.sc->done || l >= P.lsb) return;
    const Slot<TP> &S = tslot(P, s);
    TILE_LOOP(t) restrict_cell<TP, DIM>(S.lev[l].g, S.lev[l + 1].g, S.lev[l].r, S.lev[l + 1].b, c);
}

// levels lsb .. coarsest of every active problem whose plan allows it, one
// workgroup per problem, out of LDS: the single-grid kernel's copy, V-cycle
// and write-back of x.  The launch provides the largest LDS any problem
// takes.
template <typename TP, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_t_vcycle_small_lds(const BatchProb<TP> *__restrict__ probs, int s) {
    extern __shared__ uint4 lds_words[];
    const BatchProb<TP> &P = probs[blockIdx.x];
    if (P.vlds == 0 || P.sc->done) return;
    const Slot<TP> &S = tslot(P, s);
    const int l0 = P.lsb;
    char *lds = (char *)lds_words;
    const char *base = (const char *)S.lev[l0].s;
    const LdsCopy cp = P.vcp;   // a private copy: the LDS stores cannot alias it
    copy_to_lds(lds_words, (const uint4 *)base, cp);
    __syncthreads();
    vcycle_lds_dev<TP, DIM>(S, l0, lds, base);
    const TP *xl = lds_image(lds, base, S.lev[l0].x);
    TP *xg = S.lev[l0].x;
    LDS_LOOP(S.lev[l0].g.N) xg[c] = xl[c];
}

// the same levels of the other active problems, from global memory
template <typename TP, typename TB, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_t_vcycle_small(const BatchProb<TP> *__restrict__ probs, int s,
                                                               int bsel, int xsel) {
    const BatchProb<TP> &P = probs[blockIdx.x];
    if (P.vlds > 0 || P.sc->done) return;
    const Slot<TP> &S = tslot(P, s);
    const int l0 = P.lsb;
    if (l0 == 0)
        vcycle_block_dev<TP, TB, DIM>(S, 0, level_b<TP, TB>(P, S, 0, bsel), level_x(P, S, 0, xsel));
    else
        vcycle_block_dev<TP, TP, DIM>(S, l0, (const TP *)S.lev[l0].b, S.lev[l0].x);
}

// Allow k_t_vcycle_small_lds the LDS of one workgroup (once per instantiation;
// called when the tile lists are built, outside any graph capture).
template <typename TP, int DIM>
static void vcycle_small_attrs() {
    static const bool once = [] {   // thread-safe one-time initialisation
        (void)hipFuncSetAttribute((const void *)k_t_vcycle_small_lds<TP, DIM>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsVcycleBytes);
        return true;
    }();
    (void)once;
}

// ---------------------------------------------------------------------------
// preconditioned CG over the level-0 tiles; scalars per problem
// ---------------------------------------------------------------------------

// r = b - A x; partials b.b and r.r.  CH: t = L x must be current.
template <typename TP, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_cg_init(const BatchProb<TP> *__restrict__ probs,
                                                          const BTile *__restrict__ tiles, int ntiles, BatchState st,
                                                          int s, double *__restrict__ p0, double *__restrict__ p1) {
    __shared__ double lds[kTileBlock / kWave];
    BTile t;
    const bool ok = tile_of(tiles, ntiles, t);
    double bb = 0.0, rr = 0.0;
    if (ok) {
        const BatchProb<TP> &P = probs[t.prob];
        const Geo &g = P.g;
        const double *b = tb_of(P, s);
        const double *x = tx_of(P, s, st);
        double *r = P.r;
        TP *rp = P.rp;
        if (s == TS_CH) {
            const ChOp ch = P.ch;
            const double *tt = P.t;
            auto tv = [&](int e) { return tt[e]; };
            TILE_LOOP(t) {
                int ia[3];
                coords_of<DIM>(g, c, ia);
                const double Mx = x[c] - ch.a * tt[c] + ch.b * lap_at<DIM>(g, c, ia, ch.ih2, tv);
                const double bc = b[c], rc = bc - Mx;
                r[c] = rc;
                if (rp) rp[c] = (TP)rc;
                bb += bc * bc;
                rr += rc * rc;
            }
        } else {
            TILE_LOOP(t) {
                int ia[3];
                coords_of<DIM>(g, c, ia);
                const double bc = b[c], rc = bc - apply_at<double, DIM>(P.op, x, c, ia);
                r[c] = rc;
                if (rp) rp[c] = (TP)rc;
                bb += bc * bc;
                rr += rc * rc;
            }
        }
    }
    const double a0 = block_sum(bb, lds);
    const double a1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        p0[xcd_block()] = a0;
        p1[xcd_block()] = a1;
    }
}

// CH: t = L x (x the current iterate)
template <typename TP, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_ch_lap_x(const BatchProb<TP> *__restrict__ probs,
                                                           const BTile *__restrict__ tiles, int ntiles, BatchState st) {
    BTile t;
    if (!tile_of(tiles, ntiles, t)) return;
    const BatchProb<TP> &P = probs[t.prob];
    const double *x = tx_of(P, TS_CH, st);
    auto xv = [&](int e) { return x[e]; };
    TILE_LOOP(t) {
        int ia[3];
        coords_of<DIM>(P.g, c, ia);
        P.t[c] = lap_at<DIM>(P.g, c, ia, P.ch.ih2, xv);
    }
}

__device__ inline double sum_tiles(const double *__restrict__ part, int t0, int t1, double *lds) {
    double v = 0.0;
    for (int i = t0 + (int)threadIdx.x; i < t1; i += (int)blockDim.x) v += part[i];
    return block_sum_all(v, lds);
}

// one workgroup per problem: solver scalars from the b.b, r.r partials.
// round > 0 (refinement): a problem already converged stays done.
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_fin_init(const BatchProb<TP> *__restrict__ probs, int s,
                                                           const double *__restrict__ p0,
                                                           const double *__restrict__ p1) {
    __shared__ double lds[kTileBlock / kWave];
    const BatchProb<TP> &P = probs[blockIdx.x];
    const double tb = sum_tiles(p0, P.t0, P.t1, lds);
    const double tr = sum_tiles(p1, P.t0, P.t1, lds);
    if (threadIdx.x == 0) {
        Scal *sc = P.sc;
        const double rtol = s == TS_CH ? P.rtol_ch : (s == TS_P ? P.rtol_p : P.rtol_mom);
        sc->bb = tb > tr ? tb : tr;
        sc->rr = tr;
        sc->rtol2 = rtol * rtol;
        sc->max_iter = P.max_iter;
        sc->beta = 0.0;
        sc->rz = 0.0;
        sc->zmean = 0.0;
        sc->alpha = 0.0;
        sc->done = 0;
        if (!isfinite(tr) || !isfinite(tb)) {
            sc->nonfinite = 1;
            sc->done = 1;
        } else if (tr <= sc->rtol2 * sc->bb) {
            sc->done = 1;
        }
    }
}

// start of a solve: iteration counters and flags
template <typename TP>
__global__ void k_t_solve_begin(const BatchProb<TP> *__restrict__ probs, int nprob) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nprob; i += gridDim.x * blockDim.x) {
        Scal *sc = probs[i].sc;
        sc->iter = 0;
        sc->unconverged = 0;
        sc->nonfinite = 0;
    }
}

// partials of r.z, sum z, sum r
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_rz(const BatchProb<TP> *__restrict__ probs,
                                                     const BTile *__restrict__ tiles, int ntiles,
                                                     double *__restrict__ p0, double *__restrict__ p1,
                                                     double *__restrict__ p2, int singular) {
    __shared__ double lds[kTileBlock / kWave];
    BTile t;
    const bool ok = tile_of(tiles, ntiles, t);
    double arz = 0.0, az = 0.0, ar = 0.0;
    if (ok) {
        const BatchProb<TP> &P = probs[t.prob];
        if (!P.sc->done) {
            const double *r = P.r;
            const TP *z = P.z;
            TILE_LOOP(t) {
                const double rc = r[c], zc = (double)z[c];
                arz += rc * zc;
                az += zc;
                ar += rc;
            }
        }
    }
    const double s0 = block_sum(arz, lds);
    const double s1 = singular ? block_sum(az, lds) : 0.0;
    const double s2 = singular ? block_sum(ar, lds) : 0.0;
    if (threadIdx.x == 0) {
        const int i = xcd_block();
        p0[i] = s0;
        p1[i] = s1;
        p2[i] = s2;
    }
}

// one workgroup per problem: rz, zmean, beta (as in the single-grid solver)
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_fin_rz(const BatchProb<TP> *__restrict__ probs,
                                                         const double *__restrict__ p0,
                                                         const double *__restrict__ p1,
                                                         const double *__restrict__ p2, int first, int singular) {
    __shared__ double lds[kTileBlock / kWave];
    const BatchProb<TP> &P = probs[blockIdx.x];
    Scal *sc = P.sc;
    if (sc->done) return;
    const double trz = sum_tiles(p0, P.t0, P.t1, lds);
    const double tz = singular ? sum_tiles(p1, P.t0, P.t1, lds) : 0.0;
    const double tr = singular ? sum_tiles(p2, P.t0, P.t1, lds) : 0.0;
    if (threadIdx.x == 0) {
        const double zm = singular ? tz / (double)P.g.N : 0.0;
        const double rz = trz - zm * tr;
        sc->zmean = zm;
        sc->beta = (first || sc->rz == 0.0) ? 0.0 : rz / sc->rz;
        sc->rz = rz;
        if (!isfinite(rz)) {
            sc->nonfinite = 1;
            sc->done = 1;
        }
    }
}

// p_new = (z - zmean) + beta p_old; q = A p_new; partial p.q.  CH: first
// half (p_new, t = L p_new) with half = 0, second half (q) with half = 1.
// Slot operator in 2D: p of the tile's cells and one row on each side is
// formed once into an LDS window, where it was evaluated at all five stencil
// points of every cell (the same expression, so the same values; a
// neighbour outside the window, across a periodic y boundary, is evaluated
// directly).
constexpr int kApplyWin = 2048;   // window cells: tile + 2 rows (else no window)
template <typename TP, int DIM>
__global__ void __launch_bounds__(kTileBlock) k_t_apply(const BatchProb<TP> *__restrict__ probs,
                                                        const BTile *__restrict__ tiles, int ntiles, int s, int k,
                                                        int half, double *__restrict__ part) {
    __shared__ double lds[kTileBlock / kWave];
    __shared__ double pw[DIM == 2 ? kApplyWin : 1];
    BTile t;
    const bool ok = tile_of(tiles, ntiles, t);
    double acc = 0.0;
    if (ok) {
        const BatchProb<TP> &P = probs[t.prob];
        const Scal *sc = P.sc;
        if (!sc->done) {
            const Geo &g = P.g;
            double *pnew = (k & 1) ? P.p1 : P.p0;
            const double *pold = (k & 1) ? P.p0 : P.p1;
            const TP *z = P.z;
            const double beta = sc->beta, zm = sc->zmean;
            auto pv = [&](int e) { return ((double)z[e] - zm) + (beta != 0.0 ? beta * pold[e] : 0.0); };
            if (s == TS_CH) {
                const ChOp ch = P.ch;
                if (half == 0) {
                    TILE_LOOP(t) {
                        int ia[3];
                        coords_of<DIM>(g, c, ia);
                        pnew[c] = pv(c);
                        P.t[c] = lap_at<DIM>(g, c, ia, ch.ih2, pv);
                    }
                } else {
                    const double *tt = P.t;
                    auto tv = [&](int e) { return tt[e]; };
                    TILE_LOOP(t) {
                        int ia[3];
                        coords_of<DIM>(g, c, ia);
                        const double pc = pnew[c];
                        const double qc = pc - ch.a * tt[c] + ch.b * lap_at<DIM>(g, c, ia, ch.ih2, tv);
                        P.q[c] = qc;
                        acc += pc * qc;
                    }
                }
            } else {
                const Level<double> &L = P.op;
                // window [w0, w1) of cells; the tile (hence win) is uniform
                // over the workgroup, so the barrier is reached by all
                const int w0 = t.c0 - (int)g.n[0], w1 = t.c1 + (int)g.n[0];
                const bool win = DIM == 2 && w1 - w0 <= kApplyWin;
                if (win) {
                    const int N = (int)g.N;
                    for (int e = w0 + (int)threadIdx.x; e < w1; e += (int)blockDim.x)
                        if (e >= 0 && e < N) pw[e - w0] = pv(e);
                    __syncthreads();
                }
                auto pg = [&](int e) { return win && e >= w0 && e < w1 ? pw[e - w0] : pv(e); };
                TILE_LOOP(t) {
                    int ia[3];
                    coords_of<DIM>(g, c, ia);
                    const double pc = pg(c);
                    double qc = L.s[c] * pc;
#pragma unroll
                    for (int bx = 0; bx < DIM; ++bx) {
                        const int lo = nb_lo(g, c, ia[bx], bx);
                        const int hi = nb_hi(g, c, ia[bx], bx);
                        const int lc = lo >= 0 ? lo : c, hc = hi >= 0 ? hi : c;
                        const double vl = pg(lc), vh = pg(hc);
                        const double wl = L.cs[bx][c], wh = L.cs[bx][hc];
                        qc += (lo >= 0 ? wl : 0.0) * (pc - vl);
                        qc += (hi >= 0 ? wh : 0.0) * (pc - vh);
                    }
                    pnew[c] = pc;
                    P.q[c] = qc;
                    acc += pc * qc;
                }
            }
        }
    }
    if (half == 0 && s == TS_CH) return;   // uniform: no partial for the first CH half
    const double v = block_sum(acc, lds);
    if (threadIdx.x == 0) part[xcd_block()] = v;
}

// alpha = rz / (sum of the problem's p.q partials); x += alpha p;
// r -= alpha q; partial r.r
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_update(const BatchProb<TP> *__restrict__ probs,
                                                         const BTile *__restrict__ tiles, int ntiles, BatchState st,
                                                         int s, int k, const double *__restrict__ part_pq,
                                                         double *__restrict__ part_rr) {
    __shared__ double lds[kTileBlock / kWave];
    BTile t;
    const bool ok = tile_of(tiles, ntiles, t);
    double acc = 0.0;
    bool active = false;
    const BatchProb<TP> *Pp = nullptr;
    if (ok) {
        Pp = &probs[t.prob];
        active = !Pp->sc->done;
    }
    if (active) {   // uniform over the workgroup
        const BatchProb<TP> &P = *Pp;
        const double pq = sum_tiles(part_pq, P.t0, P.t1, lds);
        const double alpha = pq != 0.0 ? P.sc->rz / pq : 0.0;
        const double *pn = (k & 1) ? P.p1 : P.p0;
        double *x = tx_of(P, s, st);
        double *r = P.r;
        TP *rp = P.rp;
        const double *q = P.q;
        TILE_LOOP(t) {
            x[c] += alpha * pn[c];
            const double rc = r[c] - alpha * q[c];
            r[c] = rc;
            if (rp) rp[c] = (TP)rc;
            acc += rc * rc;
        }
    }
    const double v = block_sum(acc, lds);
    if (threadIdx.x == 0) part_rr[xcd_block()] = v;
}

// one workgroup per problem: r.r, iteration count, convergence
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_fin_rr(const BatchProb<TP> *__restrict__ probs,
                                                         const double *__restrict__ part) {
    __shared__ double lds[kTileBlock / kWave];
    const BatchProb<TP> &P = probs[blockIdx.x];
    Scal *sc = P.sc;
    if (sc->done) return;
    const double rr = sum_tiles(part, P.t0, P.t1, lds);
    if (threadIdx.x == 0) {
        sc->rr = rr;
        sc->iter += 1;
        if (!isfinite(rr)) {
            sc->nonfinite = 1;
            sc->done = 1;
        } else if (rr <= sc->rtol2 * sc->bb) {
            sc->done = 1;
        } else if (sc->iter >= sc->max_iter) {
            sc->unconverged = 1;
            sc->done = 1;
        }
    }
}

// number of problems whose solve is still running (one workgroup)
template <typename TP>
__global__ void __launch_bounds__(kTileBlock) k_t_count_active(const BatchProb<TP> *__restrict__ probs, int nprob,
                                                               int *__restrict__ out) {
    __shared__ double lds[kTileBlock / kWave];
    double v = 0.0;
    for (int i = threadIdx.x; i < nprob; i += blockDim.x) v += probs[i].sc->done ? 0.0 : 1.0;
    const double n = block_sum_all(v, lds);
    if (threadIdx.x == 0) *out = (int)n;
}

// statistics of the finished solve into the per-problem records; a problem
// that is not done here ran out of launched iterations (graph mode)
template <typename TP>
__global__ void k_t_record(const BatchProb<TP> *__restrict__ probs, int nprob, int s,
                           chns_batch_stats *__restrict__ stats) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nprob; i += gridDim.x * blockDim.x) {
        const Scal *sc = probs[i].sc;
        chns_batch_stats &S = stats[i];
        const double rel = sc->bb > 0.0 ? sqrt(sc->rr / sc->bb) : 0.0;
        const int bit = s == TS_CH ? 0 : (s == TS_P ? 4 : s);
        if (sc->unconverged || !sc->done) S.flags |= 1 << bit;
        if (sc->nonfinite) S.flags |= 1 << 5;
        S.total_iters += sc->iter;
        if (s == TS_CH) {
            S.iters_ch = sc->iter;
            S.res_ch = rel;
        } else if (s == TS_P) {
            S.iters_p = sc->iter;
            S.res_p = rel;
            S.steps += 1;   // one pressure solve per step
        } else {
            S.iters_mom[s - TS_MOM0] = sc->iter;
            S.res_mom[s - TS_MOM0] = rel;
        }
    }
}

// statistics of the direct CH solve: one application, no residual left
__global__ void k_t_record_direct(int nprob, chns_batch_stats *__restrict__ stats) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nprob; i += gridDim.x * blockDim.x) {
        stats[i].iters_ch = 1;
        stats[i].res_ch = 0.0;
        stats[i].total_iters += 1;
    }
}

}  // namespace chns

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
using namespace chns;

namespace {

#define THIPCHK(expr)                                                                                        \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess) return set_error(CHNS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename TP, int DIM>
struct Tiled {
    chns_batch *b;
    BatchState st;
    hipStream_t s;
    int graph;
    const BatchProb<TP> *probs() const { return (const BatchProb<TP> *)b->d_probs; }
    int nt(int l) const { return b->ntiles[l]; }
    const BTile *tl(int l) const { return b->d_tiles[l]; }
    int np() const { return b->count; }

    void phase(int ph, int a = 0) {
        const dim3 gr(nt(0)), bl(kTileBlock);
        switch (ph) {
            case 0: hipLaunchKernelGGL((k_t_phase<TP, DIM, 0>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
            case 1: hipLaunchKernelGGL((k_t_phase<TP, DIM, 1>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
            case 2: hipLaunchKernelGGL((k_t_phase<TP, DIM, 2>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
            case 3: hipLaunchKernelGGL((k_t_phase<TP, DIM, 3>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
            case 4: hipLaunchKernelGGL((k_t_phase<TP, DIM, 4>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
            default: hipLaunchKernelGGL((k_t_phase<TP, DIM, 5>), gr, bl, 0, s, probs(), tl(0), nt(0), st, a); break;
        }
    }
    void remove_mean(int which) {
        hipLaunchKernelGGL((k_t_sum<TP>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), st, which,
                           b->tpart0);
        hipLaunchKernelGGL((k_t_sub_mean<TP>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), st, which,
                           (const double *)b->tpart0);
    }
    void setup_var(int singular) {
        for (int l = 0; l < std::max(b->lg, 1); ++l)
            for (int op = 0; op < 2; ++op)
                hipLaunchKernelGGL((k_t_setup_level<TP, DIM>), dim3(nt(l)), dim3(kTileBlock), 0, s, probs(), tl(l),
                                   nt(l), l, op);
        hipLaunchKernelGGL((k_t_setup_small<TP, DIM>), dim3(np()), dim3(kSBThreads), 0, s, probs(), singular);
    }
    // the single-workgroup levels of every problem: out of LDS where the
    // problem's plan allows, else from global memory
    template <typename TB>
    void vcycle_small(int sv, int bsel, int xsel) {
        if (b->vlds_max > 0)
            hipLaunchKernelGGL((k_t_vcycle_small_lds<TP, DIM>), dim3(np()), dim3(kSBThreads), (size_t)b->vlds_max, s,
                               probs(), sv);
        if (b->vlds_some_global)
            hipLaunchKernelGGL((k_t_vcycle_small<TP, TB, DIM>), dim3(np()), dim3(kSBThreads), 0, s, probs(), sv,
                               bsel, xsel);
    }
    template <typename TB>
    void vcycle(int sv, int bsel, int xsel) {
        if (DIM == 2) {
            // fused passes: one launch per level on the way down and one on the way up
            for (int l = 0; l < b->lg; ++l) {
                if (l == 0)
                    hipLaunchKernelGGL((k_t_down2<TP, TB>), dim3(b->nt2[0]), dim3(kTileThreadsBatch), 0, s, probs(),
                                       b->d_t2[0], b->nt2[0], sv, 0, bsel);
                else
                    hipLaunchKernelGGL((k_t_down2<TP, TP>), dim3(b->nt2[l]), dim3(kTileThreadsBatch), 0, s, probs(),
                                       b->d_t2[l], b->nt2[l], sv, l, 0);
            }
            vcycle_small<TB>(sv, bsel, xsel);
            for (int l = b->lg - 1; l >= 0; --l) {
                if (l == 0)
                    hipLaunchKernelGGL((k_t_up2<TP, TB>), dim3(b->nt2[0]), dim3(kTileThreadsBatch), 0, s, probs(),
                                       b->d_t2[0], b->nt2[0], sv, 0, bsel, xsel);
                else
                    hipLaunchKernelGGL((k_t_up2<TP, TP>), dim3(b->nt2[l]), dim3(kTileThreadsBatch), 0, s, probs(),
                                       b->d_t2[l], b->nt2[l], sv, l, 0, 0);
            }
            return;
        }
        for (int l = 0; l < b->lg; ++l) {
            if (l == 0) {
                sweep<TB>(sv, 0, bsel, xsel, 0);
                sweep<TB>(sv, 0, bsel, xsel, 1);
            } else {
                sweep<TP>(sv, l, 0, 0, 0);
                sweep<TP>(sv, l, 0, 0, 1);
            }
            hipLaunchKernelGGL((k_t_restrict<TP, DIM>), dim3(nt(l + 1)), dim3(kTileBlock), 0, s, probs(), tl(l + 1),
                               nt(l + 1), sv, l);
        }
        vcycle_small<TB>(sv, bsel, xsel);
        for (int l = b->lg - 1; l >= 0; --l) {
            const int ops[3] = {4, 5, 6};
            for (int o = 0; o < 3; ++o) {
                if (l == 0)
                    sweep<TB>(sv, 0, bsel, xsel, ops[o]);
                else
                    sweep<TP>(sv, l, 0, 0, ops[o]);
            }
        }
    }
    template <typename TB>
    void sweep(int sv, int l, int bsel, int xsel, int op) {
        hipLaunchKernelGGL((k_t_sweep<TP, TB, DIM>), dim3(nt(l)), dim3(kTileBlock), 0, s, probs(), tl(l), nt(l), sv, l,
                           bsel, xsel, op);
    }
    // (with a lower-precision hierarchy the level-0 passes read r rounded to
    // it, written by the CG update: 4 instead of 8 bytes per cell of it)
    void precond(int sv) {
        constexpr bool low = sizeof(TP) != sizeof(double);
        if (sv == TS_CH) {
            if (low)
                vcycle<TP>(sv, 2, 1);       // r -> w
            else
                vcycle<double>(sv, 0, 1);
            vcycle<TP>(sv, 1, 0);           // w -> z
        } else {
            if (low)
                vcycle<TP>(sv, 2, 0);       // r -> z
            else
                vcycle<double>(sv, 0, 0);
        }
    }
    void rz(int sv, int first) {
        const int singular = sv == TS_P;
        hipLaunchKernelGGL((k_t_rz<TP>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), b->tpart0,
                           b->tpart1, b->tpart2, singular);
        hipLaunchKernelGGL((k_t_fin_rz<TP>), dim3(np()), dim3(kTileBlock), 0, s, probs(), (const double *)b->tpart0,
                           (const double *)b->tpart1, (const double *)b->tpart2, first, singular);
    }
    void iteration(int sv, int k) {
        if (sv == TS_CH)
            hipLaunchKernelGGL((k_t_apply<TP, DIM>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), sv, k,
                               0, b->tpart0);
        hipLaunchKernelGGL((k_t_apply<TP, DIM>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), sv, k, 1,
                           b->tpart0);
        hipLaunchKernelGGL((k_t_update<TP>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), st, sv, k,
                           (const double *)b->tpart0, b->tpart1);
        hipLaunchKernelGGL((k_t_fin_rr<TP>), dim3(np()), dim3(kTileBlock), 0, s, probs(), (const double *)b->tpart1);
        precond(sv);
        rz(sv, 0);
    }
    int active(int &n) {
        hipLaunchKernelGGL((k_t_count_active<TP>), dim3(1), dim3(kTileBlock), 0, s, probs(), np(), b->d_active);
        THIPCHK(hipMemcpyAsync(&n, b->d_active, sizeof(int), hipMemcpyDeviceToHost, s));
        THIPCHK(hipStreamSynchronize(s));
        return CHNS_OK;
    }
    // One solve for every problem.  The iteration count of a problem runs on
    // across refinement rounds (fin_init does not reset it).  Eager: rounds
    // continue while the true residual of any problem misses the tolerance,
    // iterations while any problem is active (host check per chunk).
    // Graph: round 0 launches budget iterations and, with an FP32 hierarchy,
    // one refinement round launches rbudget more (after its true-residual
    // check); problems that converge earlier skip the remaining launches.
    int solve(int sv, chns_batch_stats *stats) {
        const int kb = sv == TS_CH ? 0 : (sv == TS_P ? 2 : 1);
        const bool fp32 = sizeof(TP) < sizeof(double);
        const int rounds = graph ? (fp32 ? 2 : 1) : (fp32 ? kMaxRefine : 1);
        const int gb = (np() + 255) / 256;
        hipLaunchKernelGGL((k_t_solve_begin<TP>), dim3(gb), dim3(256), 0, s, probs(), np());
        int most0 = 0, most1 = 0;
        for (int round = 0; round < rounds; ++round) {
            if (sv == TS_CH)
                hipLaunchKernelGGL((k_t_ch_lap_x<TP, DIM>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0),
                                   st);
            hipLaunchKernelGGL((k_t_cg_init<TP, DIM>), dim3(nt(0)), dim3(kTileBlock), 0, s, probs(), tl(0), nt(0), st,
                               sv, b->tpart0, b->tpart1);
            hipLaunchKernelGGL((k_t_fin_init<TP>), dim3(np()), dim3(kTileBlock), 0, s, probs(), sv,
                               (const double *)b->tpart0, (const double *)b->tpart1);
            const int cap = graph ? (round == 0 ? b->budget[kb] : b->rbudget[kb]) : 1 << 30;
            if (graph && cap <= 0) continue;
            int n = 1;
            if (!graph) {
                if (int rc = active(n)) return rc;
                if (n == 0) break;
            }
            precond(sv);
            rz(sv, 1);
            int launched = 0;
            int chunk = round == 0 ? std::max(1, b->last_iters[kb] > 0 ? b->last_iters[kb] : 4) : 2;
            for (;;) {
                const int todo = graph ? cap : chunk;
                for (int it = 0; it < todo; ++it) iteration(sv, launched + it);
                launched += todo;
                if (graph) break;
                if (int rc = active(n)) return rc;
                if (n == 0 || launched > 100000) break;
                chunk = 2;
            }
            if (round == 0)
                most0 = launched;
            else
                most1 += launched;
        }
        if (!graph) {
            b->last_iters[kb] = std::max(1, most0);
            b->last_refine[kb] = most1;
        }
        hipLaunchKernelGGL((k_t_record<TP>), dim3(gb), dim3(256), 0, s, probs(), np(), sv, stats);
        return CHNS_OK;
    }
    int step(chns_batch_stats *stats) {
        phase(0);   // S1
        if (b->spec_on) {   // S2 by the direct solve
            const hipError_t e = spectral_batch_solve(b->spec, s);
            if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("CH direct solve: ") + hipGetErrorString(e));
            hipLaunchKernelGGL(k_t_record_direct, dim3((np() + 255) / 256), dim3(256), 0, s, np(), stats);
        } else if (int rc = solve(TS_CH, stats)) {
            return rc;
        }
        phase(1);   // S3
        phase(2);   // S4
        for (int a = 0; a < DIM; ++a) {
            phase(3, a);   // S5..S7 set-up
            setup_var(0);
            if (int rc = solve(TS_MOM0 + a, stats)) return rc;
        }
        phase(4);   // S8 set-up
        remove_mean(0);
        setup_var(1);
        if (int rc = solve(TS_P, stats)) return rc;
        remove_mean(1);
        phase(5);   // S9
        return CHNS_OK;
    }
};

template <typename TP, int DIM>
int run_tiled(chns_batch *b, const BatchState &st, int nsteps, int graph, hipStream_t s, chns_batch_stats *stats) {
    Tiled<TP, DIM> T{b, st, s, graph};
    for (int n = 0; n < nsteps; ++n)
        if (int rc = T.step(stats)) return rc;
    return CHNS_OK;
}

}  // namespace

namespace chns {

int tiled_build(chns_batch *b, int tile_cells) {
    if (tile_cells < kTileBlock || tile_cells % kTileBlock) return set_error(CHNS_EINVAL, "bad tile size");
    if (b->prec == CHNS_FP64) {
        if (b->dim == 2) vcycle_small_attrs<double, 2>(); else vcycle_small_attrs<double, 3>();
    } else {
        if (b->dim == 2) vcycle_small_attrs<float, 2>(); else vcycle_small_attrs<float, 3>();
    }
    for (int l = 0; l < kMaxLev; ++l) {
        std::vector<BTile> v;
        if (l < b->nlev_max) {
            for (int p = 0; p < b->count; ++p) {
                if (l >= b->nlev[p]) continue;
                const long long n = b->ncells[l][p];
                for (long long c0 = 0; c0 < n; c0 += tile_cells) {
                    BTile t{p, (int)c0, (int)std::min<long long>(n, c0 + tile_cells), 0};
                    v.push_back(t);
                }
            }
        }
        if (v.empty()) v.push_back(BTile{-1, 0, 0, 0});
        while (v.size() > 8 && (v.size() & 7)) v.push_back(BTile{-1, 0, 0, 0});
        if (v.size() > b->tile_cap[l]) return set_error(CHNS_EINVAL, "tile list exceeds its capacity");
        b->ntiles[l] = (int)v.size();
        if (l == 0) {
            // each problem's range of level-0 tiles (for its partial sums)
            std::vector<int> t0(b->count, 0), t1(b->count, 0);
            for (int i = (int)v.size() - 1; i >= 0; --i)
                if (v[i].prob >= 0) t0[v[i].prob] = i;
            for (int i = 0; i < (int)v.size(); ++i)
                if (v[i].prob >= 0) t1[v[i].prob] = i + 1;
            // patch the device table entries
            const size_t entry = b->prec == CHNS_FP64 ? sizeof(BatchProb<double>) : sizeof(BatchProb<float>);
            const size_t off_t0 = b->prec == CHNS_FP64 ? offsetof(BatchProb<double>, t0) : offsetof(BatchProb<float>, t0);
            for (int p = 0; p < b->count; ++p) {
                int pair[2] = {t0[p], t1[p]};
                hipError_t e = hipMemcpy((char *)b->d_probs + entry * p + off_t0, pair, sizeof pair,
                                         hipMemcpyHostToDevice);
                if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("tile table: ") + hipGetErrorString(e));
            }
        }
        hipError_t e = hipMemcpy(b->d_tiles[l], v.data(), sizeof(BTile) * v.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("tile table: ") + hipGetErrorString(e));
    }
    // 2D tiles of the fused passes (independent of tile_cells)
    for (int l = 0; l < kMaxLev; ++l) {
        std::vector<BTile> v;
        if (b->dim == 2 && l < b->lg) {
            for (int p = 0; p < b->count; ++p) {
                if (l >= b->lsb[p]) continue;
                const int ntx = (int)((b->lev_n[l][p][0] + kTFX - 1) / kTFX);
                const int nty = (int)((b->lev_n[l][p][1] + kTFY - 1) / kTFY);
                for (int ty = 0; ty < nty; ++ty)
                    for (int tx = 0; tx < ntx; ++tx) v.push_back(BTile{p, tx, ty, 0});
            }
        }
        if (v.empty()) v.push_back(BTile{-1, 0, 0, 0});
        while (v.size() > 8 && (v.size() & 7)) v.push_back(BTile{-1, 0, 0, 0});
        if (v.size() > b->t2_cap[l]) return set_error(CHNS_EINVAL, "2D tile list exceeds its capacity");
        b->nt2[l] = (int)v.size();
        hipError_t e = hipMemcpy(b->d_t2[l], v.data(), sizeof(BTile) * v.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("tile table: ") + hipGetErrorString(e));
    }
    b->tile_cells = tile_cells;
    return CHNS_OK;
}

int tiled_steps(chns_batch *b, const BatchState &st, int nsteps, int graph, hipStream_t s,
                chns_batch_stats *d_stats) {
    if (b->prec == CHNS_FP64)
        return b->dim == 2 ? run_tiled<double, 2>(b, st, nsteps, graph, s, d_stats)
                           : run_tiled<double, 3>(b, st, nsteps, graph, s, d_stats);
    return b->dim == 2 ? run_tiled<float, 2>(b, st, nsteps, graph, s, d_stats)
                       : run_tiled<float, 3>(b, st, nsteps, graph, s, d_stats);
}

}  // namespace chns
