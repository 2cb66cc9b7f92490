// Batched ensemble (gfx950): many independent problems of uneven size, each
// advanced through the whole split step S1..S9 by ONE workgroup inside a
// persistent kernel.  One launch per time step:
//   * workgroups pull problems from a device queue in longest-first order
//     (largest cell count first), so the makespan stays close to the mean
//     load; there is no synchronisation between workgroups;
//   * inside a problem every sweep is a workgroup-stride loop followed by a
//     workgroup barrier; the three kinds of linear solves run the same
//     preconditioned CG as the single-grid path (FP64 vectors and
//     reductions, the V-cycle in FP64 or, in the precision form, FP32 with an
//     FP64 true-residual refinement), with their convergence loops on the
//     device, so a step has data-independent control flow on the host and
//     nsteps launches are captured once into a hipGraph and replayed;
//   * per-cell arithmetic is shared with the single-grid kernels, so a batched
//     problem matches its own single-grid run up to the order of the sums.
// Workgroup size and workgroup count are chosen by chns_batch_autotune.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "mgdev.h"
#include "plan.h"
#include "solvers.h"
#include "stepdev.h"
#include "tile2d.h"

namespace chns {

// Solve outcome inside a workgroup.
struct PcgRes {
    int iters;
    double rel;
    int unconv, nonfinite;
};

constexpr int kBatchMaxThreads = 512;
constexpr int kBatchSBCells = 2048;   // tiled form: levels at or below this run in one workgroup

// first level of a problem that the single-workgroup part handles
static int batch_lsb(const Plan &P) {
    int lsb = 0;
    while (lsb < P.nlev - 1 && P.lev[lsb].N > kBatchSBCells) ++lsb;
    return lsb;
}

// r.z (with the singular projection), returned to every thread
template <typename TP>
__device__ inline double rz_block(int N, const double *__restrict__ r, const TP *__restrict__ z, int singular,
                                  double *red, double &zm) {
    double arz = 0.0, az = 0.0, ar = 0.0;
    BLOCK_LOOP(N) {
        const double rc = r[c], zc = (double)z[c];
        arz += rc * zc;
        az += zc;
        ar += rc;
    }
    const double trz = block_sum_all(arz, red);
    const double tz = singular ? block_sum_all(az, red) : 0.0;
    const double tr = singular ? block_sum_all(ar, red) : 0.0;
    zm = singular ? tz / (double)N : 0.0;
    return trz - zm * tr;
}

template <typename TP, int DIM>
__device__ __attribute__((noinline)) void precond_block(int kind, const Slot<TP> &SP, const double *r, TP *z, TP *w) {
    if (kind == OP_CH) {
        vcycle_block_dev<TP, double, DIM>(SP, 0, r, w);
        vcycle_block_dev<TP, TP, DIM>(SP, 0, w, z);
    } else {
        vcycle_block_dev<TP, double, DIM>(SP, 0, r, z);
    }
}

// Preconditioned CG on A x = b inside one workgroup; x holds the initial
// guess.  kind OP_SLOT: A = P.op (variable coefficients); OP_CH: the
// constant CH operator.  With an FP32 hierarchy the solve restarts from the
// FP64 true residual until it meets the tolerance (at most kMaxRefine
// rounds).  Ends with a workgroup barrier.
template <typename TP, int DIM>
__device__ __attribute__((noinline)) PcgRes pcg_block(const BatchProb<TP> &P, int kind, const Slot<TP> &SP, int singular,
                            const double *__restrict__ b, double *__restrict__ x, double rtol, int max_iter,
                            double *red) {
    const Geo &g = P.g;
    const int N = (int)g.N;
    const ChOp ch = P.ch;
    double *r = P.r, *q = P.q, *t = P.t;
    TP *z = P.z, *w = P.w;
    const double rtol2 = rtol * rtol;
    const int rounds = sizeof(TP) < sizeof(double) ? kMaxRefine : 1;
    PcgRes out{0, 0.0, 0, 0};
    for (int round = 0; round < rounds; ++round) {
        // r = b - A x
        double bb = 0.0, rr = 0.0;
        if (kind == OP_CH) {
            auto xv = [&](int e) { return x[e]; };
            BLOCK_LOOP(N) {
                int ia[3];
                coords_of<DIM>(g, c, ia);
                t[c] = lap_at<DIM>(g, c, ia, ch.ih2, xv);
            }
            __syncthreads();
            auto tv = [&](int e) { return t[e]; };
            BLOCK_LOOP(N) {
                int ia[3];
                coords_of<DIM>(g, c, ia);
                const double Mx = x[c] - ch.a * t[c] + ch.b * lap_at<DIM>(g, c, ia, ch.ih2, tv);
                const double bc = b[c], rc = bc - Mx;
                r[c] = rc;
                bb += bc * bc;
                rr += rc * rc;
            }
        } else {
            BLOCK_LOOP(N) {
                int ia[3];
                coords_of<DIM>(g, c, ia);
                const double bc = b[c], rc = bc - apply_at<double, DIM>(P.op, x, c, ia);
                r[c] = rc;
                bb += bc * bc;
                rr += rc * rc;
            }
        }
        const double tb = block_sum_all(bb, red);
        double rrt = block_sum_all(rr, red);
        const double bref = tb > rrt ? tb : rrt;
        if (!isfinite(tb) || !isfinite(rrt)) {
            out.nonfinite = 1;
            return out;
        }
        out.rel = bref > 0.0 ? sqrt(rrt / bref) : 0.0;
        if (rrt <= rtol2 * bref) {
            out.unconv = 0;
            return out;
        }
        // PCG from here
        precond_block<TP, DIM>(kind, SP, r, z, w);
        double zm = 0.0;
        double rz = rz_block<TP>(N, r, z, singular, red, zm);
        double beta = 0.0;
        double *pnew = P.p0, *pold = P.p1;
        int it = 0;
        out.unconv = 1;
        for (;;) {
            auto pv = [&](int e) { return ((double)z[e] - zm) + (beta != 0.0 ? beta * pold[e] : 0.0); };
            double pq = 0.0;
            if (kind == OP_CH) {
                BLOCK_LOOP(N) {
                    int ia[3];
                    coords_of<DIM>(g, c, ia);
                    pnew[c] = pv(c);
                    t[c] = lap_at<DIM>(g, c, ia, ch.ih2, pv);
                }
                __syncthreads();
                auto tv = [&](int e) { return t[e]; };
                BLOCK_LOOP(N) {
                    int ia[3];
                    coords_of<DIM>(g, c, ia);
                    const double pc = pnew[c];
                    const double qc = pc - ch.a * t[c] + ch.b * lap_at<DIM>(g, c, ia, ch.ih2, tv);
                    q[c] = qc;
                    pq += pc * qc;
                }
            } else {
                const Level<double> &L = P.op;
                BLOCK_LOOP(N) {
                    int ia[3];
                    coords_of<DIM>(g, c, ia);
                    const double pc = pv(c);
                    double qc = L.s[c] * pc;
#pragma unroll
                    for (int bx = 0; bx < DIM; ++bx) {
                        const int lo = nb_lo(g, c, ia[bx], bx);
                        const int hi = nb_hi(g, c, ia[bx], bx);
                        const int l = lo >= 0 ? lo : c, h = hi >= 0 ? hi : c;
                        const double vl = pv(l), vh = pv(h);
                        const double wl = L.cs[bx][c], wh = L.cs[bx][h];
                        qc += (lo >= 0 ? wl : 0.0) * (pc - vl);
                        qc += (hi >= 0 ? wh : 0.0) * (pc - vh);
                    }
                    pnew[c] = pc;
                    q[c] = qc;
                    pq += pc * qc;
                }
            }
            pq = block_sum_all(pq, red);
            const double alpha = pq != 0.0 ? rz / pq : 0.0;
            rr = 0.0;
            BLOCK_LOOP(N) {
                x[c] += alpha * pnew[c];
                const double rc = r[c] - alpha * q[c];
                r[c] = rc;
                rr += rc * rc;
            }
            rrt = block_sum_all(rr, red);
            ++it;
            out.rel = bref > 0.0 ? sqrt(rrt / bref) : 0.0;
            if (!isfinite(rrt)) {
                out.nonfinite = 1;
                out.iters += it;
                return out;
            }
            if (rrt <= rtol2 * bref) {
                out.unconv = 0;
                break;
            }
            if (it >= max_iter) break;
            precond_block<TP, DIM>(kind, SP, r, z, w);
            const double rzn = rz_block<TP>(N, r, z, singular, red, zm);
            if (!isfinite(rzn)) {
                out.nonfinite = 1;
                out.iters += it;
                return out;
            }
            beta = rz == 0.0 ? 0.0 : rzn / rz;
            rz = rzn;
            double *tmp = pnew;
            pnew = pold;
            pold = tmp;
        }
        out.iters += it;
        if (out.unconv) return out;
        // FP64 rounds are final; the precision form re-checks the true residual
    }
    return out;
}

__device__ inline void remove_mean_block(int N, double *x, double *red) {
    double acc = 0.0;
    BLOCK_LOOP(N) acc += x[c];
    const double m = block_sum_all(acc, red) / (double)N;
    BLOCK_LOOP(N) x[c] -= m;
    __syncthreads();
}

// Level-0 coefficients of a variable slot from the FP64 operator, then the
// hierarchy (inverse diagonals, coarse levels, coarsest inverse).
template <typename TP, int DIM>
__device__ __attribute__((noinline)) void prepare_slot(const BatchProb<TP> &P, const Slot<TP> &S, SetupLds &sh) {
    if (sizeof(TP) < sizeof(double)) {
        const Level<TP> &L0 = S.lev[0];
        BLOCK_LOOP(P.g.N) {
            L0.s[c] = (TP)P.op.s[c];
#pragma unroll
            for (int b = 0; b < DIM; ++b) L0.cs[b][c] = (TP)P.op.cs[b][c];
        }
        __syncthreads();
    }
    setup_block_dev<TP, DIM>(S, 0, sh);
}

// Statistics of one solve (written by thread 0 into the problem's record).
__device__ inline void record(PcgRes o, int bit, int *iters, double *res, int &flags, long long &total) {
    if (threadIdx.x == 0) {
        *iters = o.iters;
        *res = o.rel;
    }
    total += o.iters;
    if (o.unconv) flags |= 1 << bit;
    if (o.nonfinite) flags |= 1 << 5;
}

// S1..S9 of one problem by the calling workgroup.  part 0: all of them;
// part 1: S1 only; part 2: S3..S9, S2 having been solved directly in between.
template <typename TP, int DIM>
__device__ void batch_problem_step(const BatchProb<TP> &P, const BatchState &st, chns_batch_stats *S,
                                   SetupLds &sh, double *red, int part) {
    const Geo &g = P.g;
    const int N = (int)g.N;
    const StepConst &k = P.k;
    double *phi = st.phi + P.off, *mu = st.mu + P.off, *pr = st.p + P.off;
    const U3 uc{{st.u[0] + P.off, st.u[1] + P.off, DIM == 3 ? st.u[2] + P.off : nullptr}};
    const W3 uw{{st.u[0] + P.off, st.u[1] + P.off, DIM == 3 ? st.u[2] + P.off : nullptr}};
    const U3 usc{{P.ustar[0], P.ustar[1], P.ustar[2]}};
    const W3 opcs{{P.op.cs[0], P.op.cs[1], P.op.cs[2]}};
    int flags = 0;
    long long total = 0;
    PcgRes o;
    if (part != 2) {
        // S1, S2
        BLOCK_LOOP(N) ch_rhs_cell<DIM>(g, k, phi, uc, P.rch, P.phihat, c);
        __syncthreads();
        if (part == 1) return;
        o = pcg_block<TP, DIM>(P, OP_CH, P.chs, 0, P.rch, P.phihat, P.rtol_ch, P.max_iter, red);
        record(o, 0, &S->iters_ch, &S->res_ch, flags, total);
    } else {
        // S2 solved directly: one application, no residual left
        if (threadIdx.x == 0) {
            S->iters_ch = 1;
            S->res_ch = 0.0;
        }
        total += 1;
    }
    // S3, S4
    BLOCK_LOOP(N) mu_cell<DIM>(g, k, phi, P.phihat, mu, c);
    __syncthreads();
    BLOCK_LOOP(N) phi_update_cell<DIM>(g, k, phi, uc, mu, P.phi_new, c);
    __syncthreads();
    // S5..S7
    for (int a = 0; a < DIM; ++a) {
        BLOCK_LOOP(N) mom_setup_cell<DIM>(g, k, a, phi, P.phi_new, mu, uc, P.op.s, opcs, P.rhs, P.ustar[a], 0, c);
        __syncthreads();
        prepare_slot<TP, DIM>(P, P.mom, sh);
        o = pcg_block<TP, DIM>(P, OP_SLOT, P.mom, 0, P.rhs, P.ustar[a], P.rtol_mom, P.max_iter, red);
        record(o, 1 + a, &S->iters_mom[a], &S->res_mom[a], flags, total);
    }
    // S8
    BLOCK_LOOP(N) p_setup_cell<DIM>(g, k, P.phi_new, usc, P.op.s, opcs, P.rhs, kPCoef | kPRhs, c);
    __syncthreads();
    remove_mean_block(N, P.rhs, red);
    prepare_slot<TP, DIM>(P, P.pres, sh);
    o = pcg_block<TP, DIM>(P, OP_SLOT, P.pres, 1, P.rhs, pr, P.rtol_p, P.max_iter, red);
    record(o, 4, &S->iters_p, &S->res_p, flags, total);
    remove_mean_block(N, pr, red);
    // S9
    BLOCK_LOOP(N) project_cell<DIM>(g, k, P.phi_new, usc, pr, phi, uw, c);
    __syncthreads();
    if (threadIdx.x == 0) {
        S->flags |= flags;
        S->total_iters += total;
        S->steps += 1;
    }
}

// One time step of every problem.  Workgroups take problems from the queue
// (order[] lists them longest first) until it is empty.
template <typename TP, int DIM>
__global__ void __launch_bounds__(kBatchMaxThreads) k_batch_step(const BatchProb<TP> *__restrict__ probs,
                                                                 const int *__restrict__ order, int nprob,
                                                                 unsigned int *queue, BatchState st,
                                                                 chns_batch_stats *stats, int part) {
    __shared__ SetupLds sh;
    __shared__ double red[kBatchMaxThreads / kWave];
    __shared__ int s_t;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_t = (int)atomicAdd(queue, 1u);
        __syncthreads();
        // uniform across the workgroup: keep the problem index (and so every
        // table load below) in scalar registers
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        if (t >= nprob) break;
        const int i = __builtin_amdgcn_readfirstlane(order[t]);
        batch_problem_step<TP, DIM>(probs[i], st, stats + i, sh, red, part);
    }
}

// Constant CH hierarchy of every problem (one workgroup per problem).
template <typename TP, int DIM>
__global__ void __launch_bounds__(kBatchMaxThreads) k_batch_init(const BatchProb<TP> *__restrict__ probs, int nprob) {
    __shared__ SetupLds sh;
    for (int i = blockIdx.x; i < nprob; i += gridDim.x) {
        const BatchProb<TP> &P = probs[i];
        const Level<TP> &L0 = P.chs.lev[0];
        const double csv = sqrt(P.ch.b) * P.ch.ih2;
        BLOCK_LOOP(P.g.N) {
            L0.s[c] = (TP)1.0;
#pragma unroll
            for (int b = 0; b < DIM; ++b) L0.cs[b][c] = (TP)csv;
        }
        __syncthreads();
        setup_block_dev<TP, DIM>(P.chs, 0, sh);
    }
}

__global__ void k_batch_reset_queue(unsigned int *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) queue[0] = 0u;
}

__global__ void k_batch_reset_stats(chns_batch_stats *stats, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        chns_batch_stats z = {};
        stats[i] = z;
    }
}

}  // namespace chns

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace chns;

namespace {

#define BHIPCHK(expr)                                                                                         \
    do {                                                                                                      \
        hipError_t e_ = (expr);                                                                               \
        if (e_ != hipSuccess) return set_error(CHNS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename TP>
size_t layout_batch(Bump &B, int count, const Plan *plans, const chns_props *props, std::vector<BatchProb<TP>> *host,
                    chns_batch *b) {
    // tables first
    void *probs = B.take<BatchProb<TP>>((size_t)count);
    int *order = B.take<int>((size_t)count);
    unsigned int *queue = B.take<unsigned int>(64);
    chns_batch_stats *stats = B.take<chns_batch_stats>((size_t)count);
    long long tot = 0;
    for (int i = 0; i < count; ++i) tot += plans[i].lev[0].N;
    const int dim = plans[0].dim;
    double *backup = B.take<double>((size_t)tot * (3 + dim));
    // tiled form: per-problem scalars, tile lists (capacity for the smallest
    // tile), per-tile partial sums
    Scal *scal = B.take<Scal>((size_t)count);
    int *active = B.take<int>(64);
    BTile *tiles[kMaxLev];
    size_t cap[kMaxLev];
    for (int l = 0; l < kMaxLev; ++l) {
        size_t n = 8;
        for (int i = 0; i < count; ++i)
            if (l < plans[i].nlev) n += (size_t)((plans[i].lev[l].N + kTileBlock - 1) / kTileBlock);
        cap[l] = n + 8;
        tiles[l] = B.take<BTile>(cap[l]);
    }
    // 2D tiles of the fused V-cycle passes (levels above each problem's
    // single-workgroup levels)
    BTile *t2[kMaxLev];
    size_t cap2[kMaxLev];
    for (int l = 0; l < kMaxLev; ++l) {
        size_t n = 8;
        for (int i = 0; i < count; ++i) {
            const Plan &P = plans[i];
            if (P.dim != 2 || l >= batch_lsb(P)) continue;
            n += (size_t)((P.lev[l].n[0] + kTFX - 1) / kTFX) * (size_t)((P.lev[l].n[1] + kTFY - 1) / kTFY);
        }
        cap2[l] = n + 8;
        t2[l] = B.take<BTile>(cap2[l]);
    }
    double *tp0 = B.take<double>(cap[0]), *tp1 = B.take<double>(cap[0]), *tp2 = B.take<double>(cap[0]);
    if (b) {
        b->d_probs = probs;
        b->d_order = order;
        b->d_queue = queue;
        b->d_stats = stats;
        b->backup = backup;
        b->d_scal = scal;
        b->d_active = active;
        for (int l = 0; l < kMaxLev; ++l) {
            b->d_tiles[l] = tiles[l];
            b->tile_cap[l] = cap[l];
            b->d_t2[l] = t2[l];
            b->t2_cap[l] = cap2[l];
        }
        b->tpart0 = tp0;
        b->tpart1 = tp1;
        b->tpart2 = tp2;
    }
    long long off = 0;
    for (int i = 0; i < count; ++i) {
        const Plan &P = plans[i];
        const size_t N = (size_t)P.lev[0].N;
        BatchProb<TP> Q;
        memset(&Q, 0, sizeof Q);
        Q.g = P.lev[0];
        Q.off = off;
        off += (long long)N;
        Q.phi_new = B.take<double>(N);
        Q.phihat = B.take<double>(N);
        Q.rch = B.take<double>(N);
        for (int a = 0; a < 3; ++a) Q.ustar[a] = a < dim ? B.take<double>(N) : nullptr;
        Q.rhs = B.take<double>(N);
        Q.r = B.take<double>(N);
        Q.p0 = B.take<double>(N);
        Q.p1 = B.take<double>(N);
        Q.q = B.take<double>(N);
        Q.t = B.take<double>(N);
        Q.z = B.take<TP>(N);
        Q.w = B.take<TP>(N);
        Q.rp = sizeof(TP) != sizeof(double) ? B.take<TP>(N) : nullptr;
        carve_slot(B, P, Q.chs, 0);
        carve_slot(B, P, Q.mom, 0);
        Q.pres = Q.mom;
        Q.pres.singular = 1;
        const int nc = Q.mom.ncoarse;
        double *aug = nc > kLdsInverse ? B.take<double>((size_t)nc * nc) : nullptr;
        Q.chs.aug = Q.mom.aug = Q.pres.aug = aug;
        Q.op.g = Q.g;
        if (sizeof(TP) == sizeof(double)) {
            const Level<TP> &L0 = Q.mom.lev[0];
            Q.op.s = (double *)L0.s;
            for (int a = 0; a < 3; ++a) Q.op.cs[a] = (double *)L0.cs[a];
            Q.op.invd = (double *)L0.invd;
            Q.op.r = (double *)L0.r;
        } else {
            Q.op.s = B.take<double>(N);
            for (int a = 0; a < 3; ++a) Q.op.cs[a] = a < dim ? B.take<double>(N) : nullptr;
        }
        Q.sc = scal ? scal + i : nullptr;
        {
            Q.lsb = batch_lsb(P);   // first level of the single-workgroup part
            // the V-cycle of those levels out of LDS where it fits; one
            // plan serves every slot (same carving from a 256-byte boundary)
            Q.vlds = (int)lds_vcycle_bytes(Q.mom, Q.lsb);
            memset(&Q.vcp, 0, sizeof Q.vcp);
            if (Q.vlds) {
                Q.vcp = lds_copy_plan(Q.mom, Q.lsb);
                const LdsCopy c2 = lds_copy_plan(Q.chs, Q.lsb);
                if ((int)lds_vcycle_bytes(Q.chs, Q.lsb) != Q.vlds || memcmp(&c2, &Q.vcp, sizeof c2) != 0) Q.vlds = 0;
            }
            if (b) {
                b->vlds_max = std::max(b->vlds_max, Q.vlds);
                if (Q.vlds == 0) b->vlds_some_global = 1;
            }
        }
        if (host) {   // step constants and CH operator are filled in by the caller
            const chns_props &p = props[i];
            Q.rtol_ch = p.rtol_ch;
            Q.rtol_mom = p.rtol_mom;
            Q.rtol_p = p.rtol_p;
            Q.max_iter = p.max_iter;
            host->push_back(Q);
        }
    }
    if (b) b->total_cells = tot;
    // direct CH solve (2D): bases and tables of every problem shape
    bool spec_ok = dim == 2;
    for (int i = 0; i < count && spec_ok; ++i)
        for (int a = 0; a < 2; ++a)
            if (plans[i].lev[0].n[a] > kSpectralMaxN) spec_ok = false;
    std::vector<SpecGroup> groups;
    std::vector<std::vector<int>> members;
    if (spec_ok) {
        for (int i = 0; i < count; ++i) {
            const Geo &g = plans[i].lev[0];
            size_t k = 0;
            while (k < groups.size() && !(groups[k].nx == g.n[0] && groups[k].ny == g.n[1] &&
                                          groups[k].perx == g.per[0] && groups[k].pery == g.per[1]))
                ++k;
            if (k == groups.size()) {
                SpecGroup G;
                memset(&G, 0, sizeof G);
                G.nx = g.n[0];
                G.ny = g.n[1];
                G.perx = g.per[0];
                G.pery = g.per[1];
                groups.push_back(G);
                members.emplace_back();
            }
            groups[k].m += 1;
            members[k].push_back(i);
        }
        for (SpecGroup &G : groups) {
            const size_t m = (size_t)G.m;
            G.Q[0] = B.take<double>((size_t)G.nx * G.nx);
            G.Q[1] = B.take<double>((size_t)G.ny * G.ny);
            G.lam[0] = B.take<double>((size_t)G.nx);
            G.lam[1] = B.take<double>((size_t)G.ny);
            G.abh = B.take<double>(3 * m);
            G.r = (const double **)B.take<double *>(m);
            G.x = B.take<double *>(m);
            G.t0 = B.take<double *>(m);
            G.t1 = B.take<double *>(m);
        }
    }
    if (b) {
        b->spec = groups;
        b->spec_members = members;
    }
    return B.off;
}

// Tables and bases of the direct CH solve.  Off for 3D batches and for
// axes over kSpectralMaxN.
template <typename TP>
int spectral_batch_setup(chns_batch *b, const std::vector<BatchProb<TP>> &h) {
    b->spec_on = 0;
    if (b->spec.empty()) return CHNS_OK;
    for (size_t k = 0; k < b->spec.size(); ++k) {
        const SpecGroup &G = b->spec[k];
        const std::vector<int> &mem = b->spec_members[k];
        std::vector<double> Q, lam, abh;
        std::vector<const double *> r;
        std::vector<double *> x, t0, t1;
        for (int i : mem) {
            abh.push_back(h[i].ch.a);
            abh.push_back(h[i].ch.b);
            abh.push_back(h[i].ch.ih2);
            r.push_back(h[i].rch);
            x.push_back(h[i].phihat);
            t0.push_back(h[i].q);
            t1.push_back(h[i].t);
        }
        hipError_t e = hipSuccess;
        for (int a = 0; a < 2 && e == hipSuccess; ++a) {
            spectral_axis(a ? G.ny : G.nx, a ? G.pery : G.perx, 1.0, Q, lam);
            e = hipMemcpy(G.Q[a], Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(G.lam[a], lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        const size_t pm = sizeof(void *) * mem.size();
        if (e == hipSuccess) e = hipMemcpy(G.abh, abh.data(), abh.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void *)G.r, r.data(), pm, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void *)G.x, x.data(), pm, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void *)G.t0, t0.data(), pm, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void *)G.t1, t1.data(), pm, hipMemcpyHostToDevice);
        if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("CH bases: ") + hipGetErrorString(e));
    }
    b->spec_on = 1;
    return CHNS_OK;
}

int check_descs(int count, const chns_grid_desc *descs, std::vector<Plan> &plans) {
    if (count < 1) return set_error(CHNS_EINVAL, "count must be >= 1");
    if (!descs) return set_error(CHNS_EINVAL, "descs is NULL");
    plans.resize(count);
    for (int i = 0; i < count; ++i) {
        if (int rc = make_plan(&descs[i], plans[i])) return rc;
        if (descs[i].nphases != 2) return set_error(CHNS_EINVAL, "batched problems are two-phase (nphases = 2)");
        if (descs[i].dim != descs[0].dim || descs[i].precision != descs[0].precision)
            return set_error(CHNS_EINVAL, "every problem of a batch must have the same dim and precision");
    }
    return CHNS_OK;
}

template <typename TP>
size_t batch_bytes(int count, const std::vector<Plan> &plans) {
    Bump B{nullptr, 0};
    return layout_batch<TP>(B, count, plans.data(), nullptr, nullptr, nullptr) + 256;
}

// One persistent step; with the direct CH solve, S1 | S2 (batched GEMMs) |
// S3..S9.  Returns 0 or an error code.
template <typename TP, int DIM>
int launch_step(chns_batch *b, const BatchState &st, hipStream_t s) {
    const int parts[2] = {b->spec_on ? 1 : 0, 2};
    for (int k = 0; k < (b->spec_on ? 2 : 1); ++k) {
        if (k == 1) {
            const hipError_t e = spectral_batch_solve(b->spec, s);
            if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("CH direct solve: ") + hipGetErrorString(e));
        }
        hipLaunchKernelGGL(k_batch_reset_queue, dim3(1), dim3(64), 0, s, b->d_queue);
        hipLaunchKernelGGL((k_batch_step<TP, DIM>), dim3(b->grid), dim3(b->block), 0, s,
                           (const BatchProb<TP> *)b->d_probs, (const int *)b->d_order, b->count, b->d_queue, st,
                           b->d_stats, parts[k]);
    }
    return CHNS_OK;
}

// graph != 0: the launches are being captured; the per-call statistics are
// then reset by the caller before the replays (a call may replay a graph
// several times and the flags of every replay must survive).
int launch_steps(chns_batch *b, const BatchState &st, int nsteps, hipStream_t s, int graph) {
    if (!graph)
        hipLaunchKernelGGL(k_batch_reset_stats, dim3((b->count + 255) / 256), dim3(256), 0, s, b->d_stats, b->count);
    if (b->mode == CHNS_BATCH_TILED) return tiled_steps(b, st, nsteps, graph, s, b->d_stats);
    for (int n = 0; n < nsteps; ++n) {
        int rc;
        if (b->prec == CHNS_FP64)
            rc = b->dim == 2 ? launch_step<double, 2>(b, st, s) : launch_step<double, 3>(b, st, s);
        else
            rc = b->dim == 2 ? launch_step<float, 2>(b, st, s) : launch_step<float, 3>(b, st, s);
        if (rc) return rc;
    }
    return CHNS_OK;
}

void drop_graph(chns_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_steps = -1;
}

int state_of(chns_batch *b, const chns_state *packed, BatchState &st) {
    if (!packed || !packed->phi || !packed->p || !packed->mu) return set_error(CHNS_EINVAL, "state pointer is NULL");
    for (int a = 0; a < b->dim; ++a)
        if (!packed->u[a]) return set_error(CHNS_EINVAL, "velocity pointer is NULL");
    st.phi = (double *)packed->phi;
    st.p = (double *)packed->p;
    st.mu = (double *)packed->mu;
    for (int a = 0; a < 3; ++a) st.u[a] = a < b->dim ? (double *)packed->u[a] : nullptr;
    return CHNS_OK;
}

bool same_state(const BatchState &x, const BatchState &y) {
    return x.phi == y.phi && x.p == y.p && x.mu == y.mu && x.u[0] == y.u[0] && x.u[1] == y.u[1] && x.u[2] == y.u[2];
}

// Run nsteps on the batch's own stream (ordered after the caller's stream).
int copy_state(chns_batch *b, const BatchState &st, int to_backup, hipStream_t s);

// Captured graphs hold at most this many steps; longer calls replay a graph
// of the largest divisor of nsteps up to it.  (A host-side crash was seen
// while capturing 50 tiled steps of the 512-problem ensemble, ~55k kernel
// nodes; graphs of up to 20 steps have always run.  Its cause is not known,
// so longer captures are not made.)
constexpr int kGraphMaxSteps = 20;

int graph_chunk(int nsteps) {
    int c = nsteps < kGraphMaxSteps ? nsteps : kGraphMaxSteps;
    while (c > 1 && nsteps % c) --c;
    return c;
}

// keep: 1 copies the state to the backup before the steps, 2 restores it
// from the backup first (a replay with other budgets), 0 neither.
int run_steps(chns_batch *b, const BatchState &st, int nsteps, int use_graph, int keep = 0) {
    BHIPCHK(hipEventRecord(b->ev_in, b->user_stream));
    BHIPCHK(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    if (keep)
        if (int rc = copy_state(b, st, keep == 1, b->stream)) return rc;
    const int chunk = use_graph && nsteps > 0 ? graph_chunk(nsteps) : 0;
    if (use_graph && nsteps > 0) {
        const int nsteps_all = nsteps;
        nsteps = chunk;   // the captured graph holds one chunk
        if (!(b->exec && b->g_steps == nsteps && b->g_block == b->block && b->g_grid == b->grid &&
              b->g_mode == b->mode && b->g_tile == b->tile_cells && same_state(b->g_state, st))) {
            drop_graph(b);
            BHIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            const int rc = launch_steps(b, st, nsteps, b->stream, 1);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &gr);
            if (rc) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            b->graph = gr;
            e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return set_error(CHNS_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            b->g_steps = nsteps;
            b->g_block = b->block;
            b->g_grid = b->grid;
            b->g_mode = b->mode;
            b->g_tile = b->tile_cells;
            b->g_state = st;
        }
        hipLaunchKernelGGL(k_batch_reset_stats, dim3((b->count + 255) / 256), dim3(256), 0, b->stream, b->d_stats,
                           b->count);
        for (int done = 0; done < nsteps_all; done += chunk) BHIPCHK(hipGraphLaunch(b->exec, b->stream));
    } else {
        if (int rc = launch_steps(b, st, nsteps, b->stream, 0)) return rc;
    }
    BHIPCHK(hipGetLastError());
    BHIPCHK(hipEventRecord(b->ev_out, b->stream));
    BHIPCHK(hipStreamWaitEvent(b->user_stream, b->ev_out, 0));
    return CHNS_OK;
}

int copy_state(chns_batch *b, const BatchState &st, int to_backup, hipStream_t s) {
    const size_t n = (size_t)b->total_cells * sizeof(double);
    double *fields[6] = {st.phi, st.p, st.mu, st.u[0], st.u[1], st.u[2]};
    const int nf = 3 + b->dim;
    for (int f = 0; f < nf; ++f) {
        double *bk = b->backup + (size_t)f * b->total_cells;
        BHIPCHK(hipMemcpyAsync(to_backup ? bk : fields[f], to_backup ? fields[f] : bk, n, hipMemcpyDeviceToDevice, s));
    }
    return CHNS_OK;
}

}  // namespace

extern "C" {

int chns_batch_workspace_size(int count, const chns_grid_desc *descs, size_t *bytes) {
    if (!bytes) return set_error(CHNS_EINVAL, "bytes is NULL");
    std::vector<Plan> plans;
    if (int rc = check_descs(count, descs, plans)) return rc;
    *bytes = descs[0].precision == CHNS_FP64 ? batch_bytes<double>(count, plans) : batch_bytes<float>(count, plans);
    return CHNS_OK;
}

int chns_create_batch(int count, const chns_grid_desc *descs, const chns_props *props, void *workspace, size_t bytes,
                      void *hip_stream, chns_batch **out) {
    if (!out) return set_error(CHNS_EINVAL, "out is NULL");
    *out = nullptr;
    std::vector<Plan> plans;
    if (int rc = check_descs(count, descs, plans)) return rc;
    if (!props) return set_error(CHNS_EINVAL, "props is NULL");
    for (int i = 0; i < count; ++i)
        if (int rc = check_props(&props[i])) return rc;
    if (!workspace) return set_error(CHNS_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return set_error(CHNS_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    chns_batch_workspace_size(count, descs, &need);
    if (bytes < need) return set_error(CHNS_ENOMEM, "workspace smaller than chns_batch_workspace_size");
    chns_batch *b = new (std::nothrow) chns_batch();
    if (!b) return set_error(CHNS_ENOMEM, "host allocation failed");
    b->count = count;
    b->dim = descs[0].dim;
    b->prec = descs[0].precision;
    b->user_stream = (hipStream_t)hip_stream;
    b->graph = nullptr;
    b->exec = nullptr;
    b->g_steps = -1;
    b->block = 256;
    b->grid = count;
    b->mode = CHNS_BATCH_PERSISTENT;
    b->tile_cells = 1024;
    b->budget[0] = 30;
    b->budget[1] = 30;
    b->budget[2] = 60;
    b->max_iter_max = 1;
    for (int i = 0; i < count; ++i) b->max_iter_max = std::max(b->max_iter_max, props[i].max_iter);
    for (int k = 0; k < 3; ++k) {
        b->rbudget[k] = 8;
        b->last_iters[k] = b->last_refine[k] = 0;
    }
    b->nlev.resize(count);
    b->lsb.resize(count);
    b->nlev_max = 0;
    b->lg = 0;
    b->vlds_max = 0;
    b->vlds_some_global = 0;
    for (int l = 0; l < kMaxLev; ++l) {
        b->ncells[l].assign(count, 0);
        b->lev_n[l].assign(count, std::array<long long, 3>{0, 0, 0});
    }
    for (int i = 0; i < count; ++i) {
        const Plan &P = plans[i];
        b->nlev[i] = P.nlev;
        const int lsb = batch_lsb(P);
        b->lsb[i] = lsb;
        b->nlev_max = std::max(b->nlev_max, P.nlev);
        b->lg = std::max(b->lg, lsb);
        for (int l = 0; l < P.nlev; ++l) {
            b->ncells[l][i] = P.lev[l].N;
            for (int a = 0; a < 3; ++a) b->lev_n[l][i][a] = P.lev[l].n[a];
        }
    }
    Bump B{(char *)workspace, 0};
    std::vector<char> host_table;
    size_t entry = 0;
    std::function<int(chns_batch *)> spec_host;
    auto fill = [&](auto tag) {
        using TP = decltype(tag);
        std::vector<BatchProb<TP>> h;
        h.reserve(count);
        layout_batch<TP>(B, count, plans.data(), props, &h, b);
        for (int i = 0; i < count; ++i) {
            h[i].k = step_const_of(props[i], descs[i].h);
            const StepConst &k = h[i].k;
            h[i].ch = ChOp{props[i].dt * k.kM * props[i].S, props[i].dt * k.kM * props[i].Cn * props[i].Cn, k.ih2};
        }
        entry = sizeof(BatchProb<TP>);
        host_table.resize(entry * count);
        memcpy(host_table.data(), h.data(), entry * count);
        spec_host = [h](chns_batch *bb) { return spectral_batch_setup<TP>(bb, h); };
    };
    if (b->prec == CHNS_FP64) fill(double()); else fill(float());
    b->offsets.resize(count + 1);
    b->offsets[0] = 0;
    for (int i = 0; i < count; ++i) b->offsets[i + 1] = b->offsets[i] + plans[i].lev[0].N;
    // longest first (stable: equal sizes keep their index order)
    b->order.resize(count);
    for (int i = 0; i < count; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return plans[x].lev[0].N > plans[y].lev[0].N; });
    auto cleanup = [&](int rc) {
        if (b->stream) (void)hipStreamDestroy(b->stream);
        if (b->ev_in) (void)hipEventDestroy(b->ev_in);
        if (b->ev_out) (void)hipEventDestroy(b->ev_out);
        delete b;
        return rc;
    };
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemcpy(b->d_probs, host_table.data(), entry * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_order, b->order.data(), sizeof(int) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_scal, 0, sizeof(Scal) * count);
    if (e != hipSuccess) return cleanup(set_error(CHNS_EDEVICE, std::string("batch set-up: ") + hipGetErrorString(e)));
    if (int rc = tiled_build(b, b->tile_cells)) return cleanup(rc);
    const int ginit = count < 4096 ? count : 4096;
    if (b->prec == CHNS_FP64) {
        if (b->dim == 2)
            hipLaunchKernelGGL((k_batch_init<double, 2>), dim3(ginit), dim3(kBatchMaxThreads), 0, b->stream,
                               (const BatchProb<double> *)b->d_probs, count);
        else
            hipLaunchKernelGGL((k_batch_init<double, 3>), dim3(ginit), dim3(kBatchMaxThreads), 0, b->stream,
                               (const BatchProb<double> *)b->d_probs, count);
    } else {
        if (b->dim == 2)
            hipLaunchKernelGGL((k_batch_init<float, 2>), dim3(ginit), dim3(kBatchMaxThreads), 0, b->stream,
                               (const BatchProb<float> *)b->d_probs, count);
        else
            hipLaunchKernelGGL((k_batch_init<float, 3>), dim3(ginit), dim3(kBatchMaxThreads), 0, b->stream,
                               (const BatchProb<float> *)b->d_probs, count);
    }
    hipLaunchKernelGGL(k_batch_reset_stats, dim3((count + 255) / 256), dim3(256), 0, b->stream, b->d_stats, count);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return cleanup(set_error(CHNS_EDEVICE, std::string("batch init: ") + hipGetErrorString(e)));
    if (int rc = spec_host(b)) return cleanup(rc);
    *out = b;
    return CHNS_OK;
}

int chns_batch_offsets(chns_batch *b, long long *offsets) {
    if (!b || !offsets) return set_error(CHNS_EINVAL, "NULL argument");
    for (int i = 0; i <= b->count; ++i) offsets[i] = b->offsets[i];
    return CHNS_OK;
}

int chns_batch_step(chns_batch *b, const chns_state *packed, int nsteps, int use_graph, chns_batch_stats *stats) {
    if (!b) return set_error(CHNS_EINVAL, "NULL handle");
    if (nsteps < 0) return set_error(CHNS_EINVAL, "nsteps must be >= 0");
    BatchState st;
    if (int rc = state_of(b, packed, st)) return rc;
    int flags = 0;
    if (use_graph && nsteps > 0 && b->mode == CHNS_BATCH_TILED) {
        // Captured tiled steps launch a fixed number of iterations per solve
        // (the budgets).  The state is kept; when a replay reports a solve
        // that ran out of its budget, that budget grows, the state is
        // restored and the steps are captured and replayed again.  Grown
        // budgets stay for later calls.
        std::vector<chns_batch_stats> hs(stats ? 0 : b->count);
        chns_batch_stats *out = stats ? stats : hs.data();
        for (int attempt = 0;; ++attempt) {
            if (int rc = run_steps(b, st, nsteps, 1, attempt == 0 ? 1 : 2)) return rc;
            BHIPCHK(hipMemcpyAsync(out, b->d_stats, sizeof(chns_batch_stats) * b->count, hipMemcpyDeviceToHost,
                                   b->stream));
            BHIPCHK(hipStreamSynchronize(b->stream));
            flags = 0;
            for (int i = 0; i < b->count; ++i) flags |= out[i].flags;
            if (!(flags & 31) || (flags & 32)) break;
            // the flag does not tell which round of the solve ran short (the
            // iterations or, with the FP32 hierarchy, the refinement round
            // after the true-residual check), so both budgets grow
            bool grown = false;
            auto grow = [&](int kind) {
                const int nb = std::min(b->max_iter_max, b->budget[kind] + std::max(2, b->budget[kind] / 4));
                const int nr = std::min(b->max_iter_max, b->rbudget[kind] + std::max(2, b->rbudget[kind] / 2));
                if (nb > b->budget[kind] || nr > b->rbudget[kind]) {
                    b->budget[kind] = nb;
                    b->rbudget[kind] = nr;
                    grown = true;
                }
            };
            if (flags & 1) grow(0);
            if (flags & 14) grow(1);
            if (flags & 16) grow(2);
            if (!grown) break;   // at max_iter: genuinely unconverged
            drop_graph(b);
        }
    } else {
        if (int rc = run_steps(b, st, nsteps, use_graph)) return rc;
        if (!stats) return CHNS_OK;
        BHIPCHK(hipMemcpyAsync(stats, b->d_stats, sizeof(chns_batch_stats) * b->count, hipMemcpyDeviceToHost,
                               b->stream));
        BHIPCHK(hipStreamSynchronize(b->stream));
        for (int i = 0; i < b->count; ++i) flags |= stats[i].flags;
    }
    if (flags & 32) return set_error(CHNS_ENONFINITE, "non-finite residual in a batched solve");
    if (flags) {
        char buf[160];
        snprintf(buf, sizeof buf, "unconverged batched solves (bit 0 CH, 1..3 momentum, 4 pressure): mask %d", flags);
        return set_error(CHNS_ENOCONV, buf);
    }
    return CHNS_OK;
}

int chns_batch_set_launch(chns_batch *b, int block, int grid) {
    if (!b) return set_error(CHNS_EINVAL, "NULL handle");
    if (block < kWave || block > kBatchMaxThreads || block % kWave) return set_error(CHNS_EINVAL, "bad block size");
    if (grid < 1) return set_error(CHNS_EINVAL, "grid must be >= 1");
    b->mode = CHNS_BATCH_PERSISTENT;
    b->block = block;
    b->grid = grid;
    return CHNS_OK;
}

int chns_batch_set_tiled(chns_batch *b, int tile_cells) {
    if (!b) return set_error(CHNS_EINVAL, "NULL handle");
    if (tile_cells < kTileBlock || tile_cells % kTileBlock || tile_cells > (1 << 20))
        return set_error(CHNS_EINVAL, "tile_cells must be a multiple of 256 in [256, 2^20]");
    if (b->tile_cells != tile_cells)
        if (int rc = tiled_build(b, tile_cells)) return rc;
    b->mode = CHNS_BATCH_TILED;
    return CHNS_OK;
}

int chns_batch_set_budget(chns_batch *b, int iters_ch, int iters_mom, int iters_p) {
    if (!b) return set_error(CHNS_EINVAL, "NULL handle");
    if (iters_ch < 1 || iters_mom < 1 || iters_p < 1) return set_error(CHNS_EINVAL, "budgets must be >= 1");
    b->budget[0] = iters_ch;
    b->budget[1] = iters_mom;
    b->budget[2] = iters_p;
    return CHNS_OK;
}

int chns_batch_autotune(chns_batch *b, const chns_state *packed, int steps_per_trial, chns_batch_tuning *result) {
    if (!b) return set_error(CHNS_EINVAL, "NULL handle");
    if (steps_per_trial < 1) return set_error(CHNS_EINVAL, "steps_per_trial must be >= 1");
    BatchState st;
    if (int rc = state_of(b, packed, st)) return rc;
    // candidates: persistent form (threads per workgroup x workgroups) and
    // tiled form (cells per tile)
    struct Cand {
        int mode, a, g;
    };
    std::vector<Cand> cands;
    for (int bl : {256, 512})
        for (int gr : {std::min(b->count, 256), b->count}) {
            bool dup = false;
            for (const Cand &c : cands) dup |= c.mode == CHNS_BATCH_PERSISTENT && c.a == bl && c.g == gr;
            if (!dup) cands.push_back({CHNS_BATCH_PERSISTENT, bl, gr});
        }
    for (int tc : {512, 1024, 2048, 4096}) cands.push_back({CHNS_BATCH_TILED, tc, 0});
    chns_batch_tuning res;
    memset(&res, 0, sizeof res);
    hipEvent_t e0, e1;
    BHIPCHK(hipEventCreate(&e0));
    BHIPCHK(hipEventCreate(&e1));
    const int saved_mode = b->mode, saved_block = b->block, saved_grid = b->grid, saved_tile = b->tile_cells;
    BHIPCHK(hipEventRecord(b->ev_in, b->user_stream));
    BHIPCHK(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    int rc = copy_state(b, st, 1, b->stream);
    double best = 1e300;
    int most[3] = {0, 0, 0}, most_r[3] = {0, 0, 0};
    for (const Cand &c : cands) {
        if (rc || res.ncand >= CHNS_MAX_TUNING) break;
        if (c.mode == CHNS_BATCH_TILED) {
            if ((rc = tiled_build(b, c.a))) break;
            b->mode = CHNS_BATCH_TILED;
        } else {
            b->mode = CHNS_BATCH_PERSISTENT;
            b->block = c.a;
            b->grid = c.g;
        }
        // warm-up step (code objects, caches, the tiled form's chunk sizes)
        if ((rc = launch_steps(b, st, 1, b->stream, 0))) break;
        if ((rc = copy_state(b, st, 0, b->stream))) break;
        (void)hipEventRecord(e0, b->stream);
        if ((rc = launch_steps(b, st, steps_per_trial, b->stream, 0))) break;
        (void)hipEventRecord(e1, b->stream);
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = set_error(CHNS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
            break;
        }
        if (c.mode == CHNS_BATCH_TILED)
            for (int k = 0; k < 3; ++k) {
                most[k] = std::max(most[k], b->last_iters[k]);
                most_r[k] = std::max(most_r[k], b->last_refine[k]);
            }
        const double per = ms / steps_per_trial;
        res.cand_mode[res.ncand] = c.mode;
        res.cand_block[res.ncand] = c.a;
        res.cand_grid[res.ncand] = c.g;
        res.cand_ms[res.ncand] = per;
        res.ncand++;
        if (per < best) {
            best = per;
            res.mode = c.mode;
            res.block = c.mode == CHNS_BATCH_TILED ? kTileBlock : c.a;
            res.grid = c.g;
            res.tile_cells = c.mode == CHNS_BATCH_TILED ? c.a : 0;
            res.ms_per_step = per;
        }
        if ((rc = copy_state(b, st, 0, b->stream))) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc && hipStreamSynchronize(b->stream) != hipSuccess) rc = set_error(CHNS_EDEVICE, "autotune sync failed");
    if (rc) {
        b->mode = saved_mode;
        b->block = saved_block;
        b->grid = saved_grid;
        (void)tiled_build(b, saved_tile);
        return rc;
    }
    // graph budgets of the tiled form: the most iterations any problem
    // needed in the trials (eager steps), plus a margin of 2
    for (int k = 0; k < 3; ++k)
        if (most[k] > 0) {
            b->budget[k] = most[k] + 2;
            b->rbudget[k] = most_r[k] > 0 ? most_r[k] + 1 : 0;
        }
    res.budget_ch = b->budget[0];
    res.budget_mom = b->budget[1];
    res.budget_p = b->budget[2];
    if (res.mode == CHNS_BATCH_TILED) {
        if ((rc = tiled_build(b, res.tile_cells))) return rc;
        b->mode = CHNS_BATCH_TILED;
    } else {
        if ((rc = tiled_build(b, saved_tile))) return rc;
        b->mode = CHNS_BATCH_PERSISTENT;
        b->block = res.block;
        b->grid = res.grid;
    }
    drop_graph(b);
    hipLaunchKernelGGL(k_batch_reset_stats, dim3((b->count + 255) / 256), dim3(256), 0, b->stream, b->d_stats,
                       b->count);
    BHIPCHK(hipEventRecord(b->ev_out, b->stream));
    BHIPCHK(hipStreamWaitEvent(b->user_stream, b->ev_out, 0));
    if (result) *result = res;
    return CHNS_OK;
}

int chns_destroy_batch(chns_batch *b) {
    if (!b) return CHNS_OK;
    drop_graph(b);
    if (b->stream) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    delete b;
    return CHNS_OK;
}

}  // extern "C"
