// Matrix-free multigrid-preconditioned conjugate gradients on the uniform
// grid (gfx950).  The elliptic solver is not fixed by the paper (its coupled
// system goes to Krylov solvers with ASM / algebraic-multigrid
// preconditioners, and it names matrix-free multigrid as future work); this
// is a geometric cell-centred multigrid:
//   * operator       (A x)_c = s_c x_c + sum_b cs_b(c)(x_c - x_{c-e_b})
//                                       + cs_b(c+e_b)(x_c - x_{c+e_b}),
//   * smoother       red-black Gauss-Seidel; pre-smoothing (red, black) from
//                    a zero guess, post-smoothing (black, red): the V-cycle is
//                    a symmetric positive definite preconditioner;
//   * transfers      cell-centred bilinear / trilinear prolongation P and
//                    full-weighting restriction R = P^T / 2^d;
//   * coarse levels  re-discretised: s averaged over children, face
//                    coefficients averaged over the fine faces of a coarse
//                    face and divided by 4 (spacing doubles);
//   * coarsest       explicit FP64 inverse (Gauss-Jordan in one workgroup)
//                    with a rank-one shift tau 1 1^T for the singular
//                    pressure operator.
// Launch structure (a launch costs a few microseconds whatever its size):
//   * 2D levels above kSBCells cells: two tile kernels per level, one for
//     the way down (pre-smoothing, residual, restriction) and one for the
//     way up (prolongation, black sweep, red sweep), on LDS tiles with halos;
//   * 3D levels above kSBCells cells: one grid-wide kernel per pass (fused
//     zero-guess pre-smoothing, residual, restriction, prolongation, black
//     sweep, red sweep);
//   * all smaller levels: ONE single-workgroup kernel that copies their
//     storage into LDS and runs every sweep there.
// Reductions are deterministic and fence-free: per-block partials from a
// fixed grid-stride partition, summed in a fixed order either by a
// one-workgroup finalize kernel or redundantly by every block of the kernel
// that consumes them.  PCG scalars live on the device; every iteration
// kernel returns at once when the device "done" flag is set, so the host
// launches iterations in chunks and checks the flag once per chunk.
#include <cstdlib>
#include <type_traits>

#include "mgdev.h"
#include "solvers.h"
#include "tile2d.h"

namespace chns {

static int sb_cells() { return kSBCells; }

// ---------------------------------------------------------------------------
// grid-wide V-cycle kernels (one pass each)
// ---------------------------------------------------------------------------
#define GRID_LOOP(N) \
    for (int c = xcd_block() * (int)blockDim.x + (int)threadIdx.x; c < (int)(N); c += (int)(gridDim.x * blockDim.x))

template <typename T, typename TB, int DIM>
__global__ void __launch_bounds__(kBlock) k_presmooth(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                      const int *__restrict__ done) {
    if (*done) return;
    GRID_LOOP(L.g.N) presmooth_cell<T, TB, DIM>(L, b, x, c);
}

// The same pass with one thread per x-adjacent pair of cells (even x
// extent): each lane updates one red and one black cell, so a wave whose
// lanes share a row runs each colour's branch once instead of both with
// half of its lanes masked off.
template <typename T, typename TB, int DIM>
__global__ void __launch_bounds__(kBlock) k_presmooth_pair(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                           const int *__restrict__ done) {
    if (*done) return;
    GRID_LOOP(L.g.N / 2) {
        presmooth_cell<T, TB, DIM>(L, b, x, 2 * c);
        presmooth_cell<T, TB, DIM>(L, b, x, 2 * c + 1);
    }
}

template <typename T, typename TB, int DIM>
__global__ void __launch_bounds__(kBlock) k_residual(Level<T> L, const TB *__restrict__ b, const T *__restrict__ x,
                                                     const int *__restrict__ done) {
    if (*done) return;
    GRID_LOOP(L.g.N) residual_cell<T, TB, DIM>(L, b, x, c);
}

// Two consecutive values along x (the pair starts at an even index).
template <typename T>
struct Pair2 {
    T v[2];
};

// 3D prolongation x += P e, one thread per coarse cell: the 3 x 3 x 3 coarse
// neighbourhood (parent, lower and upper side neighbour per axis, from
// pro_axis) is loaded once and the eight children are updated with the taps,
// weights and summation order of prolong_at.  Needs an even fine x extent.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add3(Geo gf, Geo gc, const T *__restrict__ xc,
                                                         T *__restrict__ x, const int *__restrict__ done) {
    if (*done) return;
    using R = T;
    GRID_LOOP(gc.N) {
        int I[3];
        coords_of<3>(gc, c, I);
        int q[3][3];   // [axis][0: parent, 1: lower child's neighbour, 2: upper child's neighbour]
        R w0[3][2], w1[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a][0] = I[a];
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                int c0, c1;
                pro_axis<R>(2 * I[a] + sd, (int)gc.n[a], gc.per[a], c0, c1, w0[a][sd], w1[a][sd]);
                q[a][1 + sd] = c1;
            }
        }
        const int nx = (int)gc.n[0], nxy = nx * (int)gc.n[1];
        R X[3][3][3];
#pragma unroll
        for (int z = 0; z < 3; ++z)
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int xx = 0; xx < 3; ++xx) X[z][y][xx] = (R)xc[q[2][z] * nxy + q[1][y] * nx + q[0][xx]];
        const int fnx = (int)gf.n[0], fnxy = fnx * (int)gf.n[1];
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy) {
                const int f = 2 * I[0] + fnx * (2 * I[1] + dy) + fnxy * (2 * I[2] + dz);
                Pair2<T> pr = *(const Pair2<T> *)(x + f);
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    R v = 0.0;
#pragma unroll
                    for (int dz2 = 0; dz2 < 2; ++dz2) {
                        const R wz = dz2 ? w1[2][dz] : w0[2][dz];
                        const int zi = dz2 ? 1 + dz : 0;
#pragma unroll
                        for (int dy2 = 0; dy2 < 2; ++dy2) {
                            const R wyz = wz * (dy2 ? w1[1][dy] : w0[1][dy]);
                            const int yi = dy2 ? 1 + dy : 0;
                            v = pro_row(v, wyz, w0[0][dx], X[zi][yi][0], w1[0][dx], X[zi][yi][1 + dx]);
                        }
                    }
                    pr.v[dx] = (T)((T)pr.v[dx] + v);
                }
                *(Pair2<T> *)(x + f) = pr;
            }
    }
}

// 3D restriction through LDS: a workgroup takes a tile of kRCX x kRCY x kRCZ
// coarse cells and stages the fine cells 2I-1 .. 2I+2 of all of them once
// (wrapped on periodic axes; clamped at walls, where restrict_cell gives
// those taps weight 0 and reads the same clamped cell); each thread then
// sums the 64 taps of its coarse cell out of LDS with the weights and the
// summation order of restrict_cell.  The per-thread form read every fine
// value eight times from the caches, 64 loads per coarse cell.
constexpr int kRCX = 16, kRCY = 4, kRCZ = 4;   // coarse tile (kRCX * kRCY * kRCZ = kBlock)
constexpr int kRFX = 2 * kRCX + 2, kRFY = 2 * kRCY + 2, kRFZ = 2 * kRCZ + 2;
static_assert(kRCX * kRCY * kRCZ == kBlock, "one coarse cell per thread");

// Fine index of staged position g (>= -1): one wrap on a periodic axis (the
// taps of coarse cells inside the grid reach -1 .. n at most), clamped to the
// grid otherwise and for positions past a partial tile's last coarse cell.
__device__ inline int res_fine_index(int g, int n, int per) {
    if (per) g = g < 0 ? g + n : (g >= n ? g - n : g);
    return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict3_lds(Geo gf, Geo gc, const T *__restrict__ rf,
                                                          T *__restrict__ bc, int ntx, int nty, int ntiles,
                                                          const int *__restrict__ done) {
    using R = T;
    const int tile = xcd_block();
    if (tile >= ntiles || *done) return;
    __shared__ T sf[kRFZ][kRFY][kRFX];
    const int tz = tile / (ntx * nty), trem = tile - tz * ntx * nty, ty = trem / ntx, tx = trem - ty * ntx;
    const int X0 = tx * kRCX, Y0 = ty * kRCY, Z0 = tz * kRCZ;
    const int nfx = (int)gf.n[0], nfy = (int)gf.n[1], nfz = (int)gf.n[2];
    // every staging load of a thread is issued before its first LDS store
    constexpr int kStage = kRFX * kRFY * kRFZ, kPer = (kStage + kBlock - 1) / kBlock;
    T v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = (int)threadIdx.x + r * kBlock;
        if (e < kStage) {
            const int z = e / (kRFX * kRFY), r2 = e - z * (kRFX * kRFY), y = r2 / kRFX, x = r2 - y * kRFX;
            const int gx = res_fine_index(2 * X0 - 1 + x, nfx, gc.per[0]);
            const int gy = res_fine_index(2 * Y0 - 1 + y, nfy, gc.per[1]);
            const int gz = res_fine_index(2 * Z0 - 1 + z, nfz, gc.per[2]);
            v[r] = rf[(gz * nfy + gy) * nfx + gx];
        }
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = (int)threadIdx.x + r * kBlock;
        if (e < kStage) (&sf[0][0][0])[e] = v[r];
    }
    __syncthreads();
    const int lx = (int)threadIdx.x % kRCX, ly = ((int)threadIdx.x / kRCX) % kRCY, lz = (int)threadIdx.x / (kRCX * kRCY);
    const int I[3] = {X0 + lx, Y0 + ly, Z0 + lz};
    if (I[0] >= gc.n[0] || I[1] >= gc.n[1] || I[2] >= gc.n[2]) return;
    int f[4];
    R wx[4], wy[4], wz[4];
    res_axis<R>(I[0], gc.n[0], nfx, gc.per[0], f, wx);
    res_axis<R>(I[1], gc.n[1], nfy, gc.per[1], f, wy);
    res_axis<R>(I[2], gc.n[2], nfz, gc.per[2], f, wz);
    R acc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const R wza = wz[a];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T *row = &sf[2 * lz + a][2 * ly + q][2 * lx];
            R s = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) s = fmar(wx[e], (R)row[e], s);
            acc = fmar(wy[q] * wza, s, acc);
        }
    }
    bc[(I[2] * (int)gc.n[1] + I[1]) * (int)gc.n[0] + I[0]] = (T)acc;
}

template <typename T, typename TB, int DIM>
__global__ void __launch_bounds__(kBlock) k_gs_color(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                     int color, const int *__restrict__ done) {
    if (*done) return;
    GRID_LOOP(L.g.N) gs_color_cell<T, TB, DIM>(L, b, x, color, c);
}

// ---------------------------------------------------------------------------
// 2D tile kernels of the grid levels (bodies in tile2d.h); tiles along x
// ---------------------------------------------------------------------------
template <typename T, typename TB>
__global__ void __launch_bounds__(kTileThreads) k_down_tile2(Level<T> L, Geo gc, const TB *__restrict__ b,
                                                             T *__restrict__ xs, T *__restrict__ bc, int ntx,
                                                             int ntiles, const int *__restrict__ done) {
    const int tile = xcd_block();
    if (tile >= ntiles) return;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    down_tile2<T, kTileThreads>(L, gc, RhsStored<TB>{b}, xs, bc, tx, ty, *done);
}

template <typename T, typename TB>
__global__ void __launch_bounds__(kTileThreads) k_up_tile2(Level<T> L, Geo gc, const T *__restrict__ xc,
                                                           const TB *__restrict__ b, const T *__restrict__ xs,
                                                           T *__restrict__ x, int ntx, int ntiles,
                                                           const int *__restrict__ done) {
    const int tile = xcd_block();
    if (tile >= ntiles) return;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    up_tile2<T, kTileThreads>(L, gc, xc, RhsStored<TB>{b}, xs, x, tx, ty, *done);
}

// Level 0 of the preconditioner of CG iteration k, fused with the update
// that precedes it: alpha = rz / p.q (every block sums the apply's partials
// in the same order), x += alpha p on the tile's cells, the partial of r.r
// per tile for r - alpha q, and the way down from r - alpha q.  r itself is
// not stored here (neighbouring tiles still read the old r in their halos):
// the next operator apply stores it.
template <typename T, typename TR>
__global__ void __launch_bounds__(kTileThreads) k_down_tile2_cg(Level<T> L, Geo gc, const TR *__restrict__ r,
                                                                const TR *__restrict__ q, const TR *__restrict__ p,
                                                                TR *__restrict__ x, T *__restrict__ xs,
                                                                T *__restrict__ bc, int ntx, int ntiles, Scal *sc,
                                                                const double *__restrict__ part_pq, int npq,
                                                                double *__restrict__ part_rr) {
    const int tile = xcd_block();
    if (tile >= ntiles) return;
    if (sc->done) return;
    __shared__ double bcast;
    double pq = 0.0, u0 = 0.0, u1 = 0.0;
    for (int i = (int)threadIdx.x; i < npq; i += kTileThreads) pq += part_pq[i];
    tile_sum3<kTileThreads>(pq, u0, u1);
    if (threadIdx.x == 0) bcast = pq;
    __syncthreads();
    pq = bcast;
    const double alpha = pq != 0.0 ? sc->rz / pq : 0.0;
    if (tile == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
    }
    const int ty = tile / ntx, tx = tile - ty * ntx;
    down_tile2<T, kTileThreads>(L, gc, RhsPending<TR, T>{r, q, alpha}, xs, bc, tx, ty, 0);
    const int nx = (int)L.g.n[0], ny = (int)L.g.n[1];
    double rr = 0.0;
    u0 = u1 = 0.0;
    for (int j = (int)threadIdx.x; j < kTFX * kTFY; j += kTileThreads) {
        const int ly = j / kTFX, lx = j - ly * kTFX;
        const int gx = tx * kTFX + lx, gy = ty * kTFY + ly;
        if (gx < nx && gy < ny) {
            const int g = gx + nx * gy;
            x[g] = (TR)((double)x[g] + alpha * (double)p[g]);
            const double rc = cg_residual((double)r[g], (double)q[g], alpha);
            rr += rc * rc;
        }
    }
    tile_sum3<kTileThreads>(rr, u0, u1);
    if (threadIdx.x == 0) part_rr[tile] = rr;
}

// Level 0 of the way up inside CG: right-hand side as stored (b) or pending
// (r - alpha q, bpend); dmode 0: no partials, 1: partials of r.z, sum z,
// sum r per tile with r as stored, 2: with r pending.
template <typename T, typename TR>
__global__ void __launch_bounds__(kTileThreads) k_up_tile2_cg(Level<T> L, Geo gc, const T *__restrict__ xc,
                                                              const T *__restrict__ b, const TR *__restrict__ r,
                                                              const TR *__restrict__ q, const T *__restrict__ xs,
                                                              T *__restrict__ x, int ntx, int ntiles,
                                                              const Scal *__restrict__ sc, int bpend, int dmode,
                                                              double *__restrict__ p0, double *__restrict__ p1,
                                                              double *__restrict__ p2,
                                                              const int *__restrict__ done) {
    const int tile = xcd_block();
    if (tile >= ntiles) return;
    const int ty = tile / ntx, tx = tile - ty * ntx;
    const double alpha = (bpend || dmode == 2) ? sc->alpha : 0.0;
    const int skip = *done;
    if (dmode == 0) {
        up_tile2<T, kTileThreads>(L, gc, xc, RhsPending<TR, T>{r, q, alpha}, xs, x, tx, ty, skip);
        return;
    }
    const RzDots<TR> d{r, q, alpha, dmode == 2, p0, p1, p2, tile};
    if (bpend)
        up_tile2<T, kTileThreads>(L, gc, xc, RhsPending<TR, T>{r, q, alpha}, xs, x, tx, ty, skip, d);
    else
        up_tile2<T, kTileThreads>(L, gc, xc, RhsStored<T>{b}, xs, x, tx, ty, skip, d);
}

// ---------------------------------------------------------------------------
// single-workgroup kernels for the small levels
// ---------------------------------------------------------------------------
template <typename T, typename TB, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_vcycle_block(Slot<T> S, int l0, const TB *__restrict__ b0,
                                                             T *__restrict__ x0, const int *__restrict__ done) {
    if (*done) return;
    vcycle_block_dev<T, TB, DIM>(S, l0, b0, x0);
}

// Levels [l0, nlev) out of LDS: the segments cp of their contiguous storage
// are copied in, x of level l0 is written back.
template <typename T, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_vcycle_lds(Slot<T> S, int l0, LdsCopy cp,
                                                           const int *__restrict__ done) {
    const int dn = *done;   // tested after the copy (which only reads memory and writes LDS)
    extern __shared__ uint4 lds_words[];
    char *lds = (char *)lds_words;
    const char *base = (const char *)S.lev[l0].s;
    copy_to_lds(lds_words, (const uint4 *)base, cp);
    if (dn) return;
    __syncthreads();
    vcycle_lds_dev<T, DIM>(S, l0, lds, base);
    const T *xl = lds_image(lds, base, S.lev[l0].x);
    T *xg = S.lev[l0].x;
    LDS_LOOP(S.lev[l0].g.N) xg[c] = xl[c];
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kSBThreads) k_setup_block(Slot<T> S, int l0) {
    __shared__ SetupLdsPP sh;
    setup_block_dev<T, DIM>(S, l0, sh);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_invd(Level<T> L) {
    GRID_LOOP(L.g.N) invd_cell<T, DIM>(L, c);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_coarsen(Level<T> F, Level<T> C) {
    GRID_LOOP(C.g.N) coarsen_cell<T, DIM>(F, C, c);
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------

// fixed-order sum of partials, returned to every thread of the block
__device__ inline double sum_parts_all(const double *__restrict__ part, int nparts, double *lds) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) v += part[k];
    return block_sum_all(v, lds);
}

// Start of CG iteration k, evaluated by every block of the kernel that
// consumes it (the sums are the same in every block): rz = r.(z - zmean)
// from the partials of k_pcg_rz, zmean = mean(z) for a singular operator
// (else 0), beta = rz / rz_previous (0 for k = 0).  For a singular
// (pure Neumann / periodic) operator the preconditioned vector is projected
// onto the range: the V-cycle amplifies the constant mode, and without the
// projection rounding noise in that mode destroys the conjugacy of the
// search directions.  Block 0 stores rz in sc->rzs[k & 1] while the blocks
// read the previous value from the other entry, and publishes rz, zmean,
// beta; a non-finite rz ends the solve.  Returns false when the solve ends.
struct IterStart {
    double rz, zm, beta;
};
__device__ inline bool iter_start(Scal *sc, const double *__restrict__ p0, const double *__restrict__ p1,
                                  const double *__restrict__ p2, int nparts, long long N, int k, int singular,
                                  IterStart &o) {
    // the three sums in one pass: the same per-thread and per-wave order as
    // three separate block sums, one round of barriers
    __shared__ double wsum[3][kBlock / kWave];
    double trz = 0.0, tz = 0.0, tr = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        trz += p0[i];
        if (singular) {
            tz += p1[i];
            tr += p2[i];
        }
    }
    trz = wave_sum(trz);
    tz = wave_sum(tz);
    tr = wave_sum(tr);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) {
        wsum[0][w] = trz;
        wsum[1][w] = tz;
        wsum[2][w] = tr;
    }
    __syncthreads();
    trz = tz = tr = 0.0;
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
        trz += wsum[0][q];
        tz += wsum[1][q];
        tr += wsum[2][q];
    }
    __syncthreads();
    if (!singular) tz = tr = 0.0;
    o.zm = singular ? tz / (double)N : 0.0;
    o.rz = trz - o.zm * tr;
    const double prev = k > 0 ? sc->rzs[(k + 1) & 1] : 0.0;
    o.beta = (k == 0 || prev == 0.0) ? 0.0 : o.rz / prev;
    const bool ok = isfinite(o.rz);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            sc->rzs[k & 1] = o.rz;
            sc->rz = o.rz;
            sc->zmean = o.zm;
            sc->beta = o.beta;
        } else {
            sc->nonfinite = 1;
            sc->done = 1;
        }
    }
    return ok;
}

// p_new = (z - zmean) + beta p_old (beta = 0: p_new = z - zmean);
// q = A p_new (slot operator); partial p.q
template <typename T, typename TZ, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_apply_slot(Level<T> L, const TZ *__restrict__ z,
                                                           const T *__restrict__ pold, T *__restrict__ pnew,
                                                           T *__restrict__ q, Scal *sc, double *__restrict__ part,
                                                           const double *__restrict__ rz0,
                                                           const double *__restrict__ rz1,
                                                           const double *__restrict__ rz2, int nrz, int k,
                                                           int singular, T *__restrict__ rpend) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    const double alpha_prev = rpend ? sc->alpha : 0.0;   // read before iter_start
    IterStart it;
    if (!iter_start(sc, rz0, rz1, rz2, nrz, L.g.N, k, singular, it)) return;
    const double beta = it.beta, zm = it.zm;
    auto pv = [&](int e) { return ((double)z[e] - zm) + (beta != 0.0 ? beta * (double)pold[e] : 0.0); };
    double acc = 0.0;
    GRID_LOOP(L.g.N) {
        int ia[3];
        coords_of<DIM>(L.g, c, ia);
        // residual of the previous iteration, stored before q is overwritten
        if (rpend) rpend[c] = (T)cg_residual((double)rpend[c], (double)q[c], alpha_prev);
        const double pc = pv(c);
        // a singular (pressure) operator has s = +0: not read
        double sv = 0.0;
        if (!singular) sv = (double)L.s[c];
        double qc = sv * pc;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {   // branch-free: a missing neighbour is c itself with weight 0
            const int lo = nb_lo(L.g, c, ia[b], b);
            const int hi = nb_hi(L.g, c, ia[b], b);
            const int l = lo >= 0 ? lo : c, h = hi >= 0 ? hi : c;
            const double vl = pv(l), vh = pv(h);
            const double wl = (double)L.cs[b][c], wh = (double)L.cs[b][h];
            qc += (lo >= 0 ? wl : 0.0) * (pc - vl);
            qc += (hi >= 0 ? wh : 0.0) * (pc - vh);
        }
        pnew[c] = (T)pc;
        q[c] = (T)qc;
        acc += pc * qc;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The same apply on a 3D grid (no pending residual), marching along z:
// logical block b owns the kMX x kMY x zc cells of column tile b mod ncol and
// z chunk b / ncol, one cell per thread and plane.  p = (z - zmean) + beta p_old of
// the column and a one-cell halo is formed once per plane into a ring of
// three LDS planes, where the grid-stride form above evaluates it at all
// seven stencil points of every cell (128^3: 4 TB/s).  q, p_new and the
// per-cell arithmetic are those of k_pcg_apply_slot (a missing neighbour
// enters as the cell itself with weight 0); one p.q partial per block.
constexpr int kMX = 32, kMY = kBlock / kMX, kMW = kMX + 2, kMH = kMY + 2;
#ifndef CHNS_MARCH_PLANES
#define CHNS_MARCH_PLANES 8
#endif
constexpr int kMarchPlanes = CHNS_MARCH_PLANES;   // z planes per block (more on grids too large for the partials)
// RHO (pressure operator): the face coefficients 1/(rho_f h^2) are formed
// from the cell densities rho (a second ring of planes) with the set-up's
// expression, instead of read as s and cs[3]: 8 bytes per cell instead of 32
// for six divisions per cell.  Used on grids past the Infinity Cache (the
// marching-sweep threshold of the slot): 512^3 apply 2.00 -> 1.50 ms; at
// 128^3, where the coefficients come from the cache, the divisions cost more
// than the bytes save.
template <typename T, typename TZ, bool RHO>
__global__ void __launch_bounds__(kBlock) k_pcg_apply3_march(Level<T> L, const TZ *__restrict__ z,
                                                             const T *__restrict__ pold, T *__restrict__ pnew,
                                                             T *__restrict__ q, Scal *sc, double *__restrict__ part,
                                                             const double *__restrict__ rz0,
                                                             const double *__restrict__ rz1,
                                                             const double *__restrict__ rz2, int nrz, int k,
                                                             int singular, int ncolx, int ncol, int zc,
                                                             const double *__restrict__ rho, double rho_ih2) {
    if (sc->done) return;
    __shared__ double pl[3][kMH * kMW];
    __shared__ double rl[RHO ? 3 : 1][RHO ? kMH * kMW : 1];
    __shared__ double lds[kBlock / kWave];
    IterStart it;
    if (!iter_start(sc, rz0, rz1, rz2, nrz, L.g.N, k, singular, it)) return;
    const double beta = it.beta, zm = it.zm;
    const Geo &g = L.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    // XCD-contiguous numbering: the column tiles of a z chunk, whose halos
    // overlap, run on the same XCD and share its L2 (128^3: 32 -> 28 us)
    const int lb = xcd_block();
    const int col = lb % ncol, z0 = (lb / ncol) * zc;
    const int x0 = (col % ncolx) * kMX, y0 = (col / ncolx) * kMY;
    const int z1 = z0 + zc < nz ? z0 + zc : nz;
    // coordinate of a halo position on one axis (wrapped on a periodic axis);
    // false outside a walled one
    auto wrapc = [](int v, int n, int per, int &w) {
        if (v >= 0 && v < n) {
            w = v;
            return true;
        }
        w = v < 0 ? v + n : v - n;
        return per != 0 && w >= 0 && w < n;
    };
    // p of plane zz and its halo into P (0 outside the domain; never used
    // with a nonzero weight there)
    auto form = [&](int zz, int slot) {
        double *P = pl[slot];
        int gz;
        const bool vz = wrapc(zz, nz, g.per[2], gz);
        for (int i = (int)threadIdx.x; i < kMH * kMW; i += kBlock) {
            const int ly = i / kMW, lx = i - ly * kMW;
            int gx, gy;
            const bool vx = wrapc(x0 - 1 + lx, nx, g.per[0], gx);
            const bool vy = wrapc(y0 - 1 + ly, ny, g.per[1], gy);
            const bool v = vx && vy && vz;
            double pv = 0.0, rv = 0.0;
            if (v) {
                const int e = gx + nx * (gy + ny * gz);
                pv = ((double)z[e] - zm) + (beta != 0.0 ? beta * (double)pold[e] : 0.0);
                if (RHO) rv = rho[e];
            }
            P[i] = pv;
            if (RHO) rl[slot][i] = rv;
        }
    };
    const int tx = (int)threadIdx.x % kMX, ty = (int)threadIdx.x / kMX;
    const int gx = x0 + tx, gy = y0 + ty, li = (ty + 1) * kMW + tx + 1;
    const bool own = gx < nx && gy < ny;
    form(z0 - 1, (z0 + 2) % 3);
    form(z0, z0 % 3);
    double acc = 0.0;
    for (int zz = z0; zz < z1; ++zz) {
        form(zz + 1, (zz + 1) % 3);
        __syncthreads();
        const double *Pm = pl[(zz + 2) % 3], *P0 = pl[zz % 3], *Pp = pl[(zz + 1) % 3];
        if (own) {
            const int c = gx + nx * (gy + ny * zz);
            const int ia[3] = {gx, gy, zz};
            const double pc = P0[li];
            const double nbv[3][2] = {{P0[li - 1], P0[li + 1]}, {P0[li - kMW], P0[li + kMW]}, {Pm[li], Pp[li]}};
            double rc = 0.0, nbr[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
            if (RHO) {
                const double *Rm = rl[(zz + 2) % 3], *R0 = rl[zz % 3], *Rp = rl[(zz + 1) % 3];
                rc = R0[li];
                nbr[0][0] = R0[li - 1];
                nbr[0][1] = R0[li + 1];
                nbr[1][0] = R0[li - kMW];
                nbr[1][1] = R0[li + kMW];
                nbr[2][0] = Rm[li];
                nbr[2][1] = Rp[li];
            }
            // s = +0 on a singular (pressure) operator: not read
            double sv = 0.0;
            if (!RHO && !singular) sv = (double)L.s[c];
            double qc = sv * pc;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int lo = nb_lo(g, c, ia[b], b);
                const int hi = nb_hi(g, c, ia[b], b);
                const int h = hi >= 0 ? hi : c;
                const double vl = lo >= 0 ? nbv[b][0] : pc, vh = hi >= 0 ? nbv[b][1] : pc;
                double wl, wh;
                if (RHO) {
                    // the set-up's 1.0 / (0.5 * (rho_c + rho_lo)) * ih2 for the faces c and c + e_b
                    wl = lo >= 0 ? 1.0 / (0.5 * (rc + nbr[b][0])) * rho_ih2 : 0.0;
                    wh = hi >= 0 ? 1.0 / (0.5 * (nbr[b][1] + rc)) * rho_ih2 : 0.0;
                } else {
                    wl = (double)L.cs[b][c];
                    wh = (double)L.cs[b][h];
                }
                qc += (lo >= 0 ? wl : 0.0) * (pc - vl);
                qc += (hi >= 0 ? wh : 0.0) * (pc - vh);
            }
            pnew[c] = (T)pc;
            q[c] = (T)qc;
            acc += pc * qc;
        }
        __syncthreads();   // the next plane overwrites this iteration's lower plane
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// 3D smoother and residual sweeps marching along z (levels of at least
// Slot::march_cells cells, by default those whose arrays exceed the Infinity
// Cache): block b
// owns the kMX x kMY columns of tile b mod ncol over kSweepPlanes planes of z
// chunk b / ncol.  The value a stencil reads at the neighbours (x, or b / diag
// for the zero-guess pre-smoothing) is formed once per plane with a one-cell
// x / y halo into a ring of three LDS planes, so the z neighbours come from
// LDS instead of another pass over memory (a grid-stride sweep capped at
// 4096 workgroups spreads four z planes over the eight XCDs per round, and
// the z neighbours of a cell then sit in another XCD's L2).  Per-cell
// arithmetic and order as the grid-stride bodies (a missing neighbour enters
// as the cell itself with weight 0).
// ---------------------------------------------------------------------------
constexpr int kSweepPlanes = 16;

// Ring of three planes (with halo) of a value v(e), 0 outside the domain.
template <typename T>
struct SweepRing {
    T pl[3][kMH * kMW];
};

struct MarchTile {
    int x0, y0, z0, z1, gx, gy, li;
    bool own;
};

// Tile of logical block lb (XCD-contiguous numbering: the columns of a z
// chunk, whose halos overlap, run on the same XCD).
__device__ inline MarchTile march_tile(const Geo &g, int ncolx, int ncol, int lb) {
    MarchTile t;
    const int col = lb % ncol;
    t.z0 = (lb / ncol) * kSweepPlanes;
    t.z1 = t.z0 + kSweepPlanes < (int)g.n[2] ? t.z0 + kSweepPlanes : (int)g.n[2];
    t.x0 = (col % ncolx) * kMX;
    t.y0 = (col / ncolx) * kMY;
    const int tx = (int)threadIdx.x % kMX, ty = (int)threadIdx.x / kMX;
    t.gx = t.x0 + tx;
    t.gy = t.y0 + ty;
    t.li = (ty + 1) * kMW + tx + 1;
    t.own = t.gx < g.n[0] && t.gy < g.n[1];
    return t;
}

// fill plane slot P with v at plane zz of the tile and its halo
template <typename T, typename V>
__device__ inline void march_form(const Geo &g, const MarchTile &t, int zz, T *P, V v) {
    auto wrapc = [](int q, int n, int per, int &w) {
        if (q >= 0 && q < n) {
            w = q;
            return true;
        }
        w = q < 0 ? q + n : q - n;
        return per != 0 && w >= 0 && w < n;
    };
    int gz;
    const bool vz = wrapc(zz, (int)g.n[2], g.per[2], gz);
    for (int i = (int)threadIdx.x; i < kMH * kMW; i += kBlock) {
        const int ly = i / kMW, lx = i - ly * kMW;
        int gx, gy;
        const bool vx = wrapc(t.x0 - 1 + lx, (int)g.n[0], g.per[0], gx);
        const bool vy = wrapc(t.y0 - 1 + ly, (int)g.n[1], g.per[1], gy);
        P[i] = (vx && vy && vz) ? v(gx + (int)g.n[0] * (gy + (int)g.n[1] * gz)) : (T)0;
    }
}

// March over the tile's planes: cell(c, ia, xc, nbv) for every owned cell,
// with the ring values of the cell and its six neighbours.
template <typename T, typename V, typename Cell>
__device__ inline void march_sweep(const Geo &g, int ncolx, int ncol, int ntiles, SweepRing<T> &R, V v, Cell cell) {
    const int lb = xcd_block();
    if (lb >= ntiles) return;   // the whole block (grid rounded up to whole XCD groups)
    const MarchTile t = march_tile(g, ncolx, ncol, lb);
    march_form(g, t, t.z0 - 1, R.pl[(t.z0 + 2) % 3], v);
    march_form(g, t, t.z0, R.pl[t.z0 % 3], v);
    for (int zz = t.z0; zz < t.z1; ++zz) {
        march_form(g, t, zz + 1, R.pl[(zz + 1) % 3], v);
        __syncthreads();
        const T *Pm = R.pl[(zz + 2) % 3], *P0 = R.pl[zz % 3], *Pp = R.pl[(zz + 1) % 3];
        if (t.own) {
            const int c = t.gx + (int)g.n[0] * (t.gy + (int)g.n[1] * zz);
            const int ia[3] = {t.gx, t.gy, zz};
            const T nbv[3][2] = {{P0[t.li - 1], P0[t.li + 1]}, {P0[t.li - kMW], P0[t.li + kMW]}, {Pm[t.li], Pp[t.li]}};
            cell(c, ia, P0[t.li], nbv);
        }
        __syncthreads();   // the next plane overwrites this iteration's lower plane
    }
}

// sum_b cs * v_nb with the neighbour values of the ring
template <typename T>
__device__ inline T march_offsum(const Level<T> &L, int c, const int ia[3], T vc, const T nbv[3][2]) {
    using R = T;
    R acc = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int lo = nb_lo(L.g, c, ia[b], b);
        const int hi = nb_hi(L.g, c, ia[b], b);
        const int h = hi >= 0 ? hi : c;
        const R vl = lo >= 0 ? (R)nbv[b][0] : (R)vc, vh = hi >= 0 ? (R)nbv[b][1] : (R)vc;
        const R wl = (R)L.cs[b][c], wh = (R)L.cs[b][h];
        acc = fmar(lo >= 0 ? wl : (R)0, vl, acc);
        acc = fmar(hi >= 0 ? wh : (R)0, vh, acc);
    }
    return acc;
}

// zero-guess pre-smoothing: red x = b / d, black from those red values
template <typename T, typename TB>
__global__ void __launch_bounds__(kBlock) k_presmooth_march(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                            const int *__restrict__ done, int ncolx, int ncol,
                                                            int ntiles) {
    if (*done) return;
    using R = T;
    __shared__ SweepRing<T> ring;
    auto red = [&](int e) { return (T)((R)b[e] * (R)L.invd[e]); };
    march_sweep<T>(L.g, ncolx, ncol, ntiles, ring, red, [&](int c, const int ia[3], T vc, const T nbv[3][2]) {
        if (((ia[0] + ia[1] + ia[2]) & 1) == 0)
            x[c] = vc;
        else
            x[c] = (T)(((R)b[c] + march_offsum<T>(L, c, ia, vc, nbv)) * (R)L.invd[c]);
    });
}

// in-place Gauss-Seidel update of one colour
template <typename T, typename TB>
__global__ void __launch_bounds__(kBlock) k_gs_color_march(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                           int color, const int *__restrict__ done, int ncolx,
                                                           int ncol, int ntiles) {
    if (*done) return;
    using R = T;
    __shared__ SweepRing<T> ring;
    march_sweep<T>(L.g, ncolx, ncol, ntiles, ring, [&](int e) { return x[e]; },
                   [&](int c, const int ia[3], T vc, const T nbv[3][2]) {
                       if (((ia[0] + ia[1] + ia[2]) & 1) != color) return;
                       x[c] = (T)(((R)b[c] + march_offsum<T>(L, c, ia, vc, nbv)) * (R)L.invd[c]);
                   });
}

// r = b - A x
template <typename T, typename TB>
__global__ void __launch_bounds__(kBlock) k_residual_march(Level<T> L, const TB *__restrict__ b,
                                                           const T *__restrict__ x, const int *__restrict__ done,
                                                           int ncolx, int ncol, int ntiles) {
    if (*done) return;
    using R = T;
    __shared__ SweepRing<T> ring;
    march_sweep<T>(L.g, ncolx, ncol, ntiles, ring, [&](int e) { return x[e]; },
                   [&](int c, const int ia[3], T vc, const T nbv[3][2]) {
                       R acc = (R)L.s[c] * (R)vc;
#pragma unroll
                       for (int a = 0; a < 3; ++a) {
                           const int lo = nb_lo(L.g, c, ia[a], a);
                           const int hi = nb_hi(L.g, c, ia[a], a);
                           const int h = hi >= 0 ? hi : c;
                           const R xl = lo >= 0 ? (R)nbv[a][0] : (R)vc, xh = hi >= 0 ? (R)nbv[a][1] : (R)vc;
                           const R wl = (R)L.cs[a][c], wh = (R)L.cs[a][h];
                           acc = fmar(lo >= 0 ? wl : (R)0, (R)vc - xl, acc);
                           acc = fmar(hi >= 0 ? wh : (R)0, (R)vc - xh, acc);
                       }
                       L.r[c] = (T)((R)b[c] - acc);
                   });
}

// tiles and grid (rounded up to whole XCD groups) of a marching sweep
static inline int march_sweep_grid(const Geo &g, int &ncolx, int &ncol, int &ntiles) {
    ncolx = (int)((g.n[0] + kMX - 1) / kMX);
    ncol = ncolx * (int)((g.n[1] + kMY - 1) / kMY);
    ntiles = ncol * (int)((g.n[2] + kSweepPlanes - 1) / kSweepPlanes);
    return ntiles > 8 ? (ntiles + 7) & ~7 : ntiles;
}

// ---------------------------------------------------------------------------
// 3D V-cycle passes on cubic tiles (levels of at most Slot::tile_cells cells
// above the single-workgroup part): ONE launch per level on the way down
// (zero-guess pre-smoothing, residual, restriction) and one on the way up
// (prolongation, black sweep, red sweep), where the grid-wide form takes
// three dependent launches each -- on these levels a launch costs more than
// its sweep.  A workgroup owns a kTF^3 block of fine cells (kTC^3 coarse
// cells) and recomputes into LDS what its cells' stencils reach in the
// neighbouring tiles:
//   down: b / d of the red cells on a halo of 3, x on a halo of 2, the
//         residual on a halo of 1 (the restriction's outer taps);
//   up:   red x + P e on a halo of 2, the black GS values on a halo of 1,
//         then the red GS values of the owned cells.
// Each value is formed with the arithmetic and order of the grid-wide
// bodies (presmooth_cell, apply_at, restrict_cell, prolong_at,
// gs_color_cell), so both forms give the same bits.  The pre-smoothed x of
// the owned cells goes to the level's r array (the residual stays in LDS)
// and the way up reads it there, writing the smoothed x: a workgroup writes
// its cells while its neighbours still read their halo values.  Positions
// past a wall hold 0 and enter only with weight 0, as a missing neighbour
// does in the grid-wide bodies (the zero product added to a sum that starts
// at +0 leaves it unchanged).
// ---------------------------------------------------------------------------
constexpr int kTF = 8, kTC = kTF / 2;   // fine / coarse cells per tile edge
// Threads per tile: at most one cell of each region per thread (two of the
// widest halo), so that all loads of a tile kernel are issued together.
constexpr int kT3Threads = 1024;

// Global index and coordinates of position (lx, ly, lz) of a tile whose
// first fine cell is f0, with a halo of H cells, wrapped on periodic axes;
// ok = false past a wall (the index is then that of a cell inside).
template <int H>
__device__ inline int tile_cell(const Geo &g, const int f0[3], int lx, int ly, int lz, int ia[3], bool &ok) {
    const int l[3] = {lx, ly, lz};
    ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int p = f0[a] - H + l[a];
        if (p < 0 || p >= g.n[a]) {
            ok = ok && g.per[a] != 0;
            p %= g.n[a];
            p = p < 0 ? p + g.n[a] : p;
        }
        ia[a] = p;
    }
    return ia[0] + g.n[0] * (ia[1] + g.n[1] * ia[2]);
}

// x-pair k of a region of edge E (E even, halo H): position of the member
// of colour col (colour = parity of the global coordinates; the tile origin
// is even and periodic extents are even, so it is the parity of the
// unwrapped position)
template <int E, int H>
__device__ inline void tile_pair(int k, int col, int &lx, int &ly, int &lz) {
    const int kx = k % (E / 2), r = k / (E / 2);
    ly = r % E;
    lz = r / E;
    lx = 2 * kx + ((H + ly + lz + col) & 1);
}

template <int E>
__device__ inline void tile_split(int q, int &lx, int &ly, int &lz) {
    lx = q % E;
    const int r = q / E;
    ly = r % E;
    lz = r / E;
}

// The loads of one cell's stencil, issued at the start of a tile kernel
// (each kernel then waits on one round of loads, not one per pass):
// neighbour existence (nb_lo / nb_hi), b, the diagonal term (1 / d for a
// sweep, s for the residual) and the coefficients of the faces towards the
// neighbours.
template <typename T>
struct TileSt {
    bool lo[3], hi[3];
    T bv, dv, wl[3], wh[3];
};

template <typename T, typename TB, bool RES>
__device__ inline void tile_load(const Level<T> &L, const TB *__restrict__ b, int c, const int ia[3], TileSt<T> &S) {
    using R = T;
    S.bv = (R)b[c];
    S.dv = RES ? (R)L.s[c] : (R)L.invd[c];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int lo = nb_lo(L.g, c, ia[a], a);
        const int hi = nb_hi(L.g, c, ia[a], a);
        const int h = hi >= 0 ? hi : c;
        S.lo[a] = lo >= 0;
        S.hi[a] = hi >= 0;
        S.wl[a] = (R)L.cs[a][c];
        S.wh[a] = (R)L.cs[a][h];
    }
}

// GS value (b_c + sum_b cs * v_nb) / d_c from the neighbours' values at
// stride offsets of position q of an LDS region of edge E (offsum_at's
// order; a missing neighbour enters as 0 with weight 0)
template <typename T, int E>
__device__ inline T tile_gs(const TileSt<T> &S, const T *v, int q) {
    using R = T;
    constexpr int st[3] = {1, E, E * E};
    R acc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R vl = S.lo[a] ? (R)v[q - st[a]] : (R)0, vh = S.hi[a] ? (R)v[q + st[a]] : (R)0;
        acc = fmar(S.lo[a] ? S.wl[a] : (R)0, vl, acc);
        acc = fmar(S.hi[a] ? S.wh[a] : (R)0, vh, acc);
    }
    return (T)((S.bv + acc) * S.dv);
}

// residual b - A x at position q (apply_at's order)
template <typename T, int E>
__device__ inline T tile_res(const TileSt<T> &S, const T *v, int q) {
    using R = T;
    constexpr int st[3] = {1, E, E * E};
    const R xc = (R)v[q];
    R acc = S.dv * xc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R xl = S.lo[a] ? (R)v[q - st[a]] : xc, xh = S.hi[a] ? (R)v[q + st[a]] : xc;
        acc = fmar(S.lo[a] ? S.wl[a] : (R)0, xc - xl, acc);
        acc = fmar(S.hi[a] ? S.wh[a] : (R)0, xc - xh, acc);
    }
    return (T)(S.bv - acc);
}

// P e at fine cell fi: the eight coarse taps loaded up front, then
// prolong_at's weights and summation order
template <typename T>
struct TilePro {
    T X[2][2][2];
    T w0[3], w1[3];
};

template <typename T>
__device__ inline void pro_load(const Geo &gc, const T *__restrict__ xc, const int fi[3], TilePro<T> &P) {
    using R = T;
    int c0[3], c1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) pro_axis<R>(fi[a], gc.n[a], gc.per[a], c0[a], c1[a], P.w0[a], P.w1[a]);
    const int nx = gc.n[0], nxy = gc.n[0] * gc.n[1];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const int kz = (dz ? c1[2] : c0[2]) * nxy;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int ky = kz + (dy ? c1[1] : c0[1]) * nx;
            P.X[dz][dy][0] = xc[ky + c0[0]];
            P.X[dz][dy][1] = xc[ky + c1[0]];
        }
    }
}

template <typename T>
__device__ inline T pro_value(const TilePro<T> &P) {
    using R = T;
    R v = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const R wz = dz ? P.w1[2] : P.w0[2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const R wyz = wz * (dy ? P.w1[1] : P.w0[1]);
            v = pro_row(v, wyz, P.w0[0], (R)P.X[dz][dy][0], P.w1[0], (R)P.X[dz][dy][1]);
        }
    }
    return v;
}

template <typename T, typename TB>
__global__ void __launch_bounds__(kT3Threads) k_down3_tile(Level<T> L, Geo gc, const TB *__restrict__ b,
                                                           T *__restrict__ bc, int ntx, int nty, int ntiles,
                                                           const int *__restrict__ done) {
    using R = T;
    const int tile = xcd_block();
    if (tile >= ntiles || *done) return;
    constexpr int E3 = kTF + 6, E2 = kTF + 4, E1 = kTF + 2;
    constexpr int N3 = E3 * E3 * E3 / 2, N2 = E2 * E2 * E2 / 2, N1 = E1 * E1 * E1;
    constexpr int K3 = (N3 + kT3Threads - 1) / kT3Threads;
    static_assert(N2 <= kT3Threads && N1 <= kT3Threads, "one x pair and one residual cell per thread");
    __shared__ T sd[E3 * E3 * E3];   // red b / d, halo 3
    __shared__ T sx[E2 * E2 * E2];   // pre-smoothed x, halo 2
    __shared__ T sr[E1 * E1 * E1];   // residual, halo 1
    const Geo &g = L.g;
    const int tz = tile / (ntx * nty), trem = tile - tz * ntx * nty, ty = trem / ntx, tx = trem - ty * ntx;
    const int f0[3] = {tx * kTF, ty * kTF, tz * kTF};
    const int tid = (int)threadIdx.x;
    // loads: red b and 1 / d (halo 3), the black member of an x-pair (halo 2),
    // a residual cell (halo 1)
    R rb[K3], rd[K3];
    int rq[K3];
    bool rok[K3];
#pragma unroll
    for (int j = 0; j < K3; ++j) {
        const int k = tid + j * kT3Threads;
        int lx, ly, lz, ia[3];
        tile_pair<E3, 3>(k < N3 ? k : N3 - 1, 0, lx, ly, lz);
        const int c = tile_cell<3>(g, f0, lx, ly, lz, ia, rok[j]);
        rq[j] = lx + E3 * (ly + E3 * lz);
        rb[j] = (R)b[c];
        rd[j] = (R)L.invd[c];
    }
    int x2, y2, z2, ia2[3];
    bool ok2;
    tile_pair<E2, 2>(tid < N2 ? tid : 0, 1, x2, y2, z2);
    TileSt<T> S2;
    tile_load<T, TB, false>(L, b, tile_cell<2>(g, f0, x2, y2, z2, ia2, ok2), ia2, S2);
    int x1, y1, z1, ia1[3];
    bool ok1;
    tile_split<E1>(tid < N1 ? tid : 0, x1, y1, z1);
    TileSt<T> S1;
    tile_load<T, TB, true>(L, b, tile_cell<1>(g, f0, x1, y1, z1, ia1, ok1), ia1, S1);
#pragma unroll
    for (int j = 0; j < K3; ++j)
        if (tid + j * kT3Threads < N3) sd[rq[j]] = rok[j] ? (T)(rb[j] * rd[j]) : (T)0;
    __syncthreads();
    // x: black GS from the red neighbours' b / d, red b / d
    if (tid < N2) {
        const int q = x2 + E2 * (y2 + E2 * z2);
        const int q3 = (x2 + 1) + E3 * ((y2 + 1) + E3 * (z2 + 1));
        const T v = tile_gs<T, E3>(S2, sd, q3);
        sx[q] = ok2 ? v : (T)0;
        const int d = 1 - 2 * (x2 & 1);   // the red member of the x-pair
        sx[q + d] = sd[q3 + d];
    }
    __syncthreads();
    // r = b - A x
    if (tid < N1) {
        const T v = tile_res<T, E2>(S1, sx, (x1 + 1) + E2 * ((y1 + 1) + E2 * (z1 + 1)));
        sr[tid] = ok1 ? v : (T)0;
    }
    // the owned cells' pre-smoothed x (read back on the way up)
    if (tid < kTF * kTF * kTF) {
        int lx, ly, lz;
        tile_split<kTF>(tid, lx, ly, lz);
        const int gx = f0[0] + lx, gy = f0[1] + ly, gz = f0[2] + lz;
        if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2])
            L.r[gx + g.n[0] * (gy + g.n[1] * gz)] = sx[(lx + 2) + E2 * ((ly + 2) + E2 * (lz + 2))];
    }
    __syncthreads();
    // restriction (restrict_cell's weights and order) of the tile's coarse cells
    if (tid < kTC * kTC * kTC) {
        int cx, cy, cz;
        tile_split<kTC>(tid, cx, cy, cz);
        const int I[3] = {tx * kTC + cx, ty * kTC + cy, tz * kTC + cz};
        if (I[0] < gc.n[0] && I[1] < gc.n[1] && I[2] < gc.n[2]) {
            int f[4];
            R wx[4], wy[4], wz[4];
            res_axis<R>(I[0], gc.n[0], g.n[0], gc.per[0], f, wx);
            res_axis<R>(I[1], gc.n[1], g.n[1], gc.per[1], f, wy);
            res_axis<R>(I[2], gc.n[2], g.n[2], gc.per[2], f, wz);
            R acc = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const R wza = wz[a];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T *row = &sr[2 * cx + E1 * ((2 * cy + q) + E1 * (2 * cz + a))];
                    R s = 0.0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) s = fmar(wx[e], (R)row[e], s);
                    acc = fmar(wy[q] * wza, s, acc);
                }
            }
            bc[(I[2] * gc.n[1] + I[1]) * gc.n[0] + I[0]] = (T)acc;
        }
    }
}

template <typename T, typename TB>
__global__ void __launch_bounds__(kT3Threads) k_up3_tile(Level<T> L, Geo gc, const T *__restrict__ xc,
                                                         const TB *__restrict__ b, const T *__restrict__ xpre,
                                                         T *__restrict__ x, int ntx, int nty, int ntiles,
                                                         const int *__restrict__ done) {
    using R = T;
    const int tile = xcd_block();
    if (tile >= ntiles || *done) return;
    constexpr int E2 = kTF + 4, E1 = kTF + 2;
    constexpr int N2 = E2 * E2 * E2 / 2, N1 = E1 * E1 * E1 / 2, N0 = kTF * kTF * kTF / 2;
    static_assert(N2 <= kT3Threads, "one red cell of the halo-2 region per thread");
    __shared__ T se[E2 * E2 * E2];   // red x + P e, halo 2
    __shared__ T sb[E1 * E1 * E1];   // black GS values, halo 1
    const Geo &g = L.g;
    const int tz = tile / (ntx * nty), trem = tile - tz * ntx * nty, ty = trem / ntx, tx = trem - ty * ntx;
    const int f0[3] = {tx * kTF, ty * kTF, tz * kTF};
    const int tid = (int)threadIdx.x;
    // loads: a red cell's x and coarse taps (halo 2), a black cell (halo 1),
    // an owned x-pair
    int x2, y2, z2, ia2[3];
    bool ok2;
    tile_pair<E2, 2>(tid < N2 ? tid : 0, 0, x2, y2, z2);
    const int c2 = tile_cell<2>(g, f0, x2, y2, z2, ia2, ok2);
    const R xp = (R)xpre[c2];
    TilePro<T> P;
    pro_load<T>(gc, xc, ia2, P);
    int x1, y1, z1, ia1[3];
    bool ok1;
    tile_pair<E1, 1>(tid < N1 ? tid : 0, 1, x1, y1, z1);
    TileSt<T> S1;
    tile_load<T, TB, false>(L, b, tile_cell<1>(g, f0, x1, y1, z1, ia1, ok1), ia1, S1);
    int x0, y0, z0;
    tile_pair<kTF, 0>(tid < N0 ? tid : 0, 0, x0, y0, z0);
    int ia0[3] = {f0[0] + x0, f0[1] + y0, f0[2] + z0};
    // whole pairs (even extents): the red member inside <=> the pair inside
    const bool own0 = tid < N0 && ia0[0] < g.n[0] && ia0[1] < g.n[1] && ia0[2] < g.n[2];
    if (!own0) ia0[0] = ia0[1] = ia0[2] = 0;
    const int c0 = ia0[0] + g.n[0] * (ia0[1] + g.n[1] * ia0[2]);
    TileSt<T> S0;
    tile_load<T, TB, false>(L, b, c0, ia0, S0);
    if (tid < N2) {
        const T v = (T)(xp + pro_value<T>(P));
        se[x2 + E2 * (y2 + E2 * z2)] = ok2 ? v : (T)0;
    }
    __syncthreads();
    if (tid < N1) {
        const T v = tile_gs<T, E2>(S1, se, (x1 + 1) + E2 * ((y1 + 1) + E2 * (z1 + 1)));
        sb[x1 + E1 * (y1 + E1 * z1)] = ok1 ? v : (T)0;
    }
    __syncthreads();
    if (own0) {
        const int q1 = (x0 + 1) + E1 * ((y0 + 1) + E1 * (z0 + 1));
        const int d = 1 - 2 * (x0 & 1);   // the black member of the x-pair
        x[c0] = tile_gs<T, E1>(S0, sb, q1);
        x[c0 + d] = sb[q1 + d];
    }
}

// Whether level l of a 3D slot runs the tile passes: above the
// single-workgroup part, below march_cells and at most tile_cells cells,
// with even extents (every level that has a coarser one).
template <typename T>
static bool tile3_level(const Slot<T> &S, int l) {
    const Geo &g = S.lev[l].g;
    return l + 1 < S.nlev && g.N <= S.tile_cells && g.N < S.march_cells && (g.n[0] & 1) == 0 &&
           (g.n[1] & 1) == 0 && (g.n[2] & 1) == 0;
}

static inline int tile3_grid(const Geo &gc, int &ntx, int &nty, int &ntiles) {
    ntx = (gc.n[0] + kTC - 1) / kTC;
    nty = (gc.n[1] + kTC - 1) / kTC;
    ntiles = ntx * nty * ((gc.n[2] + kTC - 1) / kTC);
    return ntiles > 8 ? (ntiles + 7) & ~7 : ntiles;
}

// CH operator, first half: p_new = z + beta p_old, t = L p_new.
template <typename T, typename TZ, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_ch_lap(Geo g, double ih2, const TZ *__restrict__ z,
                                                       const T *__restrict__ pold, T *__restrict__ pnew,
                                                       T *__restrict__ t, Scal *sc, const double *__restrict__ rz0,
                                                       int nrz, int k, T *__restrict__ rpend,
                                                       const T *__restrict__ q) {
    if (sc->done) return;
    const double alpha_prev = rpend ? sc->alpha : 0.0;
    IterStart it;
    if (!iter_start(sc, rz0, rz0, rz0, nrz, g.N, k, 0, it)) return;
    const double beta = it.beta;
    auto pv = [&](int e) { return (double)z[e] + (beta != 0.0 ? beta * (double)pold[e] : 0.0); };
    GRID_LOOP(g.N) {
        int ia[3];
        coords_of<DIM>(g, c, ia);
        // residual of the previous iteration (q is rewritten by the second half)
        if (rpend) rpend[c] = (T)cg_residual((double)rpend[c], (double)q[c], alpha_prev);
        pnew[c] = (T)pv(c);
        t[c] = (T)lap_at<DIM>(g, c, ia, ih2, pv);
    }
}

// CH operator, second half: q = p - a t + b L t; partial p.q.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_ch_apply(Geo g, double ih2, double ca, double cb,
                                                         const T *__restrict__ p, const T *__restrict__ t,
                                                         T *__restrict__ q, const Scal *__restrict__ sc,
                                                         double *__restrict__ part) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    auto tv = [&](int e) { return (double)t[e]; };
    double acc = 0.0;
    GRID_LOOP(g.N) {
        int ia[3];
        coords_of<DIM>(g, c, ia);
        const double pc = (double)p[c];
        const double qc = pc - ca * (double)t[c] + cb * lap_at<DIM>(g, c, ia, ih2, tv);
        q[c] = (T)qc;
        acc += pc * qc;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// End of CG iteration: r.r, the iteration count and the stop flags (thread 0)
__device__ inline void pcg_fin_rr_dev(Scal *sc, double rr) {
    if (threadIdx.x != 0) return;
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

// alpha = rz / sum(part_pq) (every block, same order); x += alpha p;
// r -= alpha q; partial r.r.  TP != T: also rp = r rounded to TP (the
// right-hand side of the preconditioner in its own precision).
template <typename T, typename TP = T>
__global__ void __launch_bounds__(kBlock) k_pcg_update(int N, const T *__restrict__ p, const T *__restrict__ q,
                                                       T *__restrict__ x, T *__restrict__ r, Scal *sc,
                                                       const double *__restrict__ part_pq, int nparts,
                                                       double *__restrict__ part_rr, TP *__restrict__ rp = nullptr) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    const double pq = sum_parts_all(part_pq, nparts, lds);
    const double alpha = pq != 0.0 ? sc->rz / pq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
    }
    double acc = 0.0;
    GRID_LOOP(N) {
        x[c] = (T)((double)x[c] + alpha * (double)p[c]);
        const double rc = cg_residual((double)r[c], (double)q[c], alpha);
        r[c] = (T)rc;
        if constexpr (!std::is_same<T, TP>::value) rp[c] = (TP)(T)rc;
        acc += rc * rc;
    }
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// rp = r rounded to the preconditioner's precision
template <typename T, typename TP>
__global__ void __launch_bounds__(kBlock) k_round_vec(int N, const T *__restrict__ r, TP *__restrict__ rp) {
    GRID_LOOP(N) rp[c] = (TP)r[c];
}

// one workgroup: rr = sum(part_rr); iteration count; convergence flag
__global__ void __launch_bounds__(kBlock) k_pcg_fin_rr(Scal *sc, const double *__restrict__ part_rr, int nparts) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    pcg_fin_rr_dev(sc, sum_parts_all(part_rr, nparts, lds));
}

// partials of r.z, sum z, sum r
template <typename T, typename TZ>
__global__ void __launch_bounds__(kBlock) k_pcg_rz(int N, const T *__restrict__ r, const TZ *__restrict__ z,
                                                   const Scal *__restrict__ sc, double *__restrict__ p0,
                                                   double *__restrict__ p1, double *__restrict__ p2, int singular) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    double arz = 0.0, az = 0.0, ar = 0.0;
    GRID_LOOP(N) {
        const double rc = (double)r[c], zc = (double)z[c];
        arz += rc * zc;
        az += zc;
        ar += rc;
    }
    const double s0 = block_sum(arz, lds);
    const double s1 = singular ? block_sum(az, lds) : 0.0;
    const double s2 = singular ? block_sum(ar, lds) : 0.0;
    if (threadIdx.x == 0) {
        p0[blockIdx.x] = s0;
        p1[blockIdx.x] = s1;
        p2[blockIdx.x] = s2;
    }
}

// The last pass of a 3D preconditioner (the red sweep of level 0) with the
// partials of k_pcg_rz: the same cells per thread and block (grid-stride
// over grid_red(N) blocks) and the same sums, so the partials are those of
// the separate pass bit for bit; the z of a black cell is read back, the
// z of a red cell is its new value.
template <typename T, typename TB, int DIM, typename TR>
__global__ void __launch_bounds__(kBlock) k_gs_red_rz(Level<T> L, const TB *__restrict__ b, T *__restrict__ x,
                                                      const TR *__restrict__ r, const Scal *__restrict__ sc,
                                                      double *__restrict__ p0, double *__restrict__ p1,
                                                      double *__restrict__ p2, int singular) {
    if (sc->done) return;
    __shared__ double lds[kBlock / kWave];
    double arz = 0.0, az = 0.0, ar = 0.0;
    GRID_LOOP(L.g.N) {
        gs_color_cell<T, TB, DIM>(L, b, x, 0, c);
        const double rc = (double)r[c], zc = (double)x[c];
        arz += rc * zc;
        az += zc;
        ar += rc;
    }
    const double s0 = block_sum(arz, lds);
    const double s1 = singular ? block_sum(az, lds) : 0.0;
    const double s2 = singular ? block_sum(ar, lds) : 0.0;
    if (threadIdx.x == 0) {
        p0[blockIdx.x] = s0;
        p1[blockIdx.x] = s1;
        p2[blockIdx.x] = s2;
    }
}

// r = b - A x (slot operator); partials of b.b and r.r; rp (when given):
// r rounded to the preconditioner's precision.  conv: also the level-0
// arrays of the preconditioner's hierarchy B that the set-up would write
// (a cycle that ends on the grid needs nothing else): 1 / diag, and for a
// lower precision the rounded s and cs[b], with the arithmetic and order of
// k_invd / k_conv_coef (bit for bit).
template <typename T, int DIM, typename TP = T>
__global__ void __launch_bounds__(kBlock) k_pcg_init_slot(Level<T> L, const T *__restrict__ b,
                                                          const T *__restrict__ x, T *__restrict__ r,
                                                          double *__restrict__ p0, double *__restrict__ p1,
                                                          TP *__restrict__ rp, Level<TP> B, int conv) {
    constexpr bool kSame = std::is_same<T, TP>::value;
    __shared__ double lds[kBlock / kWave];
    double bb = 0.0, rr = 0.0;
    GRID_LOOP(L.g.N) {
        int ia[3];
        coords_of<DIM>(L.g, c, ia);
        const double bc = (double)b[c];
        const double rc = bc - apply_at<T, DIM>(L, x, c, ia);
        r[c] = (T)rc;
        if (rp) rp[c] = (TP)(T)rc;   // the preconditioner's copy (k_round_vec's value)
        bb += bc * bc;
        rr += rc * rc;
        if (conv) {
            const TP sv = (TP)L.s[c];
            if (!kSame) B.s[c] = sv;
            TP d = sv;
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const TP w = (TP)L.cs[q][c];
                if (!kSame) B.cs[q][c] = w;
                if (nb_lo(L.g, c, ia[q], q) >= 0) d += w;
                const int hi = nb_hi(L.g, c, ia[q], q);
                if (hi >= 0) d += (TP)L.cs[q][hi];
            }
            B.invd[c] = (TP)1 / d;
        }
    }
    const double s0 = block_sum(bb, lds);
    const double s1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        p0[blockIdx.x] = s0;
        p1[blockIdx.x] = s1;
    }
}

// zero initial guess: x = 0, r = b; partials of b.b (twice)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_init_zero(int N, const T *__restrict__ b, T *__restrict__ x,
                                                          T *__restrict__ r, double *__restrict__ p0,
                                                          double *__restrict__ p1) {
    __shared__ double lds[kBlock / kWave];
    double bb = 0.0;
    GRID_LOOP(N) {
        const T bc = b[c];
        x[c] = (T)0;
        r[c] = bc;
        bb += (double)bc * (double)bc;
    }
    const double s0 = block_sum(bb, lds);
    if (threadIdx.x == 0) {
        p0[blockIdx.x] = s0;
        p1[blockIdx.x] = s0;
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_ch_lap_plain(Geo g, double ih2, const T *__restrict__ x,
                                                         T *__restrict__ t) {
    auto xv = [&](int e) { return (double)x[e]; };
    GRID_LOOP(g.N) {
        int ia[3];
        coords_of<DIM>(g, c, ia);
        t[c] = (T)lap_at<DIM>(g, c, ia, ih2, xv);
    }
}

// CH: r = b - (x - a t + b L t) with t = L x; partials b.b, r.r
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_pcg_init_ch(Geo g, double ih2, double ca, double cb,
                                                        const T *__restrict__ b, const T *__restrict__ x,
                                                        const T *__restrict__ t, T *__restrict__ r,
                                                        double *__restrict__ p0, double *__restrict__ p1) {
    __shared__ double lds[kBlock / kWave];
    auto tv = [&](int e) { return (double)t[e]; };
    double bb = 0.0, rr = 0.0;
    GRID_LOOP(g.N) {
        int ia[3];
        coords_of<DIM>(g, c, ia);
        const double Mx = (double)x[c] - ca * (double)t[c] + cb * lap_at<DIM>(g, c, ia, ih2, tv);
        const double bc = (double)b[c];
        const double rc = bc - Mx;
        r[c] = (T)rc;
        bb += bc * bc;
        rr += rc * rc;
    }
    const double s0 = block_sum(bb, lds);
    const double s1 = block_sum(rr, lds);
    if (threadIdx.x == 0) {
        p0[blockIdx.x] = s0;
        p1[blockIdx.x] = s1;
    }
}

// one workgroup: initialise the scalars from the b.b and r0.r0 partials
__global__ void __launch_bounds__(kBlock) k_pcg_fin_init(Scal *sc, const double *__restrict__ p0,
                                                         const double *__restrict__ p1, int nparts, double rtol,
                                                         int max_iter) {
    __shared__ double lds[kBlock / kWave];
    const double tb = sum_parts_all(p0, nparts, lds);
    const double tr = sum_parts_all(p1, nparts, lds);
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

// mean removal: partial sums, then every block sums them and subtracts
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum(int N, const T *__restrict__ x, double *__restrict__ part) {
    __shared__ double lds[kBlock / kWave];
    double acc = 0.0;
    GRID_LOOP(N) acc += (double)x[c];
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x -= mean(x); copy (when given) receives the same values
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sub_mean(int N, T *__restrict__ x, const double *__restrict__ part,
                                                     int nparts, T *__restrict__ copy) {
    __shared__ double lds[kBlock / kWave];
    const double m = sum_parts_all(part, nparts, lds) / (double)N;
    GRID_LOOP(N) {
        const T v = (T)((double)x[c] - m);
        x[c] = v;
        if (copy) copy[c] = v;
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_slot_apply(Level<T> L, const T *__restrict__ x, T *__restrict__ y) {
    GRID_LOOP(L.g.N) {
        int ia[3];
        coords_of<DIM>(L.g, c, ia);
        y[c] = (T)apply_at<T, DIM>(L, x, c, ia);
    }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
#define LAUNCH(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_for(n)), dim3(kBlock), st, __VA_ARGS__)
#define LAUNCH1(cls, bytes, kern, threads, st, ...) TLAUNCH(cls, bytes, kern, dim3(1), dim3(threads), st, __VA_ARGS__)
// kernels that produce per-block partials use at most kRedBlocks blocks
#define LAUNCHR(cls, bytes, kern, n, st, ...) TLAUNCH(cls, bytes, kern, dim3(grid_red(n)), dim3(kBlock), st, __VA_ARGS__)

// First level handled by the single-workgroup kernel.
template <typename T>
static int single_block_level(const Slot<T> &S) {
    int l = 0;
    const int lim = sb_cells();
    while (l < S.nlev - 1 && S.lev[l].g.N > lim) ++l;
    return l;
}

// Level at which the V-cycle of S ends (-1: it runs down to the coarsest).
template <typename T>
static int trunc_level(const Slot<T> &S, int dim) {
    return dim == 3 && S.ltrunc >= 0 && S.ltrunc < S.lsb ? S.ltrunc : -1;
}

template <typename T, int DIM>
static void mg_setup_d(Slot<T> &S, hipStream_t st, bool invd0) {
    constexpr double W = sizeof(T);
    S.lsb = single_block_level(S);
    const int lsb = S.lsb;
    const int lt = trunc_level(S, DIM);
    if (lsb > 0 && invd0)
        LAUNCH(K_MG_SETUP, W * (2 + DIM) * S.lev[0].g.N, (k_invd<T, DIM>), S.lev[0].g.N, st, S.lev[0]);
    for (int l = 1; l < (lt >= 0 ? lt + 1 : lsb); ++l) {
        LAUNCH(K_MG_SETUP, W * (1 + DIM) * (S.lev[l - 1].g.N + S.lev[l].g.N), (k_coarsen<T, DIM>), S.lev[l].g.N, st,
               S.lev[l - 1], S.lev[l]);
        LAUNCH(K_MG_SETUP, W * (2 + DIM) * S.lev[l].g.N, (k_invd<T, DIM>), S.lev[l].g.N, st, S.lev[l]);
    }
    if (lt >= 0) return;   // the cycle ends at level lt: no small levels, no coarsest inverse
    double bytes = 0.0;
    for (int l = lsb; l < S.nlev; ++l) bytes += W * (2 + 2 * DIM) * S.lev[l].g.N;
    bytes += 8.0 * S.ncoarse * S.ncoarse;
    LAUNCH1(K_MG_SETUP, bytes, (k_setup_block<T, DIM>), kSBThreads, st, S, lsb);
}

template <typename T>
void mg_setup(Slot<T> &S, int dim, hipStream_t st, bool invd0) {
    if (dim == 2)
        mg_setup_d<T, 2>(S, st, invd0);
    else
        mg_setup_d<T, 3>(S, st, invd0);
}

// 2D tile grid of a level: tiles along x, rounded up to whole XCD groups
// Level-0 role of a 2D V-cycle inside CG (tile kernels only): down_upd:
// the way down also performs the CG update of the iteration
// (k_down_tile2_cg, then k_pcg_fin_rr); bpend: the right-hand side is the
// pending residual r - alpha q; dmode: partials of r.z, sum z, sum r on the
// way up (0 none, 1 r as stored, 2 r pending).
template <typename TR>
struct L0Cg {
    int down_upd, bpend, dmode;
    const TR *r, *q, *p;
    TR *x;
    Scal *sc;
    const double *part_pq;
    int npq;
    double *part_rr;
    double *rz0, *rz1, *rz2;
};

static void tile_grid2(const Geo &g, int &ntx, int &ntiles, int &grid) {
    ntx = ((int)g.n[0] + kTFX - 1) / kTFX;
    ntiles = ntx * (((int)g.n[1] + kTFY - 1) / kTFY);
    grid = ntiles > 8 ? (ntiles + 7) & ~7 : ntiles;
}

// The r.z partials of CG (k_pcg_rz) taken by the last pass of a 3D
// preconditioner, the red sweep of level 0 (k_gs_red_rz); *taken is set
// when that pass ran in the grid-wide form, which is the one that can.
template <typename TR>
struct RzFuse {
    const TR *r;
    const Scal *sc;
    double *p0, *p1, *p2;
    int singular;
    bool *taken;
};

// red sweep of level 0, with the r.z partials when rz is given
template <typename T, typename TB, int DIM, typename TR>
static void gs_red_last(Level<T> &L, const TB *b, T *x, const int *done, hipStream_t st, const RzFuse<TR> *rz) {
    const double N = (double)L.g.N;
    const double bytes = sizeof(T) * (3.5 + DIM) * N + (sizeof(TB) - sizeof(T)) * N;
    if (rz) {
        LAUNCHR(K_SMOOTH, bytes + sizeof(TR) * N, (k_gs_red_rz<T, TB, DIM, TR>), L.g.N, st, L, b, x, rz->r, rz->sc,
                rz->p0, rz->p1, rz->p2, rz->singular);
        *rz->taken = true;
    } else {
        LAUNCH(K_SMOOTH, bytes, (k_gs_color<T, TB, DIM>), L.g.N, st, L, b, x, 0, done);
    }
}

template <typename T, typename TB, int DIM, typename TR = T>
static void vcycle_down(Slot<T> &S, int l, const TB *b, T *x, const int *done, hipStream_t st,
                        const L0Cg<TR> *cg = nullptr) {
    constexpr double W = sizeof(T);
    Level<T> &lv = S.lev[l];
    const int N = (int)lv.g.N, Nc = (int)S.lev[l + 1].g.N;
    if (DIM == 2) {
        int ntx, ntiles, grid;
        tile_grid2(lv.g, ntx, ntiles, grid);
        if (cg && cg->down_upd) {
            constexpr double WR = sizeof(TR);
            // r, q, p, x in, x out; invd, s, cs in; x, bc out
            const double bytes = 5.0 * WR * N + W * (3 + DIM) * N + W * Nc;
            TLAUNCH(K_MG_DOWN, bytes, (k_down_tile2_cg<T, TR>), dim3(grid), dim3(kTileThreads), st, lv,
                    S.lev[l + 1].g, cg->r, cg->q, cg->p, cg->x, lv.r, S.lev[l + 1].b, ntx, ntiles, cg->sc,
                    cg->part_pq, cg->npq, cg->part_rr);
            LAUNCH1(K_PCG_UPDATE, 8.0 * ntiles, (k_pcg_fin_rr), kBlock, st, cg->sc, (const double *)cg->part_rr,
                    ntiles);
            return;
        }
        const double bytes = (sizeof(TB) + W * (3 + DIM)) * N + W * Nc;   // b, invd, s, cs in; x, bc out
        TLAUNCH(K_MG_DOWN, bytes, (k_down_tile2<T, TB>), dim3(grid), dim3(kTileThreads), st, lv, S.lev[l + 1].g, b,
                lv.r, S.lev[l + 1].b, ntx, ntiles, done);
        return;
    }
    const double WB = sizeof(TB) - W;   // extra bytes of a wider right-hand side
    if (DIM == 3 && tile3_level(S, l)) {
        // b, invd, s, cs in; pre-smoothed x (to r) and the coarse b out
        int ntx, nty, ntiles;
        const int grid = tile3_grid(S.lev[l + 1].g, ntx, nty, ntiles);
        TLAUNCH(K_MG_DOWN, (sizeof(TB) + W * (3 + DIM)) * N + W * Nc, (k_down3_tile<T, TB>), dim3(grid),
                dim3(kT3Threads), st, lv, S.lev[l + 1].g, b, S.lev[l + 1].b, ntx, nty, ntiles, done);
        return;
    }
    if (DIM == 3 && lv.g.N >= S.march_cells) {
        int ncolx, ncol, ntiles;
        const int grid = march_sweep_grid(lv.g, ncolx, ncol, ntiles);
        TLAUNCH(K_SMOOTH, W * (3 + DIM) * N + WB * N, (k_presmooth_march<T, TB>), dim3(grid), dim3(kBlock), st, lv, b,
                x, done, ncolx, ncol, ntiles);
        TLAUNCH(K_RESIDUAL, W * (4 + DIM) * N + WB * N, (k_residual_march<T, TB>), dim3(grid), dim3(kBlock), st, lv,
                b, (const T *)x, done, ncolx, ncol, ntiles);
    } else {
        if ((lv.g.n[0] & 1) == 0)
            LAUNCH(K_SMOOTH, W * (3 + DIM) * N + WB * N, (k_presmooth_pair<T, TB, DIM>), N / 2, st, lv, b, x, done);
        else
            LAUNCH(K_SMOOTH, W * (3 + DIM) * N + WB * N, (k_presmooth<T, TB, DIM>), N, st, lv, b, x, done);
        LAUNCH(K_RESIDUAL, W * (4 + DIM) * N + WB * N, (k_residual<T, TB, DIM>), N, st, lv, b, (const T *)x, done);
    }
    {
        const Geo &gc = S.lev[l + 1].g;
        const int ntx = (int)((gc.n[0] + kRCX - 1) / kRCX), nty = (int)((gc.n[1] + kRCY - 1) / kRCY);
        const int ntiles = ntx * nty * (int)((gc.n[2] + kRCZ - 1) / kRCZ);
        const int grid = ntiles > 8 ? (ntiles + 7) & ~7 : ntiles;
        TLAUNCH(K_RESTRICT, W * (N + Nc), (k_restrict3_lds<T>), dim3(grid), dim3(kBlock), st, lv.g, gc,
                (const T *)lv.r, S.lev[l + 1].b, ntx, nty, ntiles, done);
    }
}

template <typename T, typename TB, int DIM, typename TR = T>
static void vcycle_up(Slot<T> &S, int l, const TB *b, T *x, const int *done, hipStream_t st,
                      const L0Cg<TR> *cg = nullptr, const RzFuse<TR> *rz = nullptr) {
    constexpr double W = sizeof(T);
    Level<T> &lv = S.lev[l];
    const int N = (int)lv.g.N, Nc = (int)S.lev[l + 1].g.N;
    if (DIM == 2) {
        int ntx, ntiles, grid;
        tile_grid2(lv.g, ntx, ntiles, grid);
        if constexpr (std::is_same<TB, T>::value) {
            if (cg && (cg->bpend || cg->dmode)) {
                constexpr double WR = sizeof(TR);
                // right-hand side (r, q when pending), invd, cs, x, xc in; x out; r (and q) for the dots
                const double rhs = cg->bpend ? 2.0 * WR : (double)sizeof(TB);
                const double dots = cg->dmode == 0 ? 0.0 : (cg->bpend ? 0.0 : (cg->dmode == 2 ? 2.0 : 1.0) * WR);
                const double bytes = (rhs + dots + W * (3 + DIM)) * N + W * Nc;
                TLAUNCH(K_MG_UP, bytes, (k_up_tile2_cg<T, TR>), dim3(grid), dim3(kTileThreads), st, lv,
                        S.lev[l + 1].g, (const T *)S.lev[l + 1].x, (const T *)b, cg->r, cg->q, (const T *)lv.r, x,
                        ntx, ntiles, (const Scal *)cg->sc, cg->bpend, cg->dmode, cg->rz0, cg->rz1, cg->rz2, done);
                return;
            }
        }
        const double bytes = (sizeof(TB) + W * (3 + DIM)) * N + W * Nc;   // b, invd, cs, x, xc in; x out
        TLAUNCH(K_MG_UP, bytes, (k_up_tile2<T, TB>), dim3(grid), dim3(kTileThreads), st, lv, S.lev[l + 1].g,
                (const T *)S.lev[l + 1].x, b, (const T *)lv.r, x, ntx, ntiles, done);
        return;
    }
    const double WB = sizeof(TB) - W;
    if (DIM == 3 && tile3_level(S, l)) {
        // pre-smoothed x (from r), b, invd, cs, coarse x in; x out
        int ntx, nty, ntiles;
        const int grid = tile3_grid(S.lev[l + 1].g, ntx, nty, ntiles);
        TLAUNCH(K_MG_UP, (sizeof(TB) + W * (3 + DIM)) * N + W * Nc, (k_up3_tile<T, TB>), dim3(grid),
                dim3(kT3Threads), st, lv, S.lev[l + 1].g, (const T *)S.lev[l + 1].x, b, (const T *)lv.r, x, ntx, nty,
                ntiles, done);
        return;
    }
    if (DIM == 3) {
        // one thread per coarse cell (fine x extent is even on every level above the coarsest)
        LAUNCH(K_PROLONG, W * (2 * N + Nc), (k_prolong_add3<T>), Nc, st, lv.g, S.lev[l + 1].g,
               (const T *)S.lev[l + 1].x, x, done);
        if (lv.g.N >= S.march_cells) {
            int ncolx, ncol, ntiles;
            const int grid = march_sweep_grid(lv.g, ncolx, ncol, ntiles);
            for (int color = 1; color >= 0; --color)
                TLAUNCH(K_SMOOTH, W * (3.5 + DIM) * N + WB * N, (k_gs_color_march<T, TB>), dim3(grid), dim3(kBlock),
                        st, lv, b, x, color, done, ncolx, ncol, ntiles);
        } else {
            LAUNCH(K_SMOOTH, W * (3.5 + DIM) * N + WB * N, (k_gs_color<T, TB, DIM>), N, st, lv, b, x, 1, done);
            gs_red_last<T, TB, DIM, TR>(lv, b, x, done, st, rz);
        }
    }
}

// One V-cycle of slot S: x0 ~ A^{-1} b0 (b0 may be stored in another
// precision than the hierarchy).
template <typename T, typename TB, int DIM, typename TR = T>
static void vcycle_d(Slot<T> &S, const TB *b0, T *x0, const int *done, hipStream_t st,
                     const L0Cg<TR> *cg = nullptr, const RzFuse<TR> *rz = nullptr) {
    constexpr double W = sizeof(T);
    const int lsb = S.lsb;
    if (const int lt = trunc_level(S, DIM); lt >= 0) {
        // truncated cycle (3D): down to level lt, which is solved by one
        // symmetric red-black Gauss-Seidel sweep from zero (red, black as the
        // zero-guess pre-smoothing, then red again: the backward sweep's black
        // half would repeat the forward one), then back up; at lt = 0 the
        // preconditioner is that sweep alone
        auto sgs = [&](Level<T> &L, const auto *b, T *x, const RzFuse<TR> *rzl) {
            using TL = std::remove_cv_t<std::remove_pointer_t<decltype(b)>>;
            const double WL = sizeof(TL) - W;
            const int N = (int)L.g.N;
            if ((L.g.n[0] & 1) == 0)
                LAUNCH(K_SMOOTH, W * (3 + DIM) * N + WL * N, (k_presmooth_pair<T, TL, DIM>), N / 2, st, L, b, x, done);
            else
                LAUNCH(K_SMOOTH, W * (3 + DIM) * N + WL * N, (k_presmooth<T, TL, DIM>), N, st, L, b, x, done);
            gs_red_last<T, TL, DIM, TR>(L, b, x, done, st, rzl);
        };
        if (lt == 0) {
            sgs(S.lev[0], b0, x0, rz);
            return;
        }
        vcycle_down<T, TB, DIM, TR>(S, 0, b0, x0, done, st, cg);
        for (int l = 1; l < lt; ++l) vcycle_down<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x, done, st);
        sgs(S.lev[lt], (const T *)S.lev[lt].b, S.lev[lt].x, nullptr);
        for (int l = lt - 1; l >= 1; --l) vcycle_up<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x, done, st);
        vcycle_up<T, TB, DIM, TR>(S, 0, b0, x0, done, st, cg, rz);
        return;
    }
    if (lsb > 0) {
        vcycle_down<T, TB, DIM, TR>(S, 0, b0, x0, done, st, cg);
        for (int l = 1; l < lsb; ++l) vcycle_down<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x, done, st);
    }
    {
        // storage of the small levels: one contiguous range from lev[lsb].s
        // to the end of the coarsest inverse
        const size_t range16 = lds_vcycle_bytes(S, lsb);
        if (range16) {
            // the range is read once and x of level lsb written back
            static const bool attr = [] {   // once per instantiation, thread-safe
                (void)hipFuncSetAttribute((const void *)k_vcycle_lds<T, DIM>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, kLdsVcycleBytes);
                return true;
            }();
            (void)attr;
            const LdsCopy cp = lds_copy_plan(S, lsb);
            const double bytes = 16.0 * cp.total + W * S.lev[lsb].g.N;
            TLAUNCHS(K_COARSE_SOLVE, bytes, (k_vcycle_lds<T, DIM>), dim3(1), dim3(kSBThreads), range16, st, S, lsb,
                     cp, done);
        } else {
            double bytes = 8.0 * S.ncoarse * S.ncoarse;
            for (int l = lsb; l < S.nlev; ++l) bytes += W * 12.0 * S.lev[l].g.N;
            if (lsb == 0)
                LAUNCH1(K_COARSE_SOLVE, bytes, (k_vcycle_block<T, TB, DIM>), kSBThreads, st, S, 0, b0, x0, done);
            else
                LAUNCH1(K_COARSE_SOLVE, bytes, (k_vcycle_block<T, T, DIM>), kSBThreads, st, S, lsb,
                        (const T *)S.lev[lsb].b, S.lev[lsb].x, done);
        }
    }
    if (lsb > 0) {
        for (int l = lsb - 1; l >= 1; --l) vcycle_up<T, T, DIM>(S, l, S.lev[l].b, S.lev[l].x, done, st);
        vcycle_up<T, TB, DIM, TR>(S, 0, b0, x0, done, st, cg, rz);
    }
}

template <typename T>
void mg_vcycle(Slot<T> &S, int dim, const T *b0, T *x0, const int *done, hipStream_t st) {
    if (dim == 2)
        vcycle_d<T, T, 2>(S, b0, x0, done, st);
    else
        vcycle_d<T, T, 3>(S, b0, x0, done, st);
}

// Preconditioner z = B r with the hierarchy SP (precision TP); r in T.
// rz: the r.z partials of CG (vector precision TR) may ride on the last pass.
template <typename T, typename TP, int DIM, typename TR = T>
static void precond_d(Slot<TP> &SP, OpKind kind, const T *r, TP *z, TP *w, const int *done, hipStream_t st,
                      const RzFuse<TR> *rz = nullptr) {
    if (kind == OP_CH) {
        // M ~ (I - c L)^2 with c = sqrt(b): two V-cycles of the slot operator
        vcycle_d<TP, T, DIM>(SP, r, w, done, st);
        vcycle_d<TP, TP, DIM>(SP, w, z, done, st);
    } else {
        vcycle_d<TP, T, DIM, TR>(SP, r, z, done, st, nullptr, rz);
    }
}

// The same inside CG with the level-0 roles of cg (2D tile levels); for the
// CH operator the first V-cycle takes the update and the pending
// right-hand side, the second the dot products.
template <typename TP, int DIM, typename TR>
static void precond_cg_d(Slot<TP> &SP, OpKind kind, const TP *r, TP *z, TP *w, const int *done, hipStream_t st,
                         const L0Cg<TR> &cg) {
    if (kind == OP_CH) {
        L0Cg<TR> c1 = cg, c2 = cg;
        c1.dmode = 0;
        c2.down_upd = 0;
        c2.bpend = 0;
        vcycle_d<TP, TP, DIM, TR>(SP, r, w, done, st, &c1);
        vcycle_d<TP, TP, DIM, TR>(SP, w, z, done, st, &c2);
    } else {
        vcycle_d<TP, TP, DIM, TR>(SP, r, z, done, st, &cg);
    }
}

// PCG in precision T (operator SA level 0, vectors, updates) preconditioned
// by V-cycles of the hierarchy SP in precision TP.
template <typename T, typename TP, int DIM>
static hipError_t pcg_d(Slot<T> &SA, Slot<TP> &SP, OpKind kind, ChOp ch, const T *b, T *x, double rtol, int max_iter,
                        int predict, Red &red, const PcgVecs2<T, TP> &v, hipStream_t st, SolveOut *out,
                        int zero_guess, int conv0 = 0) {
    constexpr double W = sizeof(T);
    constexpr double WP = sizeof(TP);
    const Level<T> &L0 = SA.lev[0];
    const Geo g = L0.g;
    const int N = (int)g.N;
    const int nb = grid_red(N);
    const int singular = SP.singular;
    Scal *sc = red.scal;
    const int *done = &sc->done;
    if (zero_guess) {
        LAUNCHR(K_PCG_INIT, W * 3 * N, (k_pcg_init_zero<T>), N, st, N, b, x, v.r, red.part0, red.part1);
    } else if (kind == OP_SLOT) {
        constexpr bool split = !std::is_same<T, TP>::value;
        // conv0: the level-0 set-up of SP's cycle rides on this pass
        const double conv_bytes = conv0 ? (split ? WP * (2 + DIM) : WP) * N : 0.0;
        LAUNCHR(K_PCG_INIT, W * (4 + DIM) * N + (split ? WP * N : 0.0) + conv_bytes, (k_pcg_init_slot<T, DIM, TP>), N,
                st, L0, b, (const T *)x, v.r, red.part0, red.part1, split ? (TP *)v.rp : (TP *)nullptr, SP.lev[0],
                conv0);
    } else {
        LAUNCH(K_PCG_INIT, W * 2 * N, (k_ch_lap_plain<T, DIM>), N, st, g, ch.ih2, (const T *)x, v.t);
        LAUNCHR(K_PCG_INIT, W * 4 * N, (k_pcg_init_ch<T, DIM>), N, st, g, ch.ih2, ch.a, ch.b, b, (const T *)x,
               (const T *)v.t, v.r, red.part0, red.part1);
    }
    LAUNCH1(K_PCG_INIT, 16.0 * nb, (k_pcg_fin_init), kBlock, st, sc, (const double *)red.part0,
            (const double *)red.part1, nb, rtol, max_iter);
    Scal hs;
    // With a lower-precision hierarchy the V-cycle reads the residual
    // already rounded to its precision (the value its sweeps would round it
    // to), so the level-0 passes read 4 instead of 8 bytes per cell of it.
    constexpr bool split = !std::is_same<T, TP>::value;
    const TP *rpre = split ? (const TP *)v.rp : (const TP *)(const void *)v.r;
    if (split && !(kind == OP_SLOT && !zero_guess))   // (the slot init writes rp itself)
        LAUNCH(K_PCG_INIT, (W + WP) * N, (k_round_vec<T, TP>), N, st, N, (const T *)v.r, v.rp);
    // preconditioner, then the r.z partials (in 3D with the slot operator
    // they ride on the preconditioner's last pass where that can take them)
    auto precond_rz = [&]() {
        bool taken = false;
        const RzFuse<T> rzf{(const T *)v.r, (const Scal *)sc, red.rz0, red.rz1, red.rz2, singular, &taken};
        precond_d<TP, TP, DIM, T>(SP, kind, rpre, v.z, v.w, done, st, DIM == 3 && kind == OP_SLOT ? &rzf : nullptr);
        if (!taken)
            LAUNCHR(K_PCG_DOT, (W + WP) * N, (k_pcg_rz<T, TP>), N, st, N, (const T *)v.r, (const TP *)v.z,
                    (const Scal *)sc, red.rz0, red.rz1, red.rz2, singular);
    };
    // 2D with tiled level 0: the update and the r.z partials ride on the
    // level-0 tile passes (one partial per tile), and the residual store
    // moves to the next operator apply
    int ntiles0 = 0;
    if (DIM == 2 && SP.lsb > 0) {
        int ntx, grid;
        tile_grid2(SP.lev[0].g, ntx, ntiles0, grid);
    }
    const bool fuse = DIM == 2 && SP.lsb > 0 && ntiles0 <= kRedBlocks;
    const int nrz = fuse ? ntiles0 : nb;
    L0Cg<T> cg{0, 0, 1, (const T *)v.r, (const T *)v.q, nullptr, x, sc, (const double *)red.part0, nb,
               red.part1, red.rz0, red.rz1, red.rz2};
    if (fuse) {
        precond_cg_d<TP, DIM, T>(SP, kind, rpre, v.z, v.w, done, st, cg);
    } else {
        precond_rz();
    }
    // 3D slot operator: the z-marching apply (8 planes per block, more when
    // the grid would exceed the partial-sum slots)
    struct {
        int nb = 0, ncolx = 0, ncol = 0, zc = 0;
    } march;
    if (DIM == 3 && kind == OP_SLOT) {
        const Geo &g0 = L0.g;
        march.ncolx = (g0.n[0] + kMX - 1) / kMX;
        march.ncol = march.ncolx * ((g0.n[1] + kMY - 1) / kMY);
        if (march.ncol <= kMaxBlocks) {   // else the grid-stride apply
            march.zc = kMarchPlanes;
            while (march.zc < g0.n[2] && (long long)march.ncol * ((g0.n[2] + march.zc - 1) / march.zc) > kMaxBlocks)
                march.zc *= 2;
            march.nb = march.ncol * ((g0.n[2] + march.zc - 1) / march.zc);
        }
    }
    int launched = 0;
    int chunk = predict < 1 ? 1 : predict;
    for (;;) {
        if (chunk > max_iter - launched) chunk = max_iter - launched;
        for (int it = 0; it < chunk; ++it) {
            const int k = launched + it;
            T *pnew = (k & 1) ? v.p1 : v.p0;
            T *pold = (k & 1) ? v.p0 : v.p1;
            // the consumer of the r.z partials starts the iteration (beta);
            // fused: it also stores the previous iteration's residual
            T *rpend = fuse && k > 0 ? v.r : nullptr;
            const double WRP = rpend ? 2.0 * W : 0.0;   // r read and written
            if (kind == OP_SLOT && march.nb && SA.rho && g.N >= SA.march_cells) {
                // rho, p_old read; p_new, q written; z in its precision
                TLAUNCH(K_PCG_APPLY, 8.0 * N + 3.0 * W * N + WP * N, (k_pcg_apply3_march<T, TP, true>),
                        dim3(march.nb), dim3(kBlock), st, L0, (const TP *)v.z, (const T *)pold, pnew, v.q, sc,
                        red.part0, (const double *)red.rz0, (const double *)red.rz1, (const double *)red.rz2, nrz, k,
                        singular, march.ncolx, march.ncol, march.zc, SA.rho, SA.rho_ih2);
            } else if (kind == OP_SLOT && march.nb) {
                TLAUNCH(K_PCG_APPLY, W * (4 + DIM) * N + WP * N, (k_pcg_apply3_march<T, TP, false>), dim3(march.nb),
                        dim3(kBlock), st, L0, (const TP *)v.z, (const T *)pold, pnew, v.q, sc, red.part0,
                        (const double *)red.rz0, (const double *)red.rz1, (const double *)red.rz2, nrz, k, singular,
                        march.ncolx, march.ncol, march.zc, (const double *)nullptr, 0.0);
            } else if (kind == OP_SLOT) {
                LAUNCHR(K_PCG_APPLY, W * (4 + DIM) * N + WP * N + WRP * N, (k_pcg_apply_slot<T, TP, DIM>), N, st,
                        L0, (const TP *)v.z, (const T *)pold, pnew, v.q, sc, red.part0, (const double *)red.rz0,
                        (const double *)red.rz1, (const double *)red.rz2, nrz, k, singular, rpend);
            } else {
                LAUNCHR(K_PCG_APPLY, W * 3 * N + WP * N + WRP * N, (k_pcg_ch_lap<T, TP, DIM>), N, st, g, ch.ih2,
                        (const TP *)v.z, (const T *)pold, pnew, v.t, sc, (const double *)red.rz0, nrz, k, rpend,
                        (const T *)v.q);
                LAUNCHR(K_PCG_APPLY, W * 3 * N, (k_pcg_ch_apply<T, DIM>), N, st, g, ch.ih2, ch.a, ch.b, (const T *)pnew,
                       (const T *)v.t, v.q, (const Scal *)sc, red.part0);
            }
            if (fuse) {
                L0Cg<T> c = cg;
                c.down_upd = 1;
                c.bpend = 1;
                c.dmode = 2;
                c.p = pnew;
                precond_cg_d<TP, DIM, T>(SP, kind, rpre, v.z, v.w, done, st, c);
                continue;
            }
            // (a last-block finalize inside the update would need a
            // device-scope fence per block, which costs more than this launch)
            LAUNCHR(K_PCG_UPDATE, W * 6 * N + (split ? WP * N : 0.0), (k_pcg_update<T, TP>), N, st, N,
                    (const T *)pnew, (const T *)v.q, x, v.r, sc, (const double *)red.part0,
                    kind == OP_SLOT && march.nb ? march.nb : nb, red.part1, split ? v.rp : (TP *)nullptr);
            LAUNCH1(K_PCG_UPDATE, 8.0 * nb, (k_pcg_fin_rr), kBlock, st, sc, (const double *)red.part1, nb);
            precond_rz();
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
                     int predict, Red &red, PcgVecs<T> &v, hipStream_t st, SolveOut *out, int zero_guess,
                     int conv0) {
    const PcgVecs2<T, T> v2{v.r, v.p0, v.p1, v.q, v.t, v.z, v.t, nullptr};
    if (dim == 2)
        return pcg_d<T, T, 2>(S, S, kind, ch, b, x, rtol, max_iter, predict, red, v2, st, out, zero_guess, conv0);
    return pcg_d<T, T, 3>(S, S, kind, ch, b, x, rtol, max_iter, predict, red, v2, st, out, zero_guess, conv0);
}

// ---------------------------------------------------------------------------
// precision form: FP64 CG preconditioned by the FP32 hierarchy.  x, r, p,
// q, the level-0 operator of the CG recurrence, its updates and every dot
// product are FP64; the V-cycle runs on FP32 coefficients, sweeps and
// transfers (FP64 coarsest inverse) and returns z in FP32.  The initial
// residual is the true FP64 residual b - A x of the starting iterate and the
// recurrence residual is that of an FP64 CG, so the solve stops on the FP64
// form's test, ||r||_2 <= rtol max(||b||_2, ||r_0||_2).
// ---------------------------------------------------------------------------
template <int DIM>
// FP32 copy of the level-0 coefficients and their 1 / diag (invd_cell's
// sum, in FP32, of the rounded values: the upper faces' coefficients are
// read from the neighbours' FP64 entries and rounded the same way)
__global__ void __launch_bounds__(kBlock) k_conv_coef(Level<double> A, Level<float> B) {
    GRID_LOOP(A.g.N) {
        int ia[3];
        coords_of<DIM>(A.g, c, ia);
        const float sc = (float)A.s[c];
        B.s[c] = sc;
        float d = sc;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const float w = (float)A.cs[b][c];
            B.cs[b][c] = w;
            if (nb_lo(A.g, c, ia[b], b) >= 0) d += w;
            const int hi = nb_hi(A.g, c, ia[b], b);
            if (hi >= 0) d += (float)A.cs[b][hi];
        }
        B.invd[c] = 1.0f / d;
    }
}

void convert_level0(const Slot<double> &A, Slot<float> &B, int dim, hipStream_t st) {
    const int N = A.lev[0].g.N;
    const double bytes = (8.0 + 4.0) * (1 + dim) * N + 4.0 * N;
    if (dim == 2)
        LAUNCH(K_MG_SETUP, bytes, (k_conv_coef<2>), N, st, A.lev[0], B.lev[0]);
    else
        LAUNCH(K_MG_SETUP, bytes, (k_conv_coef<3>), N, st, A.lev[0], B.lev[0]);
}

template <int DIM>
static hipError_t refine_d(Slot<double> &S64, Slot<float> &S32, OpKind kind, ChOp ch, const double *b, double *x,
                           double rtol, int max_iter, int *predict, Red &red, const PcgVecs2<double, float> &v,
                           hipStream_t st, SolveOut *out, int conv0) {
    SolveOut o;
    hipError_t e =
        pcg_d<double, float, DIM>(S64, S32, kind, ch, b, x, rtol, max_iter, *predict, red, v, st, &o, 0, conv0);
    if (e != hipSuccess) return e;
    if (o.iters > 0) *predict = o.iters;
    if (out) *out = o;
    return hipGetLastError();
}

hipError_t refine_solve(Slot<double> &S64, Slot<float> &S32, int dim, OpKind kind, ChOp ch, const double *b,
                        double *x, double rtol, int max_iter, int *predict, Red &red,
                        const PcgVecs2<double, float> &v, hipStream_t st, SolveOut *out, int conv0) {
    if (dim == 2) return refine_d<2>(S64, S32, kind, ch, b, x, rtol, max_iter, predict, red, v, st, out, conv0);
    return refine_d<3>(S64, S32, kind, ch, b, x, rtol, max_iter, predict, red, v, st, out, conv0);
}

template <typename T>
void remove_mean(const Geo &g, T *x, Red &red, hipStream_t st, T *copy) {
    const int N = (int)g.N;
    const int nb = grid_red(N);
    LAUNCHR(K_MEAN, sizeof(T) * N, (k_sum<T>), N, st, N, (const T *)x, red.part0);
    LAUNCHR(K_MEAN, (copy ? 3.0 : 2.0) * sizeof(T) * N, (k_sub_mean<T>), N, st, N, x, (const double *)red.part0, nb,
            copy);
}

template <typename T>
void slot_apply(Slot<T> &S, int dim, const T *x, T *y, hipStream_t st) {
    if (dim == 2)
        LAUNCH(K_PCG_APPLY, 0, (k_slot_apply<T, 2>), S.lev[0].g.N, st, S.lev[0], x, y);
    else
        LAUNCH(K_PCG_APPLY, 0, (k_slot_apply<T, 3>), S.lev[0].g.N, st, S.lev[0], x, y);
}

template void mg_setup<double>(Slot<double> &, int, hipStream_t, bool);
template void mg_vcycle<double>(Slot<double> &, int, const double *, double *, const int *, hipStream_t);
template hipError_t pcg_solve<double>(Slot<double> &, int, OpKind, ChOp, const double *, double *, double, int, int,
                                      Red &, PcgVecs<double> &, hipStream_t, SolveOut *, int, int);
template void mg_setup<float>(Slot<float> &, int, hipStream_t, bool);
template hipError_t pcg_solve<float>(Slot<float> &, int, OpKind, ChOp, const float *, float *, double, int, int,
                                     Red &, PcgVecs<float> &, hipStream_t, SolveOut *, int, int);
template void remove_mean<double>(const Geo &, double *, Red &, hipStream_t, double *);
template void slot_apply<double>(Slot<double> &, int, const double *, double *, hipStream_t);

}  // namespace chns
