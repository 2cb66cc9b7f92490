// Internal definitions shared by the HIP translation units of libchns.
// Grid geometry, neighbour indexing on the uniform MAC grid, deterministic
// block reductions and the handle layout.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/chns.h"

namespace chns {
class WorkerPool;

constexpr int kMaxLev = 16;
constexpr int kMaxCoarse = 512;     // cells of the coarsest (dense) level
constexpr int kBlock = 256;         // threads per block of the linear kernels
constexpr int kMaxBlocks = 4096;    // grid-stride cap (fixes reduction order)
constexpr int kWave = 64;
constexpr int kLdsInverse = 64;     // coarsest sizes inverted in LDS
constexpr int kSBThreads = 1024;    // single-workgroup coarse-level kernels
constexpr int kLdsVcycleBytes = 160 * 1024;   // LDS of one workgroup on gfx950

// The parts of a V-cycle's storage range that it reads before writing them
// (s, cs, invd of every level, b of the first, the coarsest inverse), as at
// most kLdsCopySegs segments of 16-byte words, each copied to the same
// offset in LDS: segment i covers words [cend[i-1] + shift[i],
// cend[i] + shift[i]) of the range (cend[-1] = 0); unused segments have
// cend = total.
constexpr int kLdsCopySegs = 4;
struct LdsCopy {
    int total;                    // words to copy (>= 1)
    int cend[kLdsCopySegs];       // running end of the copied words
    int shift[kLdsCopySegs];      // range word = copied word + shift
};

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geo {
    int n[3];      // cells per axis (n[2] = 1 in 2D)
    int per[3];    // 1: periodic, 0: walled (Neumann-type at both ends)
    long long N;   // total cells
};

// Kernels index cells with 32-bit integers (grids are limited to < 2^31
// cells); coordinates come from unsigned 32-bit divisions.
__host__ __device__ inline int stride_of(const Geo &g, int a) {
    return a == 0 ? 1 : (a == 1 ? g.n[0] : g.n[0] * g.n[1]);
}

__device__ inline void cell_coords(const Geo &g, int c, int &i, int &j, int &k) {
    const unsigned uc = (unsigned)c, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];
    const unsigned t = uc / n0;
    i = (int)(uc - t * n0);
    const unsigned kk = t / n1;
    j = (int)(t - kk * n1);
    k = (int)kk;
}

// 2D: one division (the row index is j)
__device__ inline void cell_coords2(const Geo &g, int c, int &i, int &j, int &k) {
    const unsigned uc = (unsigned)c, n0 = (unsigned)g.n[0];
    const unsigned t = uc / n0;
    i = (int)(uc - t * n0);
    j = (int)t;
    k = 0;
}

// Index of c - e_a (wrapping on periodic axes); -1 outside a walled axis.
__device__ inline int nb_lo(const Geo &g, int c, int ia, int a) {
    const int s = stride_of(g, a);
    if (ia > 0) return c - s;
    return g.per[a] ? c + (g.n[a] - 1) * s : -1;
}
// Index of c + e_a; -1 outside a walled axis.
__device__ inline int nb_hi(const Geo &g, int c, int ia, int a) {
    const int s = stride_of(g, a);
    if (ia < g.n[a] - 1) return c + s;
    return g.per[a] ? c - (g.n[a] - 1) * s : -1;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;    // blocks of kernels that write partials

// Grids are rounded up to a multiple of the 8 XCDs so that xcd_block()
// below is a bijection.
inline int grid_red(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kRedBlocks) b = kRedBlocks;
    if (b > 8) b = (b + 7) & ~7LL;
    return (int)b;
}

inline int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    if (b > 8) b = (b + 7) & ~7LL;
    return (int)b;
}

// Logical block index for grid-stride sweeps.  Workgroups are dispatched
// round-robin over the 8 XCDs, each with its own L2; renumbering them so
// that XCD k sweeps one contiguous 1/8 of the cells keeps a cell's y / z
// neighbour rows in the same L2 as the cell.
__device__ inline int xcd_block() {
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// deterministic reductions: fixed element -> block mapping (grid-stride with
// a fixed grid), wave shuffles then LDS inside the block, and a fixed-order
// sum over the block partials done by the last block to finish.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, kWave));
    return v;
}

// Sum over the block; result valid in thread 0.  lds: >= blockDim/64 doubles.
__device__ inline double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) r += lds[k];
    return r;
}
__device__ inline double block_max(double v, double *lds) {
    v = wave_max(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) r = fmax(r, lds[k]);
    return r;
}

// Returns true in every thread of the block that finished last.  Thread 0
// must have written this block's partials before the call.
__device__ inline bool last_block(unsigned int *counter) {
    __shared__ int am_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int prev = atomicAdd(counter, 1u);
        am_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (am_last) __threadfence();
    return am_last != 0;
}

// Sum over the block; result returned to every thread.
__device__ inline double block_sum_all(double v, double *lds) {
    double r = block_sum(v, lds);
    __syncthreads();
    if (threadIdx.x == 0) lds[0] = r;
    __syncthreads();
    r = lds[0];
    __syncthreads();
    return r;
}

// Sum of nparts partials in a fixed order (block-wide); result in thread 0.
__device__ inline double sum_partials(const double *part, int nparts, double *lds) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) v += ((volatile const double *)part)[k];
    return block_sum(v, lds);
}

// ---------------------------------------------------------------------------
// PCG scalar block (device memory)
// ---------------------------------------------------------------------------
struct Scal {
    double rz, pq, rr, bb, alpha, beta, rtol2, sum0, sum1, zmean;
    double rzs[2];   // single-grid PCG: r.z of iteration k in rzs[k & 1]
    int done, iter, max_iter, nonfinite;
    int unconverged, pad0, pad1, pad2;
};

// ---------------------------------------------------------------------------
// multigrid operator slot:  A x = s x - sum_b D_b(cs_b G_b x) h^2,
// i.e. (A x)_c = s_c x_c + sum_b [cs_b(c) (x_c - x_{c-e_b}) + cs_b(c+e_b) (x_c - x_{c+e_b})]
// with cs_b pre-divided by the squared level spacing; walled axes carry no
// boundary term (Neumann type), Dirichlet contributions are folded into s.
// ---------------------------------------------------------------------------
template <typename T>
struct Level {
    Geo g;
    T *s;
    T *cs[3];
    T *invd;        // 1 / A_cc
    T *x, *b, *r;   // level >= 1 own x, b; every level owns r (also the
                    // scratch of the fused prolongation + smoothing pass)
};

template <typename T>
struct Slot {
    int nlev;
    int lsb;        // first level handled by the single-workgroup kernel
    int ltrunc;     // 3D: the V-cycle ends at this grid level with a symmetric
                    // Gauss-Seidel solve (-1: full cycle down to the coarsest)
    long long march_cells;   // 3D levels with at least this many cells sweep marching along z
    long long tile_cells;    // 3D levels with at most this many cells (above the single-workgroup
                             // part, below march_cells) run one tile pass per side of the cycle
    const double *rho;       // pressure slots: cell densities whose face averages give the level-0
    double rho_ih2;          // coefficients 1/(rho_f h^2) (rho_ih2 = the 1/h^2 they were formed with);
                             // the 3D CG apply forms them on the fly on grids of at least march_cells
                             // cells (null: it reads the stored cs)
    int singular;
    int ncoarse;
    Level<T> lev[kMaxLev];
    double *Ainv;   // coarsest-level inverse, ncoarse x ncoarse (FP64)
    double *aug;    // scratch for the inverse when ncoarse > kLdsInverse
};

// Default of Slot::march_cells: levels whose arrays outgrow the Infinity
// Cache (256^3 cells and up).
constexpr long long kMarchSweepCells = 1LL << 24;
// Default of Slot::tile_cells: the levels whose sweeps cost less than their
// launches (64^3 cells and below).
constexpr long long kTileCycleCells = 1LL << 18;

// Reduction scratch shared by all solves of a handle.
struct Red {
    double *part0, *part1, *part2;   // kMaxBlocks partials each
    double *rz0, *rz1, *rz2;         // kRedBlocks partials each: r.z, sum z, sum r
    unsigned int *counter;     // last-block counters (several)
    Scal *scal;                // device scalars
};

// ---------------------------------------------------------------------------
// optional per-kernel timing (hipEvent pairs around every launch, grouped by
// kernel class, with the algorithmic bytes of each launch)
// ---------------------------------------------------------------------------
enum KClass {
    K_CH_RHS = 0, K_MU, K_PHI_UPDATE, K_MOM_SETUP, K_P_SETUP, K_PROJECT,
    K_SMOOTH, K_RESIDUAL, K_RESTRICT, K_PROLONG, K_COARSE_SOLVE, K_MG_SETUP,
    K_PCG_APPLY, K_PCG_UPDATE, K_PCG_DOT, K_PCG_INIT, K_MEAN, K_DIAG, K_ADJOINT, K_MG_DOWN, K_MG_UP,
    K_CH_SPECTRAL, K_NCLASS
};

struct Prof {
    int enabled;
    int cap, n;                  // event pairs in the pool / in use
    hipEvent_t *ev;              // 2 * cap events
    int *cls;
    double *bytes;
    int launches[K_NCLASS];
    double ms[K_NCLASS];
    double total_bytes[K_NCLASS];
};

extern thread_local Prof *g_prof;
void prof_slot(int cls, double bytes, hipEvent_t *e0, hipEvent_t *e1);
int prof_flush();                // synchronise and accumulate; 0 on success
const char *kclass_name(int cls);

}  // namespace chns

// Launch with optional timing: cls = KClass, bytes = algorithmic bytes.
// In timing mode the start / stop events are recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so their difference is the kernel's execution time
// without the gaps between launches.
#define TLAUNCHS(cls, bytes, kern, grid, block, shm, st, ...)                             \
    do {                                                                                  \
        if (chns::g_prof) {                                                               \
            hipEvent_t e0_, e1_;                                                          \
            chns::prof_slot((cls), (double)(bytes), &e0_, &e1_);                          \
            hipExtLaunchKernelGGL(kern, grid, block, shm, st, e0_, e1_, 0, __VA_ARGS__);  \
        } else {                                                                          \
            hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);                  \
        }                                                                                 \
    } while (0)
#define TLAUNCH(cls, bytes, kern, grid, block, st, ...) TLAUNCHS(cls, bytes, kern, grid, block, 0, st, __VA_ARGS__)

// ---------------------------------------------------------------------------
// device buffers of the discrete adjoint (carved from the adjoint workspace)
// ---------------------------------------------------------------------------
namespace chns {
constexpr int kAdjRegions = 6;   // partial sums: 0..2 dL/dk, 3..5 dL/ds_t (one per axis)

struct AdjBufs {
    double *p_t, *mu_t;                                   // forward recomputation
    double *pbar, *zeta, *etab, *pbt, *mub, *chr, *omega, *lphi, *sbar;   // cells
    double *usb[3], *rfnb[3], *rfob[3], *aphib[3], *gmub[3], *mb[3], *nu[3], *csb[3];   // faces
    double *Fb[3];     // aliases usb (dead after the momentum adjoint solves)
    double *gpart;     // kAdjRegions x kRedBlocks partials
    double *gout;      // 4 doubles: this step's parameter derivatives
};
}  // namespace chns

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
namespace chns {
// Buffers of one momentum component solved on a stream of its own (the
// components of S7 are independent): its own hierarchy, PCG vectors,
// reduction scratch and right-hand side.
struct MomCtx {
    Slot<double> mom;
    Slot<float> mom32;
    double *rhs;
    double *vr, *vz, *vp0, *vp1, *vq, *vt;
    float *f_z, *f_t, *f_r;
    Red red;
    hipStream_t stream;
    hipEvent_t done_ev;   // recorded on stream after the solve
};

// Three-phase constants: densities, viscosities, spreading coefficients
// Sigma_i = sigma_ij + sigma_ik - sigma_jk and the weights
// w_i = Sigma_T / (3 Sigma_i) of the constrained chemical potentials.
struct TernConst {
    double rho[3], eta[3], Sg[3], w[3];
};

// Bases of the direct Cahn-Hilliard solve (spectral.h, spectral.hip).
constexpr int kSpectralMaxN = 2048;   // larger axes keep the MG-PCG solve
// Periodic axes of 2^kFftMinLog .. 2^kFftMaxLog cells are transformed by a
// radix-2 FFT instead of the product with the dense basis.
constexpr int kFftMinLog = 4, kFftMaxLog = 9;

struct Spectral {
    int carved;        // bases carved from the workspace (every axis <= kSpectralMaxN)
    int on;            // set up and in use (else the CH system is solved by MG-PCG)
    int dense;         // 1: dense transforms on every axis (no FFT)
    int dim, n[3], per[3];
    int fft[3];        // per axis: log2 n when the FFT can transform it, else 0
    double *Q[3];      // per axis: n x n basis, column-major, column k = mode k
    double *lam[3];    // per axis: eigenvalue of each mode (1/h^2 included)
    double *tw[3];     // FFT axes: cos, sin of 2 pi k / n, k < n (interleaved)
};
}  // namespace chns

struct chns_grid {
    chns_grid_desc desc;
    chns_props props;
    int props_set;
    hipStream_t stream;
    chns::Geo geo;
    int dim;
    double h;
    // state-independent workspace buffers (double, N cells each)
    double *phi_new, *phihat, *rch, *ustar[3], *rhs;
    int nph;                                 // phases: 2, or 3 (three-phase model)
    chns::TernConst tern;                    // three-phase constants (nph == 3)
    double *prho;                            // cell density of the step's pressure operator (its set-up writes it)
    double *phi_new2, *phihat2, *rch2;       // the second stored phase (nph == 3)
    double *mix3[5];                         // per-step mixture fields (nph == 3)
    double *mflux3[3];                       // per-step face mass fluxes (nph == 3)
    double *vr, *vz, *vp0, *vp1, *vq, *vt;   // PCG vectors
    chns::Slot<double> ch, mom, pres;
    // precision form (FP32 inner solves under FP64 refinement)
    int prec;
    chns::Slot<float> ch32, mom32, pres32;
    float *f_z, *f_t;   // FP32 preconditioned vector and V-cycle scratch
    float *f_r;         // FP32 copy of the CG residual (the V-cycle's right-hand side)
    int last_inner[12];
    chns::Red red;
    double *diag;                            // diagnostics scratch
    int last_iters[12];                      // iteration-count predictions
    chns::MomCtx mc[2];                      // momentum components 1, 2 (component 0 uses the buffers above)
    chns::Spectral spec;                     // direct CH solve (single grids)
    hipEvent_t ev_fork;                      // main stream -> component streams
    hipEvent_t ev_mset;                      // main stream after the momentum set-up -> component streams
    chns::WorkerPool *pool;                  // host threads of the concurrent solves (created on first use)
    hipStream_t pstream;                     // pressure set-up during the momentum solves
    hipEvent_t ev_pset;                      // recorded on pstream after that set-up
    int mc_ready;                            // streams and events of mc and the pressure set-up created
    int serial_components;                   // CHNS_OPT_SERIAL_COMPONENTS
    int scheme, picard;                      // CHNS_OPT_TIME_SCHEME, CHNS_OPT_PICARD_ITERATIONS
    int pguess;                              // CHNS_OPT_TIME_GUESS
    int in_record;                           // inside chns_step_record (no extrapolated guesses)
    double *pext[3];                         // S8 guess history: the last three steps' pressures, newest first
    double *uext[3][3];                      // S7 guess history per component: the last three u*, newest first
    double *cn_phim, *cn_phimid, *cn_dp, *cn_vt[3];   // Crank-Nicolson iterates (two-phase grids)
    const double *wall_u[3][2][3];           // moving-wall data [axis][side][component] (caller-owned)
    int walls_move;                          // any of them set
    int adj_ready;                           // adjoint workspace attached
    chns::AdjBufs adj;
    chns_step_stats last;
    chns::Prof prof;
    void *ws;
    size_t ws_bytes;
};
