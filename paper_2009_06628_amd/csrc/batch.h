// Tables of the batched ensemble, shared by the persistent (workgroup per
// problem) and the tiled (one launch per sweep over all problems) forms.
#pragma once
#include <array>
#include <vector>

#include "common.h"
#include "solvers.h"
#include "spectral.h"
#include "step.h"

namespace chns {

// ---------------------------------------------------------------------------
// device tables
// ---------------------------------------------------------------------------
template <typename TP>
struct BatchProb {
    Geo g;
    StepConst k;
    ChOp ch;
    double rtol_ch, rtol_mom, rtol_p;
    int max_iter;
    long long off;                         // first cell in the packed state arrays
    double *phi_new, *phihat, *rch, *ustar[3], *rhs;
    double *r, *p0, *p1, *q, *t;           // CG vectors (FP64)
    TP *z, *w;                             // preconditioned vector, V-cycle scratch
    TP *rp;                                // r rounded to TP (tiled form, FP32 hierarchy; else null)
    Level<double> op;                      // FP64 level-0 operator of the momentum / pressure solves
    Slot<TP> chs, mom, pres;               // CH hierarchy; momentum and pressure share arrays
    // tiled mode
    Scal *sc;                              // solver scalars of the problem
    int lsb;                               // first level handled by one workgroup
    int vlds;                              // LDS bytes of that V-cycle out of LDS (0: from global memory)
    LdsCopy vcp;                           // its copy plan (the same for every slot of the problem)
    int t0, t1;                            // the problem's tiles in the level-0 tile list
};

struct BatchState {
    double *phi, *u[3], *p, *mu;
};

// A contiguous range of cells of one level of one problem (tiled form);
// prob < 0 marks padding.
struct BTile {
    int prob, c0, c1, pad;
};

constexpr int kTileBlock = 256;   // threads per tiled-form workgroup

}  // namespace chns

struct chns_batch {
    int count, dim, prec;
    hipStream_t user_stream, stream;
    hipEvent_t ev_in, ev_out;
    void *d_probs;
    int *d_order;
    unsigned int *d_queue;
    chns_batch_stats *d_stats;
    double *backup;
    std::vector<long long> offsets;   // count + 1
    std::vector<int> order;
    long long total_cells;
    int block, grid;                  // launch shape
    // captured graph of the last chns_batch_step call with use_graph
    hipGraph_t graph;
    hipGraphExec_t exec;
    int g_steps, g_block, g_grid, g_mode, g_tile;
    chns::BatchState g_state;
    // tiled mode (one launch per sweep over the cells of all problems)
    int mode;                         // CHNS_BATCH_PERSISTENT or CHNS_BATCH_TILED
    int tile_cells;                   // cells per tile (multiple of kTileBlock)
    int lg;                           // levels swept by tiled kernels (max over problems of lsb)
    int nlev_max;
    std::vector<int> nlev, lsb;       // per problem
    std::vector<long long> ncells[chns::kMaxLev];   // per level, per problem
    std::vector<std::array<long long, 3>> lev_n[chns::kMaxLev];   // per level, per problem: extents
    chns::BTile *d_tiles[chns::kMaxLev];
    int ntiles[chns::kMaxLev];
    size_t tile_cap[chns::kMaxLev];
    // 2D: per level, the kTFX x kTFY tiles {prob, tx, ty} of every problem
    // whose level is above its single-workgroup levels (fused V-cycle passes)
    chns::BTile *d_t2[chns::kMaxLev];
    int nt2[chns::kMaxLev];
    size_t t2_cap[chns::kMaxLev];
    double *tpart0, *tpart1, *tpart2; // per-tile partial sums (level-0 tile capacity)
    chns::Scal *d_scal;
    int *d_active;                    // number of problems whose current solve is not done
    int budget[3];                    // graph mode: PCG iterations launched per solve (CH, momentum, pressure)
    int rbudget[3];                   // graph mode, FP32 hierarchy: iterations of the one refinement round
    int last_iters[3];                // eager mode: most iterations any problem needed, last step
    int last_refine[3];               // eager mode: most iterations in refinement rounds, last step
    int max_iter_max;                 // largest max_iter of the problems (graph budgets never exceed it)
    int vlds_max;                     // largest LDS of the problems' single-workgroup V-cycles
    int vlds_some_global;             // some problem runs those levels from global memory
    // direct CH solve (2D, every axis <= kSpectralMaxN): one group per
    // problem shape, and its members
    std::vector<chns::SpecGroup> spec;
    std::vector<std::vector<int>> spec_members;
    int spec_on;
};


namespace chns {
// Tiled form (batch_tiled.hip): build the tile lists for tile_cells cells
// per tile and upload them; enqueue nsteps steps on stream s.  graph != 0:
// every solve launches a fixed number of iterations (budget) and the host
// never waits, so the sequence can be captured; otherwise solves run until
// every problem has converged, checking once per chunk of iterations.
int tiled_build(chns_batch *b, int tile_cells);
int tiled_steps(chns_batch *b, const BatchState &st, int nsteps, int graph, hipStream_t s,
                chns_batch_stats *d_stats);
}  // namespace chns
