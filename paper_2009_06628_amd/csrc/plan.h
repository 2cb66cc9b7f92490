// Host-side helpers shared by the single-grid and batched entry points:
// grid plan (multigrid levels), workspace bump allocator, slot carving,
// step constants and the thread-local error message.
#pragma once
#include <string>

#include "common.h"
#include "step.h"

namespace chns {

// Record the calling thread's error message; returns code.
int set_error(int code, const std::string &msg);
// Check a property set (CHNS_OK or CHNS_EINVAL with a message).
int check_props(const chns_props *p);
// Step constants from the properties and the cell size.
StepConst step_const_of(const chns_props &p, double h);

struct Plan {
    int dim;
    int nph;       // phases (2 or 3)
    int nlev;
    Geo lev[kMaxLev];
};

// Validate a grid description and build its multigrid levels (halving every
// axis while all stay even, down to at most 64 cells where possible).
int make_plan(const chns_grid_desc *d, Plan &P);

// Bump allocator over the workspace (base == nullptr: sizing pass).
struct Bump {
    char *base;
    size_t off;
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

template <typename T>
inline void carve_slot(Bump &B, const Plan &P, Slot<T> &S, int singular) {
    S.nlev = P.nlev;
    S.lsb = 0;
    S.ltrunc = -1;
    S.march_cells = kMarchSweepCells;
    S.tile_cells = kTileCycleCells;
    S.rho = nullptr;
    S.rho_ih2 = 0.0;
    S.singular = singular;
    S.ncoarse = (int)P.lev[P.nlev - 1].N;
    for (int l = 0; l < P.nlev; ++l) {
        Level<T> &L = S.lev[l];
        L.g = P.lev[l];
        const size_t n = (size_t)L.g.N;
        L.s = B.take<T>(n);
        for (int b = 0; b < 3; ++b) L.cs[b] = b < P.dim ? B.take<T>(n) : nullptr;
        L.invd = B.take<T>(n);
        L.r = B.take<T>(n);
        L.x = l ? B.take<T>(n) : nullptr;
        L.b = l ? B.take<T>(n) : nullptr;
    }
    S.Ainv = B.take<double>((size_t)S.ncoarse * S.ncoarse);
    S.aug = nullptr;
}


}  // namespace chns
