// Host-side entry points of the multigrid-preconditioned CG machinery.
#pragma once
#include "common.h"

namespace chns {

// Multigrid levels at or below this many cells run in the single-workgroup
// kernel.
constexpr int kSBCells = 2048;


enum OpKind { OP_SLOT = 0, OP_CH = 1 };

template <typename T>
struct PcgVecs {
    T *r, *z, *p0, *p1, *q, *t;
};

// PCG vectors in precision T with the preconditioned vector z and the
// preconditioner's scratch w in precision TP.
template <typename T, typename TP>
struct PcgVecs2 {
    T *r, *p0, *p1, *q, *t;
    TP *z, *w;
    TP *rp;   // the residual rounded to the preconditioner's precision (TP != T only)
};

struct SolveOut {
    int iters;
    double rel_res;
    int unconverged;
    int nonfinite;
};

// Constant-coefficient CH operator M = I - a L + b L L and its
// preconditioner operator I + c(-L), c = sqrt(b).
struct ChOp {
    double a, b, ih2;   // M = I - a L + b L L, ih2 = 1/h^2
};

// Coarsen the slot's level-0 coefficients onto every level and invert the
// coarsest operator (deterministic, on the stream).  invd0 = false: the
// level-0 1 / diag is already in place (convert_level0 writes it).
template <typename T>
void mg_setup(Slot<T> &S, int dim, hipStream_t st, bool invd0 = true);

// One symmetric V(1,1) cycle with red-black Gauss-Seidel: x0 ~ A^{-1} b0.
template <typename T>
void mg_vcycle(Slot<T> &S, int dim, const T *b0, T *x0, const int *done, hipStream_t st);

// PCG on A x = b (A = slot operator, or the CH operator preconditioned by
// two V-cycles of the slot).  x is the initial guess on entry.  predict is
// the number of iterations launched before the first host check.
// Returns hipSuccess or the first HIP error.  conv0: the hierarchy's cycle
// ends on the grid and its level-0 1 / diag (and, in refine_solve, the FP32
// copies of s and cs) are written by the CG init pass; the caller skips them
// in the set-up.
template <typename T>
hipError_t pcg_solve(Slot<T> &S, int dim, OpKind kind, ChOp ch, const T *b, T *x, double rtol,
                     int max_iter, int predict, Red &red, PcgVecs<T> &v, hipStream_t st,
                     SolveOut *out, int zero_guess = 0, int conv0 = 0);

// Precision form: FP64 conjugate gradients (residual recurrence, operator
// apply, updates and dot products in FP64) preconditioned by FP32 V-cycles
// (FP32 coefficients, smoother sweeps and transfers; FP64 coarsest
// inverse).  Its initial residual is the true FP64 residual of the starting
// iterate and it stops on the FP64 form's test.  S64 supplies the FP64
// level-0 operator, S32 the FP32 hierarchy (level-0 coefficients converted by
// convert_level0 and coarsened by mg_setup<float> beforehand).
// FP64 refinement rounds of the batched precision form (at most).
constexpr int kMaxRefine = 4;
// FP32 copy of the level-0 coefficients of A into B, with B's level-0
// 1 / diag (then mg_setup(B, dim, st, false)).
void convert_level0(const Slot<double> &A, Slot<float> &B, int dim, hipStream_t st);
hipError_t refine_solve(Slot<double> &S64, Slot<float> &S32, int dim, OpKind kind, ChOp ch, const double *b,
                        double *x, double rtol, int max_iter, int *predict, Red &red,
                        const PcgVecs2<double, float> &v, hipStream_t st, SolveOut *out, int conv0 = 0);

// Subtract the mean of a cell array (deterministic).  Used for the
// singular pressure system (right-hand side, then the solution gauge).
// copy (when given) receives the result as well.
template <typename T>
void remove_mean(const Geo &g, T *x, Red &red, hipStream_t st, T *copy = nullptr);

// Apply the slot operator at level 0: y = A x (tests / residual checks).
template <typename T>
void slot_apply(Slot<T> &S, int dim, const T *x, T *y, hipStream_t st);

}  // namespace chns
