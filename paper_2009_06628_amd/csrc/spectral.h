// Direct solve of the Cahn-Hilliard system of the split step (S2):
// (I - a L + b L^2) x = r with constant a, b >= 0 and the cell-centred
// Laplacian L of the grid (walled axes Neumann, periodic axes wrapped).
#pragma once
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"

namespace chns {

// L is a sum of 1D second differences, one per axis, each diagonalised by
// a real orthonormal basis: DCT-II vectors on a walled axis, the real
// Fourier basis (1, cos, sin, ..., alternating signs) on a periodic one.  So
// the system matrix is Q diag(1 - a lam + b lam^2) Q^T with Q the tensor
// product of the axis bases and lam the sum of the axis eigenvalues, and
// the solve is three steps: transform every axis, divide by the
// eigenvalue, transform back.  Each transform along an axis is a product
// with an n x n matrix (a hand-written FP64 tiled kernel, vector FMAs).
// (struct Spectral and kSpectralMaxN live in common.h, inside the handle.)

// Basis and eigenvalues of the 1D second difference on n cells of spacing h
// (host; walled axis: DCT-II, periodic: real Fourier), column-major.
void spectral_axis(int n, int per, double h, std::vector<double> &Q, std::vector<double> &lam);

// Batched form (2D): the problems of one shape {nx, ny, periodic axes}
// share the bases; per problem a, b, 1/h^2 and the pointers of its arrays.
struct SpecGroup {
    int nx, ny, perx, pery, m;
    double *Q[2], *lam[2];       // bases, eigenvalues for unit spacing
    double *abh;                 // per problem: a, b, 1/h^2
    const double **r;            // per problem: right-hand side
    double **x;                  // per problem: solution
    double **t0, **t1;           // per problem: scratch
};
// x_p = (I - a_p L + b_p L^2)^{-1} r_p for every problem of every group, on st.
hipError_t spectral_batch_solve(const std::vector<SpecGroup> &groups, hipStream_t st);

// Carve the bases (sizing pass when B.base is null).
void spectral_carve(Bump &B, const Geo &g, int dim, Spectral &S);
// Build the bases on the host and upload them.  Returns 0, or a nonzero code
// with a message in err.
int spectral_init(Spectral &S, double h, std::string &err);
void spectral_release(Spectral &S);
// x = (I - a L + b L^2)^{-1} r on stream st; t0, t1: scratch of N doubles.
// Returns hipSuccess or the launch error.
hipError_t spectral_solve(Spectral &S, double a, double b, const double *r, double *x, double *t0, double *t1,
                          hipStream_t st, std::string &err);
// Whether every axis is transformed by FFT (then spectral_solve2 applies).
bool spectral_all_fft(const Spectral &S);
// The same for two right-hand sides, both in every launch (every axis an
// FFT axis); t0[i], t1[i]: scratch of N doubles per field.
hipError_t spectral_solve2(Spectral &S, double a, double b, const double *const r[2], double *const x[2],
                           double *const t0[2], double *const t1[2], hipStream_t st);

}  // namespace chns
