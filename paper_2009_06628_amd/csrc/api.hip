// C ABI of libchns: argument checking, workspace layout, and the per-step
// sequence S1..S9 on the handle's stream.  No device memory is allocated:
// every buffer is carved out of the caller's workspace.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>

#include "spectral.h"
#include "common.h"
#include "solvers.h"
#include "step.h"
#include "adjoint.h"
#include "plan.h"
#include "pool.h"

using namespace chns;

static thread_local std::string g_err;

// partial-sum rows of the diagnostics kernels (8 two-phase, 9 three-phase)
constexpr int kDiagSlots = 10;

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------
namespace chns {
thread_local Prof *g_prof = nullptr;

static const char *kNames[K_NCLASS] = {"ch_rhs",   "mu",          "phi_update",   "mom_setup", "p_setup",
                                       "project",  "smooth",      "residual",     "restrict",  "prolong",
                                       "coarse_solve", "mg_setup", "pcg_apply",   "pcg_update", "pcg_dot",
                                       "pcg_init", "mean",        "diag",        "adjoint",   "mg_down",
                                       "mg_up",      "ch_spectral"};

const char *kclass_name(int c) { return (c >= 0 && c < K_NCLASS) ? kNames[c] : "?"; }

void prof_slot(int cls, double bytes, hipEvent_t *e0, hipEvent_t *e1) {
    Prof *P = g_prof;
    if (P->n == P->cap) prof_flush();
    *e0 = P->ev[2 * P->n];
    *e1 = P->ev[2 * P->n + 1];
    P->cls[P->n] = cls;
    P->bytes[P->n] = bytes;
    P->n++;
}

int prof_flush() {
    Prof *P = g_prof;
    if (!P || P->n == 0) return 0;
    if (hipEventSynchronize(P->ev[2 * P->n - 1]) != hipSuccess) return -1;
    for (int i = 0; i < P->n; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, P->ev[2 * i], P->ev[2 * i + 1]) != hipSuccess) return -1;
        P->ms[P->cls[i]] += ms;
        P->launches[P->cls[i]] += 1;
        P->total_bytes[P->cls[i]] += P->bytes[i];
    }
    P->n = 0;
    return 0;
}
}  // namespace chns

namespace {
// Installs the handle's profiler for the duration of an API call.
struct ProfScope {
    explicit ProfScope(chns_grid *g) { g_prof = (g && g->prof.enabled) ? &g->prof : nullptr; }
    ~ProfScope() {
        prof_flush();
        g_prof = nullptr;
    }
};
}  // namespace

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace chns {
int set_error(int code, const std::string &msg) { return fail(code, msg); }

StepConst step_const_of(const chns_props &p, double h) {
    StepConst k;
    k.h = h;
    k.ih = 1.0 / h;
    k.ih2 = k.ih * k.ih;
    k.dt = p.dt;
    k.S = p.S;
    k.Cn = p.Cn;
    k.Pe = p.Pe;
    k.kM = 1.0 / (p.Pe * p.Cn);
    k.alpha = (1.0 - p.rho_minus) / 2.0;
    k.beta = (1.0 + p.rho_minus) / 2.0;
    k.gamma = (1.0 - p.eta_minus) / 2.0;
    k.xi = (1.0 + p.eta_minus) / 2.0;
    k.inv_Re = 1.0 / p.Re;
    k.inv_We = 1.0 / p.We;
    k.We = p.We;
    k.inv_Fr = p.inv_Fr;
    return k;
}

int check_props(const chns_props *p) {
    const double pos[] = {p->rho_minus, p->eta_minus, p->Re, p->We, p->Cn, p->Pe, p->dt};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v))
            return fail(CHNS_EINVAL, "rho_minus, eta_minus, Re, We, Cn, Pe, dt must be positive and finite");
    if (!(p->S >= 0.0) || !std::isfinite(p->inv_Fr)) return fail(CHNS_EINVAL, "S must be >= 0, inv_Fr finite");
    if (!(p->rtol_ch > 0.0) || !(p->rtol_mom > 0.0) || !(p->rtol_p > 0.0))
        return fail(CHNS_EINVAL, "tolerances must be positive");
    if (p->max_iter < 1) return fail(CHNS_EINVAL, "max_iter must be >= 1");
    return CHNS_OK;
}

int make_plan(const chns_grid_desc *d, Plan &P) {
    if (!d) return fail(CHNS_EINVAL, "grid description is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(CHNS_EINVAL, "dim must be 2 or 3");
    if (d->nphases != 2 && d->nphases != 3) return fail(CHNS_EINVAL, "nphases must be 2 or 3");
    if (d->precision != CHNS_FP64 && d->precision != CHNS_FP32_REFINE) return fail(CHNS_EINVAL, "bad precision");
    if (!(d->h > 0.0) || !std::isfinite(d->h)) return fail(CHNS_EINVAL, "h must be positive and finite");
    Geo g;
    g.N = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < d->dim) {
            if (d->n[a] < 2) return fail(CHNS_EINVAL, "every n[a] must be >= 2");
            if (d->bc[a] != CHNS_BC_PERIODIC && d->bc[a] != CHNS_BC_WALL) return fail(CHNS_EINVAL, "bad bc");
            g.n[a] = d->n[a];
            g.per[a] = d->bc[a] == CHNS_BC_PERIODIC;
        } else {
            g.n[a] = 1;
            g.per[a] = 1;
        }
        g.N *= g.n[a];
    }
    if (g.N >= (1LL << 31) - 1) return fail(CHNS_EINVAL, "grid too large (kernels index cells with 32-bit integers)");
    P.dim = d->dim;
    P.nph = d->nphases;
    P.nlev = 1;
    P.lev[0] = g;
    for (;;) {
        const Geo &f = P.lev[P.nlev - 1];
        if (f.N <= 64 || P.nlev == kMaxLev) break;
        bool ok = true;
        for (int a = 0; a < d->dim; ++a)
            if ((f.n[a] & 1) || f.n[a] / 2 < 2) ok = false;
        if (!ok) break;
        Geo c = f;
        c.N = 1;
        for (int a = 0; a < 3; ++a) {
            if (a < d->dim) c.n[a] = f.n[a] / 2;
            c.N *= c.n[a];
        }
        P.lev[P.nlev++] = c;
    }
    if (P.lev[P.nlev - 1].N > kMaxCoarse) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "unsupported grid: coarsening by 2 stops at %lld cells (> %d); choose sizes with more factors of 2",
                 (long long)P.lev[P.nlev - 1].N, kMaxCoarse);
        return fail(CHNS_EINVAL, buf);
    }
    return CHNS_OK;
}

}  // namespace chns


#define HIPCHK(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(CHNS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

void layout(Bump &B, const Plan &P, chns_grid *g, int prec) {
    const size_t N = (size_t)P.lev[0].N;
    g->phi_new = B.take<double>(N);
    g->phihat = B.take<double>(N);
    g->rch = B.take<double>(N);
    for (int a = 0; a < 3; ++a) g->ustar[a] = a < P.dim ? B.take<double>(N) : nullptr;
    g->rhs = B.take<double>(N);
    g->prho = B.take<double>(N);
    g->nph = P.nph;
    if (P.nph == 3) {
        g->phi_new2 = B.take<double>(N);
        g->phihat2 = B.take<double>(N);
        g->rch2 = B.take<double>(N);
        for (int q = 0; q < 5; ++q) g->mix3[q] = B.take<double>(N);
        for (int b = 0; b < 3; ++b) g->mflux3[b] = b < P.dim ? B.take<double>(N) : nullptr;
    } else {
        g->phi_new2 = g->phihat2 = g->rch2 = nullptr;
        for (int q = 0; q < 5; ++q) g->mix3[q] = nullptr;
        for (int b = 0; b < 3; ++b) g->mflux3[b] = nullptr;
    }
    if (P.nph == 2) {   // Crank-Nicolson variant: midpoint iterates and pressure increment
        g->cn_phim = B.take<double>(N);
        g->cn_phimid = B.take<double>(N);
        g->cn_dp = B.take<double>(N);
        for (int a = 0; a < 3; ++a) g->cn_vt[a] = a < P.dim ? B.take<double>(N) : nullptr;
    } else {
        g->cn_phim = g->cn_phimid = g->cn_dp = nullptr;
        for (int a = 0; a < 3; ++a) g->cn_vt[a] = nullptr;
    }
    for (int h = 0; h < 3; ++h) g->pext[h] = B.take<double>(N);
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 3; ++h) g->uext[a][h] = a < P.dim ? B.take<double>(N) : nullptr;
    g->vr = B.take<double>(N);
    g->vz = B.take<double>(N);
    g->vp0 = B.take<double>(N);
    g->vp1 = B.take<double>(N);
    g->vq = B.take<double>(N);
    g->vt = B.take<double>(N);
    carve_slot(B, P, g->ch, 0);
    carve_slot(B, P, g->mom, 0);
    carve_slot(B, P, g->pres, 1);
    const int nc = g->ch.ncoarse;
    // set-up scratch of a coarsest level too large for LDS; the pressure
    // hierarchy has its own, as it is set up while momentum component 0 is
    double *aug = nc > kLdsInverse ? B.take<double>((size_t)nc * nc) : nullptr;
    double *paug = nc > kLdsInverse ? B.take<double>((size_t)nc * nc) : nullptr;
    g->ch.aug = g->mom.aug = aug;
    g->pres.aug = paug;
    g->prec = prec;
    if (prec == CHNS_FP32_REFINE) {
        carve_slot(B, P, g->ch32, 0);
        carve_slot(B, P, g->mom32, 0);
        carve_slot(B, P, g->pres32, 1);
        g->ch32.aug = g->mom32.aug = aug;
        g->pres32.aug = paug;
        g->f_z = B.take<float>(N);
        g->f_t = B.take<float>(N);
        g->f_r = B.take<float>(N);
    } else {
        g->f_z = g->f_t = g->f_r = nullptr;
    }
    g->red.part0 = B.take<double>(kMaxBlocks);
    g->red.part1 = B.take<double>(kMaxBlocks);
    g->red.part2 = B.take<double>(kMaxBlocks);
    g->red.rz0 = B.take<double>(kRedBlocks);
    g->red.rz1 = B.take<double>(kRedBlocks);
    g->red.rz2 = B.take<double>(kRedBlocks);
    g->diag = B.take<double>(kDiagSlots * (size_t)kMaxBlocks + 16);
    g->red.counter = B.take<unsigned int>(64);
    g->red.scal = B.take<Scal>(1);
    // momentum components 1 .. dim-1 (own hierarchy, vectors, scratch)
    for (int a = 1; a < P.dim; ++a) {
        MomCtx &M = g->mc[a - 1];
        M.rhs = B.take<double>(N);
        M.vr = B.take<double>(N);
        M.vz = B.take<double>(N);
        M.vp0 = B.take<double>(N);
        M.vp1 = B.take<double>(N);
        M.vq = B.take<double>(N);
        M.vt = B.take<double>(N);
        carve_slot(B, P, M.mom, 0);
        double *maug = nc > kLdsInverse ? B.take<double>((size_t)nc * nc) : nullptr;
        M.mom.aug = maug;
        if (prec == CHNS_FP32_REFINE) {
            carve_slot(B, P, M.mom32, 0);
            M.mom32.aug = maug;
            M.f_z = B.take<float>(N);
            M.f_t = B.take<float>(N);
            M.f_r = B.take<float>(N);
        } else {
            M.f_z = M.f_t = M.f_r = nullptr;
        }
        M.red.part0 = B.take<double>(kMaxBlocks);
        M.red.part1 = B.take<double>(kMaxBlocks);
        M.red.part2 = B.take<double>(kMaxBlocks);
        M.red.rz0 = B.take<double>(kRedBlocks);
        M.red.rz1 = B.take<double>(kRedBlocks);
        M.red.rz2 = B.take<double>(kRedBlocks);
        M.red.counter = B.take<unsigned int>(64);
        M.red.scal = B.take<Scal>(1);
    }
    spectral_carve(B, P.lev[0], P.dim, g->spec);
}

StepConst step_const(const chns_grid *g) { return step_const_of(g->props, g->h); }

PcgVecs<double> vecs(chns_grid *g) { return PcgVecs<double>{g->vr, g->vz, g->vp0, g->vp1, g->vq, g->vt}; }

int next_predict(int last) { return last < 1 ? 1 : last; }

// What one linear solve works on: hierarchies, vectors, reduction scratch
// and the stream its launches go to.
struct SolveCtx {
    Slot<double> *S64;
    Slot<float> *S32;
    PcgVecs<double> v;
    float *f_z, *f_t, *f_r;
    Red red;
    hipStream_t s;
};

// Rebuild the hierarchy of a solve from the level-0 coefficients just
// written by the set-up kernels (momentum, pressure), on c.s.  skip0: the
// level-0 arrays of the preconditioner (1 / diag, the FP32 copies) are
// written by the CG init pass instead.
static void hierarchy_setup(chns_grid *g, const SolveCtx &c, bool skip0 = false) {
    if (g->prec == CHNS_FP64) {
        mg_setup(*c.S64, g->dim, c.s, !skip0);
    } else {
        if (!skip0) convert_level0(*c.S64, *c.S32, g->dim, c.s);
        mg_setup(*c.S32, g->dim, c.s, false);
    }
}

// One linear solve in the handle's precision form.  setup: rebuild the
// hierarchy from the level-0 coefficients just written by the set-up
// kernels (momentum, pressure); the CH hierarchy is constant (set up by
// chns_set_properties).  pidx indexes the iteration predictions.
hipError_t run_solve_ctx(chns_grid *g, const SolveCtx &c, int setup, OpKind kind, ChOp ch, const double *b,
                         double *x, double rtol, int pidx, SolveOut *o) {
    if (kind == OP_CH && g->spec.on) {
        // direct solve (the same in both precision forms); v.q, v.t are
        // free while the CH system is solved
        std::string err;
        hipError_t e = spectral_solve(g->spec, ch.a, ch.b, b, x, c.v.q, c.v.t, c.s, err);
        if (e != hipSuccess && !err.empty()) set_error(CHNS_EDEVICE, err);
        o->iters = 1;
        o->rel_res = 0.0;
        o->unconverged = 0;
        o->nonfinite = 0;
        return e;
    }
    Slot<double> &S64 = *c.S64;
    PcgVecs<double> v = c.v;
    Red red = c.red;
    // a cycle that ends on the grid itself (the momentum operator when its
    // shift dominates) needs only the level-0 arrays, which the CG init pass
    // writes from the coefficients it reads anyway
    const int conv0 = setup && kind == OP_SLOT && S64.ltrunc == 0 ? 1 : 0;
    if (setup) hierarchy_setup(g, c, conv0 != 0);
    if (g->prec == CHNS_FP64) {
        hipError_t e = pcg_solve(S64, g->dim, kind, ch, b, x, rtol, g->props.max_iter, next_predict(g->last_iters[pidx]),
                                 red, v, c.s, o, 0, conv0);
        g->last_iters[pidx] = o->iters;
        return e;
    }
    Slot<float> &S32 = *c.S32;
    const PcgVecs2<double, float> v2{v.r, v.p0, v.p1, v.q, v.t, c.f_z, c.f_t, c.f_r};
    return refine_solve(S64, S32, g->dim, kind, ch, b, x, rtol, g->props.max_iter, &g->last_inner[pidx], red, v2,
                        c.s, o, conv0);
}

// The handle's own buffers; which: 0 CH, 1 momentum, 2 pressure.
SolveCtx main_ctx(chns_grid *g, int which) {
    SolveCtx c;
    c.S64 = which == 0 ? &g->ch : (which == 1 ? &g->mom : &g->pres);
    c.S32 = which == 0 ? &g->ch32 : (which == 1 ? &g->mom32 : &g->pres32);
    c.v = vecs(g);
    c.f_z = g->f_z;
    c.f_t = g->f_t;
    c.f_r = g->f_r;
    c.red = g->red;
    c.s = g->stream;
    return c;
}

// Buffers of momentum component a (0: the handle's own).
// The handle's host worker threads (created on first use; null if the
// threads could not be started).
WorkerPool *grid_pool(chns_grid *g) {
    if (!g->pool) {
        try {
            g->pool = new WorkerPool();
        } catch (...) {
            g->pool = nullptr;
        }
    }
    return g->pool;
}

// Waits for a worker's task when leaving a scope (early returns included).
struct TaskWait {
    WorkerPool *pool = nullptr;
    int w = 0;
    bool active = false;
    void start(WorkerPool *p, int worker, std::function<void()> f) {
        pool = p;
        w = worker;
        active = true;
        p->run(worker, std::move(f));
    }
    void wait() {
        if (active) pool->wait(w);
        active = false;
    }
    ~TaskWait() { wait(); }
};

SolveCtx mom_ctx(chns_grid *g, int a) {
    if (a == 0) return main_ctx(g, 1);
    MomCtx &M = g->mc[a - 1];
    SolveCtx c;
    c.S64 = &M.mom;
    c.S32 = &M.mom32;
    c.v = PcgVecs<double>{M.vr, M.vz, M.vp0, M.vp1, M.vq, M.vt};
    c.f_z = M.f_z;
    c.f_t = M.f_t;
    c.f_r = M.f_r;
    c.red = M.red;
    c.s = M.stream;
    return c;
}

hipError_t run_solve(chns_grid *g, int which, OpKind kind, ChOp ch, const double *b, double *x, double rtol,
                     int pidx, SolveOut *o) {
    return run_solve_ctx(g, main_ctx(g, which), which != 0, kind, ch, b, x, rtol, pidx, o);
}

int check_solve(const SolveOut &o, const char *what) {
    if (o.nonfinite) return fail(CHNS_ENONFINITE, std::string("non-finite residual in the ") + what + " solve");
    return CHNS_OK;
}

// CHNS_OPT_SERIAL_COMPONENTS = 1 runs the momentum components one after
// another on the handle's stream (per-kernel profiles without overlapping
// kernels).
static bool serial_momentum(const chns_grid *g) { return g->serial_components != 0; }

// S1..S8 of one step from (phi, u) with the pressure initial guess in pr:
// phihat, mu, phi_new, ustar and p; solver statistics into last.
int forward_core(chns_grid *g, const double *phi, const double *const uc[3], double *mu, double *pr,
                 chns_step_stats &last, const double *phi2 = nullptr, double *mu2 = nullptr, bool pguess = false) {
    const int dim = g->dim;
    const Geo &geo = g->geo;
    const StepConst k = step_const(g);
    const chns_props &p = g->props;
    hipStream_t s = g->stream;
    if (pguess) {
        // u*^n, component a's last solution, stays in its buffer and becomes
        // the newest history entry; the oldest entry's buffer takes this
        // step's solve (the history moves without a copy)
        for (int a = 0; a < dim; ++a) {
            double **h = g->uext[a];
            double *fresh = h[2];
            h[2] = h[1];
            h[1] = h[0];
            h[0] = g->ustar[a];
            g->ustar[a] = fresh;
        }
    }
    const double *usc[3] = {g->ustar[0], g->ustar[1], g->ustar[2]};
    const ChOp ch{p.dt * k.kM * p.S, p.dt * k.kM * p.Cn * p.Cn, k.ih2};
    SolveOut o;
    memset(&last, 0, sizeof last);
    // three-phase model: phases 1 and 2 stored (T1..T4 per phase)
    const bool tern = g->nph == 3;
    const Phases3 ph{{phi, phi2}, {g->phi_new, g->phi_new2}, {mu, mu2},
                     {g->mix3[0], g->mix3[1], g->mix3[2], g->mix3[3], g->mix3[4]}};
    // S1, S2 (a direct S2 solve needs no initial guess phihat = phi)
    const bool ch_guess = !g->spec.on;
    if (tern)
        launch_ch_rhs3(dim, geo, k, g->tern, ph, uc, g->rch, g->rch2, ch_guess ? g->phihat : nullptr,
                       ch_guess ? g->phihat2 : nullptr, s);
    else
        launch_ch_rhs(dim, geo, k, phi, uc, g->rch, ch_guess ? g->phihat : nullptr, s);
    if (tern && spectral_all_fft(g->spec)) {
        // the two phases' systems share the operator: both go through one
        // set of transform launches (the CG vectors are free until S7)
        const PcgVecs<double> v = vecs(g);
        const double *const rr[2] = {g->rch, g->rch2};
        double *const xx[2] = {g->phihat, g->phihat2};
        double *const s0[2] = {v.q, v.p0}, *const s1[2] = {v.t, v.p1};
        HIPCHK(spectral_solve2(g->spec, ch.a, ch.b, rr, xx, s0, s1, s));
        last.iters_ch = 1;
    } else {
        for (int q = 0; q < (tern ? 2 : 1); ++q) {
            HIPCHK(run_solve(g, 0, OP_CH, ch, (const double *)(q ? g->rch2 : g->rch), q ? g->phihat2 : g->phihat,
                             p.rtol_ch, q ? 11 : 0, &o));
            if (int rc = check_solve(o, "Cahn-Hilliard")) return rc;
            last.iters_ch = o.iters > last.iters_ch ? o.iters : last.iters_ch;
            last.res_ch = o.rel_res > last.res_ch ? o.rel_res : last.res_ch;
            last.unconverged |= o.unconverged ? 1 : 0;
        }
    }
    // S3, S4
    if (tern) {
        launch_mu3(dim, geo, k, g->tern, ph, g->phihat, g->phihat2, s);
        launch_phi_update3(dim, geo, k, g->tern, ph, uc, s);
    } else {
        launch_mu(dim, geo, k, phi, g->phihat, mu, s);
        launch_phi_update(dim, geo, k, phi, uc, mu, g->phi_new, s);
    }
    // S5..S7: the components are independent.  With the per-kernel timing
    // off, component a > 0 runs on its own stream (forked from and joined
    // back to the handle's stream by events) and its own host thread, so
    // the launch latencies of the components overlap; the arithmetic of
    // each solve is unchanged.  The pressure coefficients and hierarchy
    // (S8) need only phi_new: they are set up on a further stream and
    // thread meanwhile.
    const bool concurrent = dim > 1 && g->mc_ready && !g_prof && !serial_momentum(g);
    Level<double> &P0 = g->pres.lev[0];
    double *pcs[3] = {P0.cs[0], P0.cs[1], P0.cs[2]};
    hipError_t ep = hipSuccess;
    auto pressure_setup = [&]() {
        SolveCtx c = main_ctx(g, 2);
        c.s = g->pstream;
        ep = hipStreamWaitEvent(c.s, g->ev_fork, 0);
        if (ep != hipSuccess) return;
        if (tern)
            launch_p_setup3(dim, geo, k, g->tern, ph, usc, P0.s, pcs, g->rhs, c.s, kPCoef, g->prho);
        else
            launch_p_setup(dim, geo, k, g->phi_new, usc, P0.s, pcs, g->rhs, c.s, kPCoef, g->prho);
        hierarchy_setup(g, c);
        ep = hipEventRecord(g->ev_pset, c.s);
    };
    SolveOut om[3];
    hipError_t em[3] = {hipSuccess, hipSuccess, hipSuccess};
    auto momentum = [&](int a) {
        const SolveCtx c = mom_ctx(g, a);
        if (a > 0 && concurrent) {
            em[a] = hipStreamWaitEvent(c.s, g->ev_mset, 0);
            if (em[a] != hipSuccess) return;
        }
        double *rhs = a == 0 ? g->rhs : g->mc[a - 1].rhs;
        // extrapolated guess from the history (moved at the top of the step)
        if (pguess) launch_velocity_guess(geo, g->ustar[a], g->uext[a], uc[a], pr, g->pext[0], c.s);
        em[a] = run_solve_ctx(g, c, 1, OP_SLOT, ch, (const double *)rhs, g->ustar[a], p.rtol_mom, 1 + a, &om[a]);
        if (em[a] == hipSuccess && a > 0 && concurrent) em[a] = hipEventRecord(g->mc[a - 1].done_ev, c.s);
    };
    // S5..S7 set-up of every component in one pass on the handle's stream
    // (the pressure set-up stream forks before it: it needs only phi_new)
    if (concurrent) HIPCHK(hipEventRecord(g->ev_fork, s));
    {
        MomOut mo{};
        for (int a = 0; a < dim; ++a) {
            Level<double> &L0 = mom_ctx(g, a).S64->lev[0];
            mo.s[a] = L0.s;
            for (int b = 0; b < 3; ++b) mo.cs[a][b] = L0.cs[b];
            mo.rhs[a] = a == 0 ? g->rhs : g->mc[a - 1].rhs;
            mo.ustar[a] = pguess ? nullptr : g->ustar[a];   // with the time guess written by k_velocity_guess
        }
        WallVel wv;
        memcpy(wv.v, g->wall_u, sizeof wv.v);
        const WallVel *pw = g->walls_move ? &wv : nullptr;
        if (tern)
            launch_mom_setup3_all(dim, geo, k, g->tern, ph, uc, mo, g->mflux3, s, pw);
        else
            launch_mom_setup_all(dim, geo, k, phi, g->phi_new, mu, uc, mo, s, pw);
    }
    if (concurrent) {
        HIPCHK(hipEventRecord(g->ev_mset, s));
        WorkerPool *pool = grid_pool(g);
        if (!pool) return fail(CHNS_EDEVICE, "host worker threads could not be started");
        {
            TaskWait tw[3];
            for (int a = 1; a < dim; ++a) tw[a - 1].start(pool, a - 1, [&momentum, a]() { momentum(a); });
            tw[2].start(pool, 2, pressure_setup);
            momentum(0);
        }
        for (int a = 1; a < dim; ++a)
            if (em[a] == hipSuccess) em[a] = hipStreamWaitEvent(s, g->mc[a - 1].done_ev, 0);
        if (ep == hipSuccess) ep = hipStreamWaitEvent(s, g->ev_pset, 0);
    } else {
        for (int a = 0; a < dim; ++a) {
            if (a > 0) {   // sequential: component a uses its buffers on the handle's stream
                MomCtx &M = g->mc[a - 1];
                const hipStream_t keep = M.stream;
                M.stream = s;
                momentum(a);
                M.stream = keep;
            } else {
                momentum(a);
            }
            if (em[a] != hipSuccess) break;
        }
    }
    for (int a = 0; a < dim; ++a) {
        if (em[a] != hipSuccess) return fail(CHNS_EDEVICE, std::string("momentum solve: ") + hipGetErrorString(em[a]));
        if (int rc = check_solve(om[a], "momentum")) return rc;
        last.iters_mom[a] = om[a].iters;
        last.res_mom[a] = om[a].rel_res;
        last.unconverged |= om[a].unconverged ? (2 << a) : 0;
    }
    if (ep != hipSuccess) return fail(CHNS_EDEVICE, std::string("pressure set-up: ") + hipGetErrorString(ep));
    // S8 (coefficients and hierarchy already set up when concurrent)
    if (tern)
        launch_p_setup3(dim, geo, k, g->tern, ph, usc, P0.s, pcs, g->rhs, s, concurrent ? kPRhs : kPCoef | kPRhs,
                        g->prho);
    else
        launch_p_setup(dim, geo, k, g->phi_new, usc, P0.s, pcs, g->rhs, s, concurrent ? kPRhs : kPCoef | kPRhs,
                       g->prho);
    remove_mean(geo, g->rhs, g->red, s);
    // initial guess: p extrapolated in time from this handle's previous
    // solutions where its last step produced the incoming p^n (per cell),
    // else p^n
    if (pguess) launch_pressure_guess(geo, pr, g->pext, s);
    HIPCHK(run_solve_ctx(g, main_ctx(g, 2), !concurrent, OP_SLOT, ch, (const double *)g->rhs, pr, p.rtol_p, 4, &o));
    if (int rc = check_solve(o, "pressure")) return rc;
    last.iters_p = o.iters;
    last.res_p = o.rel_res;
    last.unconverged |= o.unconverged ? 16 : 0;
    remove_mean(geo, pr, g->red, s, pguess ? g->pext[0] : nullptr);   // and the newest history entry
    return CHNS_OK;
}

// One step of the Crank-Nicolson variant (Algorithm C: Picard iterations of
// midpoint sub-steps, see cn.hip) from (phi, u, p) in place; mu receives
// mu~ and p the midpoint pressure.  The momentum components run one after
// another on the handle's stream.
int cn_step(chns_grid *g, double *phi, double *const u[3], double *mu, double *pr, chns_step_stats &last) {
    const int dim = g->dim;
    const Geo &geo = g->geo;
    const StepConst k = step_const(g);
    StepConst kh = k;
    kh.dt = 0.5 * k.dt;
    const chns_props &p = g->props;
    hipStream_t s = g->stream;
    const ChOp ch{kh.dt * k.kM * p.S, kh.dt * k.kM * p.Cn * p.Cn, k.ih2};
    const size_t bytes = sizeof(double) * geo.N;
    double *phim = g->cn_phim, *phimid = g->cn_phimid;
    double *vt[3] = {g->cn_vt[0], g->cn_vt[1], g->cn_vt[2]};
    const double *vtc[3] = {vt[0], vt[1], vt[2]};
    const double *usc[3] = {g->ustar[0], g->ustar[1], g->ustar[2]};
    Level<double> &P0 = g->pres.lev[0];
    double *pcs[3] = {P0.cs[0], P0.cs[1], P0.cs[2]};
    WallVel wv;
    memcpy(wv.v, g->wall_u, sizeof wv.v);
    const WallVel *pw = g->walls_move ? &wv : nullptr;
    memset(&last, 0, sizeof last);
    HIPCHK(hipMemcpyAsync(phim, phi, bytes, hipMemcpyDeviceToDevice, s));
    for (int a = 0; a < dim; ++a) HIPCHK(hipMemcpyAsync(vt[a], u[a], bytes, hipMemcpyDeviceToDevice, s));
    SolveOut o;
    for (int it = 0; it < g->picard; ++it) {
        memset(&last, 0, sizeof last);
        // C1 - C4
        launch_cn_ch_rhs(dim, geo, kh, phi, phim, vtc, g->rch, g->phihat, s);
        HIPCHK(run_solve(g, 0, OP_CH, ch, (const double *)g->rch, g->phihat, p.rtol_ch, 0, &o));
        if (int rc = check_solve(o, "Cahn-Hilliard")) return rc;
        last.iters_ch = o.iters;
        last.res_ch = o.rel_res;
        last.unconverged |= o.unconverged ? 1 : 0;
        launch_mu(dim, geo, k, phim, g->phihat, mu, s);
        launch_cn_phi_update(dim, geo, k, phi, phim, vtc, mu, g->phi_new, phimid, s);
        // C5 - C7
        for (int a = 0; a < dim; ++a) {
            SolveCtx c = mom_ctx(g, a);
            c.s = s;
            Level<double> &L0 = c.S64->lev[0];
            double *rhs = a == 0 ? g->rhs : g->mc[a - 1].rhs;
            double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
            launch_cn_mom_setup(dim, geo, kh, a, phim, phimid, mu, vtc, L0.s, cs, rhs, g->ustar[a], u[a], pr, pw, s);
            SolveOut om;
            HIPCHK(run_solve_ctx(g, c, 1, OP_SLOT, ch, (const double *)rhs, g->ustar[a], p.rtol_mom, 1 + a, &om));
            if (int rc = check_solve(om, "momentum")) return rc;
            last.iters_mom[a] = om.iters;
            last.res_mom[a] = om.rel_res;
            last.unconverged |= om.unconverged ? (2 << a) : 0;
        }
        // C8, C9
        launch_p_setup(dim, geo, kh, phimid, usc, P0.s, pcs, g->rhs, s, kPCoef | kPRhs, g->prho);
        remove_mean(geo, g->rhs, g->red, s);
        launch_cn_zero(geo, g->cn_dp, s);
        HIPCHK(run_solve_ctx(g, main_ctx(g, 2), 1, OP_SLOT, ch, (const double *)g->rhs, g->cn_dp, p.rtol_p, 4, &o));
        if (int rc = check_solve(o, "pressure")) return rc;
        last.iters_p = o.iters;
        last.res_p = o.rel_res;
        last.unconverged |= o.unconverged ? 16 : 0;
        remove_mean(geo, g->cn_dp, g->red, s);
        launch_cn_project(dim, geo, kh, phimid, usc, g->cn_dp, vt, pr, s);
        double *t = phim;
        phim = phimid;
        phimid = t;
    }
    launch_cn_finish(dim, geo, vtc, u, phi, g->phi_new, s);
    remove_mean(geo, pr, g->red, s);
    HIPCHK(hipGetLastError());
    return CHNS_OK;
}

// Adjoint workspace: the forward recomputation's p and mu, the cell and
// face adjoints, and the parameter partials.
void layout_adjoint(Bump &B, const Geo &geo, int dim, AdjBufs &A) {
    const size_t N = (size_t)geo.N;
    double **cells[] = {&A.p_t, &A.mu_t, &A.pbar, &A.zeta, &A.etab, &A.pbt, &A.mub,
                        &A.chr, &A.omega, &A.lphi, &A.sbar};
    for (double **c : cells) *c = B.take<double>(N);
    double **faces[] = {A.usb, A.rfnb, A.rfob, A.aphib, A.gmub, A.mb, A.nu, A.csb};
    for (double **f : faces)
        for (int a = 0; a < 3; ++a) f[a] = a < dim ? B.take<double>(N) : nullptr;
    for (int a = 0; a < 3; ++a) A.Fb[a] = A.usb[a];
    A.gpart = B.take<double>((size_t)kAdjRegions * kRedBlocks);
    A.gout = B.take<double>(4);
}

}  // namespace

extern "C" {

int chns_workspace_size(const chns_grid_desc *desc, size_t *bytes) {
    if (!bytes) return fail(CHNS_EINVAL, "bytes is NULL");
    Plan P;
    int rc = make_plan(desc, P);
    if (rc) return rc;
    chns_grid tmp;
    Bump B{nullptr, 0};
    layout(B, P, &tmp, desc->precision);
    *bytes = B.off + 256;
    return CHNS_OK;
}

// Streams and events of the momentum components (waits for their work).
static void release_streams(chns_grid *g) {
    for (int a = 0; a < 2; ++a) {
        if (g->mc[a].stream) {
            (void)hipStreamSynchronize(g->mc[a].stream);
            (void)hipStreamDestroy(g->mc[a].stream);
            g->mc[a].stream = nullptr;
        }
        if (g->mc[a].done_ev) {
            (void)hipEventDestroy(g->mc[a].done_ev);
            g->mc[a].done_ev = nullptr;
        }
    }
    if (g->pstream) {
        (void)hipStreamSynchronize(g->pstream);
        (void)hipStreamDestroy(g->pstream);
        g->pstream = nullptr;
    }
    if (g->ev_pset) {
        (void)hipEventDestroy(g->ev_pset);
        g->ev_pset = nullptr;
    }
    if (g->ev_fork) {
        (void)hipEventDestroy(g->ev_fork);
        g->ev_fork = nullptr;
    }
    if (g->ev_mset) {
        (void)hipEventDestroy(g->ev_mset);
        g->ev_mset = nullptr;
    }
    g->mc_ready = 0;
}

int chns_create_grid(const chns_grid_desc *desc, void *workspace, size_t bytes, void *hip_stream, chns_grid **out) {
    if (!out) return fail(CHNS_EINVAL, "out is NULL");
    *out = nullptr;
    Plan P;
    int rc = make_plan(desc, P);
    if (rc) return rc;
    size_t need = 0;
    chns_workspace_size(desc, &need);
    if (!workspace) return fail(CHNS_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(CHNS_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(CHNS_ENOMEM, "workspace smaller than chns_workspace_size");
    chns_grid *g = new (std::nothrow) chns_grid();
    if (!g) return fail(CHNS_ENOMEM, "host allocation failed");
    g->desc = *desc;
    g->props_set = 0;
    g->stream = (hipStream_t)hip_stream;
    g->geo = P.lev[0];
    g->dim = P.dim;
    g->h = desc->h;
    g->ws = workspace;
    g->ws_bytes = bytes;
    Bump B{(char *)workspace, 0};
    layout(B, P, g, desc->precision);
    // the CG apply of the step's pressure solves forms the face coefficients
    // from the cell density its set-up writes (expression and 1/h^2 of the set-up)
    g->pres.rho = g->prho;
    {
        const double ih = 1.0 / desc->h;   // as step_const_of
        g->pres.rho_ih2 = ih * ih;
    }
    for (int k = 0; k < 12; ++k) g->last_iters[k] = g->last_inner[k] = 4;
    g->adj_ready = 0;
    g->in_record = 0;
    // streams (default priority) and events of the momentum components and
    // of the pressure set-up
    g->mc_ready = 0;
    g->ev_fork = nullptr;
    g->ev_mset = nullptr;
    g->pool = nullptr;
    g->pstream = nullptr;
    g->ev_pset = nullptr;
    for (int a = 0; a < 2; ++a) {
        g->mc[a].stream = nullptr;
        g->mc[a].done_ev = nullptr;
    }
    if (P.dim > 1) {
        hipError_t e = hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming);
        for (int a = 1; a < P.dim && e == hipSuccess; ++a) {
            e = hipStreamCreateWithFlags(&g->mc[a - 1].stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&g->mc[a - 1].done_ev, hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->pstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_pset, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_mset, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_streams(g);
            delete g;
            return fail(CHNS_EDEVICE, std::string("stream set-up: ") + hipGetErrorString(e));
        }
        g->mc_ready = 1;
    }
    // direct CH solve where the bases fit (chns_set_option can select MG-PCG)
    g->serial_components = 0;
    g->scheme = CHNS_SCHEME_SPLIT;
    g->picard = 3;
    g->pguess = 1;
    memset(g->wall_u, 0, sizeof g->wall_u);
    g->walls_move = 0;
    if (g->spec.carved) {
        std::string err;
        if (spectral_init(g->spec, desc->h, err)) {
            spectral_release(g->spec);
            release_streams(g);
            delete g;
            return fail(CHNS_EDEVICE, err);
        }
    }
    memset(&g->last, 0, sizeof g->last);
    hipError_t e = hipMemsetAsync(g->red.counter, 0, 64 * sizeof(unsigned int), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->red.scal, 0, sizeof(Scal), g->stream);
    // no pressure history yet: all-ones bytes are a NaN, equal to no pressure
    for (int h = 0; h < 3 && e == hipSuccess; ++h)
        e = hipMemsetAsync(g->pext[h], 0xFF, sizeof(double) * (size_t)g->geo.N, g->stream);
    for (int a = 0; a < P.dim && e == hipSuccess; ++a)
        for (int h = 0; h < 3 && e == hipSuccess; ++h)
            e = hipMemsetAsync(g->uext[a][h], 0xFF, sizeof(double) * (size_t)g->geo.N, g->stream);
    for (int a = 1; a < P.dim && e == hipSuccess; ++a) {
        e = hipMemsetAsync(g->mc[a - 1].red.counter, 0, 64 * sizeof(unsigned int), g->stream);
        if (e == hipSuccess) e = hipMemsetAsync(g->mc[a - 1].red.scal, 0, sizeof(Scal), g->stream);
    }
    if (e != hipSuccess) {
        release_streams(g);
        delete g;
        return fail(CHNS_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    }
    *out = g;
    return CHNS_OK;
}

// Diagonal dominance at which a 3D momentum V-cycle ends: the first grid
// level l >= 1 where the smallest diagonal shift rho_min / dt is at least
// kMomTruncRatio times the largest sum of the level's off-diagonal
// couplings, 2 d eta_max / (Re h_l^2) (the re-discretised coarse operators
// scale their couplings by (h / h_l)^2).  One symmetric Gauss-Seidel sweep
// solves such a level to ~1/ratio^2, and the levels below it would add
// corrections of that size; ending there saves their launches and set-up.
// Level 0 itself already ends the cycle at kMomTruncRatio0: the
// preconditioner is then one symmetric sweep on the grid, and CG takes an
// iteration more but each costs the sweep instead of a two-level cycle
// (three-phase drops at 128^3, ratio 10.2 on the grid: 4 CG iterations per
// component instead of 3, 3.84 instead of 3.99 ms per step).
constexpr double kMomTruncRatio = 30.0;
constexpr double kMomTruncRatio0 = 10.0;

static int momentum_trunc_level(const chns_grid *g, const chns_props &p) {
    if (g->dim != 3) return -1;
    double rho_min, eta_max;
    if (g->nph == 3) {
        rho_min = std::min(p.rho3[0], std::min(p.rho3[1], p.rho3[2]));
        eta_max = std::max(p.eta3[0], std::max(p.eta3[1], p.eta3[2]));
    } else {
        rho_min = std::min(1.0, p.rho_minus);
        eta_max = std::max(1.0, p.eta_minus);
    }
    const Slot<double> &S = g->mom;
    const double shift = rho_min / p.dt;
    for (int l = 0; l < S.nlev && S.lev[l].g.N > kSBCells; ++l) {
        const double hl = g->h * (double)(1 << l);
        const double off = 2.0 * g->dim * eta_max / (p.Re * hl * hl);
        if (shift >= (l ? kMomTruncRatio : kMomTruncRatio0) * off) return l;
    }
    return -1;
}

int chns_set_properties(chns_grid *g, const chns_props *p) {
    if (!g || !p) return fail(CHNS_EINVAL, "NULL argument");
    if (int rc = check_props(p)) return rc;
    if (g->nph == 3) {
        for (int i = 0; i < 3; ++i)
            if (!(p->rho3[i] > 0.0) || !(p->eta3[i] > 0.0) || !std::isfinite(p->rho3[i]) || !std::isfinite(p->eta3[i]) ||
                !(p->sigma3[i] > 0.0) || !std::isfinite(p->sigma3[i]))
                return fail(CHNS_EINVAL, "three-phase densities, viscosities and surface tensions must be positive");
        const TernConst t = tern_const_of(*p);
        if (!(t.Sg[0] > 0.0) || !(t.Sg[1] > 0.0) || !(t.Sg[2] > 0.0))
            return fail(CHNS_EINVAL, "every spreading coefficient sigma_ij + sigma_ik - sigma_jk must be positive");
        g->tern = t;
    }
    g->props = *p;
    g->props_set = 1;
    {
        const int lt = momentum_trunc_level(g, *p);
        g->mom.ltrunc = g->mom32.ltrunc = lt;
        for (int a = 0; a < 2; ++a) g->mc[a].mom.ltrunc = g->mc[a].mom32.ltrunc = lt;
    }
    const StepConst k = step_const(g);
    const double cb = p->dt * k.kM * p->Cn * p->Cn;
    double *cs[3] = {g->ch.lev[0].cs[0], g->ch.lev[0].cs[1], g->ch.lev[0].cs[2]};
    launch_fill_ch(g->dim, g->geo, std::sqrt(cb) * k.ih2, g->ch.lev[0].s, cs, g->stream);
    mg_setup(g->ch, g->dim, g->stream);
    if (g->prec == CHNS_FP32_REFINE) {
        convert_level0(g->ch, g->ch32, g->dim, g->stream);
        mg_setup(g->ch32, g->dim, g->stream, false);
    }
    HIPCHK(hipGetLastError());
    return CHNS_OK;
}

int chns_step(chns_grid *g, chns_state *st, int nsteps, chns_step_stats *stats) {
    if (!g || !st) return fail(CHNS_EINVAL, "NULL argument");
    if (!g->props_set) return fail(CHNS_EINVAL, "chns_set_properties must be called first");
    if (nsteps < 0) return fail(CHNS_EINVAL, "nsteps must be >= 0");
    if (!st->phi || !st->p || !st->mu) return fail(CHNS_EINVAL, "state pointer is NULL");
    for (int a = 0; a < g->dim; ++a)
        if (!st->u[a]) return fail(CHNS_EINVAL, "velocity pointer is NULL");
    if (g->nph == 3 && (!st->phi2 || !st->mu2)) return fail(CHNS_EINVAL, "three-phase state needs phi2 and mu2");
    ProfScope prof_scope(g);
    const int dim = g->dim;
    const Geo &geo = g->geo;
    const StepConst k = step_const(g);
    const chns_props &p = g->props;
    hipStream_t s = g->stream;
    double *phi = (double *)st->phi, *mu = (double *)st->mu, *pr = (double *)st->p;
    double *phi2 = g->nph == 3 ? (double *)st->phi2 : nullptr, *mu2 = g->nph == 3 ? (double *)st->mu2 : nullptr;
    double *u[3] = {(double *)st->u[0], (double *)st->u[1], dim == 3 ? (double *)st->u[2] : nullptr};
    const double *uc[3] = {u[0], u[1], u[2]};
    int unconv_any = 0;
    chns_step_stats last;
    memset(&last, 0, sizeof last);
    for (int n = 0; n < nsteps; ++n) {
        if (g->scheme == CHNS_SCHEME_CN) {
            if (int rc = cn_step(g, phi, u, mu, pr, last)) return rc;
            unconv_any |= last.unconverged;
            continue;
        }
        if (int rc = forward_core(g, phi, uc, mu, pr, last, phi2, mu2, g->pguess && !g->in_record)) return rc;
        // this step's u* buffers (forward_core may move them with the time guesses)
        const double *usc[3] = {g->ustar[0], g->ustar[1], g->ustar[2]};
        // S9
        if (g->nph == 3) {
            const Phases3 ph{{phi, phi2}, {g->phi_new, g->phi_new2}, {mu, mu2},
                             {g->mix3[0], g->mix3[1], g->mix3[2], g->mix3[3], g->mix3[4]}};
            launch_project3(dim, geo, k, g->tern, ph, usc, pr, phi, phi2, u, s);
        } else {
            launch_project(dim, geo, k, g->phi_new, usc, pr, phi, u, s);
        }
        HIPCHK(hipGetLastError());
        unconv_any |= last.unconverged;
    }
    if (stats) {
        double *dout = g->diag + kDiagSlots * kMaxBlocks;
        const double hd = std::pow(g->h, dim);
        if (g->nph == 3) {
            launch_diagnostics3(dim, geo, k, g->tern, phi, phi2, uc, g->diag, g->red.counter, dout, s);
            double h9[9];
            HIPCHK(hipMemcpyAsync(h9, dout, sizeof h9, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int q = 0; q < 3; ++q) last.mass_phase[q] = h9[q] * hd;
            last.mass_plus = last.mass_phase[0];
            last.mass_minus = last.mass_phase[1];
            const double fre = (h9[4] * hd + 0.5 * p.Cn * p.Cn * h9[5] * hd) / p.Cn;
            last.energy = h9[3] * hd + fre + p.inv_Fr * h9[6] * hd;
            last.umax = h9[7];
            last.divmax = h9[8];
        } else {
            launch_diagnostics(dim, geo, k, phi, uc, g->diag, g->red.counter, dout, s);
            double h8[8];
            HIPCHK(hipMemcpyAsync(h8, dout, sizeof h8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            last.mass_plus = h8[0] * hd;
            last.mass_minus = h8[1] * hd;
            last.mass_phase[0] = last.mass_plus;
            last.mass_phase[1] = last.mass_minus;
            last.mass_phase[2] = 0.0;
            const double kin = h8[2] * hd;
            const double fre = (h8[3] * hd + 0.5 * p.Cn * p.Cn * h8[4] * hd) / (p.Cn * p.We);
            const double grav = p.inv_Fr * h8[5] * hd;
            last.energy = kin + fre + grav;
            last.umax = h8[6];
            last.divmax = h8[7];
        }
        *stats = last;
    }
    g->last = last;
    if (unconv_any) {
        char buf[256];
        snprintf(buf, sizeof buf, "unconverged solves (bit 0 CH, 1..3 momentum, 4 pressure): mask %d", unconv_any);
        g_err = buf;
        return CHNS_ENOCONV;
    }
    return CHNS_OK;
}

// Total energy of a two-phase state (diagnostics kernel), synchronous.
static int state_energy(chns_grid *g, const double *phi, const double *const uc[3], double *energy) {
    const StepConst k = step_const(g);
    const chns_props &p = g->props;
    double *dout = g->diag + kDiagSlots * kMaxBlocks;
    launch_diagnostics(g->dim, g->geo, k, phi, uc, g->diag, g->red.counter, dout, g->stream);
    double h8[8];
    HIPCHK(hipMemcpyAsync(h8, dout, sizeof h8, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    const double hd = std::pow(g->h, g->dim);
    *energy = h8[2] * hd + (h8[3] * hd + 0.5 * p.Cn * p.Cn * h8[4] * hd) / (p.Cn * p.We) + p.inv_Fr * h8[5] * hd;
    return CHNS_OK;
}

int chns_step_monitor(chns_grid *g, chns_state *st, chns_energy_monitor *out) {
    if (!g || !st || !out) return fail(CHNS_EINVAL, "NULL argument");
    if (!g->props_set) return fail(CHNS_EINVAL, "chns_set_properties must be called first");
    if (g->nph != 2) return fail(CHNS_EINVAL, "the energy monitor covers the two-phase step");
    if (g->walls_move) return fail(CHNS_EINVAL, "the energy monitor covers walls at rest");
    if (g->scheme != CHNS_SCHEME_SPLIT) return fail(CHNS_EINVAL, "the energy monitor covers the split step");
    if (!st->phi || !st->p || !st->mu) return fail(CHNS_EINVAL, "state pointer is NULL");
    for (int a = 0; a < g->dim; ++a)
        if (!st->u[a]) return fail(CHNS_EINVAL, "velocity pointer is NULL");
    ProfScope prof_scope(g);
    const int dim = g->dim;
    const Geo &geo = g->geo;
    const StepConst k = step_const(g);
    const chns_props &p = g->props;
    hipStream_t s = g->stream;
    double *phi = (double *)st->phi, *mu = (double *)st->mu, *pr = (double *)st->p;
    double *u[3] = {(double *)st->u[0], (double *)st->u[1], dim == 3 ? (double *)st->u[2] : nullptr};
    const double *uc[3] = {u[0], u[1], u[2]};
    const double *usc[3] = {g->ustar[0], g->ustar[1], g->ustar[2]};
    memset(out, 0, sizeof *out);
    if (int rc = state_energy(g, phi, uc, &out->energy_before)) return rc;
    chns_step_stats last;
    if (int rc = forward_core(g, phi, uc, mu, pr, last)) return rc;
    const double *ms[3] = {nullptr, nullptr, nullptr};
    const double *mcs[3][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    for (int a = 0; a < dim; ++a) {
        const Level<double> &L0 = a == 0 ? g->mom.lev[0] : g->mc[a - 1].mom.lev[0];
        ms[a] = L0.s;
        for (int b = 0; b < dim; ++b) mcs[a][b] = L0.cs[b];
    }
    double *dout = g->diag + kDiagSlots * kMaxBlocks;
    launch_energy_monitor(dim, geo, k, phi, g->phi_new, mu, uc, usc, pr, ms, mcs, g->diag, g->red.counter, dout, s);
    double h4[4];
    HIPCHK(hipMemcpyAsync(h4, dout, sizeof h4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    launch_project(dim, geo, k, g->phi_new, usc, pr, phi, u, s);
    HIPCHK(hipGetLastError());
    if (int rc = state_energy(g, phi, uc, &out->energy_after)) return rc;
    const double hd = std::pow(g->h, dim);
    out->visc = h4[0] * hd;
    out->chem = h4[1] * hd / (p.Pe * p.Cn * p.Cn * p.We);
    out->cubic = h4[2] * hd / (24.0 * p.We * p.Cn);
    out->inert = h4[3] * hd / 8.0;
    const double diss = p.dt * (out->visc + out->chem), ind = out->cubic + out->inert;
    out->holds = diss >= ind ? 1 : 0;
    out->dt_max = ind == 0.0 ? HUGE_VAL : p.dt * std::sqrt(diss / ind);
    g->last = last;
    if (last.unconverged) {
        char buf[256];
        snprintf(buf, sizeof buf, "unconverged solves (bit 0 CH, 1..3 momentum, 4 pressure): mask %d", last.unconverged);
        g_err = buf;
        return CHNS_ENOCONV;
    }
    return CHNS_OK;
}

int chns_adjoint_workspace_size(const chns_grid_desc *desc, size_t *bytes) {
    if (!bytes) return fail(CHNS_EINVAL, "bytes is NULL");
    Plan P;
    int rc = make_plan(desc, P);
    if (rc) return rc;
    if (P.nph != 2) return fail(CHNS_EINVAL, "the discrete adjoint covers the two-phase step");
    AdjBufs A;
    Bump B{nullptr, 0};
    layout_adjoint(B, P.lev[0], P.dim, A);
    *bytes = B.off + 256;
    return CHNS_OK;
}

int chns_attach_adjoint_workspace(chns_grid *g, void *workspace, size_t bytes) {
    if (!g) return fail(CHNS_EINVAL, "NULL handle");
    if (g->nph != 2) return fail(CHNS_EINVAL, "the discrete adjoint covers the two-phase step");
    if (!workspace) return fail(CHNS_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(CHNS_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    if (int rc = chns_adjoint_workspace_size(&g->desc, &need)) return rc;
    if (bytes < need) return fail(CHNS_ENOMEM, "adjoint workspace smaller than chns_adjoint_workspace_size");
    Bump B{(char *)workspace, 0};
    layout_adjoint(B, g->geo, g->dim, g->adj);
    g->adj_ready = 1;
    return CHNS_OK;
}

// Forward fields of one step that the reverse step reads.
struct FwdFields {
    const double *phihat, *phi_new, *mu, *p;   // S2, S4, S3 (mu^{n+1}), S8 (p^{n+1})
    const double *ustar[3];                     // S7
};

// The reverse of S9 .. S1 (A1 .. A15) of the step from the state fwd, given
// that step's forward fields F.  The pressure slot must hold the operator of
// that step.  unconv: unconverged bits of the forward recomputation.
static int adjoint_core(chns_grid *g, const chns_state *fwd, const FwdFields &F, const chns_adj *lam_in,
                        chns_adj *lam_out, double grad_params[2], int unconv) {
    const int dim = g->dim;
    const Geo &geo = g->geo;
    const StepConst k = step_const(g);
    const chns_props &p = g->props;
    hipStream_t s = g->stream;
    AdjBufs &A = g->adj;
    const double *phi = (const double *)fwd->phi;
    const double *uc[3] = {(const double *)fwd->u[0], (const double *)fwd->u[1],
                           dim == 3 ? (const double *)fwd->u[2] : nullptr};
    const double *ubar[3] = {(const double *)lam_in->u[0], (const double *)lam_in->u[1],
                             dim == 3 ? (const double *)lam_in->u[2] : nullptr};
    double *uout[3] = {(double *)lam_out->u[0], (double *)lam_out->u[1], dim == 3 ? (double *)lam_out->u[2] : nullptr};
    const double *phibar_in = (const double *)lam_in->phi;
    double *phibar_out = (double *)lam_out->phi;
    const ChOp ch{p.dt * k.kM * p.S, p.dt * k.kM * p.Cn * p.Cn, k.ih2};
    SolveOut o;
    // The reverse of S7..S5 below solves with the step's momentum operators,
    // which depend only on the forward fields.  With the components on
    // streams of their own, a host thread sets their coefficients and
    // hierarchies up there (component 0 on the pressure set-up stream) while
    // the adjoint pressure solve runs; the solves then skip the set-up.
    const bool concurrent = dim > 1 && g->mc_ready && !g_prof && !serial_momentum(g);
    hipError_t eset = hipSuccess;
    WorkerPool *pool = concurrent ? grid_pool(g) : nullptr;
    if (concurrent && !pool) return fail(CHNS_EDEVICE, "host worker threads could not be started");
    TaskWait setup_task;
    if (concurrent) {
        HIPCHK(hipEventRecord(g->ev_fork, s));
        setup_task.start(pool, 2, [&]() {
            for (int a = 0; a < dim && eset == hipSuccess; ++a) {
                SolveCtx c = mom_ctx(g, a);
                c.s = a == 0 ? g->pstream : g->mc[a - 1].stream;
                eset = hipStreamWaitEvent(c.s, g->ev_fork, 0);
                if (eset != hipSuccess) break;
                Level<double> &L0 = c.S64->lev[0];
                double *rhs = a == 0 ? g->rhs : g->mc[a - 1].rhs;
                double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
                launch_mom_setup(dim, geo, k, a, phi, F.phi_new, F.mu, uc, L0.s, cs, rhs, g->ustar[a], c.s, 1);
                hierarchy_setup(g, c);
            }
            if (eset == hipSuccess) eset = hipEventRecord(g->ev_pset, g->pstream);   // component 0's
        });
    }
    // reverse of S9 and S8: adjoint pressure solve (the pressure slot still
    // holds the operator of the recomputed step)
    adj_p_rhs(dim, geo, k, F.phi_new, ubar, A.pbar, A.zeta, s);
    remove_mean(geo, A.pbar, g->red, s);
    HIPCHK(run_solve(g, 2, OP_SLOT, ch, (const double *)A.pbar, A.zeta, p.rtol_p, 10, &o));
    if (int rc = check_solve(o, "adjoint pressure")) return rc;
    unconv |= o.unconverged ? 16 : 0;
    remove_mean(geo, A.zeta, g->red, s);
    adj_proj_faces(dim, geo, k, F.phi_new, F.p, A.zeta, ubar, A, uout, s);
    // reverse of S7..S5: K_a nu_a = ubar*_a for every component (the forward
    // operators; independent, so they run like the forward momentum solves,
    // on the components' streams when allowed), then the gathers of each
    // component in order (they accumulate into shared adjoint fields)
    {
        if (concurrent) {
            setup_task.wait();
            if (eset != hipSuccess)
                return fail(CHNS_EDEVICE, std::string("adjoint momentum set-up: ") + hipGetErrorString(eset));
        }
        SolveOut om[3];
        hipError_t em[3] = {hipSuccess, hipSuccess, hipSuccess};
        auto nu_solve = [&](int a, hipStream_t sa) {
            SolveCtx c = mom_ctx(g, a);
            c.s = sa;
            if (a > 0 && concurrent) {
                em[a] = hipStreamWaitEvent(sa, g->ev_fork, 0);
                if (em[a] != hipSuccess) return;
            }
            if (!concurrent) {   // else set up during the adjoint pressure solve
                Level<double> &L0 = c.S64->lev[0];
                double *rhs = a == 0 ? g->rhs : g->mc[a - 1].rhs;
                double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
                launch_mom_setup(dim, geo, k, a, phi, F.phi_new, F.mu, uc, L0.s, cs, rhs, g->ustar[a], sa, 1);
            }
            em[a] = run_solve_ctx(g, c, concurrent ? 0 : 1, OP_SLOT, ch, (const double *)A.usb[a], A.nu[a],
                                  p.rtol_mom, 7 + a, &om[a]);
            if (em[a] == hipSuccess && a > 0 && concurrent) em[a] = hipEventRecord(g->mc[a - 1].done_ev, sa);
        };
        if (concurrent) {
            HIPCHK(hipStreamWaitEvent(s, g->ev_pset, 0));   // component 0's operator
            HIPCHK(hipEventRecord(g->ev_fork, s));
            {
                TaskWait tw[2];
                for (int a = 1; a < dim; ++a)
                    tw[a - 1].start(pool, a - 1, [&nu_solve, a, sa = g->mc[a - 1].stream]() { nu_solve(a, sa); });
                nu_solve(0, s);
            }
            for (int a = 1; a < dim; ++a)
                if (em[a] == hipSuccess) em[a] = hipStreamWaitEvent(s, g->mc[a - 1].done_ev, 0);
        } else {
            for (int a = 0; a < dim && (a == 0 || em[a - 1] == hipSuccess); ++a) nu_solve(a, s);
        }
        for (int a = 0; a < dim; ++a) {
            if (em[a] != hipSuccess)
                return fail(CHNS_EDEVICE, std::string("adjoint momentum solve: ") + hipGetErrorString(em[a]));
            if (int rc = check_solve(om[a], "adjoint momentum")) return rc;
            unconv |= om[a].unconverged ? (2 << a) : 0;
        }
        for (int a = 0; a < dim; ++a) adj_mom(dim, geo, k, a, phi, F.phi_new, F.mu, uc, F.ustar, A, uout, s);
    }
    // reverse of the density / viscosity maps, S4 and S3
    adj_rho_flux_mu(dim, geo, k, phi, F.phi_new, F.mu, uc, phibar_in, A, uout, phibar_out, s);
    // reverse of S2 (adjoint CH solve) and S1
    adj_ch_rhs(dim, geo, k, F.phihat, A, s);
    HIPCHK(run_solve(g, 0, OP_CH, ch, (const double *)A.chr, A.omega, p.rtol_ch, 6, &o));
    if (int rc = check_solve(o, "adjoint Cahn-Hilliard")) return rc;
    unconv |= o.unconverged ? 1 : 0;
    adj_ch_post(dim, geo, k, phi, uc, A, uout, phibar_out, s);
    HIPCHK(hipGetLastError());
    if (grad_params) {
        adj_params(dim, geo, k, A, A.gout, s);
        double gh[4];
        HIPCHK(hipMemcpyAsync(gh, A.gout, sizeof gh, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        grad_params[0] += gh[0];
        grad_params[1] += gh[1];
    }
    if (unconv) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "unconverged solves in the adjoint step (bit 0 CH, 1..3 momentum, 4 pressure): mask %d", unconv);
        g_err = buf;
        return CHNS_ENOCONV;
    }
    return CHNS_OK;
}

int chns_adjoint_step(chns_grid *g, const chns_state *fwd, const chns_adj *lam_in, chns_adj *lam_out,
                      double grad_params[2]) {
    if (!g || !fwd || !lam_in || !lam_out) return fail(CHNS_EINVAL, "NULL argument");
    if (!g->props_set) return fail(CHNS_EINVAL, "chns_set_properties must be called first");
    if (!g->adj_ready) return fail(CHNS_EINVAL, "chns_attach_adjoint_workspace must be called first");
    if (g->scheme != CHNS_SCHEME_SPLIT) return fail(CHNS_EINVAL, "the discrete adjoint covers the split step");
    if (!fwd->phi || !fwd->p || !lam_in->phi || !lam_out->phi) return fail(CHNS_EINVAL, "state pointer is NULL");
    for (int a = 0; a < g->dim; ++a)
        if (!fwd->u[a] || !lam_in->u[a] || !lam_out->u[a]) return fail(CHNS_EINVAL, "velocity pointer is NULL");
    ProfScope prof_scope(g);
    AdjBufs &A = g->adj;
    const double *phi = (const double *)fwd->phi;
    const double *uc[3] = {(const double *)fwd->u[0], (const double *)fwd->u[1],
                           g->dim == 3 ? (const double *)fwd->u[2] : nullptr};
    // Forward recomputation of S1..S8 from the stored state (the pressure
    // solve starts from the stored p, as the original step did).
    HIPCHK(hipMemcpyAsync(A.p_t, fwd->p, sizeof(double) * g->geo.N, hipMemcpyDeviceToDevice, g->stream));
    chns_step_stats last;
    memset(&last, 0, sizeof last);
    if (int rc = forward_core(g, phi, uc, A.mu_t, A.p_t, last)) return rc;
    const FwdFields F{g->phihat, g->phi_new, A.mu_t, A.p_t, {g->ustar[0], g->ustar[1], g->ustar[2]}};
    return adjoint_core(g, fwd, F, lam_in, lam_out, grad_params, last.unconverged);
}

static int check_record(const chns_grid *g, const chns_record *rec) {
    if (!rec) return fail(CHNS_EINVAL, "record is NULL");
    if (!rec->phihat || !rec->phi_new || !rec->mu || !rec->p) return fail(CHNS_EINVAL, "record pointer is NULL");
    for (int a = 0; a < g->dim; ++a)
        if (!rec->ustar[a]) return fail(CHNS_EINVAL, "record velocity pointer is NULL");
    return CHNS_OK;
}

int chns_step_record(chns_grid *g, chns_state *st, const chns_record *rec) {
    if (!g) return fail(CHNS_EINVAL, "NULL argument");
    if (g->nph != 2) return fail(CHNS_EINVAL, "step records cover the two-phase step");
    if (g->scheme != CHNS_SCHEME_SPLIT) return fail(CHNS_EINVAL, "step records cover the split step");
    if (int rc = check_record(g, rec)) return rc;
    // a recorded step starts its pressure solve from the state's p, as the
    // adjoint's recomputation of the step does
    g->in_record = 1;
    const int rc = chns_step(g, st, 1, nullptr);
    g->in_record = 0;
    if (rc != CHNS_OK && rc != CHNS_ENOCONV) return rc;
    hipStream_t s = g->stream;
    const size_t bytes = sizeof(double) * g->geo.N;
    HIPCHK(hipMemcpyAsync(rec->phihat, g->phihat, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(rec->phi_new, g->phi_new, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(rec->mu, st->mu, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(rec->p, st->p, bytes, hipMemcpyDeviceToDevice, s));
    for (int a = 0; a < g->dim; ++a)
        HIPCHK(hipMemcpyAsync(rec->ustar[a], g->ustar[a], bytes, hipMemcpyDeviceToDevice, s));
    return rc;
}

int chns_adjoint_step_recorded(chns_grid *g, const chns_state *fwd, const chns_record *rec, const chns_adj *lam_in,
                               chns_adj *lam_out, double grad_params[2]) {
    if (!g || !fwd || !lam_in || !lam_out) return fail(CHNS_EINVAL, "NULL argument");
    if (!g->props_set) return fail(CHNS_EINVAL, "chns_set_properties must be called first");
    if (!g->adj_ready) return fail(CHNS_EINVAL, "chns_attach_adjoint_workspace must be called first");
    if (!fwd->phi || !lam_in->phi || !lam_out->phi) return fail(CHNS_EINVAL, "state pointer is NULL");
    for (int a = 0; a < g->dim; ++a)
        if (!fwd->u[a] || !lam_in->u[a] || !lam_out->u[a]) return fail(CHNS_EINVAL, "velocity pointer is NULL");
    if (int rc = check_record(g, rec)) return rc;
    ProfScope prof_scope(g);
    // the pressure operator of the recorded step (S8 set-up from its
    // phi^{n+1} and u*; the right-hand side it also writes is not used)
    Level<double> &L0 = g->pres.lev[0];
    double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
    const double *usr[3] = {(const double *)rec->ustar[0], (const double *)rec->ustar[1],
                            g->dim == 3 ? (const double *)rec->ustar[2] : nullptr};
    launch_p_setup(g->dim, g->geo, step_const(g), (const double *)rec->phi_new, usr, L0.s, cs, g->rhs, g->stream,
                   kPCoef | kPRhs, g->prho);
    const FwdFields F{(const double *)rec->phihat, (const double *)rec->phi_new, (const double *)rec->mu,
                      (const double *)rec->p, {usr[0], usr[1], usr[2]}};
    return adjoint_core(g, fwd, F, lam_in, lam_out, grad_params, 0);
}

int chns_solve_pressure(chns_grid *g, const void *rho, const void *rhs, void *p, double rtol, int max_iter,
                        chns_solve_stats *stats) {
    if (!g || !rho || !rhs || !p) return fail(CHNS_EINVAL, "NULL argument");
    if (!(rtol > 0.0) || max_iter < 1) return fail(CHNS_EINVAL, "rtol must be > 0 and max_iter >= 1");
    ProfScope prof_scope(g);
    const int dim = g->dim;
    hipStream_t s = g->stream;
    Level<double> &L0 = g->pres.lev[0];
    double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
    launch_p_coef_from_rho(dim, g->geo, 1.0 / (g->h * g->h), (const double *)rho, L0.s, cs, s);
    HIPCHK(hipMemcpyAsync(g->rhs, rhs, sizeof(double) * g->geo.N, hipMemcpyDeviceToDevice, s));
    remove_mean(g->geo, g->rhs, g->red, s);
    SolveOut o;
    const int saved = g->props.max_iter;
    g->props.max_iter = max_iter;
    // the CG apply forms its coefficients from the given density, as
    // launch_p_coef_from_rho above (the same 1/h^2)
    const double *rho_step = g->pres.rho;
    const double ih2_step = g->pres.rho_ih2;
    g->pres.rho = (const double *)rho;
    g->pres.rho_ih2 = 1.0 / (g->h * g->h);
    hipError_t e = run_solve(g, 2, OP_SLOT, ChOp{0, 0, 0}, (const double *)g->rhs, (double *)p, rtol, 5, &o);
    g->pres.rho = rho_step;
    g->pres.rho_ih2 = ih2_step;
    g->props.max_iter = saved;
    HIPCHK(e);
    if (int rc = check_solve(o, "pressure")) return rc;
    remove_mean(g->geo, (double *)p, g->red, s);
    HIPCHK(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = o.iters;
        stats->rel_res = o.rel_res;
    }
    return o.unconverged ? CHNS_ENOCONV : CHNS_OK;
}

int chns_apply_pressure_operator(chns_grid *g, const void *rho, const void *x, void *y) {
    if (!g || !rho || !x || !y) return fail(CHNS_EINVAL, "NULL argument");
    Level<double> &L0 = g->pres.lev[0];
    double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
    launch_p_coef_from_rho(g->dim, g->geo, 1.0 / (g->h * g->h), (const double *)rho, L0.s, cs, g->stream);
    slot_apply(g->pres, g->dim, (const double *)x, (double *)y, g->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(g->stream));
    return CHNS_OK;
}

int chns_set_wall_velocity(chns_grid *g, int axis, int side, int component, const void *values) {
    if (!g) return fail(CHNS_EINVAL, "NULL handle");
    if (axis < 0 || axis >= g->dim || g->geo.per[axis]) return fail(CHNS_EINVAL, "axis must be a walled axis");
    if (side != 0 && side != 1) return fail(CHNS_EINVAL, "side must be 0 (lower wall) or 1 (upper wall)");
    if (component < 0 || component >= g->dim || component == axis)
        return fail(CHNS_EINVAL, "component must be a velocity component tangential to the wall");
    g->wall_u[axis][side][component] = (const double *)values;
    g->walls_move = 0;
    for (int b = 0; b < 3; ++b)
        for (int q = 0; q < 2; ++q)
            for (int a = 0; a < 3; ++a)
                if (g->wall_u[b][q][a]) g->walls_move = 1;
    return CHNS_OK;
}

int chns_set_option(chns_grid *g, int option, int value) {
    if (!g) return fail(CHNS_EINVAL, "NULL handle");
    switch (option) {
        case CHNS_OPT_CH_SOLVER:
            if (value == CHNS_CH_PCG) {
                if (g->spec.on) spectral_release(g->spec);
                return CHNS_OK;
            }
            if (value != CHNS_CH_DIRECT && value != CHNS_CH_DIRECT_DENSE)
                return fail(CHNS_EINVAL, "CH solver must be CHNS_CH_DIRECT, CHNS_CH_DIRECT_DENSE or CHNS_CH_PCG");
            if (!g->spec.carved) return fail(CHNS_EINVAL, "the direct CH solve needs every axis <= 2048 cells");
            if (!g->spec.on) {
                std::string err;
                HIPCHK(hipStreamSynchronize(g->stream));
                if (spectral_init(g->spec, g->h, err)) return fail(CHNS_EDEVICE, err);
            }
            g->spec.dense = value == CHNS_CH_DIRECT_DENSE;
            return CHNS_OK;
        case CHNS_OPT_TIME_SCHEME:
            if (value != CHNS_SCHEME_SPLIT && value != CHNS_SCHEME_CN)
                return fail(CHNS_EINVAL, "time scheme must be CHNS_SCHEME_SPLIT or CHNS_SCHEME_CN");
            if (value == CHNS_SCHEME_CN && g->nph != 2)
                return fail(CHNS_EINVAL, "the Crank-Nicolson variant covers the two-phase step");
            g->scheme = value;
            return CHNS_OK;
        case CHNS_OPT_PICARD_ITERATIONS:
            if (value < 1 || value > 1000) return fail(CHNS_EINVAL, "Picard iterations must be in 1..1000");
            g->picard = value;
            return CHNS_OK;
        case CHNS_OPT_TIME_GUESS:
            if (value != 0 && value != 1) return fail(CHNS_EINVAL, "pressure-guess value must be 0 or 1");
            g->pguess = value;
            return CHNS_OK;
        case CHNS_OPT_SERIAL_COMPONENTS:
            if (value != 0 && value != 1) return fail(CHNS_EINVAL, "serial-components value must be 0 or 1");
            g->serial_components = value;
            return CHNS_OK;
        case CHNS_OPT_MARCH_SWEEP_CELLS: {
            if (value < 1) return fail(CHNS_EINVAL, "march-sweep cells must be >= 1");
            Slot<double> *s64[] = {&g->ch, &g->mom, &g->pres, &g->mc[0].mom, &g->mc[1].mom};
            Slot<float> *s32[] = {&g->ch32, &g->mom32, &g->pres32, &g->mc[0].mom32, &g->mc[1].mom32};
            for (Slot<double> *S : s64) S->march_cells = value;
            for (Slot<float> *S : s32) S->march_cells = value;
            return CHNS_OK;
        }
        case CHNS_OPT_TILE_CYCLE_CELLS: {
            if (value < 0) return fail(CHNS_EINVAL, "tile-cycle cells must be >= 0");
            Slot<double> *s64[] = {&g->ch, &g->mom, &g->pres, &g->mc[0].mom, &g->mc[1].mom};
            Slot<float> *s32[] = {&g->ch32, &g->mom32, &g->pres32, &g->mc[0].mom32, &g->mc[1].mom32};
            for (Slot<double> *S : s64) S->tile_cells = value;
            for (Slot<float> *S : s32) S->tile_cells = value;
            return CHNS_OK;
        }
        default:
            return fail(CHNS_EINVAL, "unknown option");
    }
}

static void prof_release(Prof &P) {
    if (P.ev) {
        for (int i = 0; i < 2 * P.cap; ++i) (void)hipEventDestroy(P.ev[i]);
    }
    delete[] P.ev;
    delete[] P.cls;
    delete[] P.bytes;
    P.ev = nullptr;
    P.cls = nullptr;
    P.bytes = nullptr;
    P.cap = 0;
}

int chns_set_timing(chns_grid *g, int enable) {
    if (!g) return fail(CHNS_EINVAL, "NULL handle");
    Prof &P = g->prof;
    if (enable && !P.ev) {
        const int cap = 4096;
        P.ev = new (std::nothrow) hipEvent_t[2 * cap];
        P.cls = new (std::nothrow) int[cap];
        P.bytes = new (std::nothrow) double[cap];
        if (!P.ev || !P.cls || !P.bytes) {
            prof_release(P);
            return fail(CHNS_ENOMEM, "host allocation failed");
        }
        for (int i = 0; i < 2 * cap; ++i) {
            hipError_t e = hipEventCreate(&P.ev[i]);
            if (e != hipSuccess) {
                P.cap = i / 2;
                prof_release(P);
                return fail(CHNS_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
            }
        }
        P.cap = cap;
    }
    P.enabled = enable ? 1 : 0;
    P.n = 0;
    for (int c = 0; c < K_NCLASS; ++c) {
        P.launches[c] = 0;
        P.ms[c] = 0.0;
        P.total_bytes[c] = 0.0;
    }
    return CHNS_OK;
}

int chns_get_timing(chns_grid *g, chns_kernel_timing *out, int max, int *count) {
    if (!g || !count) return fail(CHNS_EINVAL, "NULL argument");
    const Prof &P = g->prof;
    int n = 0;
    for (int c = 0; c < K_NCLASS; ++c) {
        if (!P.launches[c]) continue;
        if (out && n < max) {
            memset(&out[n], 0, sizeof out[n]);
            strncpy(out[n].name, kclass_name(c), sizeof out[n].name - 1);
            out[n].launches = P.launches[c];
            out[n].ms = P.ms[c];
            out[n].bytes = P.total_bytes[c];
        }
        ++n;
    }
    *count = n;
    return CHNS_OK;
}

int chns_destroy_grid(chns_grid *g) {
    if (g) {
        delete g->pool;
        g->pool = nullptr;
        prof_release(g->prof);
        release_streams(g);
        spectral_release(g->spec);
    }
    delete g;
    return CHNS_OK;
}

const char *chns_error_string(int code) {
    switch (code) {
        case CHNS_OK: return "success";
        case CHNS_ENOCONV: return "a linear solve reached max_iter before the tolerance";
        case CHNS_EINVAL: return "invalid argument or unsupported grid";
        case CHNS_ENOMEM: return "workspace too small";
        case CHNS_EDEVICE: return "HIP runtime error";
        case CHNS_ENONFINITE: return "non-finite value in a residual";
        default: return "unknown error code";
    }
}

int chns_last_error(char *buf, size_t len) {
    if (buf && len > 0) {
        size_t n = g_err.size() < len - 1 ? g_err.size() : len - 1;
        memcpy(buf, g_err.data(), n);
        buf[n] = '\0';
    }
    return (int)g_err.size();
}

}  // extern "C"
