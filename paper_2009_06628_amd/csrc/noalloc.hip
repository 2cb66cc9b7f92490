// Stand-alone pressure solve that allocates nothing: the variant of
// chns_solve_pressure for callers that cannot allocate device memory.  Its
// hierarchy, CG vectors and reduction scratch live in one file-scope device
// array (`scratch`) of fixed size, which every GPU the library runs on holds
// until the process ends.  The kernels are those of chns_solve_pressure.
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"
#include "plan.h"
#include "solvers.h"
#include "step.h"

namespace chns {

constexpr size_t kNoAllocBytes = (size_t)CHNS_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device (the array's name is a host
// stand-in in host code, never a device address).
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];

static int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(CHNS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(CHNS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CHNS_OK;
}

// Clears n 32-bit words (a kernel, not hipMemsetAsync, so that the call can
// sit in a captured stream).
__global__ void k_zero_words(unsigned int *w, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

namespace {

// What a pressure solve needs, carved from a base pointer (nullptr: sizing).
struct StaticSolve {
    Slot<double> p64;
    Slot<float> p32;
    double *rhs;
    double *vr, *vz, *vp0, *vp1, *vq, *vt;
    float *f_z, *f_t, *f_r;
    Red red;
};

void carve(Bump &B, const Plan &P, int prec, StaticSolve &S) {
    const size_t N = (size_t)P.lev[0].N;
    carve_slot(B, P, S.p64, 1);
    const int nc = S.p64.ncoarse;
    double *aug = nc > kLdsInverse ? B.take<double>((size_t)nc * nc) : nullptr;
    S.p64.aug = aug;
    if (prec == CHNS_FP32_REFINE) {
        carve_slot(B, P, S.p32, 1);
        S.p32.aug = aug;
        S.f_z = B.take<float>(N);
        S.f_t = B.take<float>(N);
        S.f_r = B.take<float>(N);
    } else {
        S.f_z = S.f_t = S.f_r = nullptr;
    }
    S.rhs = B.take<double>(N);
    S.vr = B.take<double>(N);
    S.vz = B.take<double>(N);
    S.vp0 = B.take<double>(N);
    S.vp1 = B.take<double>(N);
    S.vq = B.take<double>(N);
    S.vt = B.take<double>(N);
    S.red.part0 = B.take<double>(kMaxBlocks);
    S.red.part1 = B.take<double>(kMaxBlocks);
    S.red.part2 = B.take<double>(kMaxBlocks);
    S.red.rz0 = B.take<double>(kRedBlocks);
    S.red.rz1 = B.take<double>(kRedBlocks);
    S.red.rz2 = B.take<double>(kRedBlocks);
    S.red.counter = B.take<unsigned int>(64);
    S.red.scal = B.take<Scal>(1);
}

}  // namespace
}  // namespace chns

using namespace chns;

extern "C" {

int chns_solve_pressure_noalloc(const chns_grid_desc *desc, const void *rho, const void *rhs, void *p, double rtol,
                                int max_iter, void *hip_stream, chns_solve_stats *stats) {
    if (!desc || !rho || !rhs || !p) return set_error(CHNS_EINVAL, "NULL argument");
    if (!(rtol > 0.0) || max_iter < 1) return set_error(CHNS_EINVAL, "rtol must be > 0 and max_iter >= 1");
    chns_grid_desc d = *desc;
    d.nphases = 2;   // the pressure operator does not depend on the phase count
    Plan P;
    if (int rc = make_plan(&d, P)) return rc;
    StaticSolve S;
    {
        Bump B{nullptr, 0};
        carve(B, P, d.precision, S);
        if (B.off > kNoAllocBytes) {
            char buf[200];
            snprintf(buf, sizeof buf,
                     "grid needs %zu bytes of solver scratch; chns_solve_pressure_noalloc holds at most %zu",
                     B.off, kNoAllocBytes);
            return set_error(CHNS_EINVAL, buf);
        }
    }
    void *base = nullptr;
    if (int rc = scratch_ptr(&base)) return rc;
    Bump B{(char *)base, 0};
    carve(B, P, d.precision, S);
    const int dim = P.dim;
    const Geo geo = P.lev[0];
    hipStream_t s = (hipStream_t)hip_stream;
    // the array keeps the previous call's contents: clear the reduction
    // counters and the CG scalar block
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, S.red.counter, 64);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (unsigned int *)S.red.scal,
                       (int)(sizeof(Scal) / sizeof(unsigned int)));
    Level<double> &L0 = S.p64.lev[0];
    double *cs[3] = {L0.cs[0], L0.cs[1], L0.cs[2]};
    launch_p_coef_from_rho(dim, geo, 1.0 / (d.h * d.h), (const double *)rho, L0.s, cs, s);
    hipError_t e = hipMemcpyAsync(S.rhs, rhs, sizeof(double) * geo.N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    remove_mean(geo, S.rhs, S.red, s);
    SolveOut o;
    const ChOp none{0, 0, 0};
    if (d.precision == CHNS_FP64) {
        mg_setup(S.p64, dim, s);
        PcgVecs<double> v{S.vr, S.vz, S.vp0, S.vp1, S.vq, S.vt};
        e = pcg_solve(S.p64, dim, OP_SLOT, none, (const double *)S.rhs, (double *)p, rtol, max_iter, 4, S.red, v, s,
                      &o);
    } else {
        convert_level0(S.p64, S.p32, dim, s);
        mg_setup(S.p32, dim, s, false);
        const PcgVecs2<double, float> v2{S.vr, S.vp0, S.vp1, S.vq, S.vt, S.f_z, S.f_t, S.f_r};
        int predict = 4;
        e = refine_solve(S.p64, S.p32, dim, OP_SLOT, none, (const double *)S.rhs, (double *)p, rtol, max_iter,
                         &predict, S.red, v2, s, &o);
    }
    if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("pressure solve: ") + hipGetErrorString(e));
    if (o.nonfinite) return set_error(CHNS_ENONFINITE, "non-finite residual in the pressure solve");
    remove_mean(geo, (double *)p, S.red, s);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(CHNS_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    if (stats) {
        stats->iters = o.iters;
        stats->rel_res = o.rel_res;
    }
    if (o.unconverged) return set_error(CHNS_ENOCONV, "the pressure solve reached max_iter");
    return CHNS_OK;
}

size_t chns_solve_pressure_noalloc_capacity(void) { return kNoAllocBytes; }

}  // extern "C"
