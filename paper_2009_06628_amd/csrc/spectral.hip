// Direct (spectral) solve of the Cahn-Hilliard system; see spectral.h.
#include <cmath>
#include <algorithm>
#include <utility>
#include <vector>

#include "spectral.h"

namespace chns {

// log2 n for a periodic axis the FFT can transform, else 0
static int fft_log(int n, int per) {
    if (!per || (n & (n - 1)) != 0) return 0;
    int l = 0;
    while ((1 << l) < n) ++l;
    return l >= kFftMinLog && l <= kFftMaxLog ? l : 0;
}

void spectral_carve(Bump &B, const Geo &g, int dim, Spectral &S) {
    S.carved = 1;
    S.on = 0;
    S.dense = 0;
    S.dim = dim;
    for (int a = 0; a < 3; ++a) {
        S.n[a] = a < dim ? (int)g.n[a] : 1;
        S.per[a] = a < dim ? g.per[a] : 1;
        S.fft[a] = a < dim ? fft_log(S.n[a], S.per[a]) : 0;
        S.Q[a] = S.lam[a] = S.tw[a] = nullptr;
        if (a < dim && g.n[a] > kSpectralMaxN) S.carved = 0;
    }
    if (!S.carved) return;
    for (int a = 0; a < dim; ++a) {
        S.Q[a] = B.take<double>((size_t)S.n[a] * S.n[a]);
        S.lam[a] = B.take<double>((size_t)S.n[a]);
        if (S.fft[a]) S.tw[a] = B.take<double>((size_t)2 * S.n[a]);
    }
}

// Eigenbasis of the 1D cell-centred second difference with spacing h on n
// cells.  Walled (Neumann: the flux through the wall faces is zero): column
// k = sqrt((k ? 2 : 1) / n) cos(pi k (j + 1/2) / n), eigenvalue
// -(4 / h^2) sin^2(pi k / (2 n)).  Periodic: the constant, then
// sqrt(2 / n) cos(2 pi k j / n) and sqrt(2 / n) sin(2 pi k j / n) for
// 0 < k < n / 2 (eigenvalue -(4 / h^2) sin^2(pi k / n) for both), then
// (-1)^j / sqrt(n) when n is even.  Angles are reduced exactly in integers
// before the trigonometric call.
void spectral_axis(int n, int per, double h, std::vector<double> &Q, std::vector<double> &lam) {
    const double pi = std::acos(-1.0), ih2 = 1.0 / (h * h);
    Q.assign((size_t)n * n, 0.0);
    lam.assign((size_t)n, 0.0);
    if (!per) {
        for (int k = 0; k < n; ++k) {
            const double s = std::sqrt((k ? 2.0 : 1.0) / n);
            for (int j = 0; j < n; ++j) {
                const long long m = ((long long)k * (2 * j + 1)) % (4LL * n);   // angle pi m / (2 n)
                Q[j + (size_t)n * k] = s * std::cos(pi * (double)m / (2.0 * n));
            }
            const double sn = std::sin(pi * k / (2.0 * n));
            lam[k] = -4.0 * ih2 * sn * sn;
        }
        return;
    }
    const double s0 = std::sqrt(1.0 / n), s1 = std::sqrt(2.0 / n);
    for (int j = 0; j < n; ++j) Q[j] = s0;
    lam[0] = 0.0;
    int col = 1;
    for (int k = 1; 2 * k < n; ++k, col += 2) {
        for (int j = 0; j < n; ++j) {
            const long long m = ((long long)k * j) % n;   // angle 2 pi m / n
            const double ang = 2.0 * pi * (double)m / n;
            Q[j + (size_t)n * col] = s1 * std::cos(ang);
            Q[j + (size_t)n * (col + 1)] = s1 * std::sin(ang);
        }
        const double sn = std::sin(pi * k / n);
        lam[col] = lam[col + 1] = -4.0 * ih2 * sn * sn;
    }
    if (n % 2 == 0) {
        for (int j = 0; j < n; ++j) Q[j + (size_t)n * col] = (j & 1) ? -s0 : s0;
        lam[col] = -4.0 * ih2;
    }
}

int spectral_init(Spectral &S, double h, std::string &err) {
    S.on = 0;
    if (!S.carved) return 0;
    std::vector<double> Q, lam;
    for (int a = 0; a < S.dim; ++a) {
        spectral_axis(S.n[a], S.per[a], h, Q, lam);
        hipError_t e = hipMemcpy(S.Q[a], Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(S.lam[a], lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess && S.fft[a]) {
            // twiddles cos, sin of 2 pi k / n (angles reduced exactly: the
            // quadrant symmetry makes e.g. cos(pi / 2) exactly 0)
            const int n = S.n[a];
            std::vector<double> tw(2 * (size_t)n);
            const double pi = std::acos(-1.0);
            for (int k = 0; k < n; ++k) {
                const int q = (4 * k) / n, r = 4 * k - q * n;   // angle = (q + r / n) pi / 2
                const double t = 0.5 * pi * (double)r / n, c = std::cos(t), sn = std::sin(t);
                const double cs[4] = {c, -sn, -c, sn}, ss[4] = {sn, c, -sn, -c};
                tw[2 * k] = cs[q];
                tw[2 * k + 1] = ss[q];
            }
            e = hipMemcpy(S.tw[a], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            err = std::string("spectral basis upload: ") + hipGetErrorString(e);
            return 1;
        }
    }
    S.on = 1;
    return 0;
}

void spectral_release(Spectral &S) { S.on = 0; }

// ---------------------------------------------------------------------------
// axis transforms: C(m, n) = sum_k A(m, k) B(k, n) per batch entry, FP64
// FMAs on 64 x 64 output tiles of a 256-thread workgroup (4 x 4 outputs per
// thread, k in chunks of 16 staged in LDS).  Operands are addressed by
// element strides, so one kernel covers every axis and both directions.
// ---------------------------------------------------------------------------
struct AxOp {
    const double *p;            // base of batch entry 0
    const double *const *tab;   // per-entry bases, or null (then p + b * bs)
    long long bs;               // batch stride in elements
    int s0, s1;                 // element strides of the first / second index
    __device__ const double *at(int b) const { return tab ? tab[b] : p + (long long)b * bs; }
};
struct AxOut {
    double *p;
    double *const *tab;
    long long bs;
    int s0, s1;
    __device__ double *at(int b) const { return tab ? tab[b] : p + (long long)b * bs; }
};

constexpr int kGThreads = 256;

// TS x TS output tile (TS = 64 or 32): a 16 x 16 thread grid, each thread
// (TS / 16)^2 outputs.  k runs in chunks of KC = 2048 / TS staged in LDS;
// the loads of the next chunk are in flight while the current one is used.
template <int TS>
__global__ void __launch_bounds__(kGThreads) k_axis_gemm(int M, int N, int K, AxOp A, AxOp B, AxOut C) {
    constexpr int R = TS / 16, KC = 2048 / TS, PT = TS * KC / kGThreads;   // staged values per thread
    __shared__ double As[KC][TS + 1], Bs[KC][TS + 1];
    const int bz = (int)blockIdx.z;
    const double *a = A.at(bz), *bp = B.at(bz);
    double *c = C.at(bz);
    const int m0 = (int)blockIdx.y * TS, n0 = (int)blockIdx.x * TS;
    const int tid = (int)threadIdx.x, tm = tid / 16, tn = tid % 16;
    // staging positions: the index that is contiguous in memory runs
    // fastest across the threads
    auto a_pos = [&](int e, int &mm, int &kk) {
        if (A.s1 == 1) {
            kk = e % KC;
            mm = e / KC;
        } else {
            mm = e % TS;
            kk = e / TS;
        }
    };
    auto b_pos = [&](int e, int &nn, int &kk) {
        if (B.s1 == 1) {
            nn = e % TS;
            kk = e / TS;
        } else {
            kk = e % KC;
            nn = e / KC;
        }
    };
    double ra[PT], rb[PT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
            ra[r] = (gm < M && gk < K) ? a[(long long)gm * A.s0 + (long long)gk * A.s1] : 0.0;
            rb[r] = (gn < N && gkb < K) ? bp[(long long)gkb * B.s0 + (long long)gn * B.s1] : 0.0;
        }
    };
    double acc[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) acc[i][j] = 0.0;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            As[kk][mm] = ra[r];
            Bs[kb][nn] = rb[r];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);   // in flight during the products below
        const int kn = K - k0 < KC ? K - k0 : KC;
#pragma unroll 4
        for (int kk = 0; kk < kn; ++kk) {
            double av[R], bv[R];
#pragma unroll
            for (int i = 0; i < R; ++i) av[i] = As[kk][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < R; ++j) bv[j] = Bs[kk][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int gm = m0 + tm + 16 * i, gn = n0 + tn + 16 * j;
            if (gm < M && gn < N) c[(long long)gm * C.s0 + (long long)gn * C.s1] = acc[i][j];
        }
}

// 64 x 64 output tile on the FP64 matrix cores: the four waves of the
// workgroup form a 2 x 2 grid of 32 x 32 blocks, each four 16 x 16 x 4 MFMA
// accumulators.  Staging and chunks (KC = 32) as in k_axis_gemm<64>.
// Operand layout of the FP64 16 x 16 x 4 MFMA: lane l supplies A(l % 16,
// l / 16) and B(l / 16, l % 16); element v of its accumulator is
// C(4 v + l / 16, l % 16).  Values staged past M, N or K are zero, so every
// chunk runs all of its k.
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaKC = 32;   // k per staged chunk

template <int KC>
__global__ void __launch_bounds__(kGThreads) k_axis_mfma64(int M, int N, int K, AxOp A, AxOp B, AxOut C) {
    constexpr int TS = 64, PT = TS * KC / kGThreads;
    __shared__ double As[KC][TS + 1], Bs[KC][TS + 1];
    const int bz = (int)blockIdx.z;
    const double *a = A.at(bz), *bp = B.at(bz);
    double *c = C.at(bz);
    const int m0 = (int)blockIdx.y * TS, n0 = (int)blockIdx.x * TS;
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32, li = lane & 15, lk = lane >> 4;
    auto a_pos = [&](int e, int &mm, int &kk) {
        if (A.s1 == 1) {
            kk = e % KC;
            mm = e / KC;
        } else {
            mm = e % TS;
            kk = e / TS;
        }
    };
    auto b_pos = [&](int e, int &nn, int &kk) {
        if (B.s1 == 1) {
            nn = e % TS;
            kk = e / TS;
        } else {
            kk = e % KC;
            nn = e / KC;
        }
    };
    double ra[PT], rb[PT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
            ra[r] = (gm < M && gk < K) ? a[(long long)gm * A.s0 + (long long)gk * A.s1] : 0.0;
            rb[r] = (gn < N && gkb < K) ? bp[(long long)gkb * B.s0 + (long long)gn * B.s1] : 0.0;
        }
    };
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            As[kk][mm] = ra[r];
            Bs[kb][nn] = rb[r];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);   // in flight during the products below
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[k4 + lk][wm + 16 * i + li];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[k4 + lk][wn + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gm = m0 + wm + 16 * i + 4 * v + lk, gn = n0 + wn + 16 * j + li;
                if (gm < M && gn < N) c[(long long)gm * C.s0 + (long long)gn * C.s1] = acc[i][j][v];
            }
}

// 16 x 16 output tile with k split over 16 thread groups: thread t of group
// g computes the 4 x 4 block of rows t / 4 + 4 i and columns t % 4 + 4 j over
// the k of each chunk with k mod 16 = g (half an LDS read per FMA, where one
// output per thread takes two), then the 16 partial blocks are summed in
// group order.  Staging and chunks (KC = 128) as in k_axis_gemm.
__global__ void __launch_bounds__(kGThreads) k_axis_gemm16s(int M, int N, int K, AxOp A, AxOp B, AxOut C) {
    constexpr int TS = 16, KC = 2048 / TS, PT = TS * KC / kGThreads, G = kGThreads / 16;
    static_assert(2 * KC * (TS + 1) >= G * TS * TS, "partial sums reuse the staging LDS");
    __shared__ double sm[2 * KC * (TS + 1)];
    double(*As)[TS + 1] = (double(*)[TS + 1])sm;
    double(*Bs)[TS + 1] = (double(*)[TS + 1])(sm + KC * (TS + 1));
    const int bz = (int)blockIdx.z;
    const double *a = A.at(bz), *bp = B.at(bz);
    double *c = C.at(bz);
    const int m0 = (int)blockIdx.y * TS, n0 = (int)blockIdx.x * TS;
    const int tid = (int)threadIdx.x, g = tid / 16, rm = (tid % 16) / 4, rn = tid % 4;
    auto a_pos = [&](int e, int &mm, int &kk) {
        if (A.s1 == 1) {
            kk = e % KC;
            mm = e / KC;
        } else {
            mm = e % TS;
            kk = e / TS;
        }
    };
    auto b_pos = [&](int e, int &nn, int &kk) {
        if (B.s1 == 1) {
            nn = e % TS;
            kk = e / TS;
        } else {
            kk = e % KC;
            nn = e / KC;
        }
    };
    double ra[PT], rb[PT];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
            ra[r] = (gm < M && gk < K) ? a[(long long)gm * A.s0 + (long long)gk * A.s1] : 0.0;
            rb[r] = (gn < N && gkb < K) ? bp[(long long)gkb * B.s0 + (long long)gn * B.s1] : 0.0;
        }
    };
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            int mm, kk, nn, kb;
            a_pos(tid + kGThreads * r, mm, kk);
            b_pos(tid + kGThreads * r, nn, kb);
            As[kk][mm] = ra[r];
            Bs[kb][nn] = rb[r];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);   // in flight during the products below
        const int kn = K - k0 < KC ? K - k0 : KC;
#pragma unroll 2
        for (int kk = g; kk < kn; kk += G) {
            double av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][rm + 4 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][rn + 4 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
    // partial blocks of the groups (the staging LDS is free after the last
    // barrier), then one output per thread summed over the groups in order
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) sm[g * TS * TS + (rm + 4 * i) * TS + rn + 4 * j] = acc[i][j];
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) v += sm[q * TS * TS + tid];
    const int gm = m0 + tid / TS, gn = n0 + tid % TS;
    if (gm < M && gn < N) c[(long long)gm * C.s0 + (long long)gn * C.s1] = v;
}

// The widest of 64, 32, 16 output tiles that still gives every CU a
// workgroup (the smaller tiles trade operand reuse for parallelism; the
// 16-wide ones split k to keep some)
static void axis_gemm(int M, int N, int K, const AxOp &A, const AxOp &B, const AxOut &C, int batch, hipStream_t st) {
    auto tiles = [&](int t) { return (long long)((M + t - 1) / t) * ((N + t - 1) / t) * batch; };
    if (tiles(64) >= 256)
        hipLaunchKernelGGL(k_axis_mfma64<kMfmaKC>, dim3((N + 63) / 64, (M + 63) / 64, batch), dim3(kGThreads), 0, st, M,
                           N, K, A, B, C);
    else if (tiles(32) >= 256)
        hipLaunchKernelGGL(k_axis_gemm<32>, dim3((N + 31) / 32, (M + 31) / 32, batch), dim3(kGThreads), 0, st, M, N,
                           K, A, B, C);
    else
        hipLaunchKernelGGL(k_axis_gemm16s, dim3((N + 15) / 16, (M + 15) / 16, batch), dim3(kGThreads), 0, st, M, N, K,
                           A, B, C);
}

// Transform along one axis (length na, stride nb; x: nb = 1) of a field
// stored with x fastest: forward applies Q^T along the axis, inverse Q.
// Entry (mode k, index j) of Q is Q[j + na k].  Fields: ntab problems given
// by pointer tables, or (tables null) one field of `above` consecutive
// blocks of na * nb cells (x axis: `above` = rows of length na).
static void axis_transform(const double *Q, int na, int nb, int above, bool fwd, const double *in,
                           const double *const *in_tab, double *out, double *const *out_tab, int ntab,
                           hipStream_t st) {
    if (nb == 1) {
        // out(row, n) = sum_k in(row, k) B(k, n), B = Q (forward) or Q^T
        const int batch = in_tab ? ntab : 1;
        const AxOp a{in, in_tab, 0, na, 1};
        const AxOp b{Q, nullptr, 0, fwd ? 1 : na, fwd ? na : 1};
        const AxOut c{out, out_tab, 0, na, 1};
        axis_gemm(above, na, na, a, b, c, batch, st);
    } else {
        // per block: out(m, rest) = sum_k A(m, k) in(k, rest), A = Q^T or Q
        const int batch = in_tab ? ntab : above;
        const long long bs = in_tab ? 0 : (long long)na * nb;
        const AxOp a{Q, nullptr, 0, fwd ? na : 1, fwd ? 1 : na};
        const AxOp b{in, in_tab, bs, nb, 1};
        const AxOut c{out, out_tab, bs, nb, 1};
        axis_gemm(na, nb, na, a, b, c, batch, st);
    }
}

// t /= 1 - a lam + b lam^2, lam = lam_x(i) + lam_y(j) + lam_z(k)
__global__ void __launch_bounds__(kBlock) k_spectral_scale(Geo g, const double *__restrict__ lx,
                                                           const double *__restrict__ ly,
                                                           const double *__restrict__ lz, double a, double b,
                                                           double *__restrict__ t) {
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int c = xcd_block() * (int)blockDim.x + (int)threadIdx.x; c < (int)g.N; c += stride) {
        int i, j, k;
        cell_coords(g, c, i, j, k);
        const double lam = lx[i] + ly[j] + (lz ? lz[k] : 0.0);
        t[c] = t[c] / (1.0 - a * lam + b * lam * lam);
    }
}

// ---------------------------------------------------------------------------
// FFT transforms of periodic power-of-two axes.  With the DFT
// X_k = sum_j x_j e^{-2 pi i k j / n} of a pencil along such an axis
// (m = n / 2), the coefficients in the real Fourier basis are
//   mode 0 = X_0 / sqrt(n),  mode 2k-1 = sqrt(2/n) Re X_k,
//   mode 2k = -sqrt(2/n) Im X_k (0 < k < m),  mode n-1 = X_m / sqrt(n),
// and back x_j = Re sum_{k <= m} c_k e^{+2 pi i k j / n} with
// c_0 = mode 0 / sqrt(n), c_k = sqrt(2/n) (mode 2k-1 - i mode 2k),
// c_m = mode n-1 / sqrt(n): O(log n) operations per value where the basis
// product takes O(n).  A 256-thread workgroup takes P = 2048 / n complex
// pencils (each two real ones) into LDS and runs the log2 n radix-2 stages:
// decimation in time on bit-reversed input for the forward transform,
// decimation in frequency with bit-reversed output for the inverse.
// MODE 0: forward; 1: inverse; 2: forward, division by 1 - a lam + b lam^2,
// inverse (the last axis of the solve, whose pencils carry every mode of the
// other axes).  Pencil q of an axis: element j at
// (q / nin) ostride + q % nin + j nb.
// ---------------------------------------------------------------------------
struct FftAxis {
    int nb, nin, npen;
    long long ostride;
    const double *tw;   // cos, sin of 2 pi k / n
};
struct FftScale {         // MODE 2
    double a, b;
    const double *lx, *ly;   // eigenvalues of the other axes (ly null in 2D)
    const double *lz;        // eigenvalues of this axis' modes
    int nx;                  // 3D pencil q: (x, y) = (q % nx, q / nx); 2D: x = q
};

// Radix-2 stages in groups of up to three held in registers: the stages of
// half-sizes H, 2H, 4H (H = 2^r0) only pair elements within the sets
// {base + H m : m < 8}, base = hi 8H + lo (lo < H), so a thread loads a set,
// runs the group's butterflies on it (the twiddle of the pair (m, m + 2^r)
// at half-size H 2^r is W^(H (m mod 2^r) + lo)) and stores it back: one LDS
// round trip per three stages (and one twiddle read per stage: the others
// follow by eighth-turn rotations).  Element j of pencil p sits at
// p * W + j + j / 8 (one padding word per eight, so that the sets of
// consecutive threads fall in different LDS banks).
template <int LOGN>
struct FftLds {
    static constexpr int n = 1 << LOGN, P = 2048 / n, W = n + n / 8 + 1;
    __device__ static int at(int p, int j) { return p * W + j + (j >> 3); }
};

// DIT (forward, bit-reversed input) or DIF (inverse, bit-reversed output)
// group of S stages starting at half-size 2^r0; sgn: sign of the exponent.
template <int LOGN, int S, bool DIT>
__device__ inline void fft_group(double *re, double *im, const double *tw, double sgn, int r0) {
    using L = FftLds<LOGN>;
    constexpr int n = L::n, Z = 1 << S, NS = L::P * n / Z;
    static_assert(NS % kBlock == 0, "whole sets per thread");
    const int H = 1 << r0;
#pragma unroll
    for (int sg = (int)threadIdx.x; sg < NS; sg += kBlock) {
        const int p = sg / (n / Z), si = sg % (n / Z), lo = si & (H - 1), hi = si >> r0;
        const int j0 = hi * Z * H + lo;
        double xr[Z], xi[Z];
#pragma unroll
        for (int m = 0; m < Z; ++m) {
            xr[m] = re[L::at(p, j0 + H * m)];
            xi[m] = im[L::at(p, j0 + H * m)];
        }
#pragma unroll
        for (int rr = 0; rr < S; ++rr) {
            const int r = DIT ? rr : S - 1 - rr, hh = 1 << r, tstep = n / (2 * (H << r));
            // W^(H m' + lo) = W^lo e^(sgn 2 pi i e / 8) with e = m' 8 / 2^(r+1) < 4
            const double br = tw[2 * lo * tstep], bi = sgn * tw[2 * lo * tstep + 1];
#pragma unroll
            for (int m = 0; m < Z; ++m) {
                if (m & hh) continue;
                const int e = (m & (hh - 1)) * (8 >> (r + 1)), mm = m + hh;
                constexpr double c = 0.70710678118654752440;   // sqrt(1/2)
                double wr = br, wi = bi;
                if (e == 1) {
                    wr = c * (br - sgn * bi);
                    wi = c * (bi + sgn * br);
                } else if (e == 2) {
                    wr = -sgn * bi;
                    wi = sgn * br;
                } else if (e == 3) {
                    wr = -c * (br + sgn * bi);
                    wi = c * (sgn * br - bi);
                }
                if (DIT) {
                    const double tr = wr * xr[mm] - wi * xi[mm], ti = wr * xi[mm] + wi * xr[mm];
                    xr[mm] = xr[m] - tr;
                    xi[mm] = xi[m] - ti;
                    xr[m] += tr;
                    xi[m] += ti;
                } else {
                    const double dr = xr[m] - xr[mm], di = xi[m] - xi[mm];
                    xr[m] += xr[mm];
                    xi[m] += xi[mm];
                    xr[mm] = wr * dr - wi * di;
                    xi[mm] = wr * di + wi * dr;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < Z; ++m) {
            re[L::at(p, j0 + H * m)] = xr[m];
            im[L::at(p, j0 + H * m)] = xi[m];
        }
    }
    __syncthreads();
}

// all log2 n stages: DIT groups from the smallest half-size up, DIF groups
// from the largest down (three stages per group, the remainder last / first)
template <int LOGN, bool DIT>
__device__ inline void fft_run(double *re, double *im, const double *tw, double sgn) {
    constexpr int G = LOGN / 3, REM = LOGN % 3;
    if (DIT) {
#pragma unroll
        for (int g = 0; g < G; ++g) fft_group<LOGN, 3, true>(re, im, tw, sgn, 3 * g);
        if (REM) fft_group<LOGN, (REM ? REM : 1), true>(re, im, tw, sgn, 3 * G);
    } else {
        if (REM) fft_group<LOGN, (REM ? REM : 1), false>(re, im, tw, sgn, 3 * G);
#pragma unroll
        for (int g = G - 1; g >= 0; --g) fft_group<LOGN, 3, false>(re, im, tw, sgn, 3 * g);
    }
}

// the fields of one launch (blockIdx.y): up to two solves with the same operator
struct FftIo {
    const double *in[2];
    double *out[2];
};

// Two real pencils share one complex transform: pencil p of the workgroup's
// first half is the real part and pencil p + P the imaginary part of complex
// slot p, so a workgroup transforms 2P = 4096 / n real pencils with P complex
// ones.  Forward, the spectra separate as X_k = (Z_k + conj Z_(n-k)) / 2 and
// Y_k = (Z_k - conj Z_(n-k)) / 2i; backward, the two Hermitian spectra are
// joined as Z = X + i Y and the real and imaginary parts of the result are
// the two pencils.
template <int LOGN, int MODE>
__global__ void __launch_bounds__(kBlock) k_axis_fft(FftAxis ax, FftIo io, FftScale sc) {
    const double *__restrict__ in = io.in[blockIdx.y];
    double *__restrict__ out = io.out[blockIdx.y];
    using L = FftLds<LOGN>;
    constexpr int n = L::n, m = n / 2, P = L::P, P2 = 2 * P;
    __shared__ double re[P * L::W], im[P * L::W], tws[2 * n];
    __shared__ long long base[P2];
    const int tid = (int)threadIdx.x, q0 = (int)blockIdx.x * P2;
    const double s0 = 1.0 / sqrt((double)n), s1 = sqrt(2.0 / (double)n);
    for (int i = tid; i < 2 * n; i += kBlock) tws[i] = ax.tw[i];
    if (tid < P2) {
        const int q = q0 + tid;
        base[tid] = (long long)(q / ax.nin) * ax.ostride + q % ax.nin;
    }
    __syncthreads();
    auto at = [&](int pp, int j) { return base[pp] + (long long)j * ax.nb; };
    auto valid = [&](int pp) { return q0 + pp < ax.npen; };
    // element e of the workgroup's 2P pencils: the index contiguous in memory
    // runs fastest across the threads
    auto split = [&](int e, int &pp, int &j) {
        if (ax.nb == 1) {
            pp = e / n;
            j = e % n;
        } else {
            j = e / P2;
            pp = e % P2;
        }
    };
    auto brev = [](int j) { return (int)(__brev((unsigned)j) >> (32 - LOGN)); };
    if (MODE != 1) {
        // pencil pp into the real (pp < P) or imaginary part of slot pp mod P,
        // bit-reversed for the decimation-in-time forward transform
        for (int e = tid; e < P2 * n; e += kBlock) {
            int pp, j;
            split(e, pp, j);
            const double v = valid(pp) ? in[at(pp, j)] : 0.0;
            double *part = pp < P ? re : im;
            part[L::at(pp < P ? pp : pp - P, brev(j))] = v;
        }
    } else {
        // the half spectra c_k, d_k of pencils p and p + P (c_0, c_m real;
        // c_k = s1 (mode 2k-1 - i mode 2k)) as the full spectrum
        // Z_k = C_k + i D_k, with C_k = c_k / 2 and C_(n-k) = conj(c_k) / 2
        // for 0 < k < m
        for (int e = tid; e < P * (m + 1); e += kBlock) {
            const int p = e % P, k = e / P;
            double cr = 0.0, ci = 0.0, dr = 0.0, di = 0.0;
            auto coef = [&](int pp, double &vr, double &vi) {
                if (!valid(pp)) return;
                if (k == 0) {
                    vr = s0 * in[at(pp, 0)];
                } else if (k == m) {
                    vr = s0 * in[at(pp, n - 1)];
                } else {
                    vr = s1 * in[at(pp, 2 * k - 1)];
                    vi = -s1 * in[at(pp, 2 * k)];
                }
            };
            coef(p, cr, ci);
            coef(p + P, dr, di);
            if (k == 0 || k == m) {
                re[L::at(p, k)] = cr;
                im[L::at(p, k)] = dr;
            } else {
                re[L::at(p, k)] = 0.5 * (cr - di);
                im[L::at(p, k)] = 0.5 * (ci + dr);
                re[L::at(p, n - k)] = 0.5 * (cr + di);
                im[L::at(p, n - k)] = 0.5 * (dr - ci);
            }
        }
    }
    __syncthreads();
    if (MODE != 1) fft_run<LOGN, true>(re, im, tws, -1.0);
    if (MODE == 0) {
        for (int e = tid; e < P2 * n; e += kBlock) {
            int pp, c;
            split(e, pp, c);
            if (!valid(pp)) continue;
            const int p = pp < P ? pp : pp - P, k = c == n - 1 ? m : (c + 1) / 2, kn = (n - k) & (n - 1);
            const double zr = re[L::at(p, k)], zi = im[L::at(p, k)];
            const double wr = re[L::at(p, kn)], wi = im[L::at(p, kn)];
            // X_k of pencil p (pp < P) or Y_k of pencil p + P
            const double xr = pp < P ? 0.5 * (zr + wr) : 0.5 * (zi + wi);
            const double xi = pp < P ? 0.5 * (zi - wi) : 0.5 * (wr - zr);
            const double v = c == 0 || c == n - 1 ? s0 * xr : ((c & 1) ? s1 * xr : -s1 * xi);
            out[at(pp, c)] = v;
        }
        return;
    }
    if (MODE == 2) {
        // X_k, Y_k of the slot's two pencils divided by 1 - a lam + b lam^2
        // (with the inverse's 1 / n), joined again as Z_k = X_k + i Y_k and
        // Z_(n-k) = conj X_k + i conj Y_k
        const double inv_n = 1.0 / (double)n;
        auto gain = [&](int pp, int k) {
            const int q = q0 + pp;
            if (q >= ax.npen) return 0.0;
            const double lxy = sc.ly ? sc.lx[q % sc.nx] + sc.ly[q / sc.nx] : sc.lx[q];
            const double lam = lxy + sc.lz[k == 0 ? 0 : (k == m ? n - 1 : 2 * k - 1)];
            return inv_n / (1.0 - sc.a * lam + sc.b * lam * lam);
        };
        for (int e = tid; e < P * (m + 1); e += kBlock) {
            const int p = e % P, k = e / P, kn = (n - k) & (n - 1);
            const double zr = re[L::at(p, k)], zi = im[L::at(p, k)];
            const double wr = re[L::at(p, kn)], wi = im[L::at(p, kn)];
            const double gx = gain(p, k), gy = gain(p + P, k);
            const double xr = gx * (0.5 * (zr + wr)), xi = gx * (0.5 * (zi - wi));
            const double yr = gy * (0.5 * (zi + wi)), yi = gy * (0.5 * (wr - zr));
            re[L::at(p, k)] = xr - yi;
            im[L::at(p, k)] = xi + yr;
            if (kn != k) {
                re[L::at(p, kn)] = xr + yi;
                im[L::at(p, kn)] = yr - xi;
            }
        }
        __syncthreads();
    }
    fft_run<LOGN, false>(re, im, tws, 1.0);
    for (int e = tid; e < P2 * n; e += kBlock) {
        int pp, j;
        split(e, pp, j);
        if (!valid(pp)) continue;
        const int p = pp < P ? pp : pp - P;
        out[at(pp, j)] = pp < P ? re[L::at(p, brev(j))] : im[L::at(p, brev(j))];
    }
}

// Pencils of axis a of the grid n[0..2] (x fastest).
static FftAxis fft_axis_of(const Spectral &S, int a) {
    const int nx = S.n[0], ny = S.n[1], nz = S.dim == 3 ? S.n[2] : 1;
    FftAxis ax;
    ax.tw = S.tw[a];
    if (a == 0) {
        ax.nb = 1;
        ax.nin = 1;
        ax.ostride = nx;
        ax.npen = ny * nz;
    } else if (a == 1) {
        ax.nb = nx;
        ax.nin = nx;
        ax.ostride = (long long)nx * ny;
        ax.npen = nx * nz;
    } else {
        ax.nb = nx * ny;
        ax.nin = nx * ny;
        ax.ostride = 0;
        ax.npen = nx * ny;
    }
    return ax;
}

template <int LOGN>
static void fft_launch(const FftAxis &ax, int mode, const FftIo &io, int nf, const FftScale &sc, hipStream_t st) {
    constexpr int P2 = 4096 >> LOGN;   // real pencils per workgroup
    const dim3 grid((ax.npen + P2 - 1) / P2, nf);
    if (mode == 0)
        hipLaunchKernelGGL((k_axis_fft<LOGN, 0>), grid, dim3(kBlock), 0, st, ax, io, sc);
    else if (mode == 1)
        hipLaunchKernelGGL((k_axis_fft<LOGN, 1>), grid, dim3(kBlock), 0, st, ax, io, sc);
    else
        hipLaunchKernelGGL((k_axis_fft<LOGN, 2>), grid, dim3(kBlock), 0, st, ax, io, sc);
}

// transform along axis a of nf fields (io.in / io.out [0, nf))
static void fft_transform(const Spectral &S, int a, int mode, const FftIo &io, int nf, const FftScale &sc,
                          hipStream_t st) {
    const FftAxis ax = fft_axis_of(S, a);
    switch (S.fft[a]) {
        case 4: fft_launch<4>(ax, mode, io, nf, sc, st); break;
        case 5: fft_launch<5>(ax, mode, io, nf, sc, st); break;
        case 6: fft_launch<6>(ax, mode, io, nf, sc, st); break;
        case 7: fft_launch<7>(ax, mode, io, nf, sc, st); break;
        case 8: fft_launch<8>(ax, mode, io, nf, sc, st); break;
        default: fft_launch<9>(ax, mode, io, nf, sc, st); break;
    }
}

bool spectral_all_fft(const Spectral &S) {
    if (!S.on || S.dense) return false;
    for (int a = 0; a < S.dim; ++a)
        if (!S.fft[a]) return false;
    return true;
}

// Both fields in every launch: every axis is an FFT axis.
hipError_t spectral_solve2(Spectral &S, double a, double b, const double *const r[2], double *const x[2],
                           double *const t0[2], double *const t1[2], hipStream_t st) {
    const int nx = S.n[0], ny = S.n[1], nz = S.dim == 3 ? S.n[2] : 1, last = S.dim - 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_prof) {
        prof_slot(K_CH_SPECTRAL, 2.0 * 8.0 * nx * ny * nz * 2.0 * (2 * S.dim - 1), &e0, &e1);
        (void)hipEventRecord(e0, st);
    }
    const FftScale none{0.0, 0.0, nullptr, nullptr, nullptr, 1};
    FftIo io{{r[0], r[1]}, {t0[0], t0[1]}};
    fft_transform(S, 0, 0, io, 2, none, st);
    double *cur[2] = {t0[0], t0[1]}, *oth[2] = {t1[0], t1[1]};
    auto step = [&](int ax, int mode, const FftScale &sc) {
        const FftIo f{{cur[0], cur[1]}, {oth[0], oth[1]}};
        fft_transform(S, ax, mode, f, 2, sc, st);
        std::swap(cur[0], oth[0]);
        std::swap(cur[1], oth[1]);
    };
    for (int ax = 1; ax < last; ++ax) step(ax, 0, none);
    const FftScale sc{a, b, (const double *)S.lam[0], S.dim == 3 ? (const double *)S.lam[1] : nullptr,
                      (const double *)S.lam[last], nx};
    step(last, 2, sc);
    for (int ax = last - 1; ax >= 1; --ax) step(ax, 1, none);
    const FftIo fin{{cur[0], cur[1]}, {x[0], x[1]}};
    fft_transform(S, 0, 1, fin, 2, none, st);
    if (e1) (void)hipEventRecord(e1, st);
    return hipGetLastError();
}
static_assert(kFftMinLog == 4 && kFftMaxLog == 9, "fft_transform instantiates 2^4 .. 2^9");

hipError_t spectral_solve(Spectral &S, double a, double b, const double *r, double *x, double *t0, double *t1,
                          hipStream_t st, std::string &err) {
    (void)err;
    const int nx = S.n[0], ny = S.n[1], nz = S.dim == 3 ? S.n[2] : 1, last = S.dim - 1;
    auto fft_on = [&](int ax) { return !S.dense && S.fft[ax] != 0; };
    const bool fused = fft_on(last);   // forward, division and inverse along the last axis in one pass
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_prof) {
        const double N3 = (double)nx * ny * nz;
        prof_slot(K_CH_SPECTRAL, 8.0 * N3 * 2.0 * (fused ? 2 * S.dim - 1 : 2 * S.dim + 1), &e0, &e1);
        (void)hipEventRecord(e0, st);
    }
    const FftScale none{0.0, 0.0, nullptr, nullptr, nullptr, 1};
    auto transform = [&](int ax, bool fwd, const double *in, double *out) {
        if (fft_on(ax)) {
            fft_transform(S, ax, fwd ? 0 : 1, FftIo{{in, in}, {out, out}}, 1, none, st);
        } else if (ax == 0) {
            axis_transform(S.Q[0], nx, 1, ny * nz, fwd, in, nullptr, out, nullptr, 0, st);
        } else if (ax == 1) {
            axis_transform(S.Q[1], ny, nx, nz, fwd, in, nullptr, out, nullptr, 0, st);
        } else {
            axis_transform(S.Q[2], nz, nx * ny, 1, fwd, in, nullptr, out, nullptr, 0, st);
        }
    };
    // forward: x, then y (3D), into t0 / t1
    transform(0, true, r, t0);
    double *cur = t0, *oth = t1;
    for (int ax = 1; ax < last; ++ax) {
        transform(ax, true, cur, oth);
        std::swap(cur, oth);
    }
    if (fused) {
        const FftScale sc{a, b, (const double *)S.lam[0], S.dim == 3 ? (const double *)S.lam[1] : nullptr,
                          (const double *)S.lam[last], nx};
        fft_transform(S, last, 2, FftIo{{cur, cur}, {oth, oth}}, 1, sc, st);
        std::swap(cur, oth);
    } else {
        transform(last, true, cur, oth);
        std::swap(cur, oth);
        Geo g;
        g.n[0] = nx;
        g.n[1] = ny;
        g.n[2] = nz;
        g.per[0] = g.per[1] = g.per[2] = 1;
        g.N = (long long)nx * ny * nz;
        hipLaunchKernelGGL(k_spectral_scale, dim3(grid_for(g.N)), dim3(kBlock), 0, st, g, (const double *)S.lam[0],
                           (const double *)S.lam[1], (const double *)(S.dim == 3 ? S.lam[2] : nullptr), a, b, cur);
        transform(last, false, cur, oth);
        std::swap(cur, oth);
    }
    // inverse: y (3D), then x into the result
    for (int ax = last - 1; ax >= 1; --ax) {
        transform(ax, false, cur, oth);
        std::swap(cur, oth);
    }
    transform(0, false, cur, x);
    if (e1) (void)hipEventRecord(e1, st);
    return hipGetLastError();
}

// t_p /= 1 - a_p lam + b_p lam^2, lam = (lam_x(i) + lam_y(j)) / h_p^2;
// blockIdx.y = problem of the group
__global__ void __launch_bounds__(kBlock) k_spectral_scale_batch(int nx, int ny, const double *__restrict__ lx,
                                                                 const double *__restrict__ ly,
                                                                 const double *__restrict__ abh,
                                                                 double *const *__restrict__ t) {
    const int p = (int)blockIdx.y;
    const double a = abh[3 * p], b = abh[3 * p + 1], ih2 = abh[3 * p + 2];
    double *tp = t[p];
    const int n = nx * ny, stride = (int)(gridDim.x * blockDim.x);
    for (int c = (int)(blockIdx.x * blockDim.x + threadIdx.x); c < n; c += stride) {
        const int j = c / nx, i = c - j * nx;
        const double lam = ih2 * (lx[i] + ly[j]);
        tp[c] = tp[c] / (1.0 - a * lam + b * lam * lam);
    }
}

hipError_t spectral_batch_solve(const std::vector<SpecGroup> &groups, hipStream_t st) {
    for (const SpecGroup &G : groups) {
        const int nx = G.nx, ny = G.ny, m = G.m;
        axis_transform(G.Q[0], nx, 1, ny, true, nullptr, G.r, nullptr, G.t0, m, st);
        axis_transform(G.Q[1], ny, nx, 1, true, nullptr, (const double *const *)G.t0, nullptr, G.t1, m, st);
        const int bx = std::min((nx * ny + kBlock - 1) / kBlock, 64);
        hipLaunchKernelGGL(k_spectral_scale_batch, dim3(bx, m), dim3(kBlock), 0, st, nx, ny, (const double *)G.lam[0],
                           (const double *)G.lam[1], (const double *)G.abh, (double *const *)G.t1);
        axis_transform(G.Q[1], ny, nx, 1, false, nullptr, (const double *const *)G.t1, nullptr, G.t0, m, st);
        axis_transform(G.Q[0], nx, 1, ny, false, nullptr, (const double *const *)G.t0, nullptr, G.x, m, st);
    }
    return hipGetLastError();
}

}  // namespace chns
