// HIP kernels of the one-site TDVP sweep for gfx950 (complex FP64).
//
// Paper: pyTTN (arXiv 2503.15460).  The contractions implement the node
// effective generator of the local equation of motion (Sec. II C,
// (H_eff A)_{I,i} = sum_r c_r h_{IJ} H_{ij} A_{J,j}), the SPO and mean-field
// recursions (Sec. II B 1 / II C) as conj-contractions of a node tensor with
// the operator-applied tensor, the QR gauge shifts of the canonical form
// (Sec. II A), and the local exponentials of the projector-splitting sweep.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"

namespace ttn {

// ------------------------------------------------------------ complex helpers
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ void cfma(double2 &acc, double2 a, double2 b) {  // acc += a*b
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfmac(double2 &acc, double2 a, double2 b) {  // acc += conj(a)*b
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
// single-precision forms for the FP32 contraction mode
__device__ __forceinline__ void cfma(float2 &acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfmac(float2 &acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(-a.y, b.x, acc.y);
}
// element conversions between the storage type of a buffer and the compute type
template <typename T> __device__ __forceinline__ T cvt(double2 a);
template <> __device__ __forceinline__ double2 cvt<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 cvt<float2>(double2 a) {
    return make_float2((float)a.x, (float)a.y);
}
template <typename T> __device__ __forceinline__ T cvt(float2 a);
template <> __device__ __forceinline__ double2 cvt<double2>(float2 a) { return make_double2(a.x, a.y); }
template <> __device__ __forceinline__ float2 cvt<float2>(float2 a) { return a; }
template <typename T> __device__ __forceinline__ T czero();
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.0f, 0.0f); }

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ double blk_sum1(double v, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Last-block reduction: every block stores its partials, the block that
// finishes last (atomic ticket) sums them in a fixed order.
__device__ bool last_block_ticket(unsigned *counter) {
    __shared__ int is_last;
    __syncthreads();  // the block's partial-sum stores have reached L2
    if (threadIdx.x == 0) {
        __threadfence();  // release, covering the block's stores ordered by the barrier
        const unsigned prev = atomicAdd(counter, 1u);
        is_last = (prev == gridDim.x - 1);
        if (is_last) __threadfence();  // acquire before reading the other blocks' partials
    }
    __syncthreads();
    return is_last != 0;
}


// Last-block reduction of per-block partial sums: out[q] = sum_b part[b * stride + q]
// for q < K.  Chunks of the partials are first staged in LDS with independent
// loads (all threads), then 8 lanes per value sum strided partials in a fixed
// order and combine them by shuffles.  stage: LDS scratch of KRY_STAGE doubles.
constexpr int KRY_STAGE = 4096;
__device__ void blk_reduce_staged(const double *part, int nb, int stride, int K, double *out, double *stage) {
    const int tid = threadIdx.x;
    const int ch = max(1, min((int)blockDim.x / 8, KRY_STAGE / nb));  // values per chunk
    for (int v0 = 0; v0 < K; v0 += ch) {
        const int cnt = min(ch, K - v0);
        for (int e = tid; e < nb * cnt; e += blockDim.x) {
            const int b = e / cnt, t = e - b * cnt;
            stage[e] = part[(size_t)b * stride + v0 + t];
        }
        __syncthreads();
        const int t = tid / 8, sub = tid & 7;
        double acc = 0.0;
        if (t < cnt)
            for (int b = sub; b < nb; b += 8) acc += stage[b * cnt + t];
        acc += __shfl_xor(acc, 4, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 1, 64);
        if (t < cnt && sub == 0) out[v0 + t] = acc;
        __syncthreads();
    }
}

// ============================================================ mode products
// Y[l,i,r] = sum_j M[i,j] X[l,j,r] for one (L, n, R) geometry.  TS is the
// element type read (the FP64 input at stage 0, the temporaries afterwards), T
// the compute and temporary type (double2, or float2 in the FP32 mode).
template <typename TS, typename T>
__global__ void __launch_bounds__(256) k_mode_stage(ProgView p, int stage, const TS *__restrict__ in, int ldn) {
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    const int nf = E->nf;
    if (nf <= stage) return;
    const int s = E->slot[stage];
    const double2 *__restrict__ M = E->M[stage];
    const int n = p.g.dims[s];
    const uint32_t R = (uint32_t)p.g.R[s];
    const uint32_t N = (uint32_t)p.g.N;
    T *tmp = reinterpret_cast<T *>(p.tmp);
    const TS *__restrict__ src =
        stage == 0 ? in + (int64_t)E->src * p.in_stride
                   : reinterpret_cast<const TS *>(tmp + (2 * (int64_t)e + ((stage - 1) & 1)) * N);
    T *__restrict__ dst = tmp + (2 * (int64_t)e + (stage & 1)) * N;
    const int blo = E->lo[stage], bhi = E->hi[stage];
    extern __shared__ double2 smt_raw[];
    T *smt = reinterpret_cast<T *>(smt_raw);
    const bool lds = n <= ldn;  // LDS holds ldn*ldn elements
    if (lds) {
        for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
            int i = q / n, j = q - i * n;
            smt[j * n + i] = cvt<T>(M[q]);
        }
        __syncthreads();
    }
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
        uint32_t r = idx % R, t = idx / R;
        uint32_t i = t % n, l = t / n;
        const TS *xp = src + (size_t)l * n * R + r;
        T acc = czero<T>();
        const int j0 = max(0, (int)i - blo), j1 = min(n - 1, (int)i + bhi);
        if (lds) {
            for (int j = j0; j <= j1; ++j) cfma(acc, smt[j * n + i], cvt<T>(xp[(size_t)j * R]));
        } else {
            const double2 *mr = M + (size_t)i * n;
            for (int j = j0; j <= j1; ++j) cfma(acc, cvt<T>(mr[j]), cvt<T>(xp[(size_t)j * R]));
        }
        dst[idx] = acc;
    }
}

// Tiled mode product for stages whose factors are all dense with n <= 64.
// A work-group computes all rows i (padded to NP = RG * TI) of CW = CG * TC
// columns c = l * R + r, with the contraction index j staged through LDS in
// chunks of KC together with the matching columns of M.  Thread (cg, rg) keeps
// a TI x TC register block: rows rg + RG * a, columns cg + CG * b, so that each
// LDS value feeds TI or TC complex FMAs.
constexpr int MT_KC = 16;

template <typename TS, typename T, int TI, int RG>
__global__ void __launch_bounds__(256) k_mode_tile(ProgView p, int stage, const TS *__restrict__ in) {
    constexpr int CG = 256 / RG;
    constexpr int TC = 4;
    constexpr int CW = CG * TC;
    constexpr int NP = RG * TI;
    constexpr int KC = MT_KC;
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    if (E->nf <= stage) return;
    const int s = E->slot[stage];
    const int n = p.g.dims[s];
    const uint32_t R = (uint32_t)p.g.R[s];
    const uint32_t N = (uint32_t)p.g.N;
    const uint32_t ncol = N / (uint32_t)n;
    const uint32_t c0 = blockIdx.x * (uint32_t)CW;
    if (c0 >= ncol) return;
    const double2 *__restrict__ M = E->M[stage];
    T *tmp = reinterpret_cast<T *>(p.tmp);
    const TS *__restrict__ src =
        stage == 0 ? in + (int64_t)E->src * p.in_stride
                   : reinterpret_cast<const TS *>(tmp + (2 * (int64_t)e + ((stage - 1) & 1)) * N);
    T *__restrict__ dst = tmp + (2 * (int64_t)e + (stage & 1)) * N;
    __shared__ T Ms[KC * NP];  // Ms[k * NP + i] = M[i][j0 + k]
    __shared__ T Xs[KC * CW];  // Xs[k * CW + cc] = X[j0 + k] of column c0 + cc
    const int tid = threadIdx.x;
    const int cg = tid % CG, rg = tid / CG;
    T acc[TI][TC];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TC; ++b) acc[a][b] = czero<T>();
    const uint32_t nR = (uint32_t)n * R;
    for (int j0 = 0; j0 < n; j0 += KC) {
        __syncthreads();
        for (int q = tid; q < KC * NP; q += 256) {
            const int k = q / NP, i = q - k * NP;
            Ms[q] = (i < n && j0 + k < n) ? cvt<T>(M[(size_t)i * n + j0 + k]) : czero<T>();
        }
        if (R == 1) {  // columns are rows of a row-major (ncol, n) matrix: j fastest
            for (int q = tid; q < KC * CW; q += 256) {
                const int k = q % KC, cc = q / KC;
                const uint32_t c = c0 + cc;
                Xs[k * CW + cc] = (c < ncol && j0 + k < n) ? cvt<T>(src[(size_t)c * n + j0 + k]) : czero<T>();
            }
        } else {
            for (int q = tid; q < KC * CW; q += 256) {
                const int k = q / CW, cc = q - k * CW;
                const uint32_t c = c0 + cc;
                T v = czero<T>();
                if (c < ncol && j0 + k < n) {
                    const uint32_t l = c / R, r = c - l * R;
                    v = cvt<T>(src[(size_t)l * nR + (size_t)(j0 + k) * R + r]);
                }
                Xs[q] = v;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < KC; ++k) {
            T av[TI], bv[TC];
#pragma unroll
            for (int a = 0; a < TI; ++a) av[a] = Ms[k * NP + rg + RG * a];
#pragma unroll
            for (int b = 0; b < TC; ++b) bv[b] = Xs[k * CW + cg + CG * b];
#pragma unroll
            for (int a = 0; a < TI; ++a)
#pragma unroll
                for (int b = 0; b < TC; ++b) cfma(acc[a][b], av[a], bv[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < TC; ++b) {
        const uint32_t c = c0 + cg + CG * b;
        if (c >= ncol) continue;
        const uint32_t l = c / R, r = c - l * R;
        T *yp = dst + (size_t)l * nR + r;
#pragma unroll
        for (int a = 0; a < TI; ++a) {
            const int i = rg + RG * a;
            if (i < n) yp[(size_t)i * R] = acc[a][b];
        }
    }
}

// ------------------------------------------------------------ BF16x3 MFMA stage
// Complex mode product as one real GEMM per column tile.  Realified with
// interleaved parts: row 2i+a and column 2j+b of Mt hold the 2x2 real block
// [[Re, -Im], [Im, Re]] of M[i][j]; Xt row 2j+b holds part b of X[j].  The
// realified dimension RD = 32 RT covers 2n.  Every FP32 operand is split into
// bf16 hi + lo and the product taken as hi*hi + hi*lo + lo*hi
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation; the dropped lo*lo term is
// ~2^-16 relative).  Mt of every entry is split once per stage launch by
// k_mfma_prep; a work-group (4 waves x 32 columns) stages chunks of 32
// realified K of Mt and Xt in LDS; each wave holds all RT row tiles of its
// columns.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned u32x2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
// eight consecutive bf16 of an MFMA K=16 operand from two groups of four
__device__ __forceinline__ bf8v join_bf4(bf4 a, bf4 b) {
    const u32x2v x = __builtin_bit_cast(u32x2v, a), y = __builtin_bit_cast(u32x2v, b);
    const u32x4v u = {x[0], x[1], y[0], y[1]};
    return __builtin_bit_cast(bf8v, u);
}

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ void bf16_split(float x, unsigned short &hi, unsigned short &lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - __uint_as_float((unsigned)hi << 16));
}

constexpr int MF_CW = 128;  // columns per work-group
constexpr int MF_KC = 32;   // realified K per LDS chunk
constexpr int MF_KP = MF_KC / 4 + 1;  // bf4 per LDS row (one of padding)

// Mt hi / lo of every entry with a factor at this stage: mprep[(e * 2 + h) * RD * RD + row * RD + col]
__global__ void __launch_bounds__(256) k_mfma_prep(ProgView p, int stage, int RD, unsigned short *mprep) {
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    if (E->nf <= stage) return;
    const int n = p.g.dims[E->slot[stage]];
    const double2 *M = E->M[stage];
    unsigned short *hi = mprep + (size_t)e * 2 * RD * RD, *lo = hi + (size_t)RD * RD;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < RD * RD; q += gridDim.x * blockDim.x) {
        const int row = q / RD, col = q - row * RD;
        const int i = row >> 1, j = col >> 1, a = row & 1, b2 = col & 1;
        float v = 0.0f;
        if (i < n && j < n) {
            const double2 m = M[(size_t)i * n + j];
            v = a == 0 ? (b2 == 0 ? (float)m.x : -(float)m.y) : (b2 == 0 ? (float)m.y : (float)m.x);
        }
        unsigned short h, l;
        bf16_split(v, h, l);
        hi[q] = h;
        lo[q] = l;
    }
}

template <typename TS, int RT>
__global__ void __launch_bounds__(256) k_mode_mfma(ProgView p, int stage, const TS *__restrict__ in,
                                                   const unsigned short *__restrict__ mprep) {
    constexpr int RD = 32 * RT;
    __shared__ bf4 Ah[RD * MF_KP], Al[RD * MF_KP];
    __shared__ bf4 Bh[MF_CW * MF_KP], Bl[MF_CW * MF_KP];  // [col][k / 4]
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    if (E->nf <= stage) return;
    const int s = E->slot[stage];
    const int n = p.g.dims[s];
    const uint32_t R = (uint32_t)p.g.R[s];
    const uint32_t N = (uint32_t)p.g.N;
    const uint32_t ncol = N / (uint32_t)n;
    const uint32_t c0 = blockIdx.x * (uint32_t)MF_CW;
    if (c0 >= ncol) return;
    const unsigned short *mhi = mprep + (size_t)e * 2 * RD * RD, *mlo = mhi + (size_t)RD * RD;
    float2 *tmp = reinterpret_cast<float2 *>(p.tmp);
    const TS *__restrict__ src =
        stage == 0 ? in + (int64_t)E->src * p.in_stride
                   : reinterpret_cast<const TS *>(tmp + (2 * (int64_t)e + ((stage - 1) & 1)) * N);
    float2 *__restrict__ dst = tmp + (2 * (int64_t)e + (stage & 1)) * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nR = (uint32_t)n * R;
    f32x16 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
    const int kmax = min(RD, 2 * n);
    // software pipeline: the global loads of chunk k0 + 32 are in flight while
    // the matrix cores work on chunk k0
    constexpr int MQ = RD * (MF_KC / 4) / 256;   // bf4 of each Mt chunk array per thread
    constexpr int XQ = MF_CW * (MF_KC / 2) / 256;  // complex X values per thread
    bf4 mh[MQ], ml[MQ];
    float2 xv[XQ];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            const int row = q / (MF_KC / 4), g = q - row * (MF_KC / 4);
            mh[u] = *reinterpret_cast<const bf4 *>(mhi + (size_t)row * RD + k0 + 4 * g);
            ml[u] = *reinterpret_cast<const bf4 *>(mlo + (size_t)row * RD + k0 + 4 * g);
        }
        const int j0 = k0 / 2;
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            const int q = tid + 256 * u;
            int cc, jj;
            if (R == 1) {  // columns are rows of a row-major (ncol, n) matrix: j fastest
                jj = q % (MF_KC / 2);
                cc = q / (MF_KC / 2);
            } else {
                cc = q % MF_CW;
                jj = q / MF_CW;
            }
            const int j = j0 + jj;
            const uint32_t c = c0 + cc;
            float2 v = make_float2(0.0f, 0.0f);
            if (c < ncol && j < n) {
                const uint32_t l = c / R, r = c - l * R;
                const TS x = src[(size_t)l * nR + (size_t)j * R + r];
                v = make_float2((float)x.x, (float)x.y);
            }
            xv[u] = v;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            const int row = q / (MF_KC / 4), g = q - row * (MF_KC / 4);
            Ah[row * MF_KP + g] = mh[u];
            Al[row * MF_KP + g] = ml[u];
        }
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            const int q = tid + 256 * u;
            int cc, jj;
            if (R == 1) {
                jj = q % (MF_KC / 2);
                cc = q / (MF_KC / 2);
            } else {
                cc = q % MF_CW;
                jj = q / MF_CW;
            }
            unsigned short hr, lr, hi2, li;
            bf16_split(xv[u].x, hr, lr);
            bf16_split(xv[u].y, hi2, li);
            short *bh = reinterpret_cast<short *>(Bh + cc * MF_KP);
            short *bl = reinterpret_cast<short *>(Bl + cc * MF_KP);
            bh[2 * jj] = (short)hr;
            bh[2 * jj + 1] = (short)hi2;
            bl[2 * jj] = (short)lr;
            bl[2 * jj + 1] = (short)li;
        }
    };
    load_chunk(0);
    store_chunk();
    __syncthreads();
    const int col = wave * 32 + (lane & 31);
    const int kg = 2 * (lane >> 5);  // this lane's two groups of 4 within each 16-wide K step
    for (int k0 = 0; k0 < kmax; k0 += MF_KC) {
        const bool more = k0 + MF_KC < kmax;
        if (more) load_chunk(k0 + MF_KC);
#pragma unroll
        for (int ks = 0; ks < MF_KC / 4; ks += 4) {
            const bf8v bh = join_bf4(Bh[col * MF_KP + ks + kg], Bh[col * MF_KP + ks + kg + 1]);
            const bf8v bl = join_bf4(Bl[col * MF_KP + ks + kg], Bl[col * MF_KP + ks + kg + 1]);
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const int row = t * 32 + (lane & 31);
                const bf8v ah = join_bf4(Ah[row * MF_KP + ks + kg], Ah[row * MF_KP + ks + kg + 1]);
                const bf8v al = join_bf4(Al[row * MF_KP + ks + kg], Al[row * MF_KP + ks + kg + 1]);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[t], 0, 0, 0);
            }
        }
        if (more) {
            __syncthreads();
            store_chunk();
            __syncthreads();
        }
    }
    // the lane holds rows t*32 + (v/4)*8 + (lane/32)*4 + v%4: pairs (2i, 2i+1) in (v, v+1), v even
    const uint32_t c = c0 + wave * 32 + (lane & 31);
    if (c < ncol) {
        const uint32_t l = c / R, r = c - l * R;
        float2 *yp = dst + (size_t)l * nR + r;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 16; v += 2) {
                const int i = (t * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3)) >> 1;
                if (i < n) yp[(size_t)i * R] = make_float2(acc[t][v], acc[t][v + 1]);
            }
    }
}

// ------------------------------------------------------------ FP32 MFMA stage
// The same realified mode product on the FP32 matrix cores
// (v_mfma_f32_32x32x2f32) for the FP32 mode: row 2i+a, column 2j+b of the A
// operand hold the 2x2 real block [[Re, -Im], [Im, Re]] of M[i][j] (built in
// LDS from the FP64 factor), column c of the B operand the (Re, Im) parts of
// X[j] at rows 2j, 2j+1.  The realified K order is permuted so that one
// 16-byte LDS read feeds four K steps: in group g of eight, K step s of lane
// half h takes realified index 8g + 4h + s (A and B alike, so the sum is
// unchanged).  Work-group: 4 waves x 32 columns, every wave all RT row tiles of
// its columns; chunks of 16 complex j pass through LDS, the next chunk's
// global loads in flight during the current chunk's products.
constexpr int M32_CW = 128;             // columns per work-group
constexpr int M32_KC = 32;              // realified K per chunk
constexpr int M32_LD = M32_KC + 4;      // floats per LDS row (16-byte reads conflict-free)

template <typename TS, int RT>
__global__ void __launch_bounds__(256) k_mode_mfma32(ProgView p, int stage, const TS *__restrict__ in) {
    constexpr int RD = 32 * RT;
    __shared__ float As[RD * M32_LD];
    __shared__ float Bs[M32_CW * M32_LD];
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    if (E->nf <= stage) return;
    const int s = E->slot[stage];
    const int n = p.g.dims[s];
    const uint32_t R = (uint32_t)p.g.R[s];
    const uint32_t N = (uint32_t)p.g.N;
    const uint32_t ncol = N / (uint32_t)n;
    const uint32_t c0 = blockIdx.x * (uint32_t)M32_CW;
    if (c0 >= ncol) return;
    const double2 *__restrict__ M = E->M[stage];
    float2 *tmp = reinterpret_cast<float2 *>(p.tmp);
    const TS *__restrict__ src =
        stage == 0 ? in + (int64_t)E->src * p.in_stride
                   : reinterpret_cast<const TS *>(tmp + (2 * (int64_t)e + ((stage - 1) & 1)) * N);
    float2 *__restrict__ dst = tmp + (2 * (int64_t)e + (stage & 1)) * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nR = (uint32_t)n * R;
    f32x16 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
    const int kmax = min(RD, 2 * n);
    constexpr int JC = M32_KC / 2;               // complex j per chunk
    constexpr int MQ = (RD / 2) * JC / 256;      // complex M values per thread (= RT)
    constexpr int XQ = M32_CW * JC / 256;        // complex X values per thread
    double2 mv[MQ];
    TS xv[XQ];
    auto xmap = [&](int q, int &cc, int &jj) {
        if (R == 1) {  // columns are rows of a row-major (ncol, n) matrix: j fastest
            jj = q % JC;
            cc = q / JC;
        } else {
            cc = q % M32_CW;
            jj = q / M32_CW;
        }
    };
    auto load_chunk = [&](int k0) {
        const int j0 = k0 / 2;
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            const int i = q / JC, jj = q - i * JC;
            const int j = j0 + jj;
            mv[u] = (i < n && j < n) ? M[(size_t)i * n + j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            int cc, jj;
            xmap(tid + 256 * u, cc, jj);
            const int j = j0 + jj;
            const uint32_t c = c0 + cc;
            TS v{};
            if (c < ncol && j < n) {
                const uint32_t l = c / R, r = c - l * R;
                v = src[(size_t)l * nR + (size_t)j * R + r];
            }
            xv[u] = v;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            const int i = q / JC, jj = q - i * JC;
            const float re = (float)mv[u].x, im = (float)mv[u].y;
            *reinterpret_cast<float2 *>(As + (2 * i) * M32_LD + 2 * jj) = make_float2(re, -im);
            *reinterpret_cast<float2 *>(As + (2 * i + 1) * M32_LD + 2 * jj) = make_float2(im, re);
        }
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            int cc, jj;
            xmap(tid + 256 * u, cc, jj);
            *reinterpret_cast<float2 *>(Bs + cc * M32_LD + 2 * jj) = make_float2((float)xv[u].x, (float)xv[u].y);
        }
    };
    load_chunk(0);
    store_chunk();
    __syncthreads();
    const int l32 = lane & 31, h = lane >> 5;
    const int col = wave * 32 + l32;
    for (int k0 = 0; k0 < kmax; k0 += M32_KC) {
        const bool more = k0 + M32_KC < kmax;
        if (more) load_chunk(k0 + M32_KC);
#pragma unroll
        for (int g = 0; g < M32_KC / 8; ++g) {
            const f32x4v b = *reinterpret_cast<const f32x4v *>(Bs + col * M32_LD + 8 * g + 4 * h);
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const f32x4v a = *reinterpret_cast<const f32x4v *>(As + (t * 32 + l32) * M32_LD + 8 * g + 4 * h);
#pragma unroll
                for (int st = 0; st < 4; ++st)
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st], b[st], acc[t], 0, 0, 0);
            }
        }
        if (more) {
            __syncthreads();
            store_chunk();
            __syncthreads();
        }
    }
    // the lane holds rows t*32 + (v/4)*8 + h*4 + v%4: pairs (2i, 2i+1) in (v, v+1), v even
    const uint32_t c = c0 + col;
    if (c < ncol) {
        const uint32_t l = c / R, r = c - l * R;
        float2 *yp = dst + (size_t)l * nR + r;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int v = 0; v < 16; v += 2) {
                const int i = (t * 32 + (v >> 2) * 8 + h * 4 + (v & 3)) >> 1;
                if (i < n) yp[(size_t)i * R] = make_float2(acc[t][v], acc[t][v + 1]);
            }
    }
}

// ------------------------------------------------------------ FP64 MFMA stage
// The realified mode product of the FP64 mode on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): A operand rows 2i, 2i+1 hold (Re, -Im), (Im, Re)
// of M[i][j] at columns 2j, 2j+1; the B operand holds (Re, Im) of X[j] at rows
// 2j, 2j+1.  In group g of eight realified K, lane K index k takes the pair
// 8g + 2k, 8g + 2k + 1 on two consecutive K steps, so that one 16-byte LDS
// read (a complex value) feeds both.  Work-group: 4 waves x 16 columns, every
// wave all RT row tiles of 16 realified rows; chunks of 16 complex j pass
// through LDS with the next chunk's global loads in flight.  Register r of a
// lane holds row 4r + lane / 16 of column lane % 16 of a 16 x 16 tile.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int M64_CW = 64;              // columns per work-group
constexpr int M64_KC = 32;              // realified K per chunk
constexpr int M64_LD = M64_KC + 2;      // doubles per LDS row (16-byte aligned rows)

template <int RT>
__global__ void __launch_bounds__(256) k_mode_mfma64(ProgView p, int stage, const double2 *__restrict__ in) {
    constexpr int RD = 16 * RT;
    __shared__ __attribute__((aligned(16))) double As[RD * M64_LD];
    __shared__ __attribute__((aligned(16))) double Bs[M64_CW * M64_LD];
    const int e = blockIdx.y;
    const DevEntry *E = p.ent + e;
    if (E->nf <= stage) return;
    const int s = E->slot[stage];
    const int n = p.g.dims[s];
    const uint32_t R = (uint32_t)p.g.R[s];
    const uint32_t N = (uint32_t)p.g.N;
    const uint32_t ncol = N / (uint32_t)n;
    const uint32_t c0 = blockIdx.x * (uint32_t)M64_CW;
    if (c0 >= ncol) return;
    const double2 *__restrict__ M = E->M[stage];
    double2 *tmp = p.tmp;
    const double2 *__restrict__ src =
        stage == 0 ? in + (int64_t)E->src * p.in_stride : tmp + (2 * (int64_t)e + ((stage - 1) & 1)) * N;
    double2 *__restrict__ dst = tmp + (2 * (int64_t)e + (stage & 1)) * N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nR = (uint32_t)n * R;
    f64x4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int kmax = min(RD, 2 * n);
    constexpr int JC = M64_KC / 2;                          // complex j per chunk
    constexpr int MQ = ((RD / 2) * JC + 255) / 256;         // complex M values per thread
    constexpr int XQ = M64_CW * JC / 256;                   // complex X values per thread
    double2 mv[MQ], xv[XQ];
    auto xmap = [&](int q, int &cc, int &jj) {
        if (R == 1) {  // columns are rows of a row-major (ncol, n) matrix: j fastest
            jj = q % JC;
            cc = q / JC;
        } else {
            cc = q % M64_CW;
            jj = q / M64_CW;
        }
    };
    auto load_chunk = [&](int k0) {
        const int j0 = k0 / 2;
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            const int i = q / JC, jj = q - i * JC;
            const int j = j0 + jj;
            mv[u] = (q < (RD / 2) * JC && i < n && j < n) ? M[(size_t)i * n + j] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            int cc, jj;
            xmap(tid + 256 * u, cc, jj);
            const int j = j0 + jj;
            const uint32_t c = c0 + cc;
            double2 v = make_double2(0.0, 0.0);
            if (c < ncol && j < n) {
                const uint32_t l = c / R, r = c - l * R;
                v = src[(size_t)l * nR + (size_t)j * R + r];
            }
            xv[u] = v;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int u = 0; u < MQ; ++u) {
            const int q = tid + 256 * u;
            if (q >= (RD / 2) * JC) continue;
            const int i = q / JC, jj = q - i * JC;
            *reinterpret_cast<double2 *>(As + (2 * i) * M64_LD + 2 * jj) = make_double2(mv[u].x, -mv[u].y);
            *reinterpret_cast<double2 *>(As + (2 * i + 1) * M64_LD + 2 * jj) = make_double2(mv[u].y, mv[u].x);
        }
#pragma unroll
        for (int u = 0; u < XQ; ++u) {
            int cc, jj;
            xmap(tid + 256 * u, cc, jj);
            *reinterpret_cast<double2 *>(Bs + cc * M64_LD + 2 * jj) = xv[u];
        }
    };
    load_chunk(0);
    store_chunk();
    __syncthreads();
    const int l16 = lane & 15, kq = lane >> 4;
    const int col = wave * 16 + l16;
    for (int k0 = 0; k0 < kmax; k0 += M64_KC) {
        const bool more = k0 + M64_KC < kmax;
        if (more) load_chunk(k0 + M64_KC);
#pragma unroll
        for (int g = 0; g < M64_KC / 8; ++g) {
            const double2 b = *reinterpret_cast<const double2 *>(Bs + col * M64_LD + 8 * g + 2 * kq);
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const double2 a = *reinterpret_cast<const double2 *>(As + (t * 16 + l16) * M64_LD + 8 * g + 2 * kq);
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc[t], 0, 0, 0);
            }
        }
        if (more) {
            __syncthreads();
            store_chunk();
            __syncthreads();
        }
    }
    // realified row 4r + kq of tile t: complex row (16 t + 4 r + kq) / 2, part kq % 2
    const uint32_t c = c0 + col;
    if (c < ncol) {
        const uint32_t l = c / R, r = c - l * R;
        double *yp = reinterpret_cast<double *>(dst + (size_t)l * nR + r);
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i = (16 * t + 4 * rr + kq) >> 1;
                if (i < n) yp[2 * (size_t)i * R + (kq & 1)] = acc[t][rr];
            }
    }
}

// ------------------------------------------------------------ pair-operator form
// W_k[q][kappa] = sum_e c_e F_e[a][a'] P_e[b][b'] for q = (a, b), kappa = (a', b')
// (a null factor is the identity), summed in FP64 and stored row-major,
// W[q][kappa], in complex FP32.  Work-group tile: 64 pairs alpha = a n_k + a'
// by 64 pairs beta = b n_P + b'; the terms pass through LDS in chunks.
constexpr int PB_TC = 16;
__global__ void __launch_bounds__(256) k_pair_build(PairPass pp) {
    const int nk = pp.nk, np = pp.np;
    const int na = nk * nk, nbt = np * np, Q = nk * np;
    const int a0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    __shared__ double2 Fs[64 * PB_TC];  // Fs[i * PB_TC + t] = c_t F_t[a][a'] of alpha = a0 + i
    __shared__ double2 Ps[PB_TC * 64];  // Ps[t * 64 + j] = P_t[b][b'] of beta = b0 + j
    const int ta = threadIdx.x >> 4, tb = threadIdx.x & 15;
    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
    for (int t0 = 0; t0 < pp.n_terms; t0 += PB_TC) {
        const int tc = min(PB_TC, pp.n_terms - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * PB_TC; e += blockDim.x) {
            {
                const int i = e / PB_TC, t = e % PB_TC;
                const int al = a0 + i;
                double2 v = make_double2(0.0, 0.0);
                if (t < tc && al < na) {
                    const PairTerm T = pp.terms[t0 + t];
                    const int a = al / nk, ap = al - a * nk;
                    const double2 f = T.F ? T.F[(size_t)a * nk + ap] : make_double2(a == ap ? 1.0 : 0.0, 0.0);
                    v = cmul(T.coef, f);
                }
                Fs[e] = v;
            }
            {
                const int t = e / 64, j = e % 64;
                const int be = b0 + j;
                double2 w = make_double2(0.0, 0.0);
                if (t < tc && be < nbt) {
                    const PairTerm T = pp.terms[t0 + t];
                    const int b = be / np, bp = be - b * np;
                    w = T.P ? T.P[(size_t)b * np + bp] : make_double2(b == bp ? 1.0 : 0.0, 0.0);
                }
                Ps[e] = w;
            }
        }
        __syncthreads();
        for (int t = 0; t < tc; ++t) {
            double2 f[4], w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) f[i] = Fs[(4 * ta + i) * PB_TC + t];
#pragma unroll
            for (int j = 0; j < 4; ++j) w[j] = Ps[t * 64 + 4 * tb + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) cfma(acc[i][j], f[i], w[j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int al = a0 + 4 * ta + i;
        if (al >= na) continue;
        const int a = al / nk, ap = al - a * nk;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int be = b0 + 4 * tb + j;
            if (be >= nbt) continue;
            const int b = be / np, bp = be - b * np;
            pp.W[(size_t)(a * np + b) * Q + ap * np + bp] = make_float2((float)acc[i][j].x, (float)acc[i][j].y);
        }
    }
}

// out[o; q] (+)= sum_kappa W[q][kappa] in[o; kappa] for the node tensor seen as
// rows o (the indices other than slot k and the parent slot) by the pair index:
// element (o; a, b) of o = (l, m) at l n_k R_k + a R_k + m n_P + b, R_k = Mid n_P.
// One real GEMM on the FP32 matrix cores (v_mfma_f32_32x32x2f32) with the
// complex values realified: the A operand holds (Re, Im) of in[o; kappa] at
// realified columns (2 kappa, 2 kappa + 1), the B operand the 2 x 2 blocks
// [[Re W, Im W], [-Im W, Re W]] of W[q][kappa] at rows (2 kappa, 2 kappa + 1)
// and columns (2q, 2q + 1).  The input comes as complex FP32 (converted once
// per application).  Work-group tile: 128 rows by 256 realified columns, four
// waves of 64 x 128 (2 x 4 matrix-core tiles); chunks of 16 complex kappa pass
// through LDS with the parts split ([row][part][kappa]) so that one 16-byte
// LDS read feeds four K steps; the next chunk's global loads are in flight
// while the current one is multiplied.  Tiles are dealt so that the
// work-groups resident on one XCD (work-groups go to the 8 XCDs in turn) share
// row and column blocks in that XCD's L2.
constexpr int PG_BM = 128;
constexpr int PG_KS = 16;    // complex kappa per chunk (= K steps of 2 realified)
// floats per LDS row (two parts of 16, padded): A rows 36 (conflict-free
// 16-byte reads), B rows 40 (also conflict-free stores of four q per wave)
constexpr int PG_LDA = 2 * PG_KS + 4;
constexpr int PG_LDB = 2 * PG_KS + 8;
constexpr int PG_GR = 4;     // row tiles per group of the tile order

__global__ void k_to_f32(const double2 *__restrict__ x, float2 *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = make_float2((float)x[i].x, (float)x[i].y);
}

// Tile order: the tiles are dealt to the 8 XCDs in contiguous ranges (work-
// groups go to the XCDs in turn, XCD = work-group index mod 8); inside a range
// they run in groups of PG_GR row tiles by all column tiles, so that the
// work-groups resident on one XCD share row and column blocks in its L2.
__host__ __device__ inline void pair_xcd_range(unsigned ntile, unsigned x, unsigned &t0, unsigned &cnt) {
    const unsigned q8 = ntile / 8, r8 = ntile % 8;
    t0 = x * q8 + (x < r8 ? x : r8);
    cnt = q8 + (x < r8 ? 1u : 0u);
}
__device__ __forceinline__ void pair_tile_rc(unsigned t, unsigned nrt, unsigned nct, unsigned &rt, unsigned &ct) {
    const unsigned gsz = PG_GR * nct;
    const unsigned g = t / gsz, w = t - g * gsz;
    const unsigned rows_g = min((unsigned)PG_GR, nrt - g * PG_GR);
    rt = g * PG_GR + w % rows_g;
    ct = w / rows_g;
}

// Schedule of a launch: `slots` persistent work-groups (a multiple of 8, the
// resident capacity of the device), S = min(slots / 8, tiles of the range) of
// them per XCD.  The range's tiles x K chunks are cut into S equal shares of
// consecutive (tile, chunk) units; since a share is at least one tile long, a
// tile holds at most one cut.  A cut tile's two parts go to the workspace
// (part 0 from the earlier share, part 1 from the later) and k_pair_fixup adds
// them in that order, so the result does not depend on timing.  With S equal
// to the tile count every work-group takes one whole tile.
struct PairSched {
    unsigned ntile, nrt, nct, kc;  // tiles, row / column tiles, K chunks per tile
};
__device__ __forceinline__ bool pair_share(const PairSched &sc, int slots, unsigned x, unsigned pos, unsigned &t0,
                                           uint64_t &ub, uint64_t &ue, unsigned &S) {
    unsigned cnt;
    pair_xcd_range(sc.ntile, x, t0, cnt);
    S = min((unsigned)slots / 8, cnt);
    if (pos >= S) return false;
    const uint64_t U = (uint64_t)cnt * sc.kc;
    ub = pos * U / S;
    ue = (pos + 1) * U / S;
    return true;
}

// WN: matrix-core tiles per wave along the columns (the work-group covers
// 64 WN realified columns).  LDS (dynamic): two buffers of the A tile
// (128 rows of PG_LDA floats) and the B tile (64 WN columns of PG_LDB).
// Products of one tile over the K chunks [kb, ke) into acc.
// V4 (n_P a multiple of 4): each thread stages 4 consecutive kappa of 2 rows
// and of QW / 64 operator rows with 16-byte loads and 16-byte LDS stores (one
// a' per group of 4); otherwise 1 kappa of 8 rows and of QW / 16 operator rows.
template <int WN, bool V4>
__device__ __forceinline__ void pair_gemm_tile(const PairPass &pp, const float2 *__restrict__ X, unsigned rt,
                                               unsigned ct, int kb, int ke, float *pg_lds, f32x16 (&acc)[2][WN]) {
    constexpr int BN = 64 * WN;       // realified columns per work-group
    constexpr int QW = BN / 2;        // complex q per work-group
    constexpr int BU = 16 * QW / 256; // B values per thread and chunk
    constexpr int BUF = PG_BM * PG_LDA + BN * PG_LDB;  // floats per buffer
    const int nk = pp.nk, np = pp.np;
    const int Q = nk * np;
    const int64_t Mid = pp.Mid, Rk = Mid * np;
    const int64_t M = pp.L * Mid;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t o0 = (int64_t)rt * PG_BM;
    const int q0 = (int)ct * QW;
    // scalar staging: A 128 rows x 16 kappa, 8 per thread (rows (tid >> 4) + 16 u,
    // kappa offset tid & 15); B QW q x 16 kappa from the q-major W, BU per
    // thread (q offset (tid >> 4) + 16 u, kappa offset tid & 15).  V4: rows
    // (tid >> 2) + 64 u, kappa offset 4 (tid & 3).
    constexpr int AR = V4 ? 2 : 8;                 // rows of A per thread
    constexpr int RS = V4 ? 64 : 16;               // their stride
    constexpr int BR = V4 ? QW / 64 : BU;          // operator rows per thread
    constexpr int KV = V4 ? 4 : 1;                 // kappa per row and thread
    const int rsub = V4 ? (tid >> 2) : (tid >> 4);
    const int kk = V4 ? 4 * (tid & 3) : (tid & 15);
    int64_t rbase[AR];
#pragma unroll
    for (int u = 0; u < AR; ++u) {
        const int64_t o = o0 + rsub + RS * u;
        if (o < M) {
            const int64_t l = o / Mid, m = o - l * Mid;
            rbase[u] = l * nk * Rk + m * np;
        } else {
            rbase[u] = -1;
        }
    }
    float2 av[AR][KV], bv[BR][KV];
    auto load = [&](int kappa0) {
        const int ka = kappa0 + kk;
        const bool kok = ka < Q;  // V4: Q and ka are multiples of 4, all 4 or none
        const int ap = ka / np, bp = ka - ap * np;
        const int64_t off = (int64_t)ap * Rk + bp;
#pragma unroll
        for (int u = 0; u < AR; ++u) {
            if (V4) {
                float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
                if (kok && rbase[u] >= 0) {
                    const float4 *src = reinterpret_cast<const float4 *>(X + rbase[u] + off);
                    lo = src[0];
                    hi = src[1];
                }
                av[u][0] = make_float2(lo.x, lo.y);
                av[u][1 % KV] = make_float2(lo.z, lo.w);
                av[u][2 % KV] = make_float2(hi.x, hi.y);
                av[u][3 % KV] = make_float2(hi.z, hi.w);
            } else {
                av[u][0] = (kok && rbase[u] >= 0) ? X[rbase[u] + off] : make_float2(0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int u = 0; u < BR; ++u) {
            const int q = q0 + rsub + RS * u;
            if (V4) {
                float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
                if (kok && q < Q) {
                    const float4 *src = reinterpret_cast<const float4 *>(pp.W + (size_t)q * Q + ka);
                    lo = src[0];
                    hi = src[1];
                }
                bv[u][0] = make_float2(lo.x, lo.y);
                bv[u][1 % KV] = make_float2(lo.z, lo.w);
                bv[u][2 % KV] = make_float2(hi.x, hi.y);
                bv[u][3 % KV] = make_float2(hi.z, hi.w);
            } else {
                bv[u][0] = (kok && q < Q) ? pp.W[(size_t)q * Q + ka] : make_float2(0.0f, 0.0f);
            }
        }
    };
    auto store = [&](float *buf) {
        float *As = buf, *Bs = buf + PG_BM * PG_LDA;
#pragma unroll
        for (int u = 0; u < AR; ++u) {
            float *a = As + (rsub + RS * u) * PG_LDA + kk;
            if (V4) {
                *reinterpret_cast<f32x4v *>(a) = f32x4v{av[u][0].x, av[u][1 % KV].x, av[u][2 % KV].x, av[u][3 % KV].x};
                *reinterpret_cast<f32x4v *>(a + PG_KS) =
                    f32x4v{av[u][0].y, av[u][1 % KV].y, av[u][2 % KV].y, av[u][3 % KV].y};
            } else {
                a[0] = av[u][0].x;
                a[PG_KS] = av[u][0].y;
            }
        }
#pragma unroll
        for (int u = 0; u < BR; ++u) {
            const int qq = rsub + RS * u;
            float *b0 = Bs + (2 * qq) * PG_LDB + kk;  // column 2q: (Re W, -Im W) for parts (0, 1)
            float *b1 = b0 + PG_LDB;                   // column 2q + 1: (Im W, Re W)
            if (V4) {
                const float2 w0 = bv[u][0], w1 = bv[u][1 % KV], w2 = bv[u][2 % KV], w3 = bv[u][3 % KV];
                *reinterpret_cast<f32x4v *>(b0) = f32x4v{w0.x, w1.x, w2.x, w3.x};
                *reinterpret_cast<f32x4v *>(b0 + PG_KS) = f32x4v{-w0.y, -w1.y, -w2.y, -w3.y};
                *reinterpret_cast<f32x4v *>(b1) = f32x4v{w0.y, w1.y, w2.y, w3.y};
                *reinterpret_cast<f32x4v *>(b1 + PG_KS) = f32x4v{w0.x, w1.x, w2.x, w3.x};
            } else {
                b0[0] = bv[u][0].x;
                b0[PG_KS] = -bv[u][0].y;
                b1[0] = bv[u][0].y;
                b1[PG_KS] = bv[u][0].x;
            }
        }
    };
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 32 * WN;
    const int part = lane >> 5, l32 = lane & 31;
    load(kb * PG_KS);
    __syncthreads();  // the previous tile's last products have read both buffers
    store(pg_lds);
    __syncthreads();
    int cur = 0;
    for (int kc = kb; kc < ke; ++kc) {
        const bool more = kc + 1 < ke;
        if (more) load((kc + 1) * PG_KS);
        const float *As = pg_lds + cur * BUF, *Bs = As + PG_BM * PG_LDA;
#pragma unroll
        for (int t4 = 0; t4 < PG_KS; t4 += 4) {
            f32x4v a[2], b[WN];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const f32x4v *>(As + (wr + 32 * i + l32) * PG_LDA + part * PG_KS + t4);
#pragma unroll
            for (int j = 0; j < WN; ++j)
                b[j] = *reinterpret_cast<const f32x4v *>(Bs + (wc + 32 * j + l32) * PG_LDB + part * PG_KS + t4);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
        }
        if (more) {
            // the other buffer was last read before the previous barrier
            store(pg_lds + (1 - cur) * BUF);
            __syncthreads();
            cur = 1 - cur;
        }
    }
}

// Y (+)= the tile's products (FP64 output, read back when accumulating)
template <int WN>
__device__ __forceinline__ void pair_gemm_store(const PairPass &pp, double2 *__restrict__ Y, int accumulate,
                                                unsigned rt, unsigned ct, const f32x16 (&acc)[2][WN]) {
    constexpr int BN = 64 * WN;
    const int nk = pp.nk, np = pp.np;
    const int Q = nk * np;
    const int64_t Mid = pp.Mid, Rk = Mid * np;
    const int64_t M = pp.L * Mid;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t o0 = (int64_t)rt * PG_BM;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 32 * WN;
    const int part = lane >> 5, l32 = lane & 31;
    // lane holds rows 8 (v / 4) + 4 (lane / 32) + v % 4 of column lane % 32 of each 32 x 32 tile
    double *Yd = reinterpret_cast<double *>(Y);
    int64_t obase[2][4];
    int orun[2][4];  // rows of the group of four that share its l
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            // rows o0 + wr + 32 i + 8 g + 4 part + (0..3): one division per group of four
            const int64_t o = o0 + wr + 32 * i + 8 * g + 4 * part;
            const int64_t l = o / Mid, m = o - l * Mid;
            obase[i][g] = l * nk * Rk + m * np;
            orun[i][g] = (int)min<int64_t>(4, Mid - m);
        }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
        const int cr = (int)ct * BN + wc + 32 * j + l32;  // realified column
        const int q = cr >> 1, ri = cr & 1;
        if (q >= Q) continue;
        const int a = q / np, b = q - a * np;
        const int64_t cofs = (int64_t)a * Rk + b;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            size_t idx[16];
            bool ok[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t o = o0 + wr + 32 * i + 8 * (v >> 2) + 4 * part + (v & 3);
                ok[v] = o < M;
                int64_t base = obase[i][v >> 2];
                if ((v & 3) < orun[i][v >> 2]) {
                    base += (int64_t)(v & 3) * np;
                } else {  // the group of four crosses into the next l
                    const int64_t l = o / Mid, m = o - l * Mid;
                    base = l * nk * Rk + m * np;
                }
                idx[v] = 2 * (size_t)(base + cofs) + ri;
            }
            double old[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) old[v] = (accumulate && ok[v]) ? Yd[idx[v]] : 0.0;
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (ok[v]) Yd[idx[v]] = old[v] + (double)acc[i][j][v];
        }
    }
}

// workspace of the cut tiles: part p of cut c holds the 32 WN floats of every
// thread as 8 WN float4, float4 j of thread tid at ((2 c + p) 8 WN + j) 256 + tid
template <int WN>
__device__ __forceinline__ f32x4v *pair_ws_part(float *ws, unsigned cut, int p) {
    return reinterpret_cast<f32x4v *>(ws) + ((size_t)(2 * cut + p) * 8 * WN) * 256;
}

// a cut tile's part: the cut at this share's start (part 1) or at its end (part 0)
template <int WN>
__device__ __forceinline__ void pair_cut_store(float *ws, int slots, unsigned x, unsigned pos, int kb,
                                               const f32x16 (&acc)[2][WN]) {
    const unsigned cut = x * ((unsigned)slots / 8) + (kb == 0 ? pos + 1 : pos);
    f32x4v *w = pair_ws_part<WN>(ws, cut, kb == 0 ? 0 : 1);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4v v = {acc[i][j][4 * g], acc[i][j][4 * g + 1], acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]};
                w[(size_t)((i * WN + j) * 4 + g) * 256 + threadIdx.x] = v;
            }
}

template <int WN, bool V4>
__global__ void __launch_bounds__(256, WN == 2 ? 2 : 1) k_pair_gemm(PairPass pp, const float2 *__restrict__ X, double2 *__restrict__ Y,
                                                   int accumulate, float *ws, int slots, PairSched sc) {
    const unsigned x = blockIdx.x % 8, pos = blockIdx.x / 8;
    unsigned t0, S;
    uint64_t ub, ue;
    if (!pair_share(sc, slots, x, pos, t0, ub, ue, S)) return;
    extern __shared__ __attribute__((aligned(16))) float pg_lds[];
    f32x16 acc[2][WN];
    for (uint64_t u = ub; u < ue;) {
        const unsigned tl = (unsigned)(u / sc.kc);
        const int kb = (int)(u - (uint64_t)tl * sc.kc);
        const int ke = (int)min<uint64_t>(sc.kc, kb + (ue - u));
        unsigned rt, ct;
        pair_tile_rc(t0 + tl, sc.nrt, sc.nct, rt, ct);
        pair_gemm_tile<WN, V4>(pp, X, rt, ct, kb, ke, pg_lds, acc);
        if (kb == 0 && ke == (int)sc.kc) {
            pair_gemm_store<WN>(pp, Y, accumulate, rt, ct, acc);
        } else {
            pair_cut_store<WN>(ws, slots, x, pos, kb, acc);
        }
        u += (uint64_t)(ke - kb);
    }
}

// cut tiles: part 0 + part 1, then the output as for a whole tile
template <int WN>
__global__ void __launch_bounds__(256) k_pair_fixup(PairPass pp, double2 *__restrict__ Y, int accumulate,
                                                    const float *ws, int slots, PairSched sc) {
    const unsigned x = blockIdx.x % 8, pos = blockIdx.x / 8;
    unsigned t0, S;
    uint64_t ub, ue;
    if (pos == 0 || !pair_share(sc, slots, x, pos, t0, ub, ue, S)) return;
    if (ub % sc.kc == 0) return;  // the share starts on a tile boundary: no cut
    unsigned rt, ct;
    pair_tile_rc(t0 + (unsigned)(ub / sc.kc), sc.nrt, sc.nct, rt, ct);
    const unsigned cut = x * ((unsigned)slots / 8) + pos;
    const f32x4v *w0 = pair_ws_part<WN>(const_cast<float *>(ws), cut, 0);
    const f32x4v *w1 = pair_ws_part<WN>(const_cast<float *>(ws), cut, 1);
    f32x16 acc[2][WN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const size_t q = (size_t)((i * WN + j) * 4 + g) * 256 + threadIdx.x;
                const f32x4v a = w0[q], b = w1[q];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][4 * g + e] = a[e] + b[e];
            }
    pair_gemm_store<WN>(pp, Y, accumulate, rt, ct, acc);
}

// ---- BF16x3 form of the pair GEMM.  The operands are split into bf16 hi + lo
// once (the input per application, the pair operator per build) and each
// product taken as hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16 (FP32
// accumulation; the dropped lo*lo term is ~2^-16 relative).  Realified
// interleaved layout: row o of the A operand holds (Re, Im) of in[o; kappa] at
// k' = (2 kappa, 2 kappa + 1); row c' = 2q + u of the (transposed) B operand
// holds [Re W, -Im W] (u = 0) or [Im W, Re W] (u = 1) of W[q][kappa] at the same
// k'.  A lane of the MFMA reads 8 consecutive k' (16 bytes) of its row.
// Requires n_P % 32 == 0 (a chunk of 32 kappa lies within one a').
constexpr int PGB_KS = 32;               // complex kappa per chunk (64 k', 4 MFMA K-steps)
constexpr int PGB_LD = 2 * PGB_KS + 8;   // bf16 per LDS row (padded: 144 B, conflict-free 16-byte reads)
__device__ __forceinline__ unsigned pack_bf16x2(unsigned short lo_half, unsigned short hi_half) {
    return (unsigned)lo_half | ((unsigned)hi_half << 16);
}

// xh[i], xl[i]: (Re, Im) of x[i] as bf16 hi and lo parts (low half: Re)
__global__ void k_to_bf16x2(const double2 *__restrict__ x, unsigned *__restrict__ xh, unsigned *__restrict__ xl,
                            int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned short rh, rl, ih, il;
        bf16_split((float)x[i].x, rh, rl);
        bf16_split((float)x[i].y, ih, il);
        xh[i] = pack_bf16x2(rh, ih);
        xl[i] = pack_bf16x2(rl, il);
    }
}

// Wb hi / lo ([2Q][2Q] bf16 each, row c' = 2q + u, column k' = 2 kappa + s) from W[q][kappa]
__global__ void k_pair_split(PairPass pp) {
    const int Q = pp.nk * pp.np;
    const int64_t tot = (int64_t)Q * Q;
    unsigned *wh = reinterpret_cast<unsigned *>(pp.Wb);
    unsigned *wl = wh + 2 * tot;  // each array holds 4 Q^2 bf16 = 2 Q^2 pairs
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = i / Q, ka = i - q * Q;
        const float2 w = pp.W[i];
        unsigned short reh, rel, imh, iml, nih, nil;
        bf16_split(w.x, reh, rel);
        bf16_split(w.y, imh, iml);
        bf16_split(-w.y, nih, nil);
        // pair index of (row c', k' = 2 kappa): c' * Q + kappa
        const int64_t r0 = (2 * q) * Q + ka, r1 = (2 * q + 1) * Q + ka;
        wh[r0] = pack_bf16x2(reh, nih);
        wl[r0] = pack_bf16x2(rel, nil);
        wh[r1] = pack_bf16x2(imh, reh);
        wl[r1] = pack_bf16x2(iml, rel);
    }
}

// Products of one tile of the BF16x3 pair GEMM over the K chunks [kb, ke) into acc
__device__ __forceinline__ void pair_gemm_bf_tile(const PairPass &pp, const unsigned *__restrict__ Xh,
                                                  const unsigned *__restrict__ Xl, unsigned rt, unsigned ct, int kb,
                                                  int ke, unsigned short *pgb_lds, f32x16 (&acc)[2][2]) {
    constexpr int BN = 128;  // realified columns per work-group (2 waves x 2 tiles of 32)
    const int nk = pp.nk, np = pp.np;
    const int Q = nk * np;
    const int64_t Mid = pp.Mid, Rk = Mid * np;
    const int64_t M = pp.L * Mid;
    unsigned short *Ah = pgb_lds, *Al = Ah + PG_BM * PGB_LD;
    unsigned short *Bh = Al + PG_BM * PGB_LD, *Bl = Bh + BN * PGB_LD;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t o0 = (int64_t)rt * PG_BM;
    const int c0 = (int)ct * BN;  // first realified column
    // loads: thread (row or column tid >> 1, half tid & 1) takes 16 kappa = 32 k' of each part
    const int lr = tid >> 1, half = tid & 1;
    int64_t rbase = -1;
    {
        const int64_t o = o0 + lr;
        if (o < M) {
            const int64_t l = o / Mid, m = o - l * Mid;
            rbase = l * nk * Rk + m * np;
        }
    }
    const int cb = c0 + lr;  // B row (realified column) of this thread
    const unsigned *wh = reinterpret_cast<const unsigned *>(pp.Wb);
    const unsigned *wl = wh + 2 * (int64_t)Q * Q;
    uint4 ah[4], al[4], bh[4], bl[4];
    auto load = [&](int kappa0) {
        const int ap = kappa0 / np, bp = kappa0 - ap * np;  // the chunk lies in one a' (n_P % 32 == 0)
        const int ka = kappa0 + 16 * half;
        if (rbase >= 0 && ka < Q) {
            const uint4 *ph = reinterpret_cast<const uint4 *>(Xh + rbase + (int64_t)ap * Rk + bp + 16 * half);
            const uint4 *pl = reinterpret_cast<const uint4 *>(Xl + rbase + (int64_t)ap * Rk + bp + 16 * half);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ah[u] = ph[u];
                al[u] = pl[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ah[u] = make_uint4(0, 0, 0, 0);
                al[u] = make_uint4(0, 0, 0, 0);
            }
        }
        if (cb < 2 * Q && ka < Q) {
            const uint4 *ph = reinterpret_cast<const uint4 *>(wh + (int64_t)cb * Q + ka);
            const uint4 *pl = reinterpret_cast<const uint4 *>(wl + (int64_t)cb * Q + ka);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bh[u] = ph[u];
                bl[u] = pl[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bh[u] = make_uint4(0, 0, 0, 0);
                bl[u] = make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto store = [&]() {
        uint4 *dah = reinterpret_cast<uint4 *>(Ah + lr * PGB_LD + 32 * half);
        uint4 *dal = reinterpret_cast<uint4 *>(Al + lr * PGB_LD + 32 * half);
        uint4 *dbh = reinterpret_cast<uint4 *>(Bh + lr * PGB_LD + 32 * half);
        uint4 *dbl = reinterpret_cast<uint4 *>(Bl + lr * PGB_LD + 32 * half);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            dah[u] = ah[u];
            dal[u] = al[u];
            dbh[u] = bh[u];
            dbl[u] = bl[u];
        }
    };
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int g8 = (lane >> 5) * 8, l32 = lane & 31;
    load(kb * PGB_KS);
    __syncthreads();  // the previous tile's last products have read the buffers
    store();
    __syncthreads();
    for (int kc = kb; kc < ke; ++kc) {
        const bool more = kc + 1 < ke;
        if (more) load((kc + 1) * PGB_KS);
#pragma unroll
        for (int t = 0; t < 2 * PGB_KS; t += 16) {
            bf8v xh[2], xl[2], yh[2], yl[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                xh[i] = __builtin_bit_cast(bf8v, *reinterpret_cast<const uint4 *>(Ah + (wr + 32 * i + l32) * PGB_LD + t + g8));
                xl[i] = __builtin_bit_cast(bf8v, *reinterpret_cast<const uint4 *>(Al + (wr + 32 * i + l32) * PGB_LD + t + g8));
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                yh[j] = __builtin_bit_cast(bf8v, *reinterpret_cast<const uint4 *>(Bh + (wc + 32 * j + l32) * PGB_LD + t + g8));
                yl[j] = __builtin_bit_cast(bf8v, *reinterpret_cast<const uint4 *>(Bl + (wc + 32 * j + l32) * PGB_LD + t + g8));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[i], yh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], yl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], yh[j], acc[i][j], 0, 0, 0);
                }
        }
        if (more) {
            __syncthreads();
            store();
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(256, 2) k_pair_gemm_bf(PairPass pp, const unsigned *__restrict__ Xh,
                                                         const unsigned *__restrict__ Xl, double2 *__restrict__ Y,
                                                         int accumulate, float *ws, int slots, PairSched sc) {
    const unsigned x = blockIdx.x % 8, pos = blockIdx.x / 8;
    unsigned t0, S;
    uint64_t ub, ue;
    if (!pair_share(sc, slots, x, pos, t0, ub, ue, S)) return;
    extern __shared__ __attribute__((aligned(16))) unsigned short pgb_lds[];
    f32x16 acc[2][2];
    for (uint64_t u = ub; u < ue;) {
        const unsigned tl = (unsigned)(u / sc.kc);
        const int kb = (int)(u - (uint64_t)tl * sc.kc);
        const int ke = (int)min<uint64_t>(sc.kc, kb + (ue - u));
        unsigned rt, ct;
        pair_tile_rc(t0 + tl, sc.nrt, sc.nct, rt, ct);
        pair_gemm_bf_tile(pp, Xh, Xl, rt, ct, kb, ke, pgb_lds, acc);
        if (kb == 0 && ke == (int)sc.kc) pair_gemm_store<2>(pp, Y, accumulate, rt, ct, acc);
        else pair_cut_store<2>(ws, slots, x, pos, kb, acc);
        u += (uint64_t)(ke - kb);
    }
}

// Coefficient-weighted sum of the entries of each group.  Entries without
// factors read the FP64 input; the others read their last temporary (type T).
// Output: out_single (FP64, one group) or the group sums p.gsum (type T).
template <typename T>
__global__ void __launch_bounds__(256) k_group_sum(ProgView p, const double2 *__restrict__ in,
                                                   double2 *out_single) {
    const int g = blockIdx.y;
    const uint32_t N = (uint32_t)p.g.N;
    const T *tmp = reinterpret_cast<const T *>(p.tmp);
    T *gs = reinterpret_cast<T *>(p.gsum) + (size_t)g * N;
    const int q0 = p.gptr[g], q1 = p.gptr[g + 1];
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
        T acc = czero<T>();
        for (int q = q0; q < q1; ++q) {
            const int e = p.gent[q];
            const int nf = p.ent[e].nf;
            const T v = nf == 0 ? cvt<T>(in[(int64_t)p.ent[e].src * p.in_stride + idx])
                                : tmp[(2 * (size_t)e + ((nf - 1) & 1)) * N + idx];
            cfma(acc, cvt<T>(p.ent[e].coef), v);
        }
        if (out_single) out_single[idx] = cvt<double2>(acc);
        else gs[idx] = acc;
    }
}

// generic single mode product with rectangular M (n_out x n_in)
__global__ void __launch_bounds__(256) k_mode_single(const double2 *__restrict__ X, double2 *__restrict__ Y,
                                                     const double2 *__restrict__ M, uint32_t L, int nin,
                                                     int nout, uint32_t R, int transM) {
    const uint32_t NY = L * (uint32_t)nout * R;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < NY; idx += gridDim.x * blockDim.x) {
        uint32_t r = idx % R, t = idx / R;
        uint32_t i = t % nout, l = t / nout;
        const double2 *xp = X + (size_t)l * nin * R + r;
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < nin; ++j) {
            double2 m = transM ? M[(size_t)j * nout + i] : M[(size_t)i * nin + j];
            cfma(acc, m, xp[(size_t)j * R]);
        }
        Y[idx] = acc;
    }
}

// ============================================================ contractions
// out[m,n] = sum_{l,r} conj(A[l,m,r]) B[l,n,r]; pass 1 writes per-block partials.
constexpr int CT_ROWS = 32;
constexpr int CT_MAXOUT = 16;  // outputs per thread (nA*nB <= 256*16)

// T is the compute type and the element type of B (the group sums in the FP32
// mode); A is always FP64; partials are written in FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_contract_part(const double2 *__restrict__ A, const T *__restrict__ Bbase,
                                                       int64_t bstride, uint32_t L, int nA, int nB, uint32_t R,
                                                       double2 *__restrict__ part) {
    const int g = blockIdx.y;
    const T *__restrict__ B = Bbase + (size_t)g * bstride;
    const uint32_t rows = L * R;
    const uint32_t per = (rows + gridDim.x - 1) / gridDim.x;
    const uint32_t r0 = blockIdx.x * per, r1 = min(rows, r0 + per);
    extern __shared__ double2 sct_raw[];
    T *As = reinterpret_cast<T *>(sct_raw);  // CT_ROWS * nA
    T *Bs = As + CT_ROWS * nA;                // CT_ROWS * nB
    const int nout = nA * nB;
    T acc[CT_MAXOUT];
    for (int q = 0; q < CT_MAXOUT; ++q) acc[q] = czero<T>();
    for (uint32_t t0 = r0; t0 < r1; t0 += CT_ROWS) {
        const int tr = (int)min((uint32_t)CT_ROWS, r1 - t0);
        __syncthreads();
        for (int q = threadIdx.x; q < CT_ROWS * nA; q += blockDim.x) {
            int t = q % CT_ROWS, m = q / CT_ROWS;
            T v = czero<T>();
            if (t < tr) {
                uint32_t rho = t0 + t, l = rho / R, r = rho % R;
                v = cvt<T>(A[((size_t)l * nA + m) * R + r]);
            }
            As[t * nA + m] = v;
        }
        for (int q = threadIdx.x; q < CT_ROWS * nB; q += blockDim.x) {
            int t = q % CT_ROWS, m = q / CT_ROWS;
            T v = czero<T>();
            if (t < tr) {
                uint32_t rho = t0 + t, l = rho / R, r = rho % R;
                v = B[((size_t)l * nB + m) * R + r];
            }
            Bs[t * nB + m] = v;
        }
        __syncthreads();
        for (int q = 0; q < CT_MAXOUT; ++q) {
            int o = threadIdx.x + q * blockDim.x;
            if (o >= nout) break;
            int m = o / nB, nn = o - m * nB;
            T a = acc[q];
            for (int t = 0; t < tr; ++t) cfmac(a, As[t * nA + m], Bs[t * nB + nn]);
            acc[q] = a;
        }
    }
    for (int q = 0; q < CT_MAXOUT; ++q) {
        int o = threadIdx.x + q * blockDim.x;
        if (o >= nout) break;
        part[((size_t)g * gridDim.x + blockIdx.x) * nout + o] = cvt<double2>(acc[q]);
    }
}

__global__ void k_contract_reduce(const double2 *__restrict__ part, int nblk, int nout,
                                  double2 *const *gdst, double2 *single) {
    const int g = blockIdx.y;
    double2 *dst = single ? single : gdst[g];
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < nout; o += gridDim.x * blockDim.x) {
        double2 s = make_double2(0.0, 0.0);
        for (int b = 0; b < nblk; ++b) s = cadd(s, part[((size_t)g * nblk + b) * nout + o]);
        dst[o] = s;
    }
}

// FP32 mode, n up to 64: the same contraction on the FP32 matrix cores.
// out = A^H B as one real GEMM over the realified rows: the A operand holds
// (Re, Im) of A[rho][m] at K = (2 rho, 2 rho + 1); column 2n' of the B operand
// holds (Re, Im) of B[rho][n'] (giving Re sum conj(a) b) and column 2n' + 1
// holds (Im, -Re) (giving Im).  A chunk of CM_KC rows passes through LDS
// (A converted to FP32); the four waves take alternate groups of eight K (in
// the 16-byte order of the FP32 stage kernel) and are summed through LDS at
// the end.  The work-groups of one row slice (all groups g) go to one XCD
// (XCD = work-group index mod 8) so that they find the slice of A in its L2.
constexpr int CM_KC = 32;              // rows per chunk
constexpr int CM_LD = 2 * CM_KC + 4;   // floats per LDS row

template <int RT, int CT>
__global__ void __launch_bounds__(256, 2) k_contract_mfma(const double2 *__restrict__ A, const float2 *__restrict__ Bbase,
                                                       int64_t bstride, uint32_t L, int n, uint32_t R, int nb,
                                                       int ng, double2 *__restrict__ part) {
    const unsigned x = blockIdx.x % 8, pos = blockIdx.x / 8;
    const int g = (int)(pos % (unsigned)ng);
    const int slice = (int)(pos / (unsigned)ng) * 8 + (int)x;
    if (slice >= nb) return;
    __shared__ __attribute__((aligned(16))) float lds[(32 * RT + 32 * CT) * CM_LD];
    float *As = lds, *Bs = lds + 32 * RT * CM_LD;
    const float2 *__restrict__ B = Bbase + (size_t)g * bstride;
    const uint32_t rows = L * R;
    const uint32_t per = (rows + nb - 1) / nb;
    const uint32_t r0 = (uint32_t)slice * per, r1 = min(rows, r0 + per);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q = tid; q < (32 * RT + 32 * CT) * CM_LD; q += 256) lds[q] = 0.0f;  // padding rows stay zero
    f32x16 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    const int l32 = lane & 31, h = lane >> 5;
    for (uint32_t t0 = r0; t0 < r1; t0 += CM_KC) {
        const int tr = (int)min((uint32_t)CM_KC, r1 - t0);
        __syncthreads();
        for (int q = tid; q < CM_KC * n; q += 256) {
            int t, m;
            if (R == 1) {  // rows of a row-major (rows, n) matrix: m fastest
                m = q % n;
                t = q / n;
            } else {
                t = q % CM_KC;
                m = q / CM_KC;
            }
            double2 a = make_double2(0.0, 0.0);
            float2 b = make_float2(0.0f, 0.0f);
            if (t < tr) {
                const uint32_t rho = t0 + t, l = rho / R, r = rho - l * R;
                const size_t at = ((size_t)l * n + m) * R + r;
                a = A[at];
                b = B[at];
            }
            *reinterpret_cast<float2 *>(As + m * CM_LD + 2 * t) = make_float2((float)a.x, (float)a.y);
            *reinterpret_cast<float2 *>(Bs + (2 * m) * CM_LD + 2 * t) = b;
            *reinterpret_cast<float2 *>(Bs + (2 * m + 1) * CM_LD + 2 * t) = make_float2(b.y, -b.x);
        }
        __syncthreads();
#pragma unroll
        for (int gg = 0; gg < 2; ++gg) {
            const int k8 = 8 * (wave + 4 * gg) + 4 * h;
            f32x4v b[CT];
#pragma unroll
            for (int j = 0; j < CT; ++j) b[j] = *reinterpret_cast<const f32x4v *>(Bs + (j * 32 + l32) * CM_LD + k8);
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const f32x4v a = *reinterpret_cast<const f32x4v *>(As + (i * 32 + l32) * CM_LD + k8);
#pragma unroll
                for (int st = 0; st < 4; ++st)
#pragma unroll
                    for (int j = 0; j < CT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st], b[j][st], acc[i][j], 0, 0, 0);
            }
        }
    }
    // sum of the four waves' accumulators in LDS (one wave after the other), then the FP64 partial
    float *red = lds;  // RT * CT * 16 * 64 floats, element (i, j, v) of lane at ((i CT + j) 16 + v) 64 + lane
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int j = 0; j < CT; ++j)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        float *r = red + ((i * CT + j) * 16 + v) * 64 + lane;
                        *r = w == 0 ? acc[i][j][v] : *r + acc[i][j][v];
                    }
        }
    }
    __syncthreads();
    double *pd = reinterpret_cast<double *>(part + ((size_t)g * nb + slice) * n * n);
    for (int e = tid; e < RT * CT * 16 * 64; e += 256) {
        const int ln = e & 63, v = (e >> 6) & 15, ij = e >> 10;
        const int i = ij / CT, j = ij - i * CT;
        const int m = i * 32 + 8 * (v >> 2) + 4 * (ln >> 5) + (v & 3);
        const int c = j * 32 + (ln & 31);
        if (m < n && c < 2 * n) pd[2 * ((size_t)m * n + (c >> 1)) + (c & 1)] = (double)red[e];
    }
}

static int contract_blocks(uint32_t rows) {
    int b = (int)((rows + 255) / 256);
    return b < 1 ? 1 : (b > 64 ? 64 : b);
}

// ============================================================ QR (Householder)
// In-place thin QR of the matrix with rows (l, r) and columns j of A[l, j, r]
// (the index j moved last, other indices in row-major order), following the
// LAPACK zgeqr2 / zung2r convention.  One work-group.
__device__ __forceinline__ size_t qr_addr(uint32_t rho, int j, int n, uint32_t R) {
    return ((size_t)(rho / R) * n + j) * R + (rho % R);
}

__global__ void __launch_bounds__(1024) k_qr(double2 *A, uint32_t L, int n, uint32_t R, double2 *Rout, int transR,
                                             double snap, const int *gate) {
    if (gate && *gate == 0) return;
    const uint32_t m = L * R;
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ double2 tau_s[64];
    __shared__ double2 wcol[64];
    __shared__ double2 red2[16 * 64];
    __shared__ double red1[16];
    __shared__ double2 sc[2];  // [0] tau, [1] 1/(alpha-beta)
    const int CP = 64;            // column slots per pass
    const int RP = nt / CP;       // row phases
    const int jc = tid % CP, rp = tid / CP;
    // zero-snap threshold: sub-columns below snap * |M|_F count as exactly zero
    double fro = 0.0;
    for (uint32_t q = tid; q < m * (uint32_t)n; q += nt) fro += cabs2(A[q]);
    const double thr = snap * sqrt(blk_sum1(fro, red1));
    for (int i = 0; i < n; ++i) {
        double part = 0.0;
        for (uint32_t rho = i + 1 + tid; rho < m; rho += nt) part += cabs2(A[qr_addr(rho, i, n, R)]);
        double xn2 = blk_sum1(part, red1);
        if (snap > 0.0 && sqrt(xn2) <= thr) {
            for (uint32_t rho = i + 1 + tid; rho < m; rho += nt) A[qr_addr(rho, i, n, R)] = make_double2(0.0, 0.0);
            xn2 = 0.0;
            if (tid == 0) {
                double2 a = A[qr_addr(i, i, n, R)];
                if (fabs(a.y) <= thr) A[qr_addr(i, i, n, R)] = make_double2(a.x, 0.0);
            }
            __syncthreads();
        }
        double2 alpha = A[qr_addr(i, i, n, R)];
        if (tid == 0) {
            if (xn2 == 0.0 && alpha.y == 0.0) {
                sc[0] = make_double2(0.0, 0.0);
                sc[1] = make_double2(0.0, 0.0);
            } else {
                double beta = -copysign(sqrt(cabs2(alpha) + xn2), alpha.x);
                sc[0] = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                sc[1] = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
                A[qr_addr(i, i, n, R)] = make_double2(beta, 0.0);
            }
        }
        __syncthreads();
        const double2 tau = sc[0], scl = sc[1];
        if (tid == 0) tau_s[i] = tau;
        if (tau.x == 0.0 && tau.y == 0.0) {
            __syncthreads();
            continue;
        }
        for (uint32_t rho = i + 1 + tid; rho < m; rho += nt) {
            size_t a = qr_addr(rho, i, n, R);
            A[a] = cmul(A[a], scl);
        }
        __syncthreads();
        // trailing columns: w_j = sum_rho conj(v_rho) A(rho, j); A -= conj(tau) v w_j
        for (int j0 = i + 1; j0 < n; j0 += CP) {
            const int j = j0 + jc;
            double2 acc = make_double2(0.0, 0.0);
            if (j < n) {
                for (uint32_t rho = i + rp; rho < m; rho += RP) {
                    double2 v = rho == (uint32_t)i ? make_double2(1.0, 0.0) : A[qr_addr(rho, i, n, R)];
                    cfmac(acc, v, A[qr_addr(rho, j, n, R)]);
                }
            }
            red2[rp * CP + jc] = acc;
            __syncthreads();
            if (rp == 0) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < RP; ++q) s = cadd(s, red2[q * CP + jc]);
                wcol[jc] = s;
            }
            __syncthreads();
            if (j < n) {
                const double2 ctau = make_double2(tau.x, -tau.y);
                const double2 f = cmul(ctau, wcol[jc]);
                for (uint32_t rho = i + rp; rho < m; rho += RP) {
                    double2 v = rho == (uint32_t)i ? make_double2(1.0, 0.0) : A[qr_addr(rho, i, n, R)];
                    size_t a = qr_addr(rho, j, n, R);
                    A[a] = csub(A[a], cmul(v, f));
                }
            }
            __syncthreads();
        }
    }
    // R factor
    for (int q = tid; q < n * n; q += nt) {
        int i = q / n, j = q % n;
        double2 v = j >= i ? A[qr_addr(i, j, n, R)] : make_double2(0.0, 0.0);
        if (transR) Rout[j * n + i] = v;
        else Rout[i * n + j] = v;
    }
    __syncthreads();
    // form Q in place (zung2r)
    for (int i = n - 1; i >= 0; --i) {
        const double2 tau = tau_s[i];
        for (int j0 = i + 1; j0 < n; j0 += CP) {
            const int j = j0 + jc;
            double2 acc = make_double2(0.0, 0.0);
            if (j < n) {
                for (uint32_t rho = i + rp; rho < m; rho += RP) {
                    double2 v = rho == (uint32_t)i ? make_double2(1.0, 0.0) : A[qr_addr(rho, i, n, R)];
                    cfmac(acc, v, A[qr_addr(rho, j, n, R)]);
                }
            }
            red2[rp * CP + jc] = acc;
            __syncthreads();
            if (rp == 0) {
                double2 s = make_double2(0.0, 0.0);
                for (int q = 0; q < RP; ++q) s = cadd(s, red2[q * CP + jc]);
                wcol[jc] = s;
            }
            __syncthreads();
            if (j < n) {
                const double2 f = cmul(tau, wcol[jc]);
                for (uint32_t rho = i + rp; rho < m; rho += RP) {
                    double2 v = rho == (uint32_t)i ? make_double2(1.0, 0.0) : A[qr_addr(rho, i, n, R)];
                    size_t a = qr_addr(rho, j, n, R);
                    A[a] = csub(A[a], cmul(v, f));
                }
            }
            __syncthreads();
        }
        const double2 mt = make_double2(-tau.x, -tau.y);
        for (uint32_t rho = tid; rho < m; rho += nt) {
            size_t a = qr_addr(rho, i, n, R);
            if (rho > (uint32_t)i) A[a] = cmul(mt, A[a]);
            else if (rho == (uint32_t)i) A[a] = make_double2(1.0 - tau.x, -tau.y);
            else A[a] = make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
}

// ============================================================ QR (many work-groups)
// The same Householder reflectors (LAPACK convention and zero-snap) computed by
// one launch per column: launch i applies reflector i-1 to the work-group's own
// rows and, in the same pass, reduces the norm of column i below the diagonal
// and its unscaled inner products g_j = x_i^H a_j with the trailing columns
// (v_i^H a_j = a_ij + conj(1/(alpha-beta)) g_j needs no second pass).  The last
// work-group to finish forms tau_i, beta_i and w_ij.  Q = I - V T V^H (compact
// WY form, T from the reflector Gram matrix) is built by two final launches.
constexpr int QRM_MAXN = 64;
constexpr int QRM_THREADS = 256;

__device__ __forceinline__ double2 qr_v(const double2 *A, uint32_t rho, int k, int n, uint32_t R) {
    // reflector k at row rho: 0 above the diagonal, 1 on it, stored below it
    if (rho < (uint32_t)k) return make_double2(0.0, 0.0);
    if (rho == (uint32_t)k) return make_double2(1.0, 0.0);
    return A[qr_addr(rho, k, n, R)];
}

// apply reflector k (already decided) to the rows [r0, r1): scale its column,
// set the diagonal, update trailing columns j > k
__device__ void qrm_apply(double2 *A, uint32_t r0, uint32_t r1, int k, int n, uint32_t R, const QRWork &q) {
    const double2 tau = q.tau[k], scl = q.scl[k];
    const int snapped = q.snapped[k];
    const bool has = tau.x != 0.0 || tau.y != 0.0;
    const uint32_t lo = max(r0, (uint32_t)k + 1);
    for (uint32_t rho = lo + threadIdx.x; rho < r1; rho += blockDim.x) {
        size_t a = qr_addr(rho, k, n, R);
        if (snapped) A[a] = make_double2(0.0, 0.0);
        else if (has) A[a] = cmul(A[a], scl);
    }
    if (threadIdx.x == 0 && (uint32_t)k >= r0 && (uint32_t)k < r1) A[qr_addr(k, k, n, R)] = q.diag[k];
    __syncthreads();
    if (!has) return;
    const double2 ct = make_double2(tau.x, -tau.y);
    const int nt = n - k - 1;
    if (nt <= 0) return;
    const uint32_t rs = max(r0, (uint32_t)k);
    const uint32_t rows = r1 > rs ? r1 - rs : 0;
    for (uint32_t e = threadIdx.x; e < rows * (uint32_t)nt; e += blockDim.x) {
        const uint32_t rho = rs + e / nt;
        const int j = k + 1 + (int)(e % nt);
        const double2 v = qr_v(A, rho, k, n, R);
        const size_t a = qr_addr(rho, j, n, R);
        A[a] = csub(A[a], cmul(v, cmul(ct, q.w[k * QRM_MAXN + j])));
    }
    __syncthreads();
}

__global__ void __launch_bounds__(QRM_THREADS) k_qrm_step(double2 *A, uint32_t L, int n, uint32_t R, int i,
                                                          uint32_t rows_per, QRWork q, double snap) {
    if (q.gate && *q.gate == 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    const int tid = threadIdx.x;
    __shared__ double2 red2[4 * 64];
    __shared__ double red1[16];
    if (i > 0) qrm_apply(A, r0, r1, i - 1, n, R, q);
    // partial sums of column i
    const int K = 2 + 2 * QRM_MAXN;  // doubles per block: xn2, fro, g_j (complex)
    double *part = q.part + (size_t)blockIdx.x * K;
    double xp = 0.0, fp = 0.0;
    const uint32_t lo = max(r0, (uint32_t)i + 1);
    for (uint32_t rho = lo + tid; rho < r1; rho += blockDim.x) xp += cabs2(A[qr_addr(rho, i, n, R)]);
    if (i == 0)
        for (uint32_t e = tid; e < (r1 - r0) * (uint32_t)n; e += blockDim.x)
            fp += cabs2(A[qr_addr(r0 + e / n, e % n, n, R)]);
    const double xs = blk_sum1(xp, red1);
    const double fs = blk_sum1(fp, red1);
    const int jc = tid % 64, rp = tid / 64;  // 64 column slots x 4 row phases
    const int j = i + 1 + jc;
    double2 acc = make_double2(0.0, 0.0);
    if (j < n)
        for (uint32_t rho = lo + rp; rho < r1; rho += 4) cfmac(acc, A[qr_addr(rho, i, n, R)], A[qr_addr(rho, j, n, R)]);
    red2[rp * 64 + jc] = acc;
    __syncthreads();
    if (tid == 0) {
        part[0] = xs;
        part[1] = fs;
    }
    if (rp == 0 && j < n) {
        double2 g = cadd(cadd(red2[jc], red2[64 + jc]), cadd(red2[128 + jc], red2[192 + jc]));
        part[2 + 2 * j] = g.x;
        part[3 + 2 * j] = g.y;
    }
    if ((uint32_t)i >= r0 && (uint32_t)i < r1)
        for (int c = i + tid; c < n; c += blockDim.x) q.rowi[c] = A[qr_addr(i, c, n, R)];
    if (last_block_ticket(q.counter)) {
        __shared__ double sums[2 + 2 * QRM_MAXN];
        __shared__ double2 sc[2];
        __shared__ double stage[KRY_STAGE];
        blk_reduce_staged(q.part, gridDim.x, K, 2 + 2 * n, sums, stage);
        __syncthreads();
        if (tid == 0) {
            double xn2 = sums[0];
            if (i == 0) q.thr[0] = snap * sqrt(sums[1]);
            const double thr = q.thr[0];
            double2 alpha = q.rowi[i];
            int snapped = 0;
            if (snap > 0.0 && sqrt(xn2) <= thr) {
                snapped = 1;
                xn2 = 0.0;
                if (fabs(alpha.y) <= thr) alpha.y = 0.0;
            }
            double2 tau = make_double2(0.0, 0.0), scl = make_double2(0.0, 0.0), diag = alpha;
            if (!(xn2 == 0.0 && alpha.y == 0.0)) {
                const double beta = -copysign(sqrt(cabs2(alpha) + xn2), alpha.x);
                tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                scl = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
                diag = make_double2(beta, 0.0);
            }
            q.tau[i] = tau;
            q.scl[i] = scl;
            q.diag[i] = diag;
            q.snapped[i] = snapped;
            sc[0] = scl;
            sc[1] = make_double2((double)snapped, 0.0);
        }
        __syncthreads();
        const double2 cs = make_double2(sc[0].x, -sc[0].y);
        const bool snapped = sc[1].x != 0.0;
        for (int c = i + 1 + tid; c < n; c += blockDim.x) {
            const double2 g = snapped ? make_double2(0.0, 0.0) : make_double2(sums[2 + 2 * c], sums[3 + 2 * c]);
            q.w[i * QRM_MAXN + c] = cadd(q.rowi[c], cmul(cs, g));
        }
        if (tid == 0) *q.counter = 0;
    }
}

// applies the last reflector, writes R, reduces the reflector Gram matrix and
// (last block) builds K = T V_top^H
__global__ void __launch_bounds__(QRM_THREADS) k_qrm_finish(double2 *A, uint32_t L, int n, uint32_t R,
                                                            uint32_t rows_per, QRWork q, double2 *Rout, int transR) {
    if (q.gate && *q.gate == 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    const int tid = threadIdx.x;
    qrm_apply(A, r0, r1, n - 1, n, R, q);
    if (blockIdx.x == 0) {
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int i = e / n, j = e % n;
            const double2 v = j >= i ? A[qr_addr(i, j, n, R)] : make_double2(0.0, 0.0);
            if (transR) Rout[j * n + i] = v;
            else Rout[i * n + j] = v;
        }
    }
    // partial Gram S[k][l] = sum_rho conj(V[rho,k]) V[rho,l], k < l, over own rows
    const int npair = n * (n - 1) / 2;
    double2 *Sp = q.S + (size_t)blockIdx.x * npair;
    for (int pidx = tid; pidx < npair; pidx += blockDim.x) {
        // decode pair index -> (k, l) with k < l
        int k = 0, rem = pidx;
        while (rem >= n - 1 - k) {
            rem -= n - 1 - k;
            ++k;
        }
        const int l = k + 1 + rem;
        double2 acc = make_double2(0.0, 0.0);
        for (uint32_t rho = max(r0, (uint32_t)l); rho < r1; ++rho)
            cfmac(acc, qr_v(A, rho, k, n, R), qr_v(A, rho, l, n, R));
        Sp[pidx] = acc;
    }
    if (last_block_ticket(q.counter)) {
        extern __shared__ double2 sq[];
        double2 *T = sq;              // n*n
        double2 *S = sq + n * n;      // n*n
        for (int e = tid; e < n * n; e += blockDim.x) {
            T[e] = make_double2(0.0, 0.0);
            S[e] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        {
            const int sub = tid & 7;
            const double *Sd = reinterpret_cast<const double *>(q.S);
            for (int p0 = 0; p0 < 2 * npair; p0 += (int)blockDim.x / 8) {
                const int pq = p0 + tid / 8;  // double index: pair pq/2, component pq%2
                double acc = 0.0;
                if (pq < 2 * npair)
                    for (unsigned b = sub; b < gridDim.x; b += 8) acc += Sd[(size_t)b * 2 * npair + pq];
                acc += __shfl_xor(acc, 4, 64);
                acc += __shfl_xor(acc, 2, 64);
                acc += __shfl_xor(acc, 1, 64);
                if (pq < 2 * npair && sub == 0) {
                    int k = 0, rem = pq / 2;
                    while (rem >= n - 1 - k) {
                        rem -= n - 1 - k;
                        ++k;
                    }
                    const int l = k + 1 + rem;
                    double *dst = reinterpret_cast<double *>(&S[k * n + l]);
                    dst[pq % 2] = acc;
                }
            }
        }
        __syncthreads();
        // T (upper triangular): T_ii = tau_i, T[0:i, i] = -tau_i T[0:i,0:i] S[0:i, i]
        for (int i = 0; i < n; ++i) {
            const double2 ti = q.tau[i];
            double2 val = make_double2(0.0, 0.0);
            if (tid < i) {
                for (int l = tid; l < i; ++l) cfma(val, T[tid * n + l], S[l * n + i]);
                val = cmul(make_double2(-ti.x, -ti.y), val);
            }
            __syncthreads();
            if (tid < i) T[tid * n + i] = val;
            if (tid == 0) T[i * n + i] = ti;
            __syncthreads();
        }
        // K[i][c] = sum_l T[i][l] conj(Vtop[c][l])
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int i = e / n, c = e % n;
            double2 acc = make_double2(0.0, 0.0);
            for (int l = i; l < n; ++l) {
                const double2 v = qr_v(A, (uint32_t)c, l, n, R);
                acc = cadd(acc, cmul(T[i * n + l], make_double2(v.x, -v.y)));
            }
            q.K[e] = acc;
        }
        if (tid == 0) *q.counter = 0;
    }
}

// Q[rho, c] = delta_{rho c} - sum_i V[rho, i] K[i, c], in place, tiles of 16 rows
__global__ void __launch_bounds__(QRM_THREADS) k_qrm_formq(double2 *A, uint32_t L, int n, uint32_t R,
                                                           uint32_t rows_per, QRWork q) {
    if (q.gate && *q.gate == 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    extern __shared__ double2 sf[];
    double2 *Ks = sf;           // n*n
    double2 *Vt = sf + n * n;   // 16*n
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Ks[e] = q.K[e];
    for (uint32_t t0 = r0; t0 < r1; t0 += 16) {
        const uint32_t tr = min(16u, r1 - t0);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < tr * (uint32_t)n; e += blockDim.x) {
            const uint32_t rho = t0 + e / n;
            const int k = (int)(e % n);
            Vt[e] = qr_v(A, rho, k, n, R);
        }
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < tr * (uint32_t)n; e += blockDim.x) {
            const uint32_t rr = e / n, rho = t0 + rr;
            const int c = (int)(e % n);
            double2 acc = make_double2(rho == (uint32_t)c ? 1.0 : 0.0, 0.0);
            for (int i = 0; i < n; ++i) acc = csub(acc, cmul(Vt[rr * n + i], Ks[i * n + c]));
            A[qr_addr(rho, c, n, R)] = acc;
        }
    }
}

// ============================================================ QR (one cooperative launch)
constexpr int QRC_STAGE = 4096;  // doubles of LDS staging for the per-column reduction
constexpr int PROF_TS_MAX = 8192;  // cooperative launches the launch profiler times per collection
// Grid-wide barrier for a co-resident grid: every work-group adds one to a
// 64-bit arrival counter that only grows and waits until it reaches `target`
// (the host advances its base by the arrivals of each launch, so no reset and
// no second generation word sit on the critical path).  A bounded spin records
// a failure in *fail instead of waiting for ever; the arrival itself is never
// skipped, so the count stays consistent after a failure.
__device__ void grid_barrier(unsigned long long *cnt, unsigned long long target, unsigned *fail) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 24)) {
                __hip_atomic_store(fail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// The reflectors of k_qrm_step / k_qrm_finish / k_qrm_formq in a single launch:
// every work-group owns rows [r0, r1); after each column's partial sums a
// grid-wide barrier lets every work-group reduce them in the same fixed order,
// so all work-groups hold identical reflector parameters in LDS and apply
// them to their rows without another launch.  Partials are double-buffered by
// column parity (a work-group may write column i+1 while another still reads
// column i).
// The work-group's rows stay in LDS (At, row-major (rows_per, n)) from the
// first load to the final write of Q; only the per-column partial records,
// the reflector Gram partials and K pass through global memory.
__device__ __forceinline__ double2 tile_v(const double2 *At, uint32_t r0, uint32_t rho, int k, int n) {
    if (rho < (uint32_t)k) return make_double2(0.0, 0.0);
    if (rho == (uint32_t)k) return make_double2(1.0, 0.0);
    return At[(size_t)(rho - r0) * n + k];
}

__global__ void __launch_bounds__(QRM_THREADS) k_qr_coop(double2 *A, uint32_t L, int n, uint32_t R,
                                                          uint32_t rows_per, QRWork q, double2 *Rout, int transR,
                                                          double snap, unsigned long long *ts) {
    extern __shared__ double2 sq[];
    // launch profiler only: earliest work-group start and latest end on the
    // device's constant-rate clock (a cooperative launch takes no dispatch events)
    if (ts && threadIdx.x == 0) atomicMin(ts, (unsigned long long)wall_clock64());
    if (q.gate && *q.gate == 0) {
        // not needed: the work-group still makes the n + 2 barrier arrivals the
        // host has counted for this launch, then leaves
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(reinterpret_cast<unsigned long long *>(q.bar), (unsigned long long)(n + 2),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (ts) atomicMax(ts + PROF_TS_MAX, (unsigned long long)wall_clock64());
        }
        return;
    }
    const uint32_t m = L * R;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t r0 = b * rows_per, r1 = min(m, r0 + rows_per);
    const uint32_t nr = r1 - r0;
    const int tid = threadIdx.x;
    double2 *At = sq;                          // nr * n
    double2 *aux = sq + (size_t)rows_per * n;  // staging / T,S / K
    __shared__ double2 s_w[QRM_MAXN];
    __shared__ double2 s_tau, s_scl, s_diag;
    __shared__ int s_snapped;
    __shared__ double s_thr;
    __shared__ double s_sum[QRC_REC];
    __shared__ double2 red2[256];
    __shared__ double red1[16];
    unsigned long long *bar_cnt = reinterpret_cast<unsigned long long *>(q.bar);
    unsigned long long bar_tgt = q.bar_base;
    for (uint32_t e = tid; e < nr * (uint32_t)n; e += blockDim.x) {
        const uint32_t rho = r0 + e / n;
        At[e] = A[qr_addr(rho, (int)(e % n), n, R)];
    }
    __syncthreads();
    for (int i = 0; i <= n; ++i) {
        if (i > 0) {  // apply reflector k = i - 1 to the own rows
            const int k = i - 1;
            const double2 tau = s_tau, scl = s_scl;
            const bool has = tau.x != 0.0 || tau.y != 0.0;
            const uint32_t lo = max(r0, (uint32_t)k + 1);
            for (uint32_t rho = lo + tid; rho < r1; rho += blockDim.x) {
                double2 &a = At[(size_t)(rho - r0) * n + k];
                if (s_snapped) a = make_double2(0.0, 0.0);
                else if (has) a = cmul(a, scl);
            }
            if (tid == 0 && (uint32_t)k >= r0 && (uint32_t)k < r1) At[(size_t)(k - r0) * n + k] = s_diag;
            __syncthreads();
            const int nt = n - k - 1;
            if (has && nt > 0) {
                const double2 ct = make_double2(tau.x, -tau.y);
                const uint32_t rs = max(r0, (uint32_t)k);
                const uint32_t rows = r1 > rs ? r1 - rs : 0;
                for (uint32_t e = tid; e < rows * (uint32_t)nt; e += blockDim.x) {
                    const uint32_t rho = rs + e / nt;
                    const int j = k + 1 + (int)(e % nt);
                    const double2 v = tile_v(At, r0, rho, k, n);
                    double2 &a = At[(size_t)(rho - r0) * n + j];
                    a = csub(a, cmul(v, cmul(ct, s_w[j])));
                }
            }
            __syncthreads();
        }
        if (i == n) break;
        // partial sums of column i over the own rows
        double *rec = q.cpart + ((size_t)(i & 1) * QRM_BLOCKS_MAX + b) * QRC_REC;
        double xp = 0.0, fp = 0.0;
        const uint32_t lo = max(r0, (uint32_t)i + 1);
        for (uint32_t rho = lo + tid; rho < r1; rho += blockDim.x) xp += cabs2(At[(size_t)(rho - r0) * n + i]);
        if (i == 0)
            for (uint32_t e = tid; e < nr * (uint32_t)n; e += blockDim.x) fp += cabs2(At[e]);
        xp = wave_sum(xp);
        fp = wave_sum(fp);
        if ((tid & 63) == 0) {
            red1[tid >> 6] = xp;
            red1[8 + (tid >> 6)] = fp;
        }
        const int nt = n - i - 1;
        const int P = nt > 0 ? (int)blockDim.x / nt : 0;  // row phases per trailing column
        if (nt > 0 && tid < P * nt) {
            const int jc = tid % nt, ph = tid / nt;
            const int j = i + 1 + jc;
            double2 acc = make_double2(0.0, 0.0);
            for (uint32_t rho = lo + ph; rho < r1; rho += P) {
                const double2 *row = At + (size_t)(rho - r0) * n;
                cfmac(acc, row[i], row[j]);
            }
            red2[ph * nt + jc] = acc;
        }
        __syncthreads();
        if (tid == 0) {
            double xs = 0.0, fs = 0.0;
            for (int w = 0; w < ((int)blockDim.x + 63) >> 6; ++w) {
                xs += red1[w];
                fs += red1[8 + w];
            }
            rec[0] = xs;
            rec[1] = fs;
        }
        if (tid < nt) {
            double2 g = make_double2(0.0, 0.0);
            for (int ph = 0; ph < P; ++ph) g = cadd(g, red2[ph * nt + tid]);
            const int j = i + 1 + tid;
            rec[2 + 2 * j] = g.x;
            rec[3 + 2 * j] = g.y;
        }
        if ((uint32_t)i >= r0 && (uint32_t)i < r1)
            for (int c = i + tid; c < n; c += blockDim.x) {
                const double2 v = At[(size_t)(i - r0) * n + c];
                rec[2 + 2 * QRM_MAXN + 2 * c] = v.x;
                rec[3 + 2 * QRM_MAXN + 2 * c] = v.y;
            }
        grid_barrier(bar_cnt, bar_tgt += G, q.bar + 128);
        // every work-group reduces the partials in the same order: chunks of
        // values are staged through LDS with independent loads, then 8 lanes
        // per value sum strided partials and combine them by shuffles
        const double *recs = q.cpart + (size_t)(i & 1) * QRM_BLOCKS_MAX * QRC_REC;
        const uint32_t own = (uint32_t)i / rows_per;
        // the owner's row i is independent of the sums: its loads go out first
        for (int t = tid; t < 2 * n; t += blockDim.x)
            s_sum[2 + 2 * QRM_MAXN + t] = recs[(size_t)own * QRC_REC + 2 + 2 * QRM_MAXN + t];
        {
            double *stage = reinterpret_cast<double *>(aux);  // QRC_STAGE doubles
            const int nv = 2 + 2 * n;
            const int ch = max(1, min(nv, QRC_STAGE / (int)G));
            const int groups = (int)blockDim.x / 8;
            for (int v0 = 0; v0 < nv; v0 += ch) {
                const int cnt = min(ch, nv - v0);
                for (int e = tid; e < (int)G * cnt; e += blockDim.x) {
                    const int bb = e / cnt, t = e - bb * cnt;
                    stage[e] = recs[(size_t)bb * QRC_REC + v0 + t];
                }
                __syncthreads();
                const int sub = tid & 7;
                for (int t0 = 0; t0 < cnt; t0 += groups) {  // uniform trip count: every lane shuffles
                    const int t = t0 + tid / 8;
                    double sacc = 0.0;
                    if (t < cnt)
                        for (int bb = sub; bb < (int)G; bb += 8) sacc += stage[bb * cnt + t];
                    sacc += __shfl_xor(sacc, 4, 64);
                    sacc += __shfl_xor(sacc, 2, 64);
                    sacc += __shfl_xor(sacc, 1, 64);
                    if (t < cnt && sub == 0) s_sum[v0 + t] = sacc;
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            double xn2 = s_sum[0];
            if (i == 0) s_thr = snap * sqrt(s_sum[1]);
            const double thr = s_thr;
            double2 alpha = make_double2(s_sum[2 + 2 * QRM_MAXN + 2 * i], s_sum[3 + 2 * QRM_MAXN + 2 * i]);
            int snapped = 0;
            if (snap > 0.0 && sqrt(xn2) <= thr) {
                snapped = 1;
                xn2 = 0.0;
                if (fabs(alpha.y) <= thr) alpha.y = 0.0;
            }
            double2 tau = make_double2(0.0, 0.0), scl = make_double2(0.0, 0.0), diag = alpha;
            if (!(xn2 == 0.0 && alpha.y == 0.0)) {
                const double beta = -copysign(sqrt(cabs2(alpha) + xn2), alpha.x);
                tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
                scl = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
                diag = make_double2(beta, 0.0);
            }
            s_tau = tau;
            s_scl = scl;
            s_diag = diag;
            s_snapped = snapped;
            if (b == 0) q.tau[i] = tau;
        }
        __syncthreads();
        {
            const double2 cs = make_double2(s_scl.x, -s_scl.y);
            for (int c = i + 1 + tid; c < n; c += blockDim.x) {
                const double2 g = s_snapped ? make_double2(0.0, 0.0) : make_double2(s_sum[2 + 2 * c], s_sum[3 + 2 * c]);
                const double2 rowc = make_double2(s_sum[2 + 2 * QRM_MAXN + 2 * c], s_sum[3 + 2 * QRM_MAXN + 2 * c]);
                s_w[c] = cadd(rowc, cmul(cs, g));
            }
        }
        __syncthreads();
    }
    // R factor (rows 0..n-1 live in work-group 0 since rows_per >= n)
    if (b == 0)
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int i = e / n, j = e % n;
            const double2 v = j >= i ? At[(size_t)i * n + j] : make_double2(0.0, 0.0);
            if (transR) Rout[j * n + i] = v;
            else Rout[i * n + j] = v;
        }
    // partial reflector Gram matrix S[k][l] = sum_rho conj(V[rho,k]) V[rho,l], k < l, over the own rows
    const int npair = n * (n - 1) / 2;
    double2 *Sp = q.S + (size_t)b * npair;
    for (int pidx = tid; pidx < npair; pidx += blockDim.x) {
        int k = 0, rem = pidx;
        while (rem >= n - 1 - k) {
            rem -= n - 1 - k;
            ++k;
        }
        const int l = k + 1 + rem;
        double2 sacc = make_double2(0.0, 0.0);
        for (uint32_t rho = max(r0, (uint32_t)l); rho < r1; ++rho)
            cfmac(sacc, tile_v(At, r0, rho, k, n), tile_v(At, r0, rho, l, n));
        Sp[pidx] = sacc;
    }
    grid_barrier(bar_cnt, bar_tgt += G, q.bar + 128);
    if (b == 0) {  // T (compact WY) and K = T V_top^H, as in k_qrm_finish
        double2 *T = aux;          // n*n
        double2 *S = aux + n * n;  // n*n
        for (int e = tid; e < n * n; e += blockDim.x) {
            T[e] = make_double2(0.0, 0.0);
            S[e] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int pidx = tid; pidx < npair; pidx += blockDim.x) {
            double2 sacc = make_double2(0.0, 0.0);
            for (uint32_t bb = 0; bb < G; ++bb) sacc = cadd(sacc, q.S[(size_t)bb * npair + pidx]);
            int k = 0, rem = pidx;
            while (rem >= n - 1 - k) {
                rem -= n - 1 - k;
                ++k;
            }
            S[k * n + k + 1 + rem] = sacc;
        }
        __syncthreads();
        for (int i = 0; i < n; ++i) {
            const double2 ti = q.tau[i];
            double2 val = make_double2(0.0, 0.0);
            if (tid < i) {
                for (int l = tid; l < i; ++l) cfma(val, T[tid * n + l], S[l * n + i]);
                val = cmul(make_double2(-ti.x, -ti.y), val);
            }
            __syncthreads();
            if (tid < i) T[tid * n + i] = val;
            if (tid == 0) T[i * n + i] = ti;
            __syncthreads();
        }
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int i = e / n, c = e % n;
            double2 kacc = make_double2(0.0, 0.0);
            for (int l = i; l < n; ++l) {
                const double2 v = tile_v(At, 0, (uint32_t)c, l, n);
                kacc = cadd(kacc, cmul(T[i * n + l], make_double2(v.x, -v.y)));
            }
            q.K[e] = kacc;
        }
    }
    grid_barrier(bar_cnt, bar_tgt += G, q.bar + 128);
    // Q[rho, c] = delta - sum_i V[rho, i] K[i, c] on the own rows, written to A
    double2 *Ks = aux;
    for (int e = tid; e < n * n; e += blockDim.x) Ks[e] = q.K[e];
    __syncthreads();
    for (uint32_t e = tid; e < nr * (uint32_t)n; e += blockDim.x) {
        const uint32_t rr = e / n, rho = r0 + rr;
        const int c = (int)(e % n);
        double2 qacc = make_double2(rho == (uint32_t)c ? 1.0 : 0.0, 0.0);
        for (int i = 0; i < n; ++i) qacc = csub(qacc, cmul(tile_v(At, r0, rho, i, n), Ks[i * n + c]));
        A[qr_addr(rho, c, n, R)] = qacc;
    }
    if (ts) {
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(ts + PROF_TS_MAX, (unsigned long long)wall_clock64());
    }
}

// ============================================================ QR (Cholesky route)
// For a matrix A of full column rank (rows (l, r) of A[l, j, r] as in qr_addr):
// G1 = A^H A = R1^H R1, Y = A R1^{-1}, G2 = Y^H Y = R2^H R2, Q' = Y R2^{-1} and
// R' = R2 R1 (Cholesky QR applied twice: Q' orthonormal to rounding while the
// first pass leaves Y^H Y near the identity; R' has a positive real diagonal).
// Householder reflections of A and of Q' coincide (their columns differ by
// positive factors), and for orthonormal Q' the reflectors' alphas are the
// pivots p_i of the LU factorisation without pivoting of the leading block
// Q'_1 - S, S = diag(s_i), s_i = -sign(Re p_i) (the Householder reconstruction
// of Ballard, Demmel, Grigori, Jacobsen, Knight and Nguyen).  The LAPACK
// factors are then Q = Q' S and R = S R'.  The sub-column a Householder step
// would test against the zero-snap has norm R'_ii sqrt(1 - |p_i|^2); when one
// is below CQR_XTOL |A|_F, a Cholesky factorisation breaks down, or Y^H Y is
// further than CQR_ORTH_TOL from the identity, *cq_state is set to 1 and the
// Householder kernels launched behind this route (gate = cq_state) run.
constexpr double CQR_XTOL = 1e-6;
constexpr double CQR_ORTH_TOL = 0.1;
constexpr int CQR_THREADS = 256;
constexpr int CQR_RTHREADS = 512;

// tile of CQR_TILE rows starting at t0 into Xs (row stride ld), zero beyond r1
__device__ __forceinline__ void cqr_load(double2 *Xs, int ld, const double2 *A, uint32_t t0, uint32_t r1, int n,
                                         uint32_t R) {
    if (R == 1) {
        for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
            const uint32_t rho = t0 + (uint32_t)(e / n);
            const int c = e % n;
            Xs[(e / n) * ld + c] = rho < r1 ? A[(size_t)rho * n + c] : make_double2(0.0, 0.0);
        }
    } else {  // consecutive rows are consecutive addresses within one l
        for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
            const int rr = e % CQR_TILE, c = e / CQR_TILE;
            const uint32_t rho = t0 + (uint32_t)rr;
            Xs[rr * ld + c] = rho < r1 ? A[qr_addr(rho, c, n, R)] : make_double2(0.0, 0.0);
        }
    }
}

// Xs (CQR_TILE x n) <- Xs Ms for upper-triangular Ms (n x n, zeros below the
// diagonal); thread (rb, db) owns rows 4 rb.. and columns 4 db..
__device__ __forceinline__ void cqr_tile_times_upper(double2 *Xs, int ld, const double2 *Ms, int n) {
    const int rb = threadIdx.x >> 4, db = threadIdx.x & 15;
    double2 y[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) y[i][j] = make_double2(0.0, 0.0);
    if (4 * db < n) {
        const int cmax = min(n, 4 * db + 4);
        for (int c = 0; c < cmax; ++c) {
            double2 mr[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) mr[j] = 4 * db + j < n ? Ms[c * n + 4 * db + j] : make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double2 x = Xs[(4 * rb + i) * ld + c];
#pragma unroll
                for (int j = 0; j < 4; ++j) cfma(y[i][j], x, mr[j]);
            }
        }
    }
    __syncthreads();
    if (4 * db < n)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * db + j < n) Xs[(4 * rb + i) * ld + 4 * db + j] = y[i][j];
    __syncthreads();
}

// Gram partials of the work-group's rows: pass 1 of A itself; pass 2 (APPLY) of
// Y = A R1^{-1}, which is also written to cq_Y (row-major m x n)
template <bool APPLY>
__global__ void __launch_bounds__(CQR_THREADS) k_cqr_gram(const double2 *A, uint32_t L, int n, uint32_t R,
                                                          uint32_t rows_per, QRWork q) {
    if (APPLY && *q.cq_state != 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    extern __shared__ double2 sc[];
    const int ld = n + 1;
    double2 *Xs = sc;
    double2 *Ms = sc + CQR_TILE * ld;
    if (APPLY)
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) Ms[e] = q.cq_R1inv[e];
    const int cb = threadIdx.x >> 4, db = threadIdx.x & 15;
    const bool act = 4 * cb < n && 4 * db < n;
    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
    int ci[4], dj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ci[i] = min(4 * cb + i, n - 1);
        dj[i] = min(4 * db + i, n - 1);
    }
    for (uint32_t t0 = r0; t0 < r1; t0 += CQR_TILE) {
        cqr_load(Xs, ld, A, t0, r1, n, R);
        __syncthreads();
        if (APPLY) {
            cqr_tile_times_upper(Xs, ld, Ms, n);
            for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
                const uint32_t rho = t0 + (uint32_t)(e / n);
                if (rho < r1) q.cq_Y[(size_t)rho * n + e % n] = Xs[(e / n) * ld + e % n];
            }
        }
        if (act)
            for (int t = 0; t < CQR_TILE; ++t) {
                double2 a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    a[i] = Xs[t * ld + ci[i]];
                    b[i] = Xs[t * ld + dj[i]];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) cfmac(acc[i][j], a[i], b[j]);
            }
        __syncthreads();
    }
    if (act) {
        double2 *part = q.cq_part + (size_t)blockIdx.x * n * n;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * cb + i < n && 4 * db + j < n) part[(4 * cb + i) * n + 4 * db + j] = acc[i][j];
    }
}

// The same Gram partials on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// G = X^H X as one real GEMM over the realified rows of each LDS tile, the A
// operand (Re, Im) of X[t][i] at K = (2t, 2t+1), column 2j of the B operand
// (Re, Im) of X[t][j] (giving Re G[i][j]) and column 2j+1 (Im, -Re) (giving
// Im G[i][j]).  RT x CT output tiles of 16 x 16 (RT = ceil(n / 16), CT =
// ceil(2n / 16)); wave w owns the contiguous run of tiles
// [w TPW, (w + 1) TPW) over the whole K of every tile of rows.
template <bool APPLY, int RT, int CT>
__global__ void __launch_bounds__(CQR_THREADS) k_cqr_gram_mfma(const double2 *A, uint32_t L, int n, uint32_t R,
                                                               uint32_t rows_per, QRWork q) {
    constexpr int TPW = (RT * CT + 3) / 4;  // tiles per wave
    if (APPLY && *q.cq_state != 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    extern __shared__ double2 sc[];
    const int ld = n + 1;
    double2 *Xs = sc;
    double2 *Ms = sc + CQR_TILE * ld;
    if (APPLY)
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) Ms[e] = q.cq_R1inv[e];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l16 = lane & 15, kq = lane >> 4;  // operand lane: row / column l16, K index kq
    f64x4 acc[TPW];
#pragma unroll
    for (int k = 0; k < TPW; ++k) acc[k] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (uint32_t t0 = r0; t0 < r1; t0 += CQR_TILE) {
        cqr_load(Xs, ld, A, t0, r1, n, R);
        __syncthreads();
        if (APPLY) {
            cqr_tile_times_upper(Xs, ld, Ms, n);
            for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
                const uint32_t rho = t0 + (uint32_t)(e / n);
                if (rho < r1) q.cq_Y[(size_t)rho * n + e % n] = Xs[(e / n) * ld + e % n];
            }
        }
        // K step s covers tile rows 2s, 2s + 1 (both parts): lane K index kq is row 2s + kq / 2, part kq % 2
        for (int s2 = 0; s2 < CQR_TILE / 2; ++s2) {
            const int t = 2 * s2 + (kq >> 1), part = kq & 1;
            const double2 *xr = Xs + t * ld;
#pragma unroll
            for (int k = 0; k < TPW; ++k) {
                const int tau = wave * TPW + k;
                if (tau < RT * CT) {
                    const int i = (tau / CT) * 16 + l16, jc = (tau % CT) * 16 + l16;
                    const int j = jc >> 1;
                    double a = 0.0, b = 0.0;
                    if (i < n) a = part ? xr[i].y : xr[i].x;
                    if (j < n) {
                        const double2 x = xr[j];
                        b = (jc & 1) ? (part ? -x.x : x.y) : (part ? x.y : x.x);
                    }
                    acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // register r of the lane holds row 4 r + lane / 16 of column lane % 16 of each 16 x 16 tile
    double *part = reinterpret_cast<double *>(q.cq_part + (size_t)blockIdx.x * n * n);
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int tau = wave * TPW + k;
        if (tau >= RT * CT) continue;
        const int jc = (tau % CT) * 16 + l16, j = jc >> 1;
        if (j >= n) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = (tau / CT) * 16 + 4 * r + kq;
            if (i < n) part[2 * ((size_t)i * n + j) + (jc & 1)] = acc[k][r];
        }
    }
}

// in-place upper Cholesky factor of the Hermitian G (n x n in LDS, G = R^H R);
// returns false when a pivot is not positive and finite
__device__ bool cqr_cholesky(double2 *G, int n) {
    __shared__ double s_rkk;
    __shared__ int s_ok;
    if (threadIdx.x == 0) s_ok = 1;
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double d = G[k * n + k].x;
            if (!(d > 0.0) || !isfinite(d)) s_ok = 0;
            s_rkk = d > 0.0 && isfinite(d) ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double rkk = s_rkk;
        for (int j = k + threadIdx.x; j < n; j += blockDim.x)
            G[k * n + j] = j == k ? make_double2(rkk, 0.0) : cscale(G[k * n + j], 1.0 / rkk);
        __syncthreads();
        const int w = n - k - 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            if (j >= i) {
                double2 g = G[i * n + j];
                const double2 a = G[k * n + i], b = G[k * n + j];
                g.x -= a.x * b.x + a.y * b.y;  // conj(a) b
                g.y -= a.x * b.y - a.y * b.x;
                G[i * n + j] = g;
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x)
        if (e / n > e % n) G[e] = make_double2(0.0, 0.0);
    __syncthreads();
    return s_ok != 0;
}

// X = R^{-1} for upper-triangular R with a real positive diagonal (both n x n
// in LDS): back substitution row by row, 8 lanes per column
__device__ void cqr_upper_inverse(const double2 *Rm, double2 *X, int n) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) X[e] = make_double2(0.0, 0.0);
    __syncthreads();
    const int j = threadIdx.x >> 3, sub = threadIdx.x & 7;
    for (int i = n - 1; i >= 0; --i) {
        double2 acc = make_double2(0.0, 0.0);
        if (j < n && j >= i)
            for (int k = i + 1 + sub; k <= j; k += 8) cfma(acc, Rm[i * n + k], X[k * n + j]);
        acc.x += __shfl_xor(acc.x, 4, 64);
        acc.y += __shfl_xor(acc.y, 4, 64);
        acc.x += __shfl_xor(acc.x, 2, 64);
        acc.y += __shfl_xor(acc.y, 2, 64);
        acc.x += __shfl_xor(acc.x, 1, 64);
        acc.y += __shfl_xor(acc.y, 1, 64);
        if (j < n && j >= i && sub == 0) {
            const double inv = 1.0 / Rm[i * n + i].x;
            X[i * n + j] = make_double2(((i == j ? 1.0 : 0.0) - acc.x) * inv, -acc.y * inv);
        }
        __syncthreads();
    }
}

// Reduces the Gram partials (64 entries per work-group, 8 lanes each, fixed
// order); the last work-group factorises.  Pass 1: R1, R1^{-1}, |A|_F^2 and the
// state.  Pass 2: R2, the checks, the signs S, M = R2^{-1} S and R = S R2 R1.
__global__ void __launch_bounds__(CQR_RTHREADS) k_cqr_reduce(int nb, int n, int pass, QRWork q, double2 *Rout,
                                                             int transR) {
    if (pass == 2 && *q.cq_state != 0) return;
    const int nn = n * n;
    {
        const int e = blockIdx.x * (CQR_RTHREADS / 8) + (int)(threadIdx.x >> 3), sub = threadIdx.x & 7;
        double2 acc = make_double2(0.0, 0.0);
        if (e < nn)
            for (int b = sub; b < nb; b += 8) acc = cadd(acc, q.cq_part[(size_t)b * nn + e]);
        acc.x += __shfl_xor(acc.x, 4, 64);
        acc.y += __shfl_xor(acc.y, 4, 64);
        acc.x += __shfl_xor(acc.x, 2, 64);
        acc.y += __shfl_xor(acc.y, 2, 64);
        acc.x += __shfl_xor(acc.x, 1, 64);
        acc.y += __shfl_xor(acc.y, 1, 64);
        if (e < nn && sub == 0) q.cq_G[e] = acc;
    }
    if (!last_block_ticket(q.cq_counter)) return;
    extern __shared__ double2 sr[];
    double2 *Gs = sr;       // n*n: G, then its Cholesky factor
    double2 *Xs = sr + nn;  // n*n: the factor's inverse
    __shared__ double s_red[CQR_RTHREADS / 64];
    __shared__ double s_sign[64], s_rdiag[64];
    __shared__ int s_ok;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) Gs[e] = q.cq_G[e];
    __syncthreads();
    if (threadIdx.x == 0) *q.cq_counter = 0;
    if (pass == 1) {
        if (threadIdx.x == 0) {
            double fro2 = 0.0;
            for (int i = 0; i < n; ++i) fro2 += Gs[i * n + i].x;
            q.cq_scal[0] = fro2;
        }
        const bool ok = cqr_cholesky(Gs, n);
        if (ok) cqr_upper_inverse(Gs, Xs, n);
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            q.cq_R1[e] = Gs[e];
            q.cq_R1inv[e] = Xs[e];
        }
        if (threadIdx.x == 0) *q.cq_state = ok ? 0 : 1;
        return;
    }
    // pass 2: Y^H Y must be near the identity
    double dev = 0.0;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const double2 g = Gs[e];
        dev = fmax(dev, sqrt(cabs2(make_double2(g.x - (e / n == e % n ? 1.0 : 0.0), g.y))));
    }
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = 0.0;
        for (int w = 0; w < CQR_RTHREADS / 64; ++w) d = fmax(d, s_red[w]);
        s_ok = d <= CQR_ORTH_TOL;
    }
    __syncthreads();
    bool ok = s_ok != 0;
    ok = cqr_cholesky(Gs, n) && ok;
    if (ok) cqr_upper_inverse(Gs, Xs, n);
    // R' = R2 R1 (upper triangular) into cq_G, the diagonal kept for the snap test
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double2 acc = make_double2(0.0, 0.0);
        for (int k = i; k <= j; ++k) cfma(acc, Gs[i * n + k], q.cq_R1[k * n + j]);
        q.cq_G[e] = acc;
        if (i == j) s_rdiag[i] = acc.x;
    }
    __syncthreads();
    // leading block of Q' = Y R2^{-1} into Gs (R2 is no longer needed)
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double2 acc = make_double2(0.0, 0.0);
        for (int k = 0; k <= j; ++k) cfma(acc, q.cq_Y[i * n + k], Xs[k * n + j]);
        Gs[e] = acc;
    }
    __syncthreads();
    // LU without pivoting of Q'_1 - S; s_i from the pivot met at step i
    const double thr = CQR_XTOL * sqrt(q.cq_scal[0]);
    if (threadIdx.x == 0) s_ok = ok;
    for (int i = 0; i < n; ++i) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double2 p = Gs[i * n + i];
            const double s = -copysign(1.0, p.x);
            const double xn = s_rdiag[i] * sqrt(fmax(0.0, 1.0 - cabs2(p)));
            if (!(xn > thr)) s_ok = 0;
            s_sign[i] = s;
            Gs[i * n + i] = make_double2(p.x - s, p.y);
        }
        __syncthreads();
        const double2 piv = Gs[i * n + i];
        const int w = n - i - 1;
        for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
            const int r = i + 1 + e / w, c = i + 1 + e % w;
            const double2 l = cdiv(Gs[r * n + i], piv);
            Gs[r * n + c] = csub(Gs[r * n + c], cmul(l, Gs[i * n + c]));
        }
    }
    __syncthreads();
    ok = s_ok != 0;
    if (ok) {
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            const int i = e / n, j = e % n;
            q.cq_M[e] = cscale(Xs[e], s_sign[j]);
            const double2 v = cscale(q.cq_G[e], s_sign[i]);
            if (transR) Rout[j * n + i] = v;
            else Rout[e] = v;
        }
    }
    if (threadIdx.x == 0) *q.cq_state = ok ? 0 : 1;
}

// Q = Y M on the work-group's rows, written to A in its own layout
__global__ void __launch_bounds__(CQR_THREADS) k_cqr_apply(double2 *A, uint32_t L, int n, uint32_t R,
                                                           uint32_t rows_per, QRWork q) {
    if (*q.cq_state != 0) return;
    const uint32_t m = L * R;
    const uint32_t r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
    extern __shared__ double2 sc[];
    const int ld = n + 1;
    double2 *Xs = sc;
    double2 *Ms = sc + CQR_TILE * ld;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Ms[e] = q.cq_M[e];
    for (uint32_t t0 = r0; t0 < r1; t0 += CQR_TILE) {
        cqr_load(Xs, ld, q.cq_Y, t0, r1, n, 1);
        __syncthreads();
        cqr_tile_times_upper(Xs, ld, Ms, n);
        if (R == 1) {
            for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
                const uint32_t rho = t0 + (uint32_t)(e / n);
                if (rho < r1) A[(size_t)rho * n + e % n] = Xs[(e / n) * ld + e % n];
            }
        } else {
            for (int e = threadIdx.x; e < CQR_TILE * n; e += blockDim.x) {
                const int rr = e % CQR_TILE, c = e / CQR_TILE;
                const uint32_t rho = t0 + (uint32_t)rr;
                if (rho < r1) A[qr_addr(rho, c, n, R)] = Xs[rr * ld + c];
            }
        }
        __syncthreads();
    }
}

// ============================================================ small matrix exponential
// y = exp(X) e_0 for X = -i tau H (H m x m row-major in LDS, m <= SMALL_MMAX), by
// Taylor series of degree 14 after scaling to ||X||_1 <= 1/2, then squaring.
// ws: 3*m*m complex LDS.  All threads of the block must call.
__device__ void blk_expm_col0(const double2 *H, int ldh, int m, double tau, double2 *ws, double *red,
                              double2 *y) {
    const int tid = threadIdx.x, nt = blockDim.x;
    double2 *X = ws, *P = ws + m * m, *T = ws + 2 * m * m;
    for (int q = tid; q < m * m; q += nt) {
        int i = q / m, j = q % m;
        double2 h = H[i * ldh + j];
        X[q] = make_double2(tau * h.y, -tau * h.x);
    }
    __syncthreads();
    double cs = 0.0;
    if (tid < m)
        for (int i = 0; i < m; ++i) cs += sqrt(cabs2(X[i * m + tid]));
    // max over columns via reduction of maxima
    const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
    for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
    if (lane == 0) red[wave] = cs;
    __syncthreads();
    double nrm = 0.0;
    for (int w = 0; w < nw; ++w) nrm = fmax(nrm, red[w]);
    int s = 0;
    while (nrm > 0.5 && s < 60) {
        nrm *= 0.5;
        ++s;
    }
    const double scale = ldexp(1.0, -s);
    __syncthreads();
    for (int q = tid; q < m * m; q += nt) {
        X[q] = cscale(X[q], scale);
        P[q] = make_double2((q / m) == (q % m) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // Horner form P <- I + X P / k and the squarings, ping-ponging between two
    // buffers (one barrier per product)
    for (int k = 14; k >= 1; --k) {
        const double inv = 1.0 / k;
        for (int q = tid; q < m * m; q += nt) {
            int i = q / m, c = q % m;
            double2 acc = make_double2(0.0, 0.0);
            for (int t = 0; t < m; ++t) cfma(acc, X[i * m + t], P[t * m + c]);
            acc = cscale(acc, inv);
            if (i == c) acc.x += 1.0;
            T[q] = acc;
        }
        __syncthreads();
        double2 *sw = P;
        P = T;
        T = sw;
    }
    for (int r = 0; r < s; ++r) {
        for (int q = tid; q < m * m; q += nt) {
            int i = q / m, c = q % m;
            double2 acc = make_double2(0.0, 0.0);
            for (int t = 0; t < m; ++t) cfma(acc, P[i * m + t], P[t * m + c]);
            T[q] = acc;
        }
        __syncthreads();
        double2 *sw = P;
        P = T;
        T = sw;
    }
    for (int i = tid; i < m; i += nt) y[i] = P[i * m];
    __syncthreads();
}

// ============================================================ fused small solver
// One work-group owns a local problem of N <= SMALL_MAX elements (one element
// per thread).  Krylov vectors live in global scratch (L2 resident), the
// current vector, the matvec result and the temporaries in LDS.

// entry fields the two-slot matvec reads, staged in LDS once per solve
struct EntLite {
    double2 coef;
    const double2 *M0;  // slot-0 factor (null: identity on slot 0)
    const double2 *M1;  // slot-1 factor (null: identity on slot 1)
    int lo0, hi0, lo1, hi1;
};

static_assert(sizeof(EntLite) <= 48, "EntLite must fit the static LDS budget of the fused solver");

struct SmallLds {
    double2 *v, *w, *r1, *Hm, *hbuf, *ybuf;
    double2 *us;                                   // partial sums of the entry groups (batched matvec)
    double *red1;
    int *e1;        // entries with a slot-1 factor (two-slot batched matvec)
    int *tix;       // per entry: index of its slot-1 temporary, -1 if none
    EntLite *ents;  // per entry (batched matvec)
    double2 *mb;    // the entries' factor matrices in LDS when args.mlds
    double2 *vb;    // Krylov basis in LDS ((mmax + 1) x N) when args.vlds
};

__device__ void blk_mode_lds(const double2 *src, double2 *dst, const double2 *M, const Geom &g, int s, int blo,
                             int bhi) {
    const int n = g.dims[s];
    const uint32_t R = (uint32_t)g.R[s], N = (uint32_t)g.N;
    for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) {
        uint32_t r = idx % R, t = idx / R;
        uint32_t i = t % n, l = t / n;
        const double2 *xp = src + (size_t)l * n * R + r;
        const double2 *mr = M + (size_t)i * n;
        double2 acc = make_double2(0.0, 0.0);
        const int j0 = max(0, (int)i - blo), j1 = min(n - 1, (int)i + bhi);
        for (int j = j0; j <= j1; ++j) cfma(acc, mr[j], xp[(size_t)j * R]);
        dst[idx] = acc;
    }
}

// generic matvec: entries one after the other, factors applied slot by slot
__device__ void blk_matvec_seq(const SmallSolveArgs &a, const double2 *v, double2 *w, double2 *t1, double2 *t2) {
    const uint32_t N = (uint32_t)a.g.N;
    for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) w[idx] = make_double2(0.0, 0.0);
    for (int e = 0; e < a.n_ent; ++e) {
        const DevEntry *E = a.ent + e;
        const int nf = E->nf;
        const double2 *cur = v;
        for (int f = 0; f < nf; ++f) {
            double2 *dst = (f & 1) ? t2 : t1;
            __syncthreads();
            blk_mode_lds(cur, dst, E->M[f], a.g, E->slot[f], E->lo[f], E->hi[f]);
            cur = dst;
        }
        __syncthreads();
        const double2 c = E->coef;
        for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) cfma(w[idx], c, cur[idx]);
    }
    __syncthreads();
}

// two-slot local problems (leaves (d, n) and bond matrices (n, n)):
//   phase A: T_e = X x_1 M1_e for every entry with a slot-1 factor
//   phase B: Y = sum_e c_e (M0_e x_0 T_e)
__device__ void blk_matvec_two(const SmallSolveArgs &a, const double2 *v, double2 *w, double2 *T, const int *e1,
                               const int *tix, double2 *Us, const EntLite *L_ents) {
    const int n0 = a.g.dims[0], n1 = a.g.dims[1];
    const uint32_t N = (uint32_t)(n0 * n1);
    const int na = a.nA;
    const EntLite *ents = L_ents;
    for (uint32_t q = threadIdx.x; q < (uint32_t)na * N; q += blockDim.x) {
        const uint32_t k = q / N, el = q - k * N;
        const EntLite &E = ents[e1[k]];
        const uint32_t ai = el / n1, p = el - ai * n1;
        const double2 *xr = v + (size_t)ai * n1;
        double2 acc = make_double2(0.0, 0.0);
        const int j0 = max(0, (int)p - E.lo1), j1 = min(n1 - 1, (int)p + E.hi1);
        if (a.mlds) {  // LDS copy is transposed: neighbouring lanes (p) read neighbouring words
            const double2 *mc = E.M1 + p;
            for (int j = j0; j <= j1; ++j) cfma(acc, mc[(size_t)j * n1], xr[j]);
        } else {
            const double2 *mr = E.M1 + (size_t)p * n1;
            for (int j = j0; j <= j1; ++j) cfma(acc, mr[j], xr[j]);
        }
        T[q] = acc;
    }
    __syncthreads();
    // phase B: entries split over G thread groups (round robin), partial sums in LDS
    const int Np = (int)((N + 63) / 64) * 64;
    int G = (int)blockDim.x / Np;
    if (G < 1) G = 1;
    const int gsz = G > 1 ? Np : (int)blockDim.x;  // one group strides over the whole work-group
    const int grp = (int)threadIdx.x / gsz, o = (int)threadIdx.x - grp * gsz;
    if (grp < G) {
        for (uint32_t idx = o; idx < N; idx += gsz) {
            const uint32_t i = idx / n1, p = idx - i * n1;
            double2 out = make_double2(0.0, 0.0);
            for (int e = grp; e < a.n_ent; e += G) {
                const EntLite &E = ents[e];
                const int k = tix[e];
                const double2 *S = k >= 0 ? T + (size_t)k * N : v;
                double2 r = make_double2(0.0, 0.0);
                if (E.M0) {
                    const double2 *mr = E.M0 + (size_t)i * n0;
                    const int j0 = max(0, (int)i - E.lo0), j1 = min(n0 - 1, (int)i + E.hi0);
                    for (int j = j0; j <= j1; ++j) cfma(r, mr[j], S[(size_t)j * n1 + p]);
                } else {
                    r = S[idx];
                }
                cfma(out, E.coef, r);
            }
            Us[(size_t)grp * N + idx] = out;
        }
    }
    __syncthreads();
    for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) {
        double2 out = Us[idx];
        for (int g = 1; g < G; ++g) out = cadd(out, Us[(size_t)g * N + idx]);
        w[idx] = out;
    }
    __syncthreads();
}

// h_i = <V_i, w> for i < nv; result in hbuf.  One wavefront per basis vector
// (round robin): its lanes stride over the elements and a single wavefront
// reduction finishes the dot, so each wave reduces only its own vectors.
// With want_norm, hbuf[nv] additionally receives (|w|^2, 0).
__device__ void blk_dots(const double2 *V, uint32_t N, int nv, const double2 *w, double2 *hbuf,
                         bool want_norm = false) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = (blockDim.x + 63) >> 6;
    const int nt = want_norm ? nv + 1 : nv;
    for (int i = wave; i < nt; i += nw) {
        double2 c = make_double2(0.0, 0.0);
        if (i < nv) {
            const double2 *vi = V + (size_t)i * N;
            for (uint32_t idx = lane; idx < N; idx += 64) cfmac(c, vi[idx], w[idx]);
        } else {
            for (uint32_t idx = lane; idx < N; idx += 64) c.x += cabs2(w[idx]);
        }
        c.x = wave_sum(c.x);
        c.y = wave_sum(c.y);
        if (lane == 0) hbuf[i] = c;
    }
    __syncthreads();
}

// w[idx] -= sum_i h_i V_i[idx] for the thread's elements (loads eight at a time)
__device__ void blk_sub_basis(const double2 *V, uint32_t N, int nv, const double2 *h, double2 *w) {
    for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) {
        double2 wv = w[idx];
        for (int i0 = 0; i0 < nv; i0 += 8) {
            double2 c[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = (i0 + q < nv) ? V[(size_t)(i0 + q) * N + idx] : make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (i0 + q < nv) wv = csub(wv, cmul(h[i0 + q], c[q]));
        }
        w[idx] = wv;
    }
}

// Lowest eigenpair of the real symmetric tridiagonal T (diagonal a[0..m),
// off-diagonal b[0..m-1)), one thread: the eigenvalue by bisection on the
// Sturm count of the LDL^T pivots of T - s I inside the Gershgorin interval;
// the eigenvector by inverse iteration with the shift sigma just below it, so
// that T - sigma I is positive definite and its LDL^T solve needs no pivoting;
// returns the Rayleigh quotient, y receives the unit eigenvector (y[0] >= 0).
__device__ double tridiag_ground(const double *a, const double *b, int m, double *y, double *work) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    auto below = [&](double sft) {  // eigenvalues of T below sft
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = a[i] - sft - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    const double scale = fmax(1.0, fmax(fabs(lo), fabs(hi)));
    for (int it = 0; it < 200 && hi - lo > 4e-16 * scale; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= 1) hi = mid;
        else lo = mid;
    }
    const double sigma = lo - 1e-12 * scale;  // below the lowest eigenvalue: T - sigma I positive definite
    double *dd = work, *ll = work + m;
    dd[0] = a[0] - sigma;
    for (int i = 0; i + 1 < m; ++i) {
        ll[i] = b[i] / dd[i];
        dd[i + 1] = a[i + 1] - sigma - ll[i] * b[i];
    }
    for (int i = 0; i < m; ++i) y[i] = 1.0;
    for (int rep = 0; rep < 3; ++rep) {
        for (int i = 1; i < m; ++i) y[i] -= ll[i - 1] * y[i - 1];  // L z = y
        for (int i = 0; i < m; ++i) y[i] /= dd[i];                 // D w = z
        for (int i = m - 2; i >= 0; --i) y[i] -= ll[i] * y[i + 1]; // L^T v = w
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += y[i] * y[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) y[i] /= nrm;
    }
    int imax = 0;
    for (int i = 1; i < m; ++i)
        if (fabs(y[i]) > fabs(y[imax])) imax = i;
    if (y[imax] < 0.0)
        for (int i = 0; i < m; ++i) y[i] = -y[i];
    double rq = 0.0;
    for (int i = 0; i < m; ++i) {
        double ty = a[i] * y[i];
        if (i > 0) ty += b[i - 1] * y[i - 1];
        if (i + 1 < m) ty += b[i] * y[i + 1];
        rq += y[i] * ty;
    }
    return rq;
}

// One Krylov exponential x <- exp(-i tau G) x; returns true when converged.
// Ground-state mode (a.ground): at the same checkpoints the lowest Ritz pair of
// the Lanczos matrix instead of the exponential; converged when the residual
// |beta y_last| is below tol max(1, |value|); x then receives the Ritz vector
// (unit norm).  At the last allowed dimension x receives the Ritz vector even
// when it has not converged (a restart then begins from it).
__device__ bool blk_krylov_once(const SmallSolveArgs &a, double tau, double2 *x, const SmallLds &L, int &m_used,
                                int &matvecs, double &err_out, double *lambda = nullptr) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t N = (uint32_t)a.g.N;
    const int mmax = a.mmax;
    double2 *V = a.vlds ? L.vb : a.V;
    double part = 0.0;
    for (uint32_t idx = tid; idx < N; idx += nt) part += cabs2(x[idx]);
    const double beta0 = sqrt(blk_sum1(part, L.red1));
    if (beta0 == 0.0) {
        m_used = 0;
        err_out = 0.0;
        return true;
    }
    for (uint32_t idx = tid; idx < N; idx += nt) {
        double2 q = cscale(x[idx], 1.0 / beta0);
        L.v[idx] = q;
        V[idx] = q;
    }
    for (int q = tid; q < (mmax + 1) * mmax; q += nt) L.Hm[q] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int j = 0; j < mmax; ++j) {
        if (a.batched) blk_matvec_two(a, L.v, L.w, L.r1, L.e1, L.tix, L.us, L.ents);
        else blk_matvec_seq(a, L.v, L.w, L.r1, L.r1 + N);
        ++matvecs;
        double wn2 = 0.0;
        for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
            // the second pass also reduces |w|^2: |w - V h|^2 = |w|^2 - |h|^2 (h ~ eps there)
            blk_dots(V, N, j + 1, L.w, L.hbuf, pass == 1);
            if (pass == 1) {
                wn2 = L.hbuf[j + 1].x;
                for (int i = 0; i <= j; ++i) wn2 -= cabs2(L.hbuf[i]);
            }
            blk_sub_basis(V, N, j + 1, L.hbuf, L.w);
            if (tid <= j) L.Hm[tid * mmax + j] = cadd(L.Hm[tid * mmax + j], L.hbuf[tid]);
            __syncthreads();
        }
        const double beta = sqrt(fmax(wn2, 0.0));
        if (tid == 0) L.Hm[(j + 1) * mmax + j] = make_double2(beta, 0.0);
        __syncthreads();
        const bool breakdown = beta <= 1e-14 * beta0;
        if (a.ground && (breakdown || j + 1 >= a.m_hint - 1 || j == mmax - 1)) {
            const int m = j + 1;
            double *ta = reinterpret_cast<double *>(L.r1), *tb = ta + m, *ty = tb + m, *tw = ty + m;
            __shared__ double s_lam;
            if (tid == 0) {
                for (int i = 0; i < m; ++i) {
                    ta[i] = L.Hm[i * mmax + i].x;
                    if (i + 1 < m) tb[i] = L.Hm[(i + 1) * mmax + i].x;
                }
                s_lam = tridiag_ground(ta, tb, m, ty, tw);
                for (int i = 0; i < m; ++i) L.ybuf[i] = make_double2(ty[i], 0.0);
            }
            __syncthreads();
            const double lam = s_lam;
            const double err = breakdown ? 0.0 : beta * fabs(L.ybuf[j].x) / fmax(1.0, fabs(lam));
            const bool conv = breakdown || err <= a.tol;
            if (conv || j == mmax - 1) {
                for (uint32_t idx = tid; idx < N; idx += nt) x[idx] = make_double2(0.0, 0.0);
                blk_sub_basis(V, N, m, L.ybuf, x);  // x = -sum_i y_i V_i
                for (uint32_t idx = tid; idx < N; idx += nt) x[idx] = cscale(x[idx], -1.0);
                m_used = m;
                err_out = err;
                if (lambda) *lambda = lam;
                __syncthreads();
                return conv;
            }
            err_out = err;
        } else if (breakdown || j + 1 >= a.m_hint - 1 || j == mmax - 1) {
            // projected matrix of dimension j+1 (tridiagonal for Hermitian G)
            double2 *Hs = L.r1;
            const int m = j + 1;
            for (int q = tid; q < m * m; q += nt) {
                int r = q / m, c = q % m;
                double2 h;
                if (a.hermitian) {
                    if (r == c) h = make_double2(L.Hm[r * mmax + r].x, 0.0);
                    else if (r == c + 1) h = L.Hm[r * mmax + c];
                    else if (c == r + 1) h = L.Hm[c * mmax + r];
                    else h = make_double2(0.0, 0.0);
                } else {
                    h = L.Hm[r * mmax + c];
                }
                Hs[q] = h;
            }
            __syncthreads();
            blk_expm_col0(Hs, m, m, tau, L.r1 + m * m, L.red1, L.ybuf);
            const double err = beta0 * beta * sqrt(cabs2(L.ybuf[j]));
            if (breakdown || err <= a.tol * beta0) {
                for (uint32_t idx = tid; idx < N; idx += nt) x[idx] = make_double2(0.0, 0.0);
                blk_sub_basis(V, N, j + 1, L.ybuf, x);  // x = -sum_i y_i V_i
                for (uint32_t idx = tid; idx < N; idx += nt) x[idx] = cscale(x[idx], -beta0);
                m_used = j + 1;
                err_out = breakdown ? 0.0 : err / beta0;
                __syncthreads();
                return true;
            }
            err_out = err / beta0;
        }
        if (j == mmax - 1) break;
        const double ib = 1.0 / beta;
        for (uint32_t idx = tid; idx < N; idx += nt) {
            double2 q = cscale(L.w[idx], ib);
            L.v[idx] = q;
            V[(size_t)(j + 1) * N + idx] = q;
        }
        __syncthreads();
    }
    m_used = mmax;
    return false;
}

__host__ __device__ inline size_t small_r1_elems(int64_t N, int mmax, int batched, int nA) {
    size_t a = batched ? (size_t)nA * N : 2 * (size_t)N;
    size_t b = 4 * (size_t)mmax * mmax;
    return a > b ? a : b;
}

__device__ void small_solve(const SmallSolveArgs &a);

__global__ void __launch_bounds__(SMALL_THREADS) k_small_solve(SmallSolveArgs a) { small_solve(a); }

// Grouped form: work-group b solves problem args[b] (independent problems of
// several instances in one launch; dynamic LDS and threads for the largest).
__global__ void __launch_bounds__(SMALL_THREADS) k_small_solve_group(const SmallSolveArgs *__restrict__ args) {
    const SmallSolveArgs a = args[blockIdx.x];
    small_solve(a);
}

__device__ void small_solve(const SmallSolveArgs &a) {
    extern __shared__ double2 sm[];
    __shared__ int e1[SMALL_MAXENT];
    __shared__ int tix[SMALL_MAXENT];
    __shared__ EntLite ents[SMALL_MAXENT];
    __shared__ int moff[SMALL_MAXENT];
    const uint32_t N = (uint32_t)a.g.N;
    const int mmax = a.mmax;
    SmallLds L;
    L.v = sm;
    L.w = L.v + N;
    L.r1 = L.w + N;
    L.Hm = L.r1 + small_r1_elems(N, mmax, a.batched, a.nA);
    L.hbuf = L.Hm + (mmax + 1) * mmax;
    L.ybuf = L.hbuf + (mmax + 1);
    L.red1 = reinterpret_cast<double *>(L.ybuf + mmax);
    L.us = reinterpret_cast<double2 *>(L.red1 + 16);
    L.mb = L.us + (a.batched ? SMALL_US : 0);
    L.vb = L.mb + (a.mlds ? a.mlds_elems : 0);
    L.e1 = e1;
    L.tix = tix;
    L.ents = ents;
    if (a.batched) {
        // one thread per entry stages its fields (independent loads), then
        // thread 0 numbers the entries with a slot-1 factor from LDS
        for (int e = threadIdx.x; e < a.n_ent; e += blockDim.x) {
            const DevEntry *E = a.ent + e;
            const int nf = E->nf;
            EntLite el;
            el.coef = E->coef;
            const bool has0 = nf >= 1 && E->slot[0] == 0;
            const bool has1 = nf >= 1 && E->slot[nf - 1] == 1;
            el.M0 = has0 ? E->M[0] : nullptr;
            el.lo0 = has0 ? E->lo[0] : 0;
            el.hi0 = has0 ? E->hi[0] : 0;
            el.M1 = has1 ? E->M[nf - 1] : nullptr;
            el.lo1 = has1 ? E->lo[nf - 1] : 0;
            el.hi1 = has1 ? E->hi[nf - 1] : 0;
            ents[e] = el;
        }
        __syncthreads();
        const int n0 = a.g.dims[0], n1 = a.g.dims[1];
        if (threadIdx.x == 0) {
            int k = 0, off = 0;
            for (int e = 0; e < a.n_ent; ++e) {
                if (ents[e].M1) {
                    tix[e] = k;
                    e1[k++] = e;
                } else {
                    tix[e] = -1;
                }
                moff[e] = off;
                off += (ents[e].M0 ? n0 * n0 : 0) + (ents[e].M1 ? n1 * n1 : 0);
            }
        }
        __syncthreads();
        if (a.mlds) {
            // the factor matrices are read on every matvec: copy them to LDS once
            for (int e = 0; e < a.n_ent; ++e) {
                double2 *dst = L.mb + moff[e];
                const double2 *m0 = ents[e].M0, *m1 = ents[e].M1;
                const int s0 = m0 ? n0 * n0 : 0, s1 = m1 ? n1 * n1 : 0;
                // slot-1 factors are stored transposed (phase A reads them by column)
                for (int q = threadIdx.x; q < s0 + s1; q += blockDim.x) {
                    if (q < s0) {
                        dst[q] = m0[q];
                    } else {
                        const int t = q - s0, j = t / n1, p = t - j * n1;
                        dst[q] = m1[p * n1 + j];
                    }
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < a.n_ent; e += blockDim.x) {
                double2 *base = L.mb + moff[e];
                const bool has0 = ents[e].M0 != nullptr;
                if (has0) ents[e].M0 = base;
                if (ents[e].M1) ents[e].M1 = base + (has0 ? n0 * n0 : 0);
            }
        }
    }
    double2 *x = a.x;
    double2 *xorig = a.V + (size_t)(SMALL_MMAX + 1) * N;
    for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) xorig[idx] = x[idx];
    __syncthreads();
    int m_used = 0, matvecs = 0, level = 0;
    double err = 0.0;
    bool ok = false;
    if (a.ground) {  // Lanczos restarted from the last Ritz vector until the residual converges
        double lam = 0.0;
        for (level = 0; level < 8 && !ok; ++level) ok = blk_krylov_once(a, 0.0, x, L, m_used, matvecs, err, &lam);
        if (threadIdx.x == 0 && a.stat) {
            a.stat->m = m_used;
            a.stat->level = level - 1;
            a.stat->fail = ok ? 0 : 1;
            a.stat->matvecs = matvecs;
            a.stat->err = err;
            a.stat->err_lo = 0.0;
            a.stat->eval = lam;
        }
        return;
    }
    for (level = 0; level <= 8; ++level) {
        if (level > 0) {
            for (uint32_t idx = threadIdx.x; idx < N; idx += blockDim.x) x[idx] = xorig[idx];
            __syncthreads();
        }
        const int nsub = 1 << level;
        ok = true;
        for (int q = 0; q < nsub && ok; ++q) ok = blk_krylov_once(a, a.tau / nsub, x, L, m_used, matvecs, err);
        if (ok) break;
    }
    if (threadIdx.x == 0 && a.stat) {
        a.stat->m = m_used;
        a.stat->level = ok ? level : -1;
        a.stat->fail = ok ? 0 : 1;
        a.stat->matvecs = matvecs;
        a.stat->err = err;
        a.stat->err_lo = 0.0;
    }
}

size_t small_solve_lds_bytes(int64_t N, int mmax, int batched, int nA) {
    return sizeof(double2) * (size_t)(2 * N + small_r1_elems(N, mmax, batched, nA) + (mmax + 1) * mmax +
                                      (mmax + 1) + mmax + (batched ? SMALL_US : 0)) +
           16 * sizeof(double);
}

// ============================================================ multi-kernel Krylov
__global__ void __launch_bounds__(VEC_THREADS) k_kry_norm0(const double2 *__restrict__ x, uint32_t N, BigKrylov k) {
    __shared__ double red1[16];
    double part = 0.0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) part += cabs2(x[i]);
    double s = blk_sum1(part, red1);
    if (threadIdx.x == 0) k.part[blockIdx.x] = s;
    if (last_block_ticket(k.counter)) {
        __shared__ double stage[KRY_STAGE];
        __shared__ double tot[1];
        blk_reduce_staged(k.part, gridDim.x, 1, 1, tot, stage);
        if (threadIdx.x == 0) {
            k.scal[0] = sqrt(tot[0]);
            *k.meff = 0;
            *k.counter = 0;
        }
    }
}

__global__ void __launch_bounds__(VEC_THREADS) k_kry_scale0(const double2 *__restrict__ x, uint32_t N, BigKrylov k) {
    const double b0 = k.scal[0];
    const double ib = b0 > 0.0 ? 1.0 / b0 : 0.0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
        k.V[i] = cscale(x[i], ib);
}

// Classical Gram-Schmidt, twice, for w = V[j+1] against V[0..j]:
//   pass 0: h0 = V^H w                                  -> Hm[:, j] = h0
//   pass 1: w -= V h0; h1 = V^H w and |w|^2               -> Hm[:, j] += h1,
//           beta^2 = |w|^2 - |h1|^2 (h1 is rounding-size, no cancellation)
// k_kry_finalize then forms (w - V h1) / beta.
__global__ void __launch_bounds__(VEC_THREADS) k_kry_orth(BigKrylov k, uint32_t N, int j, int mmax, int pass) {
    if (*k.meff) return;
    __shared__ double2 hb[64];
    __shared__ double red1[16];
    __shared__ double stage[KRY_STAGE];
    const int nv = j + 1;
    double2 *w = k.V + (size_t)(j + 1) * N;
    double wn = 0.0;
    if (pass > 0) {
        for (int q = threadIdx.x; q < nv; q += blockDim.x) hb[q] = k.h[q];
        __syncthreads();
        for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
            double2 wv = w[idx];
            for (int i = 0; i < nv; ++i) wv = csub(wv, cmul(hb[i], k.V[(size_t)i * N + idx]));
            w[idx] = wv;
            wn += cabs2(wv);
        }
        __syncthreads();
    }
    const int K = nv + 1;  // doubles pairs per block: h (complex) and |w|^2
    double *part = k.part;
    {  // one wavefront per basis vector over the block's elements, one wave reduction per dot
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        const uint32_t stride = gridDim.x * blockDim.x;
        for (int i = wave; i < nv; i += nw) {
            const double2 *vi = k.V + (size_t)i * N;
            double2 c = make_double2(0.0, 0.0);
            for (uint32_t base = blockIdx.x * blockDim.x; base < N; base += stride)
                for (uint32_t t = lane; t < blockDim.x; t += 64) {
                    const uint32_t idx = base + t;
                    if (idx < N) cfmac(c, vi[idx], w[idx]);
                }
            c.x = wave_sum(c.x);
            c.y = wave_sum(c.y);
            if (lane == 0) hb[i] = c;
        }
        __syncthreads();
    }
    const double wns = pass == 1 ? blk_sum1(wn, red1) : 0.0;
    if (threadIdx.x < nv) {
        part[2 * ((size_t)blockIdx.x * K + threadIdx.x)] = hb[threadIdx.x].x;
        part[2 * ((size_t)blockIdx.x * K + threadIdx.x) + 1] = hb[threadIdx.x].y;
    }
    if (threadIdx.x == 0) {
        part[2 * ((size_t)blockIdx.x * K + nv)] = wns;
        part[2 * ((size_t)blockIdx.x * K + nv) + 1] = 0.0;
    }
    if (last_block_ticket(k.counter)) {
        __shared__ double sums[2 * 65];
        blk_reduce_staged(part, gridDim.x, 2 * K, 2 * K, sums, stage);
        __syncthreads();
        double2 *hcol = k.Hm + (size_t)j * (mmax + 1);
        for (int q = threadIdx.x; q < nv; q += blockDim.x) {
            const double2 sv = make_double2(sums[2 * q], sums[2 * q + 1]);
            k.h[q] = sv;
            hcol[q] = pass == 0 ? sv : cadd(hcol[q], sv);
        }
        if (pass == 1 && threadIdx.x == 0) {
            double b2 = sums[2 * nv];
            for (int q = 0; q < nv; ++q) b2 -= sums[2 * q] * sums[2 * q] + sums[2 * q + 1] * sums[2 * q + 1];
            const double beta = sqrt(fmax(b2, 0.0));
            k.scal[1] = beta;
            hcol[j + 1] = make_double2(beta, 0.0);
            if (beta <= 1e-14 * k.scal[0]) *k.meff = j + 1;
        }
        if (threadIdx.x == 0) *k.counter = 0;
    }
}

// w = (w - V h1) / beta (no-op after a breakdown)
__global__ void __launch_bounds__(VEC_THREADS) k_kry_finalize(BigKrylov k, uint32_t N, int j) {
    if (*k.meff) return;
    __shared__ double2 hb[64];
    const int nv = j + 1;
    for (int q = threadIdx.x; q < nv; q += blockDim.x) hb[q] = k.h[q];
    __syncthreads();
    const double ib = 1.0 / k.scal[1];
    double2 *w = k.V + (size_t)(j + 1) * N;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
        double2 wv = w[idx];
        for (int i = 0; i < nv; ++i) wv = csub(wv, cmul(hb[i], k.V[(size_t)i * N + idx]));
        w[idx] = cscale(wv, ib);
    }
}

// Gram-Schmidt for w = V[j+1] against V[0..j] with one pass over the basis for
// the dots and one for the update.  Twice-applied classical Gram-Schmidt
// forms w - V (h1 + h2) with h1 = V^H w and h2 = V^H (w - V h1); the second
// dots equal h1 - G h1 with G = V^H V, the Gram matrix of the stored basis,
// whose column j (v_i^H v_j) comes from the same pass as h1.  So
//   k_kry_dots1:   h1 = V^H w, G[:, j] = V^H v_j, |w|^2 -> c = 2 h1 - G h1 = Hm[:, j]
//   k_kry_update1: w -= V c, |w|^2 -> beta
// When the update cancels most of w (|w - V c|^2 < 1e-4 |w|^2: w nearly inside
// the span), its rounding is not orthogonal to V; a classical pass on the
// result then follows (k_kry_refine1, gated: h3 = V^H w, w -= V h3, Hm[:, j] += h3).
// k_kry_scale1 divides by beta.
constexpr double KRY_CANCEL = 1e-4;
// The dots stream the basis in chunks of KD_C vectors: each thread reads w and
// v_j once per chunk into registers and the chunk's vectors with independent
// loads (KD_C + 2 in flight per element, two elements per iteration), keeping
// 2 KD_C complex accumulators; the block then reduces them across its waves.
constexpr int KD_C = 8;
constexpr int KD_THREADS = 512;  // two waves per SIMD: twice the loads in flight of the 256-thread kernels
__global__ void __launch_bounds__(KD_THREADS) k_kry_dots1(BigKrylov k, uint32_t N, int j, int mmax) {
    if (*k.meff) return;
    __shared__ double2 hb[64], gb[64];
    __shared__ double red1[16];
    __shared__ double wred[KD_THREADS / 64][4 * KD_C];
    __shared__ double stage[KRY_STAGE];
    const int nv = j + 1;
    const double2 *__restrict__ V = k.V;
    const double2 *__restrict__ w = V + (size_t)(j + 1) * N;
    const double2 *__restrict__ vj = V + (size_t)j * N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t stride = gridDim.x * blockDim.x;
    double wn = 0.0;
    for (int c0 = 0; c0 < nv; c0 += KD_C) {
        const int cnt = min(KD_C, nv - c0);
        const double2 *__restrict__ vc = V + (size_t)c0 * N;
        double2 ch[KD_C], cg[KD_C];
#pragma unroll
        for (int c = 0; c < KD_C; ++c) ch[c] = cg[c] = make_double2(0.0, 0.0);
#pragma unroll 2
        for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += stride) {
            const double2 wv = w[idx], jv = vj[idx];
            if (c0 == 0) wn += cabs2(wv);
#pragma unroll
            for (int c = 0; c < KD_C; ++c)
                if (c < cnt) {
                    const double2 v = vc[(size_t)c * N + idx];
                    cfmac(ch[c], v, wv);
                    cfmac(cg[c], v, jv);
                }
        }
#pragma unroll
        for (int c = 0; c < KD_C; ++c) {
            if (c < cnt) {
                const double a = wave_sum(ch[c].x), b = wave_sum(ch[c].y);
                const double d = wave_sum(cg[c].x), e = wave_sum(cg[c].y);
                if (lane == 0) {
                    wred[wave][4 * c] = a;
                    wred[wave][4 * c + 1] = b;
                    wred[wave][4 * c + 2] = d;
                    wred[wave][4 * c + 3] = e;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 4 * cnt) {
            double s = 0.0;
            for (int q = 0; q < nw; ++q) s += wred[q][threadIdx.x];
            const int c = threadIdx.x >> 2, r = threadIdx.x & 3;
            double *dst = r < 2 ? reinterpret_cast<double *>(&hb[c0 + c]) : reinterpret_cast<double *>(&gb[c0 + c]);
            dst[r & 1] = s;
        }
        __syncthreads();
    }
    const double wns = blk_sum1(wn, red1);  // synchronises: hb, gb complete
    const int K = 2 * nv + 1;  // complex slots per block: h1, g, |w|^2
    double *part = k.part + (size_t)blockIdx.x * 2 * K;
    if (threadIdx.x < nv) {
        part[2 * threadIdx.x] = hb[threadIdx.x].x;
        part[2 * threadIdx.x + 1] = hb[threadIdx.x].y;
        part[2 * (nv + threadIdx.x)] = gb[threadIdx.x].x;
        part[2 * (nv + threadIdx.x) + 1] = gb[threadIdx.x].y;
    }
    if (threadIdx.x == 0) {
        part[2 * (2 * nv)] = wns;
        part[2 * (2 * nv) + 1] = 0.0;
    }
    if (last_block_ticket(k.counter)) {
        __shared__ double sums[2 * (2 * 65 + 1)];
        blk_reduce_staged(k.part, gridDim.x, 2 * K, 2 * K, sums, stage);
        __syncthreads();
        const int ld = mmax + 1;
        // G[q][l] = v_q^H v_l: column l (l >= q) of the stored Gram matrix, or
        // the conjugate of column q; column j is the one just reduced
        auto gram = [&](int q, int l) -> double2 {
            if (l >= q)
                return l == j ? make_double2(sums[2 * (nv + q)], sums[2 * (nv + q) + 1]) : k.G[(size_t)l * ld + q];
            double2 g = q == j ? make_double2(sums[2 * (nv + l)], sums[2 * (nv + l) + 1]) : k.G[(size_t)q * ld + l];
            g.y = -g.y;
            return g;
        };
        double2 *hcol = k.Hm + (size_t)j * (mmax + 1);
        for (int q = threadIdx.x; q < nv; q += blockDim.x) {
            double2 gh = make_double2(0.0, 0.0);
            for (int l = 0; l < nv; ++l) cfma(gh, gram(q, l), make_double2(sums[2 * l], sums[2 * l + 1]));
            const double2 h = make_double2(sums[2 * q], sums[2 * q + 1]);
            const double2 c = make_double2(2.0 * h.x - gh.x, 2.0 * h.y - gh.y);
            k.h[q] = c;
            hcol[q] = c;
            k.G[(size_t)j * ld + q] = make_double2(sums[2 * (nv + q)], sums[2 * (nv + q) + 1]);
        }
        if (threadIdx.x == 0) {
            k.scal[2] = sums[2 * (2 * nv)];
            *k.counter = 0;
        }
    }
}

// w -= V c (c = k.h) and |w|^2; last block: beta, Hm[j+1][j], the refinement
// flag and the breakdown test
__global__ void __launch_bounds__(VEC_THREADS) k_kry_update1(BigKrylov k, uint32_t N, int j, int mmax, int refine) {
    if (*k.meff) return;
    if (refine && !*k.refine) return;
    __shared__ double2 hb[64];
    __shared__ double red1[16];
    __shared__ double stage[KRY_STAGE];
    const int nv = j + 1;
    for (int q = threadIdx.x; q < nv; q += blockDim.x) hb[q] = k.h[q];
    __syncthreads();
    double2 *w = k.V + (size_t)(j + 1) * N;
    double wn = 0.0;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
        double2 wv = w[idx];
        for (int i = 0; i < nv; ++i) wv = csub(wv, cmul(hb[i], k.V[(size_t)i * N + idx]));
        w[idx] = wv;
        wn += cabs2(wv);
    }
    const double wns = blk_sum1(wn, red1);
    if (threadIdx.x == 0) k.part[blockIdx.x] = wns;
    if (last_block_ticket(k.counter)) {
        __shared__ double tot[1];
        blk_reduce_staged(k.part, gridDim.x, 1, 1, tot, stage);
        __syncthreads();
        if (threadIdx.x == 0) {
            const double b2 = tot[0];
            const double beta = sqrt(b2);
            // refinement: once, when the update cancelled most of w
            const int again = (!refine && b2 < KRY_CANCEL * k.scal[2]) ? 1 : 0;
            *k.refine = again;
            k.scal[2] = b2;
            k.scal[1] = beta;
            k.Hm[(size_t)j * (mmax + 1) + j + 1] = make_double2(beta, 0.0);
            if (!again && beta <= 1e-14 * k.scal[0]) *k.meff = j + 1;
            *k.counter = 0;
        }
    }
}

// refinement dots (gated): h3 = V^H w -> k.h, Hm[:, j] += h3
__global__ void __launch_bounds__(VEC_THREADS) k_kry_refine1(BigKrylov k, uint32_t N, int j, int mmax) {
    if (*k.meff || !*k.refine) return;
    __shared__ double2 hb[64];
    __shared__ double stage[KRY_STAGE];
    const int nv = j + 1;
    const double2 *w = k.V + (size_t)(j + 1) * N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (int i = wave; i < nv; i += nw) {
        const double2 *vi = k.V + (size_t)i * N;
        double2 c = make_double2(0.0, 0.0);
        for (uint32_t base = blockIdx.x * blockDim.x; base < N; base += stride)
            for (uint32_t t = lane; t < blockDim.x; t += 64) {
                const uint32_t idx = base + t;
                if (idx < N) cfmac(c, vi[idx], w[idx]);
            }
        c.x = wave_sum(c.x);
        c.y = wave_sum(c.y);
        if (lane == 0) hb[i] = c;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        k.part[2 * ((size_t)blockIdx.x * nv + threadIdx.x)] = hb[threadIdx.x].x;
        k.part[2 * ((size_t)blockIdx.x * nv + threadIdx.x) + 1] = hb[threadIdx.x].y;
    }
    if (last_block_ticket(k.counter)) {
        __shared__ double sums[2 * 65];
        blk_reduce_staged(k.part, gridDim.x, 2 * nv, 2 * nv, sums, stage);
        __syncthreads();
        double2 *hcol = k.Hm + (size_t)j * (mmax + 1);
        for (int q = threadIdx.x; q < nv; q += blockDim.x) {
            const double2 sv = make_double2(sums[2 * q], sums[2 * q + 1]);
            k.h[q] = sv;
            hcol[q] = cadd(hcol[q], sv);
        }
        if (threadIdx.x == 0) *k.counter = 0;
    }
}

// w /= beta (no-op after a breakdown)
__global__ void __launch_bounds__(VEC_THREADS) k_kry_scale1(BigKrylov k, uint32_t N, int j) {
    if (*k.meff) return;
    const double ib = 1.0 / k.scal[1];
    double2 *w = k.V + (size_t)(j + 1) * N;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x)
        w[idx] = cscale(w[idx], ib);
}

// exp of the projected matrix (one work-group); y = beta0 exp(-i tau H_m) e_0
__global__ void __launch_bounds__(1024) k_kry_expm(BigKrylov k, int m, int mmax, double tau, double tol,
                                                   int hermitian, SolveStat *stat) {
    extern __shared__ double2 sme[];
    __shared__ double red1[16];
    const int meff = *k.meff;
    const int mm = meff ? meff : m;
    double2 *Hs = sme;               // mm^2
    double2 *ws = sme + mm * mm;     // 3 mm^2
    double2 *y = ws + 3 * mm * mm;   // mm
    const double beta0 = k.scal[0];
    double errs[2] = {0.0, 0.0};
    for (int pass = 0; pass < 2; ++pass) {
        const int md = pass == 0 ? mm : mm - 2;
        if (md < 1) break;
        for (int q = threadIdx.x; q < md * md; q += blockDim.x) {
            int r = q / md, c = q % md;
            double2 h;
            const double2 *col = k.Hm + (size_t)c * (mmax + 1);
            if (hermitian) {
                if (r == c) h = make_double2(col[r].x, 0.0);
                else if (r == c + 1) h = col[r];
                else if (c == r + 1) h = k.Hm[(size_t)r * (mmax + 1) + c];
                else h = make_double2(0.0, 0.0);
            } else {
                // upper Hessenberg: entries below the subdiagonal are never written
                h = r <= c + 1 ? col[r] : make_double2(0.0, 0.0);
            }
            Hs[q] = h;
        }
        __syncthreads();
        blk_expm_col0(Hs, md, md, tau, ws, red1, y);
        const double hnext = k.Hm[(size_t)(md - 1) * (mmax + 1) + md].x;
        errs[pass] = (pass == 0 && meff) ? 0.0 : hnext * sqrt(cabs2(y[md - 1]));
        if (pass == 0) {
            for (int q = threadIdx.x; q < mm; q += blockDim.x) k.y[q] = cscale(y[q], beta0);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && stat) {
        stat->m = mm;
        stat->level = 0;
        stat->fail = errs[0] > tol ? 1 : 0;
        stat->matvecs = mm;
        stat->err = errs[0];
        stat->err_lo = (mm - 2 >= 1) ? errs[1] : 1.0;
    }
}

// ground-state finish of the multi-kernel Lanczos (one work-group): k.y <- the
// unit Ritz vector of the lowest Ritz value, stat: value and residual estimate
__global__ void __launch_bounds__(64) k_kry_ground(BigKrylov k, int m, int mmax, SolveStat *stat) {
    __shared__ double ta[64], tb[64], ty[64], tw[128];
    const int meff = *k.meff;
    const int mm = meff ? meff : m;
    if (threadIdx.x == 0) {
        const int ld = mmax + 1;
        for (int i = 0; i < mm; ++i) {
            ta[i] = k.Hm[(size_t)i * ld + i].x;
            if (i + 1 < mm) tb[i] = k.Hm[(size_t)i * ld + i + 1].x;
        }
        const double lam = tridiag_ground(ta, tb, mm, ty, tw);
        const double beta = meff ? 0.0 : k.Hm[(size_t)(mm - 1) * ld + mm].x;
        for (int i = 0; i < mm; ++i) k.y[i] = make_double2(ty[i], 0.0);
        stat->m = mm;
        stat->level = 0;
        stat->matvecs = m;
        stat->err = beta * fabs(ty[mm - 1]) / fmax(1.0, fabs(lam));
        stat->err_lo = 0.0;
        stat->fail = 0;
        stat->eval = lam;
    }
}

__global__ void __launch_bounds__(VEC_THREADS) k_kry_combine(BigKrylov k, uint32_t N, int m, double2 *x) {
    const int meff = *k.meff;
    const int mm = meff ? meff : m;
    __shared__ double2 yb[64];
    for (int q = threadIdx.x; q < mm; q += blockDim.x) yb[q] = k.y[q];
    __syncthreads();
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += gridDim.x * blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < mm; ++i) cfma(acc, yb[i], k.V[(size_t)i * N + idx]);
        x[idx] = acc;
    }
}

// ============================================================ misc
__global__ void __launch_bounds__(256) k_combine(const CombJob *__restrict__ jobs, const CombSrc *__restrict__ srcs) {
    const CombJob J = jobs[blockIdx.y];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < J.n2; i += gridDim.x * blockDim.x) {
        // element read for output i: transposed modes read (col, row)
        const int si = (J.mode & 1) ? (i % J.n) * J.n + i / J.n : i;
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < J.count; ++q) {
            const CombSrc S = srcs[J.first + q];
            double2 v = S.src[si];
            if (J.mode & 2) v.y = -v.y;
            cfma(acc, S.coef, v);
        }
        J.dst[i] = acc;
    }
}

__global__ void k_copy(double2 *dst, const double2 *src, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}
__global__ void k_transpose(double2 *dst, const double2 *src, int n) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n * n; q += gridDim.x * blockDim.x) {
        int i = q / n, j = q % n;
        dst[j * n + i] = src[q];
    }
}

// ============================================================ subspace expansion
// out[g, j] = sum_{l,r} op(A[l, j, r]) B_g[l, r]: threads (j, row phase), rows of
// the block's chunk; per-block partials reduced by k_ts_reduce.
__global__ void __launch_bounds__(256) k_ts_contract_part(const double2 *__restrict__ A, uint32_t L, int n,
                                                          uint32_t R, int conjA, const double2 *__restrict__ B,
                                                          int64_t bstride, double2 *__restrict__ part) {
    const int g = blockIdx.y;
    const uint32_t rows = L * R;
    const uint32_t per = (rows + gridDim.x - 1) / gridDim.x;
    const uint32_t r0 = blockIdx.x * per, r1 = min(rows, r0 + per);
    const int nph = (int)blockDim.x / 64;
    const int j = threadIdx.x % 64, ph = threadIdx.x / 64;
    const double2 *Bg = B + (int64_t)g * bstride;
    double2 acc = make_double2(0.0, 0.0);
    if (j < n)
        for (uint32_t rho = r0 + ph; rho < r1; rho += nph) {
            const uint32_t l = rho / R, r = rho - l * R;
            double2 a = A[((size_t)l * n + j) * R + r];
            if (conjA) a.y = -a.y;
            cfma(acc, a, Bg[rho]);
        }
    __shared__ double2 red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (ph == 0 && j < n) {
        double2 s = red[j];
        for (int q = 1; q < nph; ++q) s = cadd(s, red[q * 64 + j]);
        part[((size_t)g * gridDim.x + blockIdx.x) * n + j] = s;
    }
}

__global__ void k_ts_reduce(const double2 *__restrict__ part, int nblk, int n, int groups, double2 *out) {
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < n * groups; o += gridDim.x * blockDim.x) {
        const int g = o / n, j = o - g * n;
        double2 s = make_double2(0.0, 0.0);
        for (int b = 0; b < nblk; ++b) s = cadd(s, part[((size_t)g * nblk + b) * n + j]);
        out[o] = s;
    }
}

// out[g, l, r] = (base ? base[g, l, r] : 0) -+ sum_j op(A[l, j, r]) S[g, j]: one row per
// thread, eight groups at a time, S staged in LDS
__global__ void __launch_bounds__(256) k_ts_expand(const double2 *__restrict__ A, uint32_t L, int n, uint32_t R,
                                                   int conjA, const double2 *__restrict__ S, int groups,
                                                   const double2 *__restrict__ base, int negate,
                                                   double2 *__restrict__ out) {
    extern __shared__ double2 Ss[];
    for (int q = threadIdx.x; q < groups * n; q += blockDim.x) Ss[q] = S[q];
    __syncthreads();
    const uint32_t rows = L * R;
    for (uint32_t rho = blockIdx.x * blockDim.x + threadIdx.x; rho < rows; rho += gridDim.x * blockDim.x) {
        const uint32_t l = rho / R, r = rho - l * R;
        const double2 *ap = A + (size_t)l * n * R + r;
        for (int g0 = 0; g0 < groups; g0 += 8) {
            double2 acc[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = make_double2(0.0, 0.0);
            for (int j = 0; j < n; ++j) {
                double2 a = ap[(size_t)j * R];
                if (conjA) a.y = -a.y;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (g0 + q < groups) cfma(acc[q], a, Ss[(g0 + q) * n + j]);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (g0 + q < groups) {
                    const size_t o = (size_t)(g0 + q) * rows + rho;
                    double2 v = negate ? make_double2(-acc[q].x, -acc[q].y) : acc[q];
                    if (base) v = cadd(base[o], v);
                    out[o] = v;
                }
        }
    }
}

__global__ void __launch_bounds__(256) k_repack(const double2 *__restrict__ X, double2 *__restrict__ Y, uint32_t L,
                                                int n_old, int n_new, uint32_t R, const double2 *__restrict__ V,
                                                int64_t vstride, int conjV) {
    const uint32_t NY = L * (uint32_t)n_new * R;
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < NY; idx += gridDim.x * blockDim.x) {
        const uint32_t r = idx % R, t = idx / R;
        const int j = (int)(t % (uint32_t)n_new);
        const uint32_t l = t / (uint32_t)n_new;
        double2 v = make_double2(0.0, 0.0);
        if (j < n_old) {
            v = X[((size_t)l * n_old + j) * R + r];
        } else if (V) {
            v = V[(int64_t)(j - n_old) * vstride + (int64_t)l * R + r];
            if (conjV) v.y = -v.y;
        }
        Y[idx] = v;
    }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    // SplitMix64 (Steele, Lea, Flood 2014): the state x advanced by the golden gamma, then mixed
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_seed_vector(double2 *v, uint32_t N, uint64_t seed) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed + 2ull * i), b = splitmix64(seed + 2ull * i + 1ull);
        v[i] = make_double2(2.0 * ((double)(a >> 11) * 0x1.0p-53) - 1.0, 2.0 * ((double)(b >> 11) * 0x1.0p-53) - 1.0);
    }
}

// One-sided Jacobi SVD of the real n x n upper bidiagonal (one wavefront; row i
// of the working matrix and of V on lane i).  Columns are rotated until every
// pair is orthogonal to 1e-15 relative; singular values are the column norms.
constexpr int SVD_NMAX = 48;  // largest bidiagonal (LDS of the working matrix and of V)
__global__ void __launch_bounds__(64) k_bidiag_svd(const double *alpha, const double *beta, const int *nptr, int nmax,
                                                   double *s_out, double *U, double *V) {
    __shared__ double W[SVD_NMAX * SVD_NMAX], Vs[SVD_NMAX * SVD_NMAX], sv[SVD_NMAX];
    __shared__ int perm[SVD_NMAX];
    const int i = threadIdx.x;
    const int n = min(*nptr, min(nmax, SVD_NMAX));
    for (int q = i; q < SVD_NMAX * SVD_NMAX; q += 64) {
        W[q] = 0.0;
        Vs[q] = 0.0;
    }
    __syncthreads();
    if (i < n) {
        W[i * SVD_NMAX + i] = alpha[i];
        if (i + 1 < n) W[i * SVD_NMAX + i + 1] = beta[i];
        Vs[i * SVD_NMAX + i] = 1.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double ap = i < n ? W[i * SVD_NMAX + p] : 0.0, aq = i < n ? W[i * SVD_NMAX + q] : 0.0;
                const double a = wave_sum(ap * ap), b = wave_sum(aq * aq), g = wave_sum(ap * aq);
                if (fabs(g) <= 1e-15 * sqrt(a * b) || g == 0.0) continue;
                rotated = 1;
                const double zeta = (b - a) / (2.0 * g);
                const double tn = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + tn * tn), sn = c * tn;
                if (i < n) {
                    W[i * SVD_NMAX + p] = c * ap - sn * aq;
                    W[i * SVD_NMAX + q] = sn * ap + c * aq;
                    const double vp = Vs[i * SVD_NMAX + p], vq = Vs[i * SVD_NMAX + q];
                    Vs[i * SVD_NMAX + p] = c * vp - sn * vq;
                    Vs[i * SVD_NMAX + q] = sn * vp + c * vq;
                }
                __syncthreads();
            }
        if (!rotated) break;
    }
    for (int j = 0; j < n; ++j) {
        const double w = i < n ? W[i * SVD_NMAX + j] : 0.0;
        const double nr = sqrt(wave_sum(w * w));
        if (i == 0) sv[j] = nr;
    }
    __syncthreads();
    if (i == 0) {  // descending order
        for (int j = 0; j < n; ++j) perm[j] = j;
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b < n; ++b)
                if (sv[perm[b]] > sv[perm[a]]) {
                    const int t = perm[a];
                    perm[a] = perm[b];
                    perm[b] = t;
                }
    }
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const int c = perm[j];
        const double sg = sv[c];
        if (i == 0) s_out[j] = sg;
        if (i < n) {
            U[i * nmax + j] = sg > 0.0 ? W[i * SVD_NMAX + c] / sg : 0.0;
            V[i * nmax + j] = Vs[i * SVD_NMAX + c];
        }
    }
}

__global__ void k_basis_combine(const double2 *__restrict__ V, uint32_t N, const int *nptr, const double *W, int ldw,
                                int ncols, double2 *out) {
    const int n = *nptr;
    const int c = blockIdx.y;
    if (c >= ncols) return;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < n; ++q) {
            const double w = W[q * ldw + c];
            const double2 v = V[(size_t)q * N + i];
            acc.x = fma(w, v.x, acc.x);
            acc.y = fma(w, v.y, acc.y);
        }
        out[(size_t)c * N + i] = acc;
    }
}

// Dimension of the Golub-Kahan-Lanczos bidiagonal after m steps: the first
// vanishing alpha (left side) or beta (right side) ends it; alpha_0 = 0 leaves none.
__global__ void k_gkl_count(const int *meffP, const int *meffQ, const double *alpha0, int m, int *n) {
    if (threadIdx.x != 0) return;
    int k = m;
    if (*meffP > 0) k = min(k, *meffP);
    if (*meffQ > 0) k = min(k, *meffQ);
    if (!(*alpha0 > 0.0)) k = 0;
    *n = k;
}

// rows and columns keep.. of an n x n matrix set to zero
__global__ void k_zero_tail(double2 *C, int n, int keep) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n * n; q += gridDim.x * blockDim.x)
        if (q / n >= keep || q % n >= keep) C[q] = make_double2(0.0, 0.0);
}

__global__ void k_copy_scalars(double *dst, const double *src, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src[i];
}

// ============================================================ launch profiler
// Optional: every launch carries a start and a stop HIP event that the runtime
// stamps from the dispatch itself (hipExtLaunchKernelGGL), so the elapsed time
// is the kernel's own execution time without the marker packets a pair of
// hipEventRecord calls would add; per kernel name the summed elapsed time, call
// count and algorithmic flops / bytes.
namespace prof {
struct Rec {
    const char *name;
    hipEvent_t a, b;  // dispatch-stamped events, or null for a kernel-clock slot
    double flops, bytes;
    int ts_slot;  // >= 0: duration from the kernel's own start / end clock readings
};
static bool on = false;
static thread_local bool suspended = false;  // this thread's launches go untimed
// kernel-clock slots: ts[i] = earliest start, ts[PROF_TS_MAX + i] = latest end
static unsigned long long *ts = nullptr;
static int ts_used = 0;
static bool ts_fresh = false;  // slots initialised for the current collection
static double ts_khz = 0.0;
static unsigned long long *take_ts() {
    if (!ts) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0 ||
            hipMalloc((void **)&ts, sizeof(unsigned long long) * 2 * PROF_TS_MAX) != hipSuccess)
            throw std::runtime_error("launch profiler: kernel clock unavailable");
        ts_khz = khz;
    }
    if (!ts_fresh) {  // starts to the maximum, ends to zero
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemset(ts, 0xff, sizeof(unsigned long long) * PROF_TS_MAX) != hipSuccess ||
            hipMemset(ts + PROF_TS_MAX, 0, sizeof(unsigned long long) * PROF_TS_MAX) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            throw std::runtime_error("launch profiler: kernel clock slots");
        ts_used = 0;
        ts_fresh = true;
    }
    if (ts_used >= PROF_TS_MAX) return nullptr;  // slots exhausted: the launch runs untimed
    return ts + ts_used++;
}
static std::vector<hipEvent_t> pool;
static size_t used = 0;
static std::vector<Rec> recs;
static std::map<std::string, double> extra_flops;
static hipEvent_t take() {
    if (used == pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
        pool.push_back(e);
    }
    return pool[used++];
}
}  // namespace prof

#define TTN_LAUNCH(NAME, FL, BY, KER, GRID, BLOCK, LDS, ST, ...)                                     \
    do {                                                                                             \
        if (prof::on && !prof::suspended) {                                                          \
            hipEvent_t ea_ = prof::take(), eb_ = prof::take();                                       \
            hipExtLaunchKernelGGL(KER, dim3(GRID), dim3(BLOCK), LDS, ST, ea_, eb_, 0, __VA_ARGS__);   \
            prof::recs.push_back({NAME, ea_, eb_, (double)(FL), (double)(BY), -1});                  \
        } else {                                                                                     \
            hipLaunchKernelGGL(KER, GRID, BLOCK, LDS, ST, __VA_ARGS__);                              \
        }                                                                                            \
    } while (0)

void profile_enable(bool enable) {
    prof::on = enable;
    prof::used = 0;
    prof::recs.clear();
    prof::extra_flops.clear();
    prof::ts_used = 0;
    prof::ts_fresh = false;  // slots are initialised at the first cooperative launch
}

bool profile_enabled() { return prof::on; }

ProfileSuspend::ProfileSuspend() : prev(prof::suspended) { prof::suspended = true; }
ProfileSuspend::~ProfileSuspend() { prof::suspended = prev; }

void release_process_resources() {
    prof::on = false;
    prof::recs.clear();
    prof::extra_flops.clear();
    for (hipEvent_t e : prof::pool) (void)hipEventDestroy(e);
    prof::pool.clear();
    prof::used = 0;
    if (prof::ts) (void)hipFree(prof::ts);
    prof::ts = nullptr;
    prof::ts_used = 0;
    prof::ts_fresh = false;
}

void profile_add_flops(const char *name, double flops) { prof::extra_flops[name] += flops; }

std::vector<KernelStat> profile_collect() {
    if (hipDeviceSynchronize() != hipSuccess) throw std::runtime_error("hipDeviceSynchronize failed");
    std::map<std::string, KernelStat> agg;
    std::vector<unsigned long long> tsv;
    if (prof::ts && prof::ts_fresh && prof::ts_used > 0) {
        tsv.resize(2 * PROF_TS_MAX);
        if (hipMemcpy(tsv.data(), prof::ts, sizeof(unsigned long long) * 2 * PROF_TS_MAX, hipMemcpyDeviceToHost) !=
            hipSuccess)
            throw std::runtime_error("launch profiler: kernel clock read-back");
    }
    for (auto &r : prof::recs) {
        float ms = 0.f;
        if (r.ts_slot >= 0) {
            if (tsv.empty()) throw std::runtime_error("launch profiler: kernel clock slots lost");
            const unsigned long long t0 = tsv[r.ts_slot], t1 = tsv[PROF_TS_MAX + r.ts_slot];
            ms = t1 > t0 ? (float)((double)(t1 - t0) / prof::ts_khz) : 0.f;
        } else if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            throw std::runtime_error("hipEventElapsedTime failed");
        }
        KernelStat &k = agg[r.name];
        k.name = r.name;
        k.calls += 1;
        k.ms += ms;
        k.flops += r.flops;
        k.bytes += r.bytes;
    }
    for (auto &kv : prof::extra_flops) agg[kv.first].flops += kv.second;
    std::vector<KernelStat> out;
    for (auto &kv : agg) out.push_back(kv.second);
    prof::used = 0;
    prof::recs.clear();
    prof::extra_flops.clear();
    prof::ts_used = 0;
    prof::ts_fresh = false;
    return out;
}

// ============================================================ launchers
// Raise a kernel's dynamic LDS limit when a launch needs more than the default
// 64 KiB (gfx950 work-groups may use up to 160 KiB).
static void set_lds_limit(const void *fn, size_t bytes) {
    if (bytes <= 64 * 1024) return;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) throw std::runtime_error(std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
}

static inline unsigned grid_for(int64_t n, int threads, int cap = 2048) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// ------------------------------------------------------------ tile autotuner
// The tiled stage is instantiated for several register tiles (TI rows per
// thread, RG row groups, NP = TI * RG >= the stage's largest factor).  Without
// a table entry the tile comes from a fixed rule of the factor size; the
// autotuner times every admissible tile on the stage itself (same program,
// same launch shape) and records the fastest under a key of the stage's shape.
// The tile does not change the order of any accumulation, so results are bit
// for bit the same whichever tile runs.
struct TileCand {
    int ti, rg;
};
static const TileCand TILE_CANDS[] = {{1, 8}, {2, 8}, {4, 8}, {1, 16}, {2, 16}, {3, 16}, {4, 16}, {1, 32}, {2, 32}};
struct TileChoice {
    int ti, rg;
    double us;
};
static std::map<std::string, TileChoice> &tile_table() {
    static std::map<std::string, TileChoice> t;
    return t;
}

static std::string tile_key(const ProgView &p, int s) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s|nmax=%d|nmin=%d|N=%lld|ents=%d|R1=%d", p.f32 ? "f32" : "f64", p.snmax[s],
             p.snmin[s], (long long)p.g.N, p.n_ent, p.g.R[p.g.D - 1] == 1 ? 1 : 0);
    return buf;
}

static TileCand tile_rule(int nmax) {
    if (nmax <= 8) return {1, 8};
    if (nmax <= 16) return {1, 16};
    if (nmax <= 32) return {2, 16};
    if (nmax <= 48) return {3, 16};
    return {4, 16};
}

template <typename TS, typename T>
static void launch_tile_cfg(const ProgView &p, int s, const TS *in, hipStream_t st, const char *name, TileCand c) {
    const uint32_t maxcol = (uint32_t)(p.g.N / p.snmin[s]);
    auto go = [&](auto kern, int rg) {
        const int cw = 4 * (256 / rg);
        dim3 grid((maxcol + cw - 1) / cw, p.n_ent);
        TTN_LAUNCH(name, p.sflops[s], p.sbytes[s], kern, grid, dim3(256), 0, st, p, s, in);
    };
#define TTN_TILE(TI, RG) \
    if (c.ti == TI && c.rg == RG) return go(k_mode_tile<TS, T, TI, RG>, RG);
    TTN_TILE(1, 8) TTN_TILE(2, 8) TTN_TILE(4, 8) TTN_TILE(1, 16) TTN_TILE(2, 16) TTN_TILE(3, 16) TTN_TILE(4, 16)
    TTN_TILE(1, 32) TTN_TILE(2, 32)
#undef TTN_TILE
    throw std::runtime_error("tile configuration not instantiated");
}

// tiled stage: the tile from the autotuner's table, else from the rule
template <typename TS, typename T>
static void launch_mode_tile_t(const ProgView &p, int s, const TS *in, hipStream_t st, const char *name) {
    TileCand c = tile_rule(p.snmax[s]);
    auto &tab = tile_table();
    if (!tab.empty()) {
        auto it = tab.find(tile_key(p, s));
        if (it != tab.end()) c = {it->second.ti, it->second.rg};
    }
    launch_tile_cfg<TS, T>(p, s, in, st, name, c);
}

template <typename TS, typename T>
static void tune_stage(const ProgView &p, int s, const TS *in, hipStream_t st) {
    const std::string key = tile_key(p, s);
    if (tile_table().count(key)) return;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        throw std::runtime_error("autotuner: hipEventCreate failed");
    TileChoice best{0, 0, 1e30};
    const int nmax = p.snmax[s];
    for (const TileCand &c : TILE_CANDS) {
        const int np = c.ti * c.rg;
        if (np < nmax || np > std::max(16, 2 * nmax)) continue;
        launch_tile_cfg<TS, T>(p, s, in, st, "k_mode_tile_tune", c);  // warm-up
        double t = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            float ms = 0.f;
            if (hipEventRecord(a, st) != hipSuccess) throw std::runtime_error("autotuner: event record");
            launch_tile_cfg<TS, T>(p, s, in, st, "k_mode_tile_tune", c);
            if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                hipEventElapsedTime(&ms, a, b) != hipSuccess)
                throw std::runtime_error("autotuner: timing failed");
            t = std::min(t, 1e3 * (double)ms);
        }
        if (t < best.us) best = {c.ti, c.rg, t};
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (best.ti > 0) tile_table()[key] = best;
}

static int stage_on_mfma(const ProgView &p, int s);

void tune_prog_stages(const ProgView &p, const double2 *in, hipStream_t st) {
    if (p.n_ent == 0) return;
    ProfileSuspend quiet;  // the trial launches are not part of any profile
    for (int s = 0; s < p.max_nf; ++s) {
        if (!p.stile[s] || stage_on_mfma(p, s)) continue;
        if (p.f32) {
            if (s == 0) tune_stage<double2, float2>(p, s, in, st);
            else tune_stage<float2, float2>(p, s, (const float2 *)nullptr, st);
        } else {
            tune_stage<double2, double2>(p, s, in, st);
        }
    }
}

size_t tile_table_size() { return tile_table().size(); }

// One entry per line: ["key", ti, rg, microseconds]
void tile_table_save(const char *path) {
    FILE *f = fopen(path, "w");
    if (!f) throw std::runtime_error(std::string("cannot write ") + path);
    fprintf(f, "{\"ttn_tile_table\": 1, \"entries\": [\n");
    size_t i = 0;
    for (auto &kv : tile_table())
        fprintf(f, " [\"%s\", %d, %d, %.3f]%s\n", kv.first.c_str(), kv.second.ti, kv.second.rg, kv.second.us,
                ++i < tile_table().size() ? "," : "");
    fprintf(f, "]}\n");
    fclose(f);
}

int tile_table_load(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) throw std::runtime_error(std::string("cannot read ") + path);
    char line[512];
    int n = 0;
    while (fgets(line, sizeof line, f)) {
        const char *q = strstr(line, "[\"");
        if (!q) continue;
        char key[256];
        int ti = 0, rg = 0;
        double us = 0.0;
        if (sscanf(q, "[\"%255[^\"]\", %d, %d, %lf]", key, &ti, &rg, &us) != 4) continue;
        bool ok = false;
        for (const TileCand &c : TILE_CANDS) ok |= c.ti == ti && c.rg == rg;
        if (!ok) continue;  // not a tile this build instantiates
        tile_table()[key] = {ti, rg, us};
        ++n;
    }
    fclose(f);
    return n;
}

void tile_table_clear() { tile_table().clear(); }

static void launch_mode_mfma(const ProgView &p, int s, const double2 *in, const float2 *in32, hipStream_t st) {
    const uint32_t maxcol = (uint32_t)(p.g.N / p.snmin[s]);
    dim3 grid((maxcol + MF_CW - 1) / MF_CW, p.n_ent);
    const int RT = (p.snmax[s] + 15) / 16;
    const int RD = 32 * RT;
    TTN_LAUNCH("k_mfma_prep", 0.0, 4.0 * RD * RD * p.n_ent, k_mfma_prep, dim3(4, p.n_ent), dim3(256), 0, st, p, s,
               RD, p.mprep);
    const unsigned short *mp = p.mprep;
    const float2 *f = s == 0 ? in32 : nullptr;
#define TTN_MFMA_CASE(RTV)                                                                                      \
    case RTV:                                                                                                   \
        if (s == 0 && !in32)                                                                                    \
            TTN_LAUNCH("k_mode_mfma", p.sflops[s], p.sbytes[s], (k_mode_mfma<double2, RTV>), grid, dim3(256), 0, \
                       st, p, s, in, mp);                                                                       \
        else                                                                                                    \
            TTN_LAUNCH("k_mode_mfma", p.sflops[s], p.sbytes[s], (k_mode_mfma<float2, RTV>), grid, dim3(256), 0,  \
                       st, p, s, f, mp);                                                                        \
        break;
    switch (RT) {
        TTN_MFMA_CASE(2)
        TTN_MFMA_CASE(3)
        TTN_MFMA_CASE(4)
    default: throw std::runtime_error("MFMA stage shape out of range");
    }
#undef TTN_MFMA_CASE
}

static void launch_mode_mfma32(const ProgView &p, int s, const double2 *in, const float2 *in32, hipStream_t st) {
    const uint32_t maxcol = (uint32_t)(p.g.N / p.snmin[s]);
    dim3 grid((maxcol + M32_CW - 1) / M32_CW, p.n_ent);
    const int RT = (p.snmax[s] + 15) / 16;
    const float2 *f = s == 0 ? in32 : nullptr;
#define TTN_M32_CASE(RTV)                                                                                          \
    case RTV:                                                                                                      \
        if (s == 0 && !in32)                                                                                       \
            TTN_LAUNCH("k_mode_mfma32", p.sflops[s], p.sbytes[s], (k_mode_mfma32<double2, RTV>), grid, dim3(256), \
                       0, st, p, s, in);                                                                           \
        else                                                                                                       \
            TTN_LAUNCH("k_mode_mfma32", p.sflops[s], p.sbytes[s], (k_mode_mfma32<float2, RTV>), grid, dim3(256),  \
                       0, st, p, s, f);                                                                            \
        break;
    switch (RT) {
        TTN_M32_CASE(2)
        TTN_M32_CASE(3)
        TTN_M32_CASE(4)
    default: throw std::runtime_error("MFMA stage shape out of range");
    }
#undef TTN_M32_CASE
}

static void launch_mode_mfma64(const ProgView &p, int s, const double2 *in, hipStream_t st) {
    const uint32_t maxcol = (uint32_t)(p.g.N / p.snmin[s]);
    dim3 grid((maxcol + M64_CW - 1) / M64_CW, p.n_ent);
    const int need = (2 * p.snmax[s] + 15) / 16;
    const double2 *x = s == 0 ? in : nullptr;
#define TTN_M64(RTV) \
    TTN_LAUNCH("k_mode_mfma64", p.sflops[s], p.sbytes[s], (k_mode_mfma64<RTV>), grid, dim3(256), 0, st, p, s, x)
    if (need <= 2) TTN_M64(2);
    else if (need <= 3) TTN_M64(3);
    else if (need <= 4) TTN_M64(4);
    else if (need <= 6) TTN_M64(6);
    else TTN_M64(8);
#undef TTN_M64
}

// dense stages go to the matrix cores: factors of 24..64 in BF16x3 in the
// BF16x3 mode and in FP32 in the FP32 mode, of 16..64 in FP64 in the FP64 mode
// (when enabled)
static int stage_on_mfma(const ProgView &p, int s) {
    if (!p.stile[s] || p.snmax[s] > 64) return 0;
    if (p.bf16x3 && p.mprep) return p.snmin[s] >= 24 ? 1 : 0;
    if (p.f32 && !p.bf16x3 && p.mfma32) return p.snmin[s] >= 24 ? 2 : 0;
    if (!p.f32 && p.mfma64) return p.snmin[s] >= 16 ? 3 : 0;
    return 0;
}

static void launch_mode_tile(const ProgView &p, int s, const double2 *in, const float2 *in32, hipStream_t st) {
    switch (stage_on_mfma(p, s)) {
    case 1: launch_mode_mfma(p, s, in, in32, st); return;
    case 2: launch_mode_mfma32(p, s, in, in32, st); return;
    case 3: launch_mode_mfma64(p, s, in, st); return;
    default: break;
    }
    if (p.f32) {
        if (s == 0 && !in32) launch_mode_tile_t<double2, float2>(p, s, in, st, "k_mode_tile_f32");
        else launch_mode_tile_t<float2, float2>(p, s, s == 0 ? in32 : nullptr, st, "k_mode_tile_f32");
    } else {
        launch_mode_tile_t<double2, double2>(p, s, in, st, "k_mode_tile");
    }
}

void launch_prog_stages(const ProgView &p, const double2 *in, hipStream_t st, float2 *x32) {
    if (p.n_ent == 0) return;
    int maxn = 0;
    for (int s = 0; s < p.g.D; ++s) maxn = maxn > p.g.dims[s] ? maxn : p.g.dims[s];
    const int ldn = maxn <= 64 ? maxn : 0;
    const size_t lds = sizeof(double2) * (size_t)ldn * ldn;
    // one conversion of the shared input instead of one per entry (every entry
    // reads the same input when in_stride is 0)
    const float2 *in32 = nullptr;
    if (p.f32 && x32 && p.in_stride == 0 && p.n_ent >= 4 && p.max_nf > 0) {
        launch_to_f32(in, x32, p.g.N, st);
        in32 = x32;
    }
    for (int s = 0; s < p.max_nf; ++s) {
        if (p.stile[s]) {
            launch_mode_tile(p, s, in, in32, st);
            continue;
        }
        dim3 grid(grid_for(p.g.N, 256), p.n_ent);
        if (p.f32) {
            const size_t l32 = lds / 2;
            if (s == 0 && !in32)
                TTN_LAUNCH("k_mode_stage_f32", p.sflops[s], p.sbytes[s], (k_mode_stage<double2, float2>), grid,
                           dim3(256), l32, st, p, s, in, ldn);
            else
                TTN_LAUNCH("k_mode_stage_f32", p.sflops[s], p.sbytes[s], (k_mode_stage<float2, float2>), grid,
                           dim3(256), l32, st, p, s, s == 0 ? in32 : (const float2 *)nullptr, ldn);
        } else {
            TTN_LAUNCH("k_mode_stage", p.sflops[s], p.sbytes[s], (k_mode_stage<double2, double2>), grid, dim3(256),
                       lds, st, p, s, in, ldn);
        }
    }
}

void launch_prog_sum(const ProgView &p, const double2 *in, double2 *out_single, hipStream_t st) {
    dim3 grid(grid_for(p.g.N, 256), out_single ? 1 : p.n_groups);
    const double es = p.f32 ? 8.0 : 16.0;
    const double by = es * p.g.N * p.n_ent + (out_single ? 16.0 : es * p.n_groups) * p.g.N;
    if (p.f32)
        TTN_LAUNCH("k_group_sum_f32", 8.0 * p.g.N * p.n_ent, by, k_group_sum<float2>, grid, dim3(256), 0, st, p, in,
                   out_single);
    else
        TTN_LAUNCH("k_group_sum", 8.0 * p.g.N * p.n_ent, by, k_group_sum<double2>, grid, dim3(256), 0, st, p, in,
                   out_single);
}

void launch_prog_contract(const ProgView &p, const double2 *A, hipStream_t st) {
    const int s = p.contract_slot;
    const int n = p.g.dims[s];
    const uint32_t L = (uint32_t)p.g.L[s], R = (uint32_t)p.g.R[s];
    const int nb = contract_blocks(L * R);
    const size_t lds = sizeof(double2) * (size_t)CT_ROWS * 2 * n;
    if (p.f32 && p.mfma32 && n <= 64) {
        const unsigned grid = 8 * (unsigned)((nb + 7) / 8) * (unsigned)p.n_groups;
        const double fl = 8.0 * p.g.N * n * p.n_groups, by = (16.0 + 8.0) * p.g.N * p.n_groups;
#define TTN_CM(RTV, CTV)                                                                                            \
    TTN_LAUNCH("k_contract_mfma", fl, by, (k_contract_mfma<RTV, CTV>), dim3(grid), dim3(256), 0, st, A,             \
               (const float2 *)p.gsum, p.g.N, L, n, R, nb, p.n_groups, p.cpart)
        if (n <= 16) TTN_CM(1, 1);
        else if (n <= 32) TTN_CM(1, 2);
        else if (n <= 48) TTN_CM(2, 3);
        else TTN_CM(2, 4);
#undef TTN_CM
    } else if (p.f32)
        TTN_LAUNCH("k_contract_part_f32", 8.0 * p.g.N * n * p.n_groups, 16.0 * p.g.N + 8.0 * p.g.N * p.n_groups,
                   k_contract_part<float2>, dim3(nb, p.n_groups), dim3(256), lds / 2, st, A,
                   (const float2 *)p.gsum, p.g.N, L, n, n, R, p.cpart);
    else
        TTN_LAUNCH("k_contract_part", 8.0 * p.g.N * n * p.n_groups, 16.0 * p.g.N * (1 + p.n_groups),
                   k_contract_part<double2>, dim3(nb, p.n_groups), dim3(256), lds, st, A, (const double2 *)p.gsum,
                   p.g.N, L, n, n, R, p.cpart);
    TTN_LAUNCH("k_contract_reduce", 2.0 * nb * n * n * p.n_groups, 16.0 * nb * n * n * p.n_groups, k_contract_reduce,
               dim3(grid_for(n * n, 256), p.n_groups), dim3(256), 0, st, (const double2 *)p.cpart, nb, n * n, p.gdst,
               (double2 *)nullptr);
}

void launch_mode_product(const double2 *X, double2 *Y, const double2 *M, int64_t L, int n_in, int n_out,
                         int64_t R, int transM, hipStream_t st) {
    const int64_t NY = L * n_out * R;
    TTN_LAUNCH("k_mode_single", 8.0 * NY * n_in, 16.0 * (L * n_in * R + NY + (int64_t)n_in * n_out), k_mode_single,
               dim3(grid_for(NY, 256)), dim3(256), 0, st, X, Y, M, (uint32_t)L, n_in, n_out, (uint32_t)R, transM);
}

void launch_contract(const double2 *A, const double2 *B, double2 *out, int64_t L, int nA, int nB, int64_t R,
                     double2 *part, hipStream_t st) {
    const int nb = contract_blocks((uint32_t)(L * R));
    const size_t lds = sizeof(double2) * (size_t)CT_ROWS * (nA + nB);
    TTN_LAUNCH("k_contract_part", 8.0 * L * R * nA * nB, 16.0 * L * R * (nA + nB), k_contract_part<double2>, dim3(nb, 1),
               dim3(256), lds, st, A, B, (int64_t)0, (uint32_t)L, nA, nB, (uint32_t)R, part);
    TTN_LAUNCH("k_contract_reduce", 2.0 * nb * nA * nB, 16.0 * nb * nA * nB, k_contract_reduce,
               dim3(grid_for(nA * nB, 256), 1), dim3(256), 0, st, (const double2 *)part, nb, nA * nB,
               (double2 *const *)nullptr, out);
}

void launch_qr(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, hipStream_t st,
               const int *gate) {
    if (n > 64 || L * R < n) throw std::runtime_error("QR shape out of range");
    const double mm = (double)L * R;
    TTN_LAUNCH("k_qr", 16.0 * mm * n * n, 16.0 * mm * n * 4, k_qr, dim3(1), dim3(1024), 0, st, A, (uint32_t)L, n,
               (uint32_t)R, Rout, transR, QR_SNAP, gate);
}

void launch_qr_multi(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, const QRWork &q,
                     hipStream_t st) {
    const int64_t m = L * R;
    if (n > QRM_MAXN || m < n) throw std::runtime_error("QR shape out of range");
    int64_t rows_per = (m + QRM_BLOCKS_MAX - 1) / QRM_BLOCKS_MAX;
    if (rows_per < 64) rows_per = 64;
    const unsigned nb = (unsigned)((m + rows_per - 1) / rows_per);
    for (int i = 0; i < n; ++i)
        TTN_LAUNCH("k_qrm_step", 16.0 * m * (n - i), 32.0 * m * (n - i), k_qrm_step, dim3(nb), dim3(QRM_THREADS), 0, st,
                   A, (uint32_t)L, n, (uint32_t)R, i, (uint32_t)rows_per, q, QR_SNAP);
    const size_t lds_fin = sizeof(double2) * 2 * n * n;
    set_lds_limit((const void *)k_qrm_finish, lds_fin);
    TTN_LAUNCH("k_qrm_finish", 4.0 * m * n * n, 16.0 * m * n, k_qrm_finish, dim3(nb), dim3(QRM_THREADS), lds_fin, st,
               A, (uint32_t)L, n, (uint32_t)R, (uint32_t)rows_per, q, Rout, transR);
    const size_t lds_q = sizeof(double2) * (size_t)(n * n + 16 * n);
    set_lds_limit((const void *)k_qrm_formq, lds_q);
    TTN_LAUNCH("k_qrm_formq", 8.0 * m * n * n, 32.0 * m * n, k_qrm_formq, dim3(nb), dim3(QRM_THREADS), lds_q, st, A,
               (uint32_t)L, n, (uint32_t)R, (uint32_t)rows_per, q);
}

bool launch_qr_coop(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, QRWork &q,
                    hipStream_t st) {
    const int64_t m = L * R;
    if (n > QRM_MAXN || m < n) throw std::runtime_error("QR shape out of range");
    // LDS: the row tile plus an auxiliary region (reduction staging, T and S, K)
    const size_t aux = std::max<size_t>((size_t)2 * n * n, QRC_STAGE / 2);
    const size_t budget = 150 * 1024 / sizeof(double2);  // elements
    if (aux + (size_t)64 * n > budget) return false;
    const int64_t tile_rows = (int64_t)((budget - aux) / n);
    // at least 2048 matrix elements per work-group, and few enough work-groups
    // (about 64, within the tile) that the per-column exchange of partial
    // records stays small: every work-group reads every record of a column
    int64_t rows_per = std::max<int64_t>({64, (2048 + n - 1) / n, (m + 63) / 64});
    if (rows_per > tile_rows) rows_per = tile_rows;
    if ((m + rows_per - 1) / rows_per > QRM_BLOCKS_MAX) rows_per = (m + QRM_BLOCKS_MAX - 1) / QRM_BLOCKS_MAX;
    if (rows_per > tile_rows || rows_per < n) return false;
    const unsigned nb = (unsigned)((m + rows_per - 1) / rows_per);
    const size_t lds = sizeof(double2) * ((size_t)rows_per * n + aux);
    set_lds_limit((const void *)k_qr_coop, lds);
    // co-residency of the whole grid (queried once per device and LDS size)
    static std::map<std::pair<int, size_t>, int> cap;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    auto key = std::make_pair(dev, lds);
    if (!cap.count(key)) {
        int per_cu = 0, cus = 0, coop = 0;
        if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_qr_coop, QRM_THREADS, lds) !=
                hipSuccess)
            cap[key] = 0;
        else
            cap[key] = per_cu * cus;
    }
    if ((int)nb > cap[key] || nb > (unsigned)QRM_BLOCKS_MAX) return false;
    uint32_t Lu = (uint32_t)L, Ru = (uint32_t)R, rp = (uint32_t)rows_per;
    double snap = QR_SNAP;
    QRWork qq = q;
    unsigned long long *ts = nullptr;
    int slot = -1;
    if (prof::on && !prof::suspended) {
        ts = prof::take_ts();
        if (ts) slot = (int)(ts - prof::ts);
    }
    void *args[] = {&A, &Lu, &n, &Ru, &rp, &qq, &Rout, &transR, &snap, &ts};
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_qr_coop, dim3(nb), dim3(QRM_THREADS), args, lds, st);
    if (e != hipSuccess) throw std::runtime_error(std::string("hipLaunchCooperativeKernel: ") + hipGetErrorString(e));
    q.bar_base += (unsigned long long)nb * (unsigned long long)(n + 2);  // n column barriers, Gram, K
    if (prof::on && slot >= 0)
        prof::recs.push_back({"k_qr_coop", nullptr, nullptr, 16.0 * (double)m * n * n, 32.0 * (double)m * n, slot});
    return true;
}

// Gram partials of the Cholesky route on the FP64 matrix cores (TTN_CQR_MFMA=0:
// the vector-ALU kernel)
static bool cqr_mfma_setting() {
    static const bool v = [] {
        const char *e = getenv("TTN_CQR_MFMA");
        return e ? atoi(e) != 0 : true;
    }();
    return v;
}

bool launch_qr_chol(double2 *A, int64_t L, int n, int64_t R, double2 *Rout, int transR, const QRWork &q,
                    hipStream_t st) {
    const int64_t m = L * R;
    if (!q.cq_part || !q.cq_state || n < 1 || n > 64 || m < n || m * n > q.cq_ycap || m > (int64_t)UINT32_MAX)
        return false;
    int64_t rows_per = std::max<int64_t>(CQR_TILE, (m + CQR_BLOCKS_MAX - 1) / CQR_BLOCKS_MAX);
    rows_per = (rows_per + CQR_TILE - 1) / CQR_TILE * CQR_TILE;
    const unsigned nb = (unsigned)((m + rows_per - 1) / rows_per);
    if (nb > (unsigned)CQR_BLOCKS_MAX) return false;
    const size_t lds_tile = sizeof(double2) * (size_t)CQR_TILE * (n + 1);
    const size_t lds_mat = sizeof(double2) * (size_t)n * n;
    const unsigned nbr = (unsigned)((n * n + CQR_RTHREADS / 8 - 1) / (CQR_RTHREADS / 8));
    const double mm = (double)m, nn = (double)n * n;
    set_lds_limit((const void *)k_cqr_gram<false>, lds_tile);
    set_lds_limit((const void *)k_cqr_gram<true>, lds_tile + lds_mat);
    set_lds_limit((const void *)k_cqr_reduce, 2 * lds_mat);
    set_lds_limit((const void *)k_cqr_apply, lds_tile + lds_mat);
    const uint32_t Lu = (uint32_t)L, Ru = (uint32_t)R, rp = (uint32_t)rows_per;
    const double2 *Ac = A;
    const bool mf = cqr_mfma_setting();
    auto gram = [&](auto tag) {
        constexpr bool AP = decltype(tag)::value;
        const double fl = AP ? 12.0 * mm * nn : 8.0 * mm * nn;
        const double by = AP ? 16.0 * (2 * mm * n + nb * nn) : 16.0 * (mm * n + nb * nn);
        const size_t lds = AP ? lds_tile + lds_mat : lds_tile;
        if (!mf) {
            TTN_LAUNCH("k_cqr_gram", fl, by, k_cqr_gram<AP>, dim3(nb), dim3(CQR_THREADS), lds, st, Ac, Lu, n, Ru, rp, q);
            return;
        }
#define TTN_CQG(RTV, CTV)                                                                                          \
    do {                                                                                                           \
        set_lds_limit((const void *)k_cqr_gram_mfma<AP, RTV, CTV>, lds);                                           \
        TTN_LAUNCH("k_cqr_gram_mfma", fl, by, (k_cqr_gram_mfma<AP, RTV, CTV>), dim3(nb), dim3(CQR_THREADS), lds, st, \
                   Ac, Lu, n, Ru, rp, q);                                                                          \
    } while (0)
        if (n <= 16) TTN_CQG(1, 2);
        else if (n <= 32) TTN_CQG(2, 4);
        else if (n <= 48) TTN_CQG(3, 6);
        else TTN_CQG(4, 8);
#undef TTN_CQG
    };
    gram(std::false_type{});
    TTN_LAUNCH("k_cqr_reduce", 2.0 * nb * nn, 16.0 * nb * nn, k_cqr_reduce, dim3(nbr), dim3(CQR_RTHREADS), 2 * lds_mat,
               st, (int)nb, n, 1, q, Rout, transR);
    gram(std::true_type{});
    TTN_LAUNCH("k_cqr_reduce", 2.0 * nb * nn, 16.0 * nb * nn, k_cqr_reduce, dim3(nbr), dim3(CQR_RTHREADS), 2 * lds_mat,
               st, (int)nb, n, 2, q, Rout, transR);
    TTN_LAUNCH("k_cqr_apply", 4.0 * mm * nn, 32.0 * mm * n, k_cqr_apply, dim3(nb), dim3(CQR_THREADS),
               lds_tile + lds_mat, st, A, Lu, n, Ru, rp, q);
    return true;
}

void launch_zero_tail(double2 *C, int n, int keep, hipStream_t st) {
    TTN_LAUNCH("k_zero_tail", 0.0, 16.0 * n * n, k_zero_tail, dim3(grid_for((int64_t)n * n, 256)), dim3(256), 0, st, C,
               n, keep);
}

void launch_pair_build(const PairPass &pp, hipStream_t st) {
    const int na = pp.nk * pp.nk, nb = pp.np * pp.np;
    dim3 grid((unsigned)((na + 63) / 64), (unsigned)((nb + 63) / 64));
    TTN_LAUNCH("k_pair_build", 8.0 * na * nb * pp.n_terms, 8.0 * na * nb + 16.0 * pp.n_terms * (pp.nk * pp.nk + nb),
               k_pair_build, grid, dim3(256), 0, st, pp);
}

// column tiles per wave of the pair GEMM: 2, 4, or 0 for the size rule (TTN_PAIR_WN)
static int pair_gemm_wn_setting() {
    static const int v = [] {
        const char *e = getenv("TTN_PAIR_WN");
        const int w = e ? atoi(e) : 0;
        return (w == 2 || w == 4) ? w : 0;
    }();
    return v;
}

void launch_to_bf16x2(const double2 *x, unsigned *xh, unsigned *xl, int64_t n, hipStream_t st) {
    TTN_LAUNCH("k_to_bf16x2", 0.0, 24.0 * n, k_to_bf16x2, dim3(grid_for(n, 256)), dim3(256), 0, st, x, xh, xl, n);
}

void launch_pair_split(const PairPass &pp, hipStream_t st) {
    const int64_t q2 = (int64_t)pp.nk * pp.np * pp.nk * pp.np;
    TTN_LAUNCH("k_pair_split", 0.0, 24.0 * q2, k_pair_split, dim3(grid_for(q2, 256)), dim3(256), 0, st, pp);
}

static int resident_slots(const void *kern, size_t lds);
static size_t pair_gemm_bf_lds() { return sizeof(unsigned short) * (size_t)(2 * PG_BM + 2 * 128) * PGB_LD; }

void launch_pair_gemm_bf(const PairPass &pp, const unsigned *xh, const unsigned *xl, double2 *out, int accumulate,
                         double flops, float *ws, int ws_slots, hipStream_t st) {
    const int Q = pp.nk * pp.np;
    const int64_t M = pp.L * pp.Mid;
    const double N = (double)M * Q;
    PairSched sc;
    sc.nct = (unsigned)((2 * Q + 127) / 128);
    sc.nrt = (unsigned)((M + PG_BM - 1) / PG_BM);
    sc.ntile = sc.nrt * sc.nct;
    sc.kc = (unsigned)((Q + PGB_KS - 1) / PGB_KS);
    const size_t lds = pair_gemm_bf_lds();
    set_lds_limit((const void *)k_pair_gemm_bf, lds);
    const unsigned per_xcd = (sc.ntile + 7) / 8;
    const int slots = ws ? (ws_slots > 0 ? std::max(8, ws_slots / 8 * 8)
                                         : resident_slots((const void *)k_pair_gemm_bf, lds))
                         : (int)(8 * per_xcd);
    const unsigned grid = 8 * std::min<unsigned>((unsigned)slots / 8, per_xcd);
    TTN_LAUNCH("k_pair_gemm_bf", flops, 8.0 * N + 16.0 * N * (accumulate ? 2 : 1) + 16.0 * Q * Q, k_pair_gemm_bf,
               dim3(grid), dim3(256), lds, st, pp, xh, xl, out, accumulate, ws, slots, sc);
    if ((unsigned)slots / 8 < per_xcd) {  // some tiles are cut
        const double fb = (double)slots * 256 * 64 * 4 * 2 + 16.0 * (double)slots * PG_BM * 64;
        TTN_LAUNCH("k_pair_fixup", 0.0, fb, k_pair_fixup<2>, dim3(slots), dim3(256), 0, st, pp, out, accumulate,
                   (const float *)ws, slots, sc);
    }
}

void launch_to_f32(const double2 *x, float2 *y, int64_t n, hipStream_t st) {
    TTN_LAUNCH("k_to_f32", 0.0, 24.0 * n, k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, x, y, n);
}

template <int WN> static size_t pair_gemm_lds() { return sizeof(float) * 2 * (PG_BM * PG_LDA + 64 * WN * PG_LDB); }

// resident work-groups of a kernel (256 threads, `lds` bytes of LDS) on the
// current device, a multiple of 8 (the schedules deal whole rounds of the 8
// XCDs), computed once per device and kernel
static int resident_slots(const void *kern, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, kern});
    if (it != cache.end()) return it->second;
    set_lds_limit(kern, lds);
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess)
        throw std::runtime_error("pair GEMM: device occupancy query failed");
    const int slots = std::max(8, (cus * std::max(1, per_cu)) / 8 * 8);
    cache[{dev, kern}] = slots;
    return slots;
}
template <int WN> static int pair_gemm_slots() {
    return resident_slots((const void *)k_pair_gemm<WN, true>, pair_gemm_lds<WN>());
}

template <int WN> static int pair_slots_or(int slots) {
    return slots > 0 ? std::max(8, slots / 8 * 8) : pair_gemm_slots<WN>();
}

size_t pair_gemm_ws_bytes(int slots, int bf16x3) {
    // part 0 and part 1 of at most one cut per work-group slot, 32 WN floats per thread each
    if (bf16x3) {
        const int sl = slots > 0 ? std::max(8, slots / 8 * 8) : resident_slots((const void *)k_pair_gemm_bf,
                                                                                pair_gemm_bf_lds());
        return (size_t)sl * 2 * 256 * 32 * 2 * sizeof(float);
    }
    return pair_gemm_wn_setting() == 4 ? (size_t)pair_slots_or<4>(slots) * 2 * 256 * 32 * 4 * sizeof(float)
                                       : (size_t)pair_slots_or<2>(slots) * 2 * 256 * 32 * 2 * sizeof(float);
}

template <int WN>
static void pair_gemm_go(const PairPass &pp, const float2 *in, double2 *out, int accumulate, double flops, double by,
                         float *ws, int ws_slots, hipStream_t st) {
    const int Q = pp.nk * pp.np;
    const int64_t M = pp.L * pp.Mid;
    PairSched sc;
    sc.nrt = (unsigned)((M + PG_BM - 1) / PG_BM);
    sc.nct = (unsigned)((2 * Q + 64 * WN - 1) / (64 * WN));
    sc.ntile = sc.nrt * sc.nct;
    sc.kc = (unsigned)((Q + PG_KS - 1) / PG_KS);
    const size_t lds = pair_gemm_lds<WN>();
    const unsigned per_xcd = (sc.ntile + 7) / 8;  // largest tile range of an XCD
    // without a workspace: one work-group per tile (shares never cut a tile)
    const int slots = ws ? pair_slots_or<WN>(ws_slots) : (int)(8 * per_xcd);
    const unsigned grid = 8 * std::min<unsigned>((unsigned)slots / 8, per_xcd);
    if (pp.v4 && pp.np % 4 == 0) {  // 16-byte staging
        set_lds_limit((const void *)k_pair_gemm<WN, true>, lds);
        TTN_LAUNCH("k_pair_gemm", flops, by, (k_pair_gemm<WN, true>), dim3(grid), dim3(256), lds, st, pp, in, out,
                   accumulate, ws, slots, sc);
    } else {
        set_lds_limit((const void *)k_pair_gemm<WN, false>, lds);
        TTN_LAUNCH("k_pair_gemm", flops, by, (k_pair_gemm<WN, false>), dim3(grid), dim3(256), lds, st, pp, in, out,
                   accumulate, ws, slots, sc);
    }
    if ((unsigned)slots / 8 < per_xcd) {  // some tiles are cut
        const double fb = (double)slots * 256 * 32 * WN * 4 * 2 + 16.0 * (double)slots * PG_BM * 32 * WN;
        TTN_LAUNCH("k_pair_fixup", 0.0, fb, k_pair_fixup<WN>, dim3(slots), dim3(256), 0, st, pp, out, accumulate,
                   (const float *)ws, slots, sc);
    }
}

void launch_pair_gemm(const PairPass &pp, const float2 *in, double2 *out, int accumulate, double flops, float *ws,
                      int ws_slots, hipStream_t st) {
    const int Q = pp.nk * pp.np;
    const int64_t M = pp.L * pp.Mid;
    const double N = (double)M * Q;
    const double by = 8.0 * N + 16.0 * N * (accumulate ? 2 : 1) + 8.0 * Q * Q;
    // wider column tiles halve the re-reads of the input where the column count allows
    if (pair_gemm_wn_setting() == 4) pair_gemm_go<4>(pp, in, out, accumulate, flops, by, ws, ws_slots, st);
    else pair_gemm_go<2>(pp, in, out, accumulate, flops, by, ws, ws_slots, st);
}

static size_t small_solve_total_lds(const SmallSolveArgs &a) {
    return small_solve_lds_bytes(a.g.N, a.mmax, a.batched, a.nA) + (a.vlds ? small_solve_vlds_bytes(a.g.N, a.mmax) : 0) +
           (a.mlds ? sizeof(double2) * (size_t)a.mlds_elems : 0);
}

static int small_solve_threads(const SmallSolveArgs &a);

void launch_small_solve_group(const SmallSolveArgs *d_args, const std::vector<SmallSolveArgs> &h_args,
                              hipStream_t st) {
    if (h_args.empty()) return;
    size_t lds = 0;
    int threads = 64;
    for (auto &a : h_args) {
        const size_t l = small_solve_total_lds(a);
        if (a.g.N > SMALL_MAX || a.mmax > SMALL_MMAX || l + SMALL_STATIC_LDS > 160 * 1024 || (a.mlds && !a.batched) ||
            (a.batched && (a.g.D != 2 || a.n_ent > SMALL_MAXENT || a.g.dims[0] * a.g.dims[0] > SMALL_UB)))
            throw std::runtime_error("grouped small solve out of range");
        lds = std::max(lds, l);
        threads = std::max(threads, small_solve_threads(a));
    }
    set_lds_limit((const void *)k_small_solve_group, lds);
    TTN_LAUNCH("k_small_solve", 0.0, 0.0, k_small_solve_group, dim3((unsigned)h_args.size()), dim3(threads), lds, st,
               d_args);
}

void launch_small_solve(const SmallSolveArgs &a, hipStream_t st) {
    const size_t lds0 = small_solve_lds_bytes(a.g.N, a.mmax, a.batched, a.nA);
    const size_t lds = lds0 + (a.vlds ? small_solve_vlds_bytes(a.g.N, a.mmax) : 0) +
                       (a.mlds ? sizeof(double2) * (size_t)a.mlds_elems : 0);
    if (a.mlds && !a.batched) throw std::runtime_error("factor staging needs the batched matvec");
    if (a.g.N > SMALL_MAX || a.mmax > SMALL_MMAX || lds + SMALL_STATIC_LDS > 160 * 1024 ||
        (a.batched && (a.g.D != 2 || a.n_ent > SMALL_MAXENT || a.g.dims[0] * a.g.dims[0] > SMALL_UB)))
        throw std::runtime_error("small solve out of range");
    set_lds_limit((const void *)k_small_solve, lds);
    TTN_LAUNCH("k_small_solve", 0.0, 0.0, k_small_solve, dim3(1), dim3(small_solve_threads(a)), lds, st, a);
}

// work-group size: the problem size rounded up to a wavefront, capped
static int small_solve_threads(const SmallSolveArgs &a) {
    static int cap = -1;
    if (cap < 0) {
        const char *env = getenv("TTN_SMALL_THREADS");
        cap = env ? atoi(env) : 512;
        if (cap < 64 || cap > SMALL_THREADS) cap = 512;
    }
    int threads = (int)((a.g.N + 63) / 64) * 64;
    if (threads < 64) threads = 64;
    if (threads > cap) threads = cap;
    // batched: phase B splits the entries over the spare threads; beyond ~100
    // elements a full 1024-thread work-group (four waves per SIMD) hides the
    // LDS latency of the matvec and of the Gram-Schmidt dots better
    if (a.batched && threads < 256) threads = 256;
    if (a.batched && a.g.N > 96) threads = SMALL_THREADS;
    return threads;
}

void launch_copy(double2 *dst, const double2 *src, int64_t n, hipStream_t st) {
    TTN_LAUNCH("k_copy", 0.0, 32.0 * n, k_copy, dim3(grid_for(n, 256)), dim3(256), 0, st, dst, src, (uint32_t)n);
}

void launch_combine(const CombJob *jobs, const CombSrc *srcs, int n_jobs, int max_n2, hipStream_t st) {
    if (n_jobs <= 0) return;
    TTN_LAUNCH("k_combine", 0.0, 32.0 * max_n2 * n_jobs, k_combine, dim3(grid_for(max_n2, 256, 64), n_jobs),
               dim3(256), 0, st, jobs, srcs);
}

void launch_ts_contract(const double2 *A, int64_t L, int n, int64_t R, int conjA, const double2 *B,
                        int64_t bstride, int groups, double2 *out, double2 *part, hipStream_t st) {
    if (n > 64 || groups < 1) throw std::runtime_error("two-site contraction shape out of range");
    const int64_t rows = L * R;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(64, (rows + 1023) / 1024));
    TTN_LAUNCH("k_ts_contract_part", 8.0 * rows * n * groups, 16.0 * rows * (n + groups), k_ts_contract_part,
               dim3(nb, groups), dim3(256), 0, st, A, (uint32_t)L, n, (uint32_t)R, conjA, B, bstride, part);
    TTN_LAUNCH("k_ts_reduce", 0.0, 16.0 * nb * n * groups, k_ts_reduce, dim3(grid_for((int64_t)n * groups, 256)),
               dim3(256), 0, st, (const double2 *)part, nb, n, groups, out);
}

void launch_ts_expand(const double2 *A, int64_t L, int n, int64_t R, int conjA, const double2 *S, int groups,
                      const double2 *base, int negate, double2 *out, hipStream_t st) {
    if (n > 64 || groups < 1 || (size_t)groups * n * sizeof(double2) > 60 * 1024)
        throw std::runtime_error("two-site expansion shape out of range");
    const int64_t rows = L * R;
    TTN_LAUNCH("k_ts_expand", 8.0 * rows * n * groups, 16.0 * rows * (n * ((groups + 7) / 8) + groups), k_ts_expand,
               dim3(grid_for(rows, 256)), dim3(256), sizeof(double2) * groups * n, st, A, (uint32_t)L, n,
               (uint32_t)R, conjA, S, groups, base, negate, out);
}

void launch_repack(const double2 *X, double2 *Y, int64_t L, int n_old, int n_new, int64_t R, const double2 *V,
                   int64_t vstride, int conjV, hipStream_t st) {
    const int64_t NY = L * n_new * R;
    TTN_LAUNCH("k_repack", 0.0, 32.0 * NY, k_repack, dim3(grid_for(NY, 256)), dim3(256), 0, st, X, Y, (uint32_t)L,
               n_old, n_new, (uint32_t)R, V, vstride, conjV);
}

void launch_seed_vector(double2 *v, int64_t N, uint64_t seed, hipStream_t st) {
    TTN_LAUNCH("k_seed_vector", 0.0, 16.0 * N, k_seed_vector, dim3(grid_for(N, 256)), dim3(256), 0, st, v,
               (uint32_t)N, seed);
}

void launch_bidiag_svd(const double *alpha, const double *beta, const int *nptr, int nmax, double *s, double *U,
                       double *V, hipStream_t st) {
    if (nmax < 1) throw std::runtime_error("bidiagonal SVD: bad leading dimension");
    TTN_LAUNCH("k_bidiag_svd", 0.0, 0.0, k_bidiag_svd, dim3(1), dim3(64), 0, st, alpha, beta, nptr, nmax, s, U, V);
}

void launch_basis_combine(const double2 *V, int64_t N, const int *nptr, const double *W, int ldw, int ncols,
                          double2 *out, hipStream_t st) {
    if (ncols <= 0) return;
    TTN_LAUNCH("k_basis_combine", 0.0, 16.0 * N * ncols, k_basis_combine, dim3(grid_for(N, 256), ncols), dim3(256), 0,
               st, V, (uint32_t)N, nptr, W, ldw, ncols, out);
}

void launch_gkl_count(const int *meffP, const int *meffQ, const double *alpha0, int m, int *n, hipStream_t st) {
    TTN_LAUNCH("k_gkl_count", 0.0, 0.0, k_gkl_count, dim3(1), dim3(64), 0, st, meffP, meffQ, alpha0, m, n);
}

void launch_copy_scalars(double *dst, const double *src, int count, hipStream_t st) {
    TTN_LAUNCH("k_copy_scalars", 0.0, 16.0 * count, k_copy_scalars, dim3(1), dim3(64), 0, st, dst, src, count);
}

void launch_transpose(double2 *dst, const double2 *src, int n, hipStream_t st) {
    TTN_LAUNCH("k_transpose", 0.0, 32.0 * n * n, k_transpose, dim3(grid_for((int64_t)n * n, 256)), dim3(256), 0, st,
               dst, src, n);
}

static unsigned vec_blocks(int64_t N) {
    int64_t b = (N + 1023) / 1024;
    return (unsigned)(b < 1 ? 1 : (b > VEC_BLOCKS ? VEC_BLOCKS : b));
}

void launch_krylov_start(const double2 *x, int64_t N, const BigKrylov &k, hipStream_t st) {
    TTN_LAUNCH("k_kry_norm0", 4.0 * N, 16.0 * N, k_kry_norm0, dim3(vec_blocks(N)), dim3(VEC_THREADS), 0, st, x,
               (uint32_t)N, k);
    TTN_LAUNCH("k_kry_scale0", 2.0 * N, 32.0 * N, k_kry_scale0, dim3(grid_for(N, VEC_THREADS)), dim3(VEC_THREADS), 0,
               st, x, (uint32_t)N, k);
}

void launch_krylov_orth(const BigKrylov &k, int64_t N, int j, int mmax, hipStream_t st) {
    const unsigned nb = vec_blocks(N);
    const double nv = j + 1;
    TTN_LAUNCH("k_kry_orth", 8.0 * N * nv, 16.0 * N * (nv + 1), k_kry_orth, dim3(nb), dim3(VEC_THREADS), 0, st, k,
               (uint32_t)N, j, mmax, 0);
    TTN_LAUNCH("k_kry_orth", 16.0 * N * nv + 4.0 * N, 16.0 * N * (2 * nv + 2), k_kry_orth, dim3(nb),
               dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j, mmax, 1);
    TTN_LAUNCH("k_kry_finalize", 8.0 * N * nv + 2.0 * N, 16.0 * N * (nv + 2), k_kry_finalize,
               dim3(grid_for(N, VEC_THREADS)), dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j);
}

void launch_krylov_orth1(const BigKrylov &k, int64_t N, int j, int mmax, hipStream_t st) {
    const unsigned nb = vec_blocks(N);
    const double nv = j + 1;
    TTN_LAUNCH("k_kry_dots1", 16.0 * N * nv + 4.0 * N, 16.0 * N * (nv + 1), k_kry_dots1, dim3(nb), dim3(KD_THREADS),
               0, st, k, (uint32_t)N, j, mmax);
    TTN_LAUNCH("k_kry_update1", 8.0 * N * nv + 4.0 * N, 16.0 * N * (nv + 2), k_kry_update1, dim3(nb),
               dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j, mmax, 0);
    // refinement after heavy cancellation (both launches return at once otherwise)
    TTN_LAUNCH("k_kry_refine1", 0.0, 0.0, k_kry_refine1, dim3(nb), dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j, mmax);
    TTN_LAUNCH("k_kry_update1", 0.0, 0.0, k_kry_update1, dim3(nb), dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j, mmax,
               1);
    TTN_LAUNCH("k_kry_scale1", 0.0, 32.0 * N, k_kry_scale1, dim3(nb), dim3(VEC_THREADS), 0, st, k, (uint32_t)N, j);
}

void launch_krylov_ground(const BigKrylov &k, int64_t N, int m, int mmax, double2 *x, SolveStat *stat,
                          hipStream_t st) {
    if (m > 63) throw std::runtime_error("ground-state Lanczos dimension above 63");
    TTN_LAUNCH("k_kry_ground", 0.0, 0.0, k_kry_ground, dim3(1), dim3(64), 0, st, k, m, mmax, stat);
    TTN_LAUNCH("k_kry_combine", 8.0 * N * m, 16.0 * N * (m + 1), k_kry_combine, dim3(grid_for(N, VEC_THREADS)),
               dim3(VEC_THREADS), 0, st, k, (uint32_t)N, m, x);
}

void launch_krylov_finish(const BigKrylov &k, int64_t N, int m, int mmax, double tau, double tol, int hermitian,
                          double2 *x, SolveStat *stat, hipStream_t st) {
    const size_t lds = sizeof(double2) * (size_t)(4 * m * m + m);
    set_lds_limit((const void *)k_kry_expm, lds);
    TTN_LAUNCH("k_kry_expm", 0.0, 0.0, k_kry_expm, dim3(1), dim3(1024), lds, st, k, m, mmax, tau, tol, hermitian,
               stat);
    TTN_LAUNCH("k_kry_combine", 8.0 * N * m, 16.0 * N * (m + 1), k_kry_combine, dim3(grid_for(N, VEC_THREADS)),
               dim3(VEC_THREADS), 0, st, k, (uint32_t)N, m,
                       x);
}

}  // namespace ttn
