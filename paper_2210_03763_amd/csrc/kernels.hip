// Device kernels of the TTN/TDVP library for gfx950 (CDNA4, wave64), apart
// from the contractions: Lanczos reductions with device-resident scalars, the
// tridiagonal exponential of the Krylov projection (scaled Taylor series),
// Cholesky + triangular inverse for CholeskyQR2 gauge moves, precision
// conversions and small helpers.
#include <hip/hip_runtime.h>

#include <initializer_list>

#include <cmath>
#include <cstdint>
#include <cstdio>

#include "ttn_internal.h"

namespace ttn {

// ---------------------------------------------------------------------------
// reductions for Lanczos
// ---------------------------------------------------------------------------
namespace {

constexpr int RED_THREADS = 256;

__device__ inline double block_sum(double v, double* sh) {
    // wave64 shuffle reduction, then across the four waves of the block
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) r += sh[i];
    return r;   // valid in thread 0
}

// block_sum with the total returned in every thread (sh: blockDim / 64 + 1
// doubles).
__device__ inline double block_sum_all(double v, double* sh) {
    const double r = block_sum(v, sh);
    if (threadIdx.x == 0) sh[blockDim.x / 64] = r;
    __syncthreads();
    const double t = sh[blockDim.x / 64];
    __syncthreads();
    return t;
}

// Sums P values (P a power of two, 2 <= P <= 32) over the block with one
// barrier: a butterfly inside each wave leaves value (l >> 1) & (P - 1),
// summed over the wave, in lane l; the waves' results meet in sh (P per wave,
// at most four waves).  Returns the block total of value threadIdx.x in
// threads 0 .. P-1.
template <int H, int P>
__device__ inline void butterfly_step(double (&a)[P], int lane) {
    // lanes that differ in bit 2H exchange one half of their first 2H values
    const bool hi = (lane & (2 * H)) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = hi ? a[i] : a[i + H];
        const double keep = hi ? a[i + H] : a[i];
        a[i] = keep + __shfl_xor(send, 2 * H, 64);
    }
}

template <int P>
__device__ inline double block_sum_p(double (&a)[P], double* sh) {
    static_assert(P >= 2 && P <= 32 && (P & (P - 1)) == 0, "P must be a power of two in [2, 32]");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if constexpr (P >= 32) butterfly_step<16>(a, lane);
    if constexpr (P >= 16) butterfly_step<8>(a, lane);
    if constexpr (P >= 8) butterfly_step<4>(a, lane);
    if constexpr (P >= 4) butterfly_step<2>(a, lane);
    butterfly_step<1>(a, lane);
    a[0] += __shfl_xor(a[0], 1, 64);
#pragma unroll
    for (int b = 2 * P; b < 64; b <<= 1) a[0] += __shfl_xor(a[0], b, 64);
    const int idx = (lane >> 1) & (P - 1);
    __syncthreads();
    if ((lane & 1) == 0 && lane < 2 * P) sh[P * wv + idx] = a[0];
    __syncthreads();
    double r = 0;
    if (threadIdx.x < P)
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) r += sh[P * w2 + threadIdx.x];
    return r;
}

__device__ inline double block_sum32(double (&a)[32], double* sh) { return block_sum_p<32>(a, sh); }

// smallest power of two >= 2 kc
constexpr int pow2_pairs(int kc) {
    int p = 2;
    while (p < 2 * kc) p *= 2;
    return p;
}

__global__ void k_norm2_partial(const double* x, int64_t n, double* partial, const int* skip) {
    if (skip && *skip) return;
    __shared__ double sh[16];
    double acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = x[i], b = x[i + n];
        acc += a * a + b * b;
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Sum of p[start], p[start + step], ... below count, with eight loads in
// flight per thread (independent accumulators) instead of one.
__device__ inline double strided_sum(const double* p, int count, int start, int step) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = start;
    for (; i + 7 * step < count; i += 8 * step) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += p[i + u * step];
    }
    for (; i < count; i += step) acc[0] += p[i];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__device__ inline double wave_sum_partials(const double* partial, int nb) {
    double s = strided_sum(partial, nb, threadIdx.x, 64);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    return s;   // valid in lane 0
}

__global__ void k_lz_begin(const double* partial, int nb, LanczosDev* lz, int nonherm) {
    const double s = wave_sum_partials(partial, nb);
    if (threadIdx.x == 0) {
        lz->beta0 = sqrt(s);
        lz->zero = (s == 0.0) ? 1 : 0;
        lz->done = lz->zero;
        lz->m_eff = 0;
        lz->nonherm = nonherm;
    }
}

// y = x / beta (FP64), and its FP32 copy yf when yf != nullptr (the input of
// the next mixed-precision matvec); y planar (S == 0) or a slot of a chunked
// Krylov basis with chunk stride S
__global__ void k_scale_by(const double* x, int64_t n, double* y, int64_t S, const LanczosDev* lz, int use_beta0,
                           int j, float* yf) {
    if (lz->done) return;
    const double s = 1.0 / (use_beta0 ? lz->beta0 : lz->beta[j]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i] * s;
        y[S ? kch_elem(i, n, S) : i] = v;
        if (yf) yf[i] = (float)v;
    }
}

// v_{j+1} = w / beta_j (y planar, S == 0, or a chunked basis slot) with
// beta_j totalled by every block from the nb
// norm partials of k_sub_fused<2> and the breakdown test of k_lz_beta taken
// alike in every block (block 0 records beta_j, or the breakdown); also the
// FP32 copy yf when yf != nullptr.
__global__ __launch_bounds__(256) void k_scale_next(const double* x, int64_t n, double* y, int64_t S,
                                                  LanczosDev* lz, const double* pnorm, int nb, int j, double tol,
                                                  float* yf) {
    if (lz->done) return;
    __shared__ double sh[16];
    __shared__ double s_b;
    const double t = block_sum(strided_sum(pnorm, nb, threadIdx.x, blockDim.x), sh);
    if (threadIdx.x == 0) s_b = sqrt(t);
    __syncthreads();
    const double b = s_b;
    const double bprev = j > 0 ? lz->beta[j - 1] : 0.0;
    const bool stop = !(b > tol * (fabs(lz->alpha[j]) + bprev));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (stop)
            lz->done = 1;
        else
            lz->beta[j] = b;
    }
    if (stop) return;
    const double inv = 1.0 / b;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i] * inv;
        y[S ? kch_elem(i, n, S) : i] = v;
        if (yf) yf[i] = (float)v;
    }
}

// partial[blk][k] = sum_i conj(V_k[i]) w[i] for k < KC (2 KC reals per
// block); with wf != nullptr w is first widened from the FP32 matvec output
// wf (and stored).  KC is a template argument so that the per-thread arrays
// hold exactly the vectors in use.
template <int KC, int W>
__device__ inline void multidot_body(const double* V, int64_t S, const double* w, int64_t n, const float* wf,
                                     double (&re)[KC], double (&im)[KC]) {
    // W consecutive elements per thread and step (16-byte loads for W = 2)
    typedef double dv __attribute__((ext_vector_type(W)));
    typedef float fv __attribute__((ext_vector_type(W)));
    const int64_t nw = n / W;
    // slot and plane strides: chunked basis (S > 0) or planar vectors (S == 0)
    const int64_t ks = S ? 2 * KCH : 2 * n, ps = S ? KCH : n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nw; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q * W;
        const double* Vi = V + (S ? kch_ofs(i, S) : i);
        dv vr[KC], vi[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            vr[k] = *(const dv*)(Vi + ks * k);
            vi[k] = *(const dv*)(Vi + ks * k + ps);
        }
        dv wr, wi;
        if (wf) {
            const fv a = *(const fv*)(wf + i), b = *(const fv*)(wf + i + n);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                wr[e] = (double)a[e];
                wi[e] = (double)b[e];
            }
            *(dv*)(const_cast<double*>(w) + i) = wr;
            *(dv*)(const_cast<double*>(w) + i + n) = wi;
        } else {
            wr = *(const dv*)(w + i);
            wi = *(const dv*)(w + i + n);
        }
#pragma unroll
        for (int e = 0; e < W; ++e)
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                re[k] += vr[k][e] * wr[e] + vi[k][e] * wi[e];
                im[k] += vr[k][e] * wi[e] - vi[k][e] * wr[e];
            }
    }
}

// partial[blk][k] = sum_i conj(V_k[i]) w[i] for k < KC (2 KC reals per
// block); with wf != nullptr w is first widened from the FP32 matvec output
// wf (and stored).  KC is a template argument so that the per-thread arrays
// hold exactly the vectors in use; vectors of even length are read two
// elements at a time.
template <int KC>
__global__ __launch_bounds__(256) void k_multidot_partial(const double* V, int64_t S, const double* w, int64_t n,
                                                         double* partial, const LanczosDev* lz, const float* wf) {
    if (lz->done) return;
    constexpr int P = pow2_pairs(KC);
    __shared__ double shp[4 * P];
    double re[KC], im[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) re[k] = im[k] = 0;
    if (n % 2 == 0 && (((uintptr_t)V | (uintptr_t)w | (uintptr_t)wf) & 15) == 0)
        multidot_body<KC, 2>(V, S, w, n, wf, re, im);
    else
        multidot_body<KC, 1>(V, S, w, n, wf, re, im);
    double a[P];
#pragma unroll
    for (int k = 0; k < P / 2; ++k) {
        a[2 * k] = k < KC ? re[k] : 0.0;
        a[2 * k + 1] = k < KC ? im[k] : 0.0;
    }
    const double t = block_sum_p<P>(a, shp);
    if (threadIdx.x < 2 * KC) partial[blockIdx.x * 2 * KC + threadIdx.x] = t;
}

// Records the projections tot[2k], tot[2k + 1] (k < kcount) of one
// Gram-Schmidt pass in the Lanczos state; called by thread k of one block.
// alpha_index >= 0 marks the first pass of iteration alpha_index (alpha_j,
// and for an Arnoldi basis the Hessenberg column), -1 the second pass (its
// projections are added to the Hessenberg column).
__device__ inline void lz_record_projection(LanczosDev* lz, const double* tot, int kcount, int alpha_index,
                                            int k) {
    const double re = tot[2 * k], im = tot[2 * k + 1];
    lz->c[2 * k] = re;
    lz->c[2 * k + 1] = im;
    if (k == alpha_index) {
        lz->alpha[k] = re;
        lz->m_eff = k + 1;
    }
    if (lz->nonherm) {
        double* hp = lz->hs + 2 * ((kcount - 1) * KRYLOV_MAX + k);
        if (alpha_index >= 0) {
            hp[0] = re;
            hp[1] = im;
        } else {
            hp[0] += re;
            hp[1] += im;
        }
    }
}

// Totals of the nv <= 32 reals per block of nb block partials (layout
// [block][nv]) into out[0..nv), in an order that does not depend on the
// calling block; 256 threads, sh holds 256 doubles.
__device__ inline void block_partials_total(const double* p, int nb, int nv, double* sh, double* out) {
    const int v = threadIdx.x & 31, g = threadIdx.x >> 5, ng = blockDim.x >> 5;
    double u[4] = {0, 0, 0, 0};
    if (v < nv) {
        int b = g;
        for (; b + 3 * ng < nb; b += 4 * ng) {
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] += p[(int64_t)(b + q * ng) * nv + v];
        }
        for (; b < nb; b += ng) u[0] += p[(int64_t)b * nv + v];
    }
    sh[32 * g + v] = (u[0] + u[1]) + (u[2] + u[3]);
    __syncthreads();
    if (threadIdx.x < nv) {
        double r = 0;
        for (int q = 0; q < ng; ++q) r += sh[32 * q + threadIdx.x];
        out[threadIdx.x] = r;
    }
    __syncthreads();
}

// Totals of the 2 kcount reals per block (layout of k_multidot_partial) into
// the Lanczos state.  1024 threads: thread (g, v) = (t / 32, t % 32) sums value
// v of blocks g, g + 32, ..., so that each step of the 32 groups reads one
// contiguous stretch of the partials.
__global__ __launch_bounds__(1024) void k_multidot_final(const double* partial, int nb, int kcount,
                                                         LanczosDev* lz, int alpha_index) {
    if (lz->done) return;
    __shared__ double sh[32][33];
    __shared__ double tot[32];
    const int v = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int nv = 2 * kcount;
    double acc = 0;
    if (v < nv) {
        double u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int b = g;
        for (; b + 7 * 32 < nb; b += 8 * 32) {
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] += partial[(int64_t)(b + 32 * q) * nv + v];
        }
        for (; b < nb; b += 32) u[0] += partial[(int64_t)b * nv + v];
        acc = ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
    }
    sh[g][v] = acc;
    __syncthreads();
    if (threadIdx.x < 32) {
        double r = 0;
        for (int q = 0; q < 32; ++q) r += sh[q][threadIdx.x];
        tot[threadIdx.x] = r;
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k >= kcount) return;
    lz_record_projection(lz, tot, kcount, alpha_index, k);
}

// w -= sum_k c_k V_k; then, per block, partial sums of either the new
// projections conj(V_k) w (mode 1, 2 KC reals per block) or |w|^2 (mode 2,
// one real per block).  The coefficients c come from
// the Lanczos state, or, with pin != nullptr, every block totals them from
// the previous pass's nbin block partials itself (the same sums in every
// block) and block 0 records them in the state (alpha_index as in
// lz_record_projection); pin must not alias partial.
template <int MODE, int KC, int W>
__device__ inline void sub_fused_body(const double* V, int64_t S, double* w, int64_t n, const double* c,
                                      double (&pr)[KC], double (&pi)[KC], double& nrm) {
    // W consecutive elements per thread and step (16-byte loads for W = 2)
    typedef double dv __attribute__((ext_vector_type(W)));
    const int64_t nw = n / W;
    // slot and plane strides: chunked basis (S > 0) or planar vectors (S == 0)
    const int64_t ks = S ? 2 * KCH : 2 * n, ps = S ? KCH : n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nw; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q * W;
        const double* Vi = V + (S ? kch_ofs(i, S) : i);
        dv vr[KC], vi[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            vr[k] = *(const dv*)(Vi + ks * k);
            vi[k] = *(const dv*)(Vi + ks * k + ps);
        }
        dv wr = *(const dv*)(w + i), wi = *(const dv*)(w + i + n);
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const double cr = c[2 * k], ci = c[2 * k + 1];
#pragma unroll
            for (int e = 0; e < W; ++e) {
                wr[e] -= cr * vr[k][e] - ci * vi[k][e];
                wi[e] -= cr * vi[k][e] + ci * vr[k][e];
            }
        }
        *(dv*)(w + i) = wr;
        *(dv*)(w + i + n) = wi;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            if (MODE == 1) {
#pragma unroll
                for (int k = 0; k < KC; ++k) {
                    pr[k] += vr[k][e] * wr[e] + vi[k][e] * wi[e];
                    pi[k] += vr[k][e] * wi[e] - vi[k][e] * wr[e];
                }
            } else if (MODE == 2) {
                nrm += wr[e] * wr[e] + wi[e] * wi[e];
            }
        }
    }
}

template <int MODE, int KC>
__global__ __launch_bounds__(256) void k_sub_fused(const double* V, int64_t S, double* w, int64_t n, double* partial,
                                                   LanczosDev* lz, const double* pin, int nbin, int alpha_index) {
    if (lz->done) return;
    constexpr int P = pow2_pairs(KC);
    __shared__ double c[32];
    __shared__ double sh[16];
    __shared__ double shp[4 * P];
    __shared__ double shq[256];
    if (pin) {
        block_partials_total(pin, nbin, 2 * KC, shq, c);
        if (blockIdx.x == 0 && threadIdx.x < KC) lz_record_projection(lz, c, KC, alpha_index, threadIdx.x);
    } else {
        if (threadIdx.x < 2 * KC) c[threadIdx.x] = lz->c[threadIdx.x];
        __syncthreads();
    }
    double pr[KC], pi[KC], nrm = 0;
#pragma unroll
    for (int k = 0; k < KC; ++k) pr[k] = pi[k] = 0;
    if (n % 2 == 0 && (((uintptr_t)V | (uintptr_t)w) & 15) == 0)
        sub_fused_body<MODE, KC, 2>(V, S, w, n, c, pr, pi, nrm);
    else
        sub_fused_body<MODE, KC, 1>(V, S, w, n, c, pr, pi, nrm);
    if (MODE == 1) {
        double a[P];
#pragma unroll
        for (int k = 0; k < P / 2; ++k) {
            a[2 * k] = k < KC ? pr[k] : 0.0;
            a[2 * k + 1] = k < KC ? pi[k] : 0.0;
        }
        const double t = block_sum_p<P>(a, shp);
        if (threadIdx.x < 2 * KC) partial[blockIdx.x * 2 * KC + threadIdx.x] = t;
    } else if (MODE == 2) {
        const double a = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = a;
    }
}

// One whole Lanczos iteration after the matvec for short vectors (one block):
// c = V^H w (alpha_j = Re c_j); unless j is the last index: w -= V c,
// c' = V^H w, w -= V c', beta_j = |w| with the breakdown test, v_{j+1} = w / beta_j.
__global__ __launch_bounds__(256) void k_lz_iter_small(double* V, int j, int m, double* w, int64_t n, LanczosDev* lz,
                                                       double tol) {
    if (lz->done) return;
    __shared__ double sh32[4 * 32];
    __shared__ double c[32];
    __shared__ double s_beta;
    __shared__ int s_stop;
    const int kc = j + 1;
    double a[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) a[k] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double wr = w[i], wi = w[i + n];
#pragma unroll
        for (int k = 0; k < KRYLOV_MAX; ++k)
            if (k < kc) {
                const double vr = V[2 * n * k + i], vi = V[2 * n * k + n + i];
                a[2 * k] += vr * wr + vi * wi;
                a[2 * k + 1] += vr * wi - vi * wr;
            }
    }
    double t = block_sum32(a, sh32);
    if (threadIdx.x < 32) c[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        lz->alpha[j] = c[2 * j];
        lz->m_eff = j + 1;
    }
    const int nonherm = lz->nonherm;
    if (nonherm && threadIdx.x < 2 * kc) lz->hs[2 * j * KRYLOV_MAX + threadIdx.x] = c[threadIdx.x];
    if (j == m - 1) return;
    // subtract, second projection
#pragma unroll
    for (int k = 0; k < 32; ++k) a[k] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double wr = w[i], wi = w[i + n];
        double vr[KRYLOV_MAX], vi[KRYLOV_MAX];
#pragma unroll
        for (int k = 0; k < KRYLOV_MAX; ++k)
            if (k < kc) {
                vr[k] = V[2 * n * k + i];
                vi[k] = V[2 * n * k + n + i];
                wr -= c[2 * k] * vr[k] - c[2 * k + 1] * vi[k];
                wi -= c[2 * k] * vi[k] + c[2 * k + 1] * vr[k];
            }
        w[i] = wr;
        w[i + n] = wi;
#pragma unroll
        for (int k = 0; k < KRYLOV_MAX; ++k)
            if (k < kc) {
                a[2 * k] += vr[k] * wr + vi[k] * wi;
                a[2 * k + 1] += vr[k] * wi - vi[k] * wr;
            }
    }
    t = block_sum32(a, sh32);
    __syncthreads();
    if (threadIdx.x < 32) c[threadIdx.x] = t;
    if (nonherm && threadIdx.x < 2 * kc) lz->hs[2 * j * KRYLOV_MAX + threadIdx.x] += t;
    __syncthreads();
    // subtract again, norm
    double nrm[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) nrm[k] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double wr = w[i], wi = w[i + n];
#pragma unroll
        for (int k = 0; k < KRYLOV_MAX; ++k)
            if (k < kc) {
                const double vr = V[2 * n * k + i], vi = V[2 * n * k + n + i];
                wr -= c[2 * k] * vr - c[2 * k + 1] * vi;
                wi -= c[2 * k] * vi + c[2 * k + 1] * vr;
            }
        w[i] = wr;
        w[i + n] = wi;
        nrm[0] += wr * wr + wi * wi;
    }
    t = block_sum32(nrm, sh32);
    if (threadIdx.x == 0) {
        const double b = sqrt(t);
        const double bprev = j > 0 ? lz->beta[j - 1] : 0.0;
        const bool stop = !(b > tol * (fabs(lz->alpha[j]) + bprev));
        if (stop)
            lz->done = 1;
        else
            lz->beta[j] = b;
        s_stop = stop;
        s_beta = b;
    }
    __syncthreads();
    if (s_stop) return;
    const double inv = 1.0 / s_beta;
    double* vn = V + 2 * n * (j + 1);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        vn[i] = w[i] * inv;
        vn[i + n] = w[i + n] * inv;
    }
}

__global__ __launch_bounds__(256) void k_lz_beta(const double* partial, int nb, LanczosDev* lz, int j,
                                                 double tol) {
    if (lz->done) return;
    __shared__ double sh[16];
    const double s = block_sum(strided_sum(partial, nb, threadIdx.x, blockDim.x), sh);
    if (threadIdx.x == 0) {
        const double b = sqrt(s);
        const double bprev = j > 0 ? lz->beta[j - 1] : 0.0;
        if (!(b > tol * (fabs(lz->alpha[j]) + bprev)))
            lz->done = 1;
        else
            lz->beta[j] = b;
    }
}

// y = exp(-i tau H) e_1 for the m_eff x m_eff projection H of the Krylov
// basis: the Taylor series of exp(B/s), B = -i tau H, applied s times to the
// vector, with s chosen so that ||B/s||_1 <= 1/4 and as many terms as make
// the remainder bound of the series fall below double precision.  H is the
// real symmetric tridiagonal (alpha, beta) of a Lanczos basis, or the complex
// upper Hessenberg matrix of an Arnoldi basis (columns in hs, subdiagonal
// beta) when lz->nonherm.  The first wave does all of it, lane t holding row
// t of H and element t of the vectors (products with H by lane shuffles, the
// norm by one wave reduction); the other waves of the block only meet it at
// the closing barrier.

// entry (row, col) of the projection (re, im), zero outside m x m
__device__ inline double2 lz_h_entry(const LanczosDev* lz, bool herm, int m, int row, int col) {
    double a = 0.0, b = 0.0;
    if (row < 0 || col < 0 || row >= m || col >= m) return make_double2(a, b);
    if (herm) {
        if (row == col)
            a = lz->alpha[col];
        else if (row == col + 1)
            a = lz->beta[col];
        else if (col == row + 1)
            a = lz->beta[row];
    } else if (row <= col) {
        a = lz->hs[2 * (col * KRYLOV_MAX + row)];
        b = lz->hs[2 * (col * KRYLOV_MAX + row) + 1];
    } else if (row == col + 1) {
        a = lz->beta[col];
    }
    return make_double2(a, b);
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ void lz_expm_hessenberg(LanczosDev* lz, double tau, StepDev* st) {
    constexpr int KM = KRYLOV_MAX;
    const int t = threadIdx.x;
    if (t < 64) {
        const int m = lz->m_eff;
        const bool herm = !lz->nonherm;
        // row t of H (Hessenberg case; the tridiagonal case reads its three
        // entries below)
        double hr[KM], hi[KM];
#pragma unroll
        for (int c = 0; c < KM; ++c) {
            const double2 e = herm ? make_double2(0.0, 0.0) : lz_h_entry(lz, false, m, t, c);
            hr[c] = e.x;
            hi[c] = e.y;
        }
        // H[t][t-1], H[t][t], H[t][t+1] (tridiagonal)
        const double dl = herm ? lz_h_entry(lz, true, m, t, t - 1).x : 0.0;
        const double dd = herm ? lz_h_entry(lz, true, m, t, t).x : 0.0;
        const double du = herm ? lz_h_entry(lz, true, m, t, t + 1).x : 0.0;
        // 1-norm bound of tau H: the largest column sum (lane t sums column t
        // in row order)
        double cs = 0;
        for (int row = 0; row < m; ++row) {
            const double2 e = lz_h_entry(lz, herm, m, row, t);
            cs += fabs(e.x) + fabs(e.y);
        }
        double nrm = wave_max(t < m ? cs : 0.0) * fabs(tau);
        int ns = (int)ceil(nrm / 0.25);
        if (ns < 1) ns = 1;
        const double h = tau / ns;
        // number of Taylor terms K: with theta = ||h H||_1 <= 1/4 the
        // remainder after K terms is at most theta^(K+1) / (K+1)! e^theta
        // (e^theta < 1.3) of the vector, kept below 1e-18 (the same K in
        // every lane, no reductions inside the series)
        const double theta = nrm / ns;
        int K = 0;
        for (double a = 1.0; K < 40; ++K) {
            a *= theta / (K + 1);   // theta^(K+1) / (K+1)!
            if (1.3 * a <= 1e-18) break;
        }
        double vr = t == 0 ? 1.0 : 0.0, vi = 0.0;
        for (int rep = 0; rep < ns; ++rep) {
            double tr = vr, ti = vi, wr = vr, wi = vi;
            for (int k = 1; k <= K; ++k) {
                // term <- (-i h H term) / k
                double sr = 0, si = 0;
                if (herm) {
                    const double trl = __shfl(tr, t > 0 ? t - 1 : 0, 64), til = __shfl(ti, t > 0 ? t - 1 : 0, 64);
                    const double tru = __shfl(tr, t < 63 ? t + 1 : 63, 64), tiu = __shfl(ti, t < 63 ? t + 1 : 63, 64);
                    sr = dl * trl + dd * tr + du * tru;
                    si = dl * til + dd * ti + du * tiu;
                } else {
#pragma unroll
                    for (int c = 0; c < KM; ++c) {
                        const double trc = __shfl(tr, c, 64), tic = __shfl(ti, c, 64);
                        sr += hr[c] * trc - hi[c] * tic;
                        si += hr[c] * tic + hi[c] * trc;
                    }
                }
                const double f = h / k;
                if (t < m) {
                    tr = f * si;
                    ti = -f * sr;
                    wr += tr;
                    wi += ti;
                }
            }
            vr = wr;
            vi = wi;
        }
        if (t < KM) {
            lz->y[2 * t] = t < m ? vr : 0.0;
            lz->y[2 * t + 1] = t < m ? vi : 0.0;
        }
        if (t == 0) atomicMin(&st->min_krylov, m);
    }
    __syncthreads();
}

__global__ void k_lz_expm(LanczosDev* lz, double tau, StepDev* st) {
    if (lz->zero) return;
    lz_expm_hessenberg(lz, tau, st);
}

// ---------------------------------------------------------------------------
// Fused evolution of a small operator: x <- exp(-i tau Op) x for an
// effective Hamiltonian with n = DL DR DP <= SMALL_EVOLVE_N entries in one
// workgroup, every vector and operator stack in LDS, FP64 throughout: the
// matvec (the same four stages as the GEMM path), the Krylov recursion with
// two Gram-Schmidt passes, the small exponential and the recombination.
// Replaces about a hundred launches per evolution of the bottom nodes and
// their bonds.
// ---------------------------------------------------------------------------
constexpr int SMALL_THREADS = 1024;

// Two ownerships of the elements i < n <= SMALL_EVOLVE_N.  In the matvec
// four lanes share each element and split its terms (images and operator
// stacks dealt round-robin), summed by two lane exchanges: lane e + 16 q of
// wave w (e < 16, q < 4) takes part q of the elements i = e + 16 w +
// SMALL_GROUPS t, t < SMALL_PER.  Each 16-lane row of a wave then reads 16
// consecutive entries of one vector and one operator entry (no LDS bank
// conflicts; the four parts of an element on adjacent lanes had put three
// vectors 4 KB apart on the same banks).  The (l, r, p) split of every
// element is tabulated in LDS once per launch (10 bits each).  The
// projections give wave k Krylov vector k; the subtractions, norms and
// scaling give thread i element i.
constexpr int SMALL_SPLIT = 4;
constexpr int SMALL_GROUPS = SMALL_THREADS / SMALL_SPLIT;
constexpr int SMALL_PER = (int)(SMALL_EVOLVE_N / SMALL_GROUPS);
static_assert(SMALL_PER * SMALL_GROUPS == SMALL_EVOLVE_N, "elements must split evenly over the quads");
static_assert(SMALL_EVOLVE_N == SMALL_THREADS, "one element per thread in the vector passes");
static_assert(SMALL_SPLIT * 16 == 64 && SMALL_GROUPS == 16 * (SMALL_THREADS / 64), "four 16-lane parts per wave");
static_assert(SMALL_EVOLVE_N <= 1024, "leg dimensions must fit the 10-bit fields of the index table");

// acc += sum_q op[o + D q] src[base + sq q], q < D (complex, planar op of D^2
// entries and src of n entries)
__device__ inline void small_term(const double* op, int D, int o, const double* src, int n, int base, int sq,
                                  double& ar, double& ai) {
    const int D2 = D * D;
#pragma unroll 4
    for (int q = 0; q < D; ++q) {
        const double orr = op[o + D * q], oi = op[D2 + o + D * q];
        const double xr = src[base + sq * q], xi = src[n + base + sq * q];
        ar += orr * xr - oi * xi;
        ai += orr * xi + oi * xr;
    }
}

// y = Op x; S holds the left (U_k = L_k x_L x, k = 1..sL) and right (Z_j =
// R_j x_R x) images, slot stride 2n.  Ends with a barrier (y is complete).
__device__ void small_matvec(const double* L, const double* Rr, const double* B, const double* W, int DL, int DR,
                             int DP, int sL, int sR, const int* sidx, const double* x, double* S, double* y) {
    const int n = DL * DR * DP;
    const int nz = (W && sR > 0) ? sR : 0;
    const int q = (threadIdx.x >> 4) & (SMALL_SPLIT - 1), g = (threadIdx.x & 15) + 16 * (threadIdx.x >> 6);
    // images: lane q of a quad forms images k = q, q + 4, ... of its elements
    for (int k = q; k < sL + nz; k += SMALL_SPLIT) {
        const bool left = k < sL;
#pragma unroll 1
        for (int t = 0; t < SMALL_PER; ++t) {
            const int i = g + SMALL_GROUPS * t;
            if (i < n) {
                const int lx = sidx[i] & 1023, rx = (sidx[i] >> 10) & 1023;
                double ar = 0, ai = 0;
                if (left)
                    small_term(L + 2 * DL * DL * (k + 1), DL, lx, x, n, i - lx, 1, ar, ai);
                else
                    small_term(Rr + 2 * DR * DR * (k - sL + 1), DR, rx, x, n, i - DL * rx, DL, ar, ai);
                S[2 * n * k + i] = ar;
                S[2 * n * k + n + i] = ai;
            }
        }
    }
    __syncthreads();
    // sums: unit 0 is the left block Hamiltonian, units 1..sL+1 the right-leg
    // stack (H_R x, A_i U_i), the next sL+nz+1 the parent-leg stack (H_P x,
    // W U, W Z); lane q takes the units u = q mod 4
    const int uW = 1 + (B ? sL + 1 : 0);
#pragma unroll 1
    for (int t = 0; t < SMALL_PER; ++t) {
        const int i = g + SMALL_GROUPS * t;
        double ar = 0, ai = 0;
        if (i < n) {
            const int e = sidx[i];
            const int l = e & 1023, r = (e >> 10) & 1023, p = e >> 20;
            if (q == 0) small_term(L, DL, l, x, n, i - l, 1, ar, ai);
            if (B)
                for (int k = (q - 1) & (SMALL_SPLIT - 1); k <= sL; k += SMALL_SPLIT)
                    small_term(B + 2 * DR * DR * k, DR, r, k == 0 ? x : S + 2 * n * (k - 1), n, i - DL * r, DL,
                               ar, ai);
            if (W)
                for (int k = (q - uW) & (SMALL_SPLIT - 1); k <= sL + nz; k += SMALL_SPLIT)
                    small_term(W + 2 * DP * DP * k, DP, p, k == 0 ? x : S + 2 * n * (k - 1), n,
                               i - DL * DR * p, DL * DR, ar, ai);
        }
        // the four lanes of element i (16 apart) all take part
        ar += __shfl_xor(ar, 16, 64);
        ai += __shfl_xor(ai, 16, 64);
        ar += __shfl_xor(ar, 32, 64);
        ai += __shfl_xor(ai, 32, 64);
        if (q == 0 && i < n) {
            y[i] = ar;
            y[n + i] = ai;
        }
    }
    __syncthreads();
}

// c_k = <v_k, w> for k < kc (planar vectors of n in LDS, w complete on
// entry): wave k forms product k over all n elements and reduces it across
// its lanes; the totals land in c[2 kc] (LDS) behind one barrier.
static_assert(KRYLOV_MAX <= SMALL_THREADS / 64, "one wave per Krylov vector in the projections");
__device__ void small_project(const double* V, int kc, const double* w, int n, double* c) {
    const int lane = threadIdx.x & 63, k = threadIdx.x >> 6;
    if (k < kc) {
        const double* v = V + 2 * n * k;
        double re = 0, im = 0;
        for (int i = lane; i < n; i += 64) {
            const double vr = v[i], vi = v[n + i], wr = w[i], wi = w[n + i];
            re += vr * wr + vi * wi;
            im += vr * wi - vi * wr;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            re += __shfl_xor(re, o, 64);
            im += __shfl_xor(im, o, 64);
        }
        if (lane == 0) {
            c[2 * k] = re;
            c[2 * k + 1] = im;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(SMALL_THREADS) void k_small_evolve(const double* gL, const double* gR, const double* gB,
                                                             const double* gW, int DL, int DR, int DP, int sL,
                                                             int sR, int m, double tau, double tol, int nonherm,
                                                             double* x, StepDev* st) {
    __shared__ double pool[SMALL_EVOLVE_POOL];
    __shared__ LanczosDev lz;
    __shared__ double sh2[2 * (SMALL_THREADS / 64)];
    __shared__ int sidx[SMALL_EVOLVE_N];
    __shared__ double c[32];
    __shared__ double s_beta;
    __shared__ int s_stop;
    const int n = DL * DR * DP;
    const int L2 = DL * DL, R2 = DR * DR, P2 = DP * DP;
    const int nz = (gW && sR > 0) ? sR : 0;
    // carve: V[(m+1)], w, S[sL + nz], L, R, B, W
    double* V = pool;
    double* w = V + 2 * n * (m + 1);
    double* S = w + 2 * n;
    double* L = S + 2 * n * (sL + nz);
    double* Rr = L + 2 * L2 * (1 + sL);
    double* B = Rr + (nz ? 2 * R2 * (1 + sR) : 0);
    double* W = B + (gB ? 2 * R2 * (1 + sL) : 0);
    for (int e = threadIdx.x; e < 2 * L2 * (1 + sL); e += blockDim.x) L[e] = gL[e];
    if (nz)
        for (int e = threadIdx.x; e < 2 * R2 * (1 + sR); e += blockDim.x) Rr[e] = gR[e];
    if (gB)
        for (int e = threadIdx.x; e < 2 * R2 * (1 + sL); e += blockDim.x) B[e] = gB[e];
    if (gW)
        for (int e = threadIdx.x; e < 2 * P2 * (1 + sL + sR); e += blockDim.x) W[e] = gW[e];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sidx[i] = (i % DL) | ((i / DL) % DR) << 10 | (i / (DL * DR)) << 20;
    const int me_i = threadIdx.x;   // this thread's element in the vector passes
    // v_0 = x / ||x||
    double a[2] = {0.0, 0.0};
    if (me_i < n) {
        const double xr = x[me_i], xi = x[n + me_i];
        w[me_i] = xr;
        w[n + me_i] = xi;
        a[0] += xr * xr + xi * xi;
    }
    double tot = block_sum_p<2>(a, sh2);
    if (threadIdx.x == 0) {
        lz.beta0 = sqrt(tot);
        lz.zero = tot == 0.0 ? 1 : 0;
        lz.done = lz.zero;
        lz.m_eff = 0;
        lz.nonherm = nonherm;
    }
    __syncthreads();
    if (lz.zero) return;   // x = 0 stays 0
    {
        const double inv = 1.0 / lz.beta0;
        for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) V[i] = w[i] * inv;
    }
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        const int kc = j + 1;
        small_matvec(L, nz ? Rr : nullptr, gB ? B : nullptr, gW ? W : nullptr, DL, DR, DP, sL, sR, sidx,
                     V + 2 * n * j, S, w);
        small_project(V, kc, w, n, c);
        if (threadIdx.x == 0) {
            lz.alpha[j] = c[2 * j];
            lz.m_eff = j + 1;
        }
        if (nonherm && threadIdx.x < 2 * kc) lz.hs[2 * j * KRYLOV_MAX + threadIdx.x] = c[threadIdx.x];
        if (j == m - 1) break;
        // w -= V c, second projection, w -= V c' (each thread on its own
        // element; the second projection reads all of w, behind a barrier)
        a[0] = 0.0;
        a[1] = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            if (me_i < n) {
                const int i = me_i;
                double wr = w[i], wi = w[n + i];
#pragma unroll 2
                for (int k = 0; k < kc; ++k) {
                    const double vr = V[2 * n * k + i], vi = V[2 * n * k + n + i];
                    wr -= c[2 * k] * vr - c[2 * k + 1] * vi;
                    wi -= c[2 * k] * vi + c[2 * k + 1] * vr;
                }
                w[i] = wr;
                w[n + i] = wi;
                if (pass == 1) a[0] += wr * wr + wi * wi;
            }
            if (pass == 0) {
                __syncthreads();
                small_project(V, kc, w, n, c);
                if (nonherm && threadIdx.x < 2 * kc) lz.hs[2 * j * KRYLOV_MAX + threadIdx.x] += c[threadIdx.x];
            }
        }
        tot = block_sum_p<2>(a, sh2);
        if (threadIdx.x == 0) {
            const double b = sqrt(tot);
            const double bprev = j > 0 ? lz.beta[j - 1] : 0.0;
            const bool stop = !(b > tol * (fabs(lz.alpha[j]) + bprev));
            if (stop)
                lz.done = 1;
            else
                lz.beta[j] = b;
            s_stop = stop;
            s_beta = b;
        }
        __syncthreads();
        if (s_stop) break;
        const double inv = 1.0 / s_beta;
        for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) V[2 * n * (j + 1) + i] = w[i] * inv;
        __syncthreads();
    }
    // y = exp(-i tau H_m) e_1, then x = beta0 sum_k y_k v_k
    lz_expm_hessenberg(&lz, tau, st);
    __syncthreads();
    const int me = lz.m_eff;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double re = 0, im = 0;
        for (int k = 0; k < me; ++k) {
            const double yr = lz.y[2 * k] * lz.beta0, yi = lz.y[2 * k + 1] * lz.beta0;
            const double vr = V[2 * n * k + i], vi = V[2 * n * k + n + i];
            re += yr * vr - yi * vi;
            im += yr * vi + yi * vr;
        }
        x[i] = re;
        x[n + i] = im;
    }
}

// out[k][plane][n] = slot k of the chunked basis V, k < slots (planar copy)
__global__ void k_unchunk(const double* V, int64_t S, int64_t n, int slots, double* out, const int* skip) {
    if (skip && *skip) return;
    const int64_t total = 2 * n * slots;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / (2 * n), r = e - k * 2 * n;
        out[e] = V[2 * KCH * k + kch_elem(r, n, S)];
    }
}

// out = beta0 sum_k y_k v_k; V planar (S == 0, slot stride 2 n) or chunked
__global__ void k_lz_combine(const double* V, int64_t S, int64_t n, double* out, const LanczosDev* lz) {
    if (lz->zero) return;
    __shared__ double y[2 * KRYLOV_MAX];
    const int m = lz->m_eff;
    if (threadIdx.x < 2 * KRYLOV_MAX) y[threadIdx.x] = lz->y[threadIdx.x] * lz->beta0;
    __syncthreads();
    if (n % 2 == 0 && (((uintptr_t)V | (uintptr_t)out) & 15) == 0) {   // two elements per step, 16-byte loads
        typedef double d2 __attribute__((ext_vector_type(2)));
        for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n / 2;
             q += (int64_t)gridDim.x * blockDim.x) {
            const int64_t i = 2 * q;
            d2 re = {0, 0}, im = {0, 0};
            const double* Vi = V + (S ? kch_ofs(i, S) : i);
            const int64_t ks = S ? 2 * KCH : 2 * n, ps = S ? KCH : n;
            for (int k = 0; k < m; ++k) {
                const double* v = Vi + ks * k;
                const d2 vr = *(const d2*)v, vi = *(const d2*)(v + ps);
                re += y[2 * k] * vr - y[2 * k + 1] * vi;
                im += y[2 * k] * vi + y[2 * k + 1] * vr;
            }
            *(d2*)(out + i) = re;
            *(d2*)(out + i + n) = im;
        }
        return;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double re = 0, im = 0;
        const double* Vi = V + (S ? kch_ofs(i, S) : i);
        const int64_t ks = S ? 2 * KCH : 2 * n, ps = S ? KCH : n;
        for (int k = 0; k < m; ++k) {
            const double* v = Vi + ks * k;
            const double vr = v[0], vi = v[ps];
            re += y[2 * k] * vr - y[2 * k + 1] * vi;
            im += y[2 * k] * vi + y[2 * k + 1] * vr;
        }
        out[i] = re;
        out[i + n] = im;
    }
}

inline int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

}  // namespace

void lz_start(const double* x, int64_t n, double* v0, int64_t S, LanczosDev* lz, double* partial, int nb,
              hipStream_t s, int nonherm, float* v0f) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_norm2_partial, dim3(nb), dim3(RED_THREADS), 0, s, x, n, partial,
                       (const int*)nullptr);
    hipLaunchKernelGGL(k_lz_begin, dim3(1), dim3(64), 0, s, partial, nb, lz, nonherm);
    hipLaunchKernelGGL(k_scale_by, dim3(grid_for(2 * n)), dim3(256), 0, s, x, n, v0, S, lz, 1, 0, v0f);
}

// Instantiates a launch for every basis size 1 .. KRYLOV_MAX.
#define TTN_KC_DISPATCH(kc, LAUNCH)                    \
    do {                                               \
        switch (kc) {                                  \
            case 1: LAUNCH(1); break;                  \
            case 2: LAUNCH(2); break;                  \
            case 3: LAUNCH(3); break;                  \
            case 4: LAUNCH(4); break;                  \
            case 5: LAUNCH(5); break;                  \
            case 6: LAUNCH(6); break;                  \
            case 7: LAUNCH(7); break;                  \
            case 8: LAUNCH(8); break;                  \
            case 9: LAUNCH(9); break;                  \
            case 10: LAUNCH(10); break;                \
            case 11: LAUNCH(11); break;                \
            case 12: LAUNCH(12); break;                \
            case 13: LAUNCH(13); break;                \
            case 14: LAUNCH(14); break;                \
            case 15: LAUNCH(15); break;                \
            case 16: LAUNCH(16); break;                \
            default: break;                            \
        }                                              \
    } while (0)
static_assert(KRYLOV_MAX == 16, "TTN_KC_DISPATCH covers basis sizes up to 16");

void lz_project(const double* V, int64_t S, int kcount, const double* w, int64_t n, double* partial, int nb,
                LanczosDev* lz, int alpha_index, hipStream_t s, const float* wf, bool total) {
    if (g_dry_run) return;
#define TTN_L(KC) \
    hipLaunchKernelGGL(k_multidot_partial<KC>, dim3(nb), dim3(RED_THREADS), 0, s, V, S, w, n, partial, lz, wf)
    TTN_KC_DISPATCH(kcount, TTN_L);
#undef TTN_L
    if (total)
        hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(1024), 0, s, partial, nb, kcount, lz, alpha_index);
}

// With fuse (nb <= LZ_FUSE_NB) the totals of the first pass are taken inside
// k_sub_fused<1> from the partials lz_project left at `partial`, and its own
// partials go to partial + LZ_PARTIAL_HALF.
void lz_subtract_project(const double* V, int64_t S, int kcount, double* w, int64_t n, double* partial, int nb,
                         LanczosDev* lz, hipStream_t s, bool fuse) {
    if (g_dry_run) return;
    if (fuse) {
#define TTN_L(KC)                                                                                             \
    hipLaunchKernelGGL((k_sub_fused<1, KC>), dim3(nb), dim3(256), 0, s, V, S, w, n, partial + LZ_PARTIAL_HALF, lz, \
                       (const double*)partial, nb, kcount - 1)
        TTN_KC_DISPATCH(kcount, TTN_L);
#undef TTN_L
        return;
    }
#define TTN_L(KC)                                                                                         \
    hipLaunchKernelGGL((k_sub_fused<1, KC>), dim3(nb), dim3(256), 0, s, V, S, w, n, partial, lz, \
                       (const double*)nullptr, 0, 0)
    TTN_KC_DISPATCH(kcount, TTN_L);
#undef TTN_L
    hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(1024), 0, s, partial, nb, kcount, lz, -1);
}

// With fuse the second pass's totals are taken inside k_sub_fused<2> from
// partial + LZ_PARTIAL_HALF, and beta_j inside the scaling kernel.
void lz_subtract_next(const double* V, int64_t S, int kcount, double* w, int64_t n, double* vnext, LanczosDev* lz,
                      int j, double* partial, int nb, double tol, hipStream_t s, float* vnextf, bool fuse) {
    if (g_dry_run) return;
    if (fuse) {
#define TTN_L(KC)                                                                                              \
    hipLaunchKernelGGL((k_sub_fused<2, KC>), dim3(nb), dim3(256), 0, s, V, S, w, n, partial, lz,               \
                       (const double*)(partial + LZ_PARTIAL_HALF), nb, -1)
        TTN_KC_DISPATCH(kcount, TTN_L);
#undef TTN_L
        hipLaunchKernelGGL(k_scale_next, dim3(grid_for(2 * n)), dim3(256), 0, s, w, n, vnext, S, lz,
                           (const double*)partial, nb, j, tol, vnextf);
        return;
    }
#define TTN_L(KC)                                                                                         \
    hipLaunchKernelGGL((k_sub_fused<2, KC>), dim3(nb), dim3(256), 0, s, V, S, w, n, partial, lz, \
                       (const double*)nullptr, 0, 0)
    TTN_KC_DISPATCH(kcount, TTN_L);
#undef TTN_L
    hipLaunchKernelGGL(k_lz_beta, dim3(1), dim3(256), 0, s, partial, nb, lz, j, tol);
    hipLaunchKernelGGL(k_scale_by, dim3(grid_for(2 * n)), dim3(256), 0, s, w, n, vnext, S, lz, 0, j, vnextf);
}

void lz_iter_small(double* V, int j, int m, double* w, int64_t n, LanczosDev* lz, double tol, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_lz_iter_small, dim3(1), dim3(256), 0, s, V, j, m, w, n, lz, tol);
}

void lz_expm(LanczosDev* lz, double tau, StepDev* st, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_lz_expm, dim3(1), dim3(64), 0, s, lz, tau, st);
}

int64_t small_evolve_doubles(int DL, int DR, int DP, int sL, int sR, int m, bool hasB, bool hasW) {
    const int64_t n = (int64_t)DL * DR * DP;
    const int64_t nz = (hasW && sR > 0) ? sR : 0;
    return 2 * n * (m + 1) + 2 * n + 2 * n * (sL + nz) + 2 * (int64_t)DL * DL * (1 + sL) +
           (nz ? 2 * (int64_t)DR * DR * (1 + sR) : 0) + (hasB ? 2 * (int64_t)DR * DR * (1 + sL) : 0) +
           (hasW ? 2 * (int64_t)DP * DP * (1 + sL + sR) : 0);
}

void small_evolve(const double* L, const double* R, const double* B, const double* W, int DL, int DR, int DP,
                  int sL, int sR, int m, double tau, double tol, bool nonherm, double* x, StepDev* st,
                  hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_small_evolve, dim3(1), dim3(SMALL_THREADS), 0, s, L, R, B, W, DL, DR, DP, sL, sR, m, tau,
                       tol, nonherm ? 1 : 0, x, st);
}

void lz_combine(const double* V, int64_t S, int64_t n, double* out, LanczosDev* lz, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_lz_combine, dim3(grid_for(n)), dim3(256), 0, s, V, S, n, out, lz);
}

void krylov_unchunk(const double* V, int64_t S, int64_t n, int slots, double* out, const int* skip, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_unchunk, dim3(grid_for(2 * n * slots)), dim3(256), 0, s, V, S, n, slots, out, skip);
}

// ---------------------------------------------------------------------------
// conversions / copies
// ---------------------------------------------------------------------------
namespace {
__global__ void k_d2f(const double* x, float* y, int64_t c, const int* skip) {
    if (skip && *skip) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

// several conversions in one launch: the concatenated index space of the
// arrays, each element converted exactly as by k_d2f
__global__ void k_d2f_batch(D2FBatch b, int64_t total, const int* skip) {
    if (skip && *skip) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        int64_t off = i;
        while (k < b.n - 1 && off >= b.c[k]) {
            off -= b.c[k];
            ++k;
        }
        const int D = b.eye[k];
        b.y[k][off] = D ? ((off < (int64_t)D * D && off % (D + 1) == 0) ? 1.0f : 0.0f) : (float)b.x[k][off];
    }
}
__global__ void k_f2d(const float* x, double* y, int64_t c, const int* skip) {
    if (skip && *skip) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}
__global__ void k_copy(const double* x, double* y, int64_t c, const int* skip) {
    if (skip && *skip) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}
__global__ void k_zero(double* y, int64_t c) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 0.0;
}
// y[c + cols*r] = x[r + rows*c] (planar complex, column-major)
__global__ void k_transpose(const double* x, double* y, int rows, int cols) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % rows), c = (int)(e / rows);
        y[c + (int64_t)cols * r] = x[e];
        y[n + c + (int64_t)cols * r] = x[n + e];
    }
}
__global__ void k_herm_f2d(const float* in, double* out, int D, int count, int raw_first) {
    const int64_t D2 = (int64_t)D * D, total = D2 * count;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / D2, ab = e % D2;
        const int a = (int)(ab % D), b = (int)(ab / D);
        const float* m = in + 2 * D2 * k;
        if (k == 0 && raw_first) {
            out[ab] = (double)m[ab];
            out[D2 + ab] = (double)m[D2 + ab];
            continue;
        }
        const int64_t t = b + (int64_t)D * a;
        out[2 * D2 * k + ab] = 0.5 * ((double)m[ab] + (double)m[t]);
        out[2 * D2 * k + D2 + ab] = 0.5 * ((double)m[D2 + ab] - (double)m[D2 + t]);
    }
}
__global__ void k_sum_mats(const double* src, int64_t D2, int count, double* dst) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * D2;
         e += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int k = 0; k < count; ++k) a += src[2 * D2 * k + e];
        dst[e] = a;
    }
}
}  // namespace

void herm_f2d(const float* in, double* out, int D, int count, hipStream_t s, bool raw_first) {
    if (g_dry_run) return;
    const int64_t total = (int64_t)D * D * count;
    hipLaunchKernelGGL(k_herm_f2d, dim3(grid_for(total)), dim3(256), 0, s, in, out, D, count, raw_first ? 1 : 0);
}

void sum_mats(const double* src, int D, int count, double* dst, hipStream_t s) {
    if (g_dry_run) return;
    const int64_t D2 = (int64_t)D * D;
    hipLaunchKernelGGL(k_sum_mats, dim3(grid_for(2 * D2)), dim3(256), 0, s, src, D2, count, dst);
}

void convert_d2f(const double* x, float* y, int64_t count, const int* skip, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_d2f, dim3(grid_for(count)), dim3(256), 0, s, x, y, count, skip);
}
void convert_d2f_many(std::initializer_list<D2FItem> items, const int* skip, hipStream_t s) {
    if (g_dry_run) return;
    D2FBatch b{};
    int64_t total = 0;
    for (const D2FItem& it : items) {
        if ((!it.x && it.eye <= 0) || it.count <= 0) continue;
        if (b.n == D2F_MAX) {   // full: flush
            hipLaunchKernelGGL(k_d2f_batch, dim3(grid_for(total)), dim3(256), 0, s, b, total, skip);
            b = D2FBatch{};
            total = 0;
        }
        b.x[b.n] = it.x;
        b.y[b.n] = it.y;
        b.c[b.n] = it.count;
        b.eye[b.n] = it.eye > 0 ? it.eye : 0;
        ++b.n;
        total += it.count;
    }
    if (b.n > 0) hipLaunchKernelGGL(k_d2f_batch, dim3(grid_for(total)), dim3(256), 0, s, b, total, skip);
}
void convert_f2d(const float* x, double* y, int64_t count, const int* skip, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_f2d, dim3(grid_for(count)), dim3(256), 0, s, x, y, count, skip);
}
void copy_d(const double* x, double* y, int64_t count, const int* skip, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(count)), dim3(256), 0, s, x, y, count, skip);
}
void fill_zero_d(double* y, int64_t count, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(count)), dim3(256), 0, s, y, count);
}
void transpose_c(const double* x, double* y, int rows, int cols, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_transpose, dim3(grid_for((int64_t)rows * cols)), dim3(256), 0, s, x, y,
                       rows, cols);
}

// ---------------------------------------------------------------------------
// Cholesky + inverse for CholeskyQR2
// ---------------------------------------------------------------------------
namespace {

constexpr int CHOL_THREADS = 512;
constexpr int CHOL_PANEL = 16;
constexpr int CHOL_LDS_MAX = 128;   // packed lower triangle of 128 x 128 fits LDS

__device__ inline int64_t pidx(int i, int j, int D) {   // packed lower, column-major, i >= j
    return (int64_t)j * D - (int64_t)j * (j - 1) / 2 + (i - j);
}

// Panel-blocked Cholesky G = L L^H and in-place inverse X = L^{-1} (lower,
// packed, column-major).  Each panel of P columns (Cholesky) or P rows
// (inverse) is processed by the first wave with the panel held in registers
// (RPL rows or columns per lane) and pivots / column entries broadcast by
// cross-lane shuffles; the rank-P updates of the rest of the matrix use the
// whole workgroup between barriers.
template <bool LDS, int RPL, int P>
__global__ __launch_bounds__(CHOL_THREADS) void k_chol_inv(const double* G, int D, double* Linv,
                                                           double* R, const double* Rprev,
                                                           double* work, StepDev* st) {
    __shared__ double sLre[LDS ? CHOL_LDS_MAX * (CHOL_LDS_MAX + 1) / 2 : 1];
    __shared__ double sLim[LDS ? CHOL_LDS_MAX * (CHOL_LDS_MAX + 1) / 2 : 1];
    __shared__ int s_bad;
    const int64_t np = (int64_t)D * (D + 1) / 2;
    double* Lre = LDS ? sLre : work;
    double* Lim = LDS ? sLim : work + np;
    double* Tre = work + 2 * np;                 // rows x P copy of L for the inverse
    double* Tim = Tre + (int64_t)D * P;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int64_t DD = (int64_t)D * D;
    if (tid == 0) s_bad = 0;
    for (int64_t e = tid; e < DD; e += CHOL_THREADS) {
        const int i = (int)(e % D), j = (int)(e / D);
        if (i >= j) {
            Lre[pidx(i, j, D)] = G[e];
            Lim[pidx(i, j, D)] = G[DD + e];
        }
    }
    __syncthreads();
    // ---------------- Cholesky ----------------
    for (int p0 = 0; p0 < D; p0 += P) {
        const int pe = min(p0 + P, D);
        if (wave == 0) {
            double xr[RPL][P], xi[RPL][P];   // rows p0 + lane + 64 r, columns p0 + c
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = p0 + lane + 64 * r;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    const bool ok = i < D && p0 + c < pe && p0 + c <= i;
                    const int64_t q = ok ? pidx(i, p0 + c, D) : 0;
                    xr[r][c] = ok ? Lre[q] : 0.0;
                    xi[r][c] = ok ? Lim[q] : 0.0;
                }
            }
            bool bad = false;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                if (p0 + j < pe) {
                    const double piv = __shfl(xr[0][j], j, 64);   // diagonal: row p0 + j is lane j
                    bad = bad || !(piv > 1e-290);
                    const double d = sqrt(piv > 1e-290 ? piv : 1e-290), dinv = 1.0 / d;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const int i = p0 + lane + 64 * r;
                        if (i == p0 + j) {
                            xr[r][j] = d;
                            xi[r][j] = 0.0;
                        } else if (i > p0 + j) {
                            xr[r][j] *= dinv;
                            xi[r][j] *= dinv;
                        }
                    }
#pragma unroll
                    for (int k = j + 1; k < P; ++k) {
                        if (p0 + k < pe) {
                            const double lr = __shfl(xr[0][j], k, 64), li = __shfl(xi[0][j], k, 64);
#pragma unroll
                            for (int r = 0; r < RPL; ++r) {
                                const int i = p0 + lane + 64 * r;
                                if (i >= p0 + k) {   // L[i][k] -= L[i][j] conj(L[k][j])
                                    xr[r][k] -= xr[r][j] * lr + xi[r][j] * li;
                                    xi[r][k] -= xi[r][j] * lr - xr[r][j] * li;
                                }
                            }
                        }
                    }
                }
            }
            if (bad && lane == 0) s_bad = 1;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = p0 + lane + 64 * r;
#pragma unroll
                for (int c = 0; c < P; ++c)
                    if (i < D && p0 + c < pe && p0 + c <= i) {
                        const int64_t q = pidx(i, p0 + c, D);
                        Lre[q] = xr[r][c];
                        Lim[q] = xi[r][c];
                    }
            }
        }
        __syncthreads();
        // trailing update: L[i][k] -= sum_{j in panel} L[i][j] conj(L[k][j]), pe <= k <= i
        const int rn = D - pe;
        for (int64_t e = tid; e < (int64_t)rn * rn; e += CHOL_THREADS) {
            const int ii = (int)(e % rn), kk = (int)(e / rn);
            if (ii < kk) continue;
            const int i = pe + ii, k = pe + kk;
            double sr = 0, si = 0;
            for (int j = p0; j < pe; ++j) {
                const int64_t cj = pidx(j, j, D) - j;
                const double ar = Lre[cj + i], ai = Lim[cj + i];
                const double br = Lre[cj + k], bi = Lim[cj + k];
                sr += ar * br + ai * bi;
                si += ai * br - ar * bi;
            }
            const int64_t q = pidx(i, k, D);
            Lre[q] -= sr;
            Lim[q] -= si;
        }
        __syncthreads();
    }
    // R = L^H, or L^H Rprev:  R[k][a] = sum_{j=k}^{a} conj(L[j][k]) Rprev[j][a]
    for (int64_t e = tid; e < DD; e += CHOL_THREADS) {
        const int k = (int)(e % D), a = (int)(e / D);
        double rr = 0, ri = 0;
        if (a >= k) {
            const int64_t ck = pidx(k, k, D) - k;
            if (!Rprev) {
                rr = Lre[ck + a];
                ri = -Lim[ck + a];
            } else {
                for (int j = k; j <= a; ++j) {
                    const double lr = Lre[ck + j], li = -Lim[ck + j];
                    const double pr = Rprev[j + (int64_t)D * a], pi = Rprev[DD + j + (int64_t)D * a];
                    rr += lr * pr - li * pi;
                    ri += lr * pi + li * pr;
                }
            }
        }
        R[e] = rr;
        R[DD + e] = ri;
    }
    __syncthreads();
    if (tid == 0) {
        double mn = 1e308;
        for (int k = 0; k < D; ++k) {
            const double v = R[k + (int64_t)D * k];
            mn = v < mn ? v : mn;
        }
        if (s_bad || !(mn == mn)) atomicExch(&st->bad, 1);
    }
    // ---------------- inverse by elimination on the identity ----------------
    // Position (i, j), i > j, holds L[i][j] until step j and the partial
    // X[i][j] afterwards; the diagonal becomes 1 / L[i][i].
    for (int p0 = 0; p0 < D; p0 += P) {
        const int pe = min(p0 + P, D);
        if (wave == 0) {
            double yr[P][RPL], yi[P][RPL];   // panel rows p0 + t, columns lane + 64 s
#pragma unroll
            for (int t = 0; t < P; ++t)
#pragma unroll
                for (int sl = 0; sl < RPL; ++sl) {
                    const int c = lane + 64 * sl, k = p0 + t;
                    const bool ok = k < pe && c <= k;
                    const int64_t q = ok ? pidx(k, c, D) : 0;
                    yr[t][sl] = ok ? Lre[q] : 0.0;
                    yi[t][sl] = ok ? Lim[q] : 0.0;
                }
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const int k = p0 + t;
                if (k < pe) {
                    const int kl = k & 63, ks = k >> 6;
                    double sel = 0.0;
#pragma unroll
                    for (int sl = 0; sl < RPL; ++sl)
                        if (sl == ks) sel = yr[t][sl];
                    const double d = 1.0 / __shfl(sel, kl, 64);
                    // column k of the later panel rows (still L values)
                    double cr[P], ci[P];
#pragma unroll
                    for (int u = t + 1; u < P; ++u) {
                        double a = 0.0, b2 = 0.0;
#pragma unroll
                        for (int sl = 0; sl < RPL; ++sl)
                            if (sl == ks) {
                                a = yr[u][sl];
                                b2 = yi[u][sl];
                            }
                        cr[u] = __shfl(a, kl, 64);
                        ci[u] = __shfl(b2, kl, 64);
                    }
#pragma unroll
                    for (int sl = 0; sl < RPL; ++sl) {
                        const int c = lane + 64 * sl;
                        if (c < k) {
                            yr[t][sl] *= d;
                            yi[t][sl] *= d;
                        } else if (c == k) {
                            yr[t][sl] = d;
                            yi[t][sl] = 0.0;
                        }
                    }
#pragma unroll
                    for (int u = t + 1; u < P; ++u) {
                        if (p0 + u < pe) {
#pragma unroll
                            for (int sl = 0; sl < RPL; ++sl) {
                                const int c = lane + 64 * sl;
                                if (c <= k) {
                                    const double orr = (c == k) ? 0.0 : yr[u][sl];
                                    const double oii = (c == k) ? 0.0 : yi[u][sl];
                                    yr[u][sl] = orr - (cr[u] * yr[t][sl] - ci[u] * yi[t][sl]);
                                    yi[u][sl] = oii - (cr[u] * yi[t][sl] + ci[u] * yr[t][sl]);
                                }
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < P; ++t)
#pragma unroll
                for (int sl = 0; sl < RPL; ++sl) {
                    const int c = lane + 64 * sl, k = p0 + t;
                    if (k < pe && c <= k) {
                        const int64_t q = pidx(k, c, D);
                        Lre[q] = yr[t][sl];
                        Lim[q] = yi[t][sl];
                    }
                }
        }
        const int rn = D - pe;
        // copy L[i][panel] for the rows below the panel (not touched by wave 0)
        for (int e = tid; e < rn * (pe - p0); e += CHOL_THREADS) {
            const int r = e % rn, c = e / rn;
            const int64_t q = pidx(pe + r, p0 + c, D);
            Tre[r + (int64_t)D * c] = Lre[q];
            Tim[r + (int64_t)D * c] = Lim[q];
        }
        __syncthreads();
        // rows i >= pe: X[i][j] = (j in panel ? 0 : X[i][j]) - sum_{k in panel, k >= j} L[i][k] X[k][j]
        for (int64_t e = tid; e < (int64_t)rn * pe; e += CHOL_THREADS) {
            const int r = (int)(e % rn), j = (int)(e / rn);
            const int i = pe + r;
            double sr = 0, si = 0;
            for (int k = max(j, p0); k < pe; ++k) {
                const double lr = Tre[r + (int64_t)D * (k - p0)], li = Tim[r + (int64_t)D * (k - p0)];
                const int64_t qk = pidx(k, j, D);
                const double xr = Lre[qk], xi = Lim[qk];
                sr += lr * xr - li * xi;
                si += lr * xi + li * xr;
            }
            const int64_t qi = pidx(i, j, D);
            const double or_ = (j >= p0) ? 0.0 : Lre[qi];
            const double oi = (j >= p0) ? 0.0 : Lim[qi];
            Lre[qi] = or_ - sr;
            Lim[qi] = oi - si;
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < DD; e += CHOL_THREADS) {
        const int i = (int)(e % D), j = (int)(e / D);
        double xr = 0, xi = 0;
        if (i >= j) {
            xr = Lre[pidx(i, j, D)];
            xi = Lim[pidx(i, j, D)];
        }
        Linv[e] = xr;
        Linv[DD + e] = xi;
    }
}

}  // namespace

namespace {

// Blocked Cholesky + inverse for D <= 128 in one workgroup: the lower
// triangle in 16 x 16 blocks in LDS (36 blocks, 144 KB).  Right-looking by
// block columns: one wave factors the diagonal block (pivots broadcast with
// readlane, columns through LDS), the panel rows are solved by substitution
// (one lane per row), the trailing blocks are updated with the FP64 matrix
// cores while one wave already updates and factors the next diagonal block.
// The inverse: every diagonal block inverted by its own wave, then the block
// diagonals X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ, one level at a time, on
// the matrix cores (the output fragments of one product are the B operand
// fragments of the next).  Sizes that are not a multiple of 16 are padded
// with an identity block.
constexpr int CB = 16;
constexpr int CB_MAXNB = 8;
constexpr int CB_NBLK = CB_MAXNB * (CB_MAXNB + 1) / 2;
constexpr int CB_THREADS = 512;
constexpr int CB_WAVES = CB_THREADS / 64;

__device__ inline int cb_bidx(int I, int J) { return I * (I + 1) / 2 + J; }

__device__ inline double cb_readlane(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

__device__ inline void cb_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef double cb_d4 __attribute__((ext_vector_type(4)));

__device__ inline cb_d4 cb_mfma(double a, double b, cb_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// O -= A B^H on a 16 x 16 block by one wave with the FP64 matrix cores.
// Fragments: A lane l -> A[l%16][k], B lane l -> B[k][l%16], k = kk + l/16;
// the output register r of lane l is row l/16 + 4 r, column l%16.  The
// products are formed transposed (B as the first operand, A^T as the
// second), so that lane l holds O[l%16][l/16 + 4 r]: the 16 lanes of a row
// group then touch 16 consecutive entries of a column of O in LDS, where
// the untransposed layout strode 16 entries and put them on one bank.
__device__ inline void cb_sub_abh_mfma(const double* Ar, const double* Ai, const double* Br, const double* Bi,
                                       double* Or, double* Oi, int lane) {
    const int m = lane & 15, q = lane >> 4;
    // three real products per complex product (Gauss): with C = conj(B),
    // P1 = Ar Cr^T, P2 = Ai Ci^T, P3 = (Ar + Ai)(Cr + Ci)^T, Re = P1 - P2 and
    // Im = P3 - P1 - P2; independent accumulator chains
    cb_d4 d1 = {0, 0, 0, 0}, d2 = {0, 0, 0, 0}, d3 = {0, 0, 0, 0};
    double ar[4], ai[4], br[4], bi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ia = m + CB * (4 * t + q);   // A[m][kk+q]; B^H[kk+q][m] = conj(B[m][kk+q])
        ar[t] = Ar[ia];
        ai[t] = Ai[ia];
        br[t] = Br[ia];
        bi[t] = Bi[ia];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        d1 = cb_mfma(br[t], ar[t], d1);                    // P1^T
        d2 = cb_mfma(-bi[t], ai[t], d2);                   // P2^T
        d3 = cb_mfma(br[t] - bi[t], ar[t] + ai[t], d3);    // P3^T
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = m + CB * (q + 4 * r);
        Or[o] -= d1[r] - d2[r];
        Oi[o] -= d3[r] - d1[r] - d2[r];
    }
}

// Cholesky of the 16 x 16 Hermitian block (br, bi) in place by one wave:
// L lower (upper zeroed); dinv[j] = 1 / L_jj to ds[0..15]; cs: 128 doubles.
// Lane (r, g) holds row r of columns 4 g .. 4 g + 3.  The columns go in four
// groups of four: the 16 lanes of group g factor its columns in registers
// (each pivot and each entry L[c][j] the group's later columns need comes by
// a lane read, no memory round trip), publish the four columns through LDS
// once, and the lanes of the later groups take the rank-4 update.  Every
// entry sees its subtractions in the order j = 0, 1, .., as in the
// column-by-column form.
__device__ inline void cb_chol_diag(double* br, double* bi, double* ds, double* cs, int lane, int& bad) {
    const int r = lane & 15, cg = lane >> 4;
    double a_r[4], a_i[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        a_r[s] = br[r + CB * (4 * cg + s)];
        a_i[s] = bi[r + CB * (4 * cg + s)];
    }
    double* cre = cs;            // [4 columns][16 rows]
    double* cim = cs + 4 * CB;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const bool mine = cg == G;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = 4 * G + s;
            const double piv = cb_readlane(a_r[s], j + CB * G);
            bad |= !(piv > 1e-290);
            const double pv = piv > 1e-290 ? piv : 1e-290;
            double y = __builtin_amdgcn_rsq(pv);   // 1/sqrt refined by two Newton steps
            y = y * (1.5 - 0.5 * pv * y * y);
            y = y * (1.5 - 0.5 * pv * y * y);
            if (lane == 0) ds[j] = y;
            {
                const double vr = r > j ? a_r[s] * y : (r == j ? pv * y : 0.0);
                const double vi = r > j ? a_i[s] * y : 0.0;
                a_r[s] = mine ? vr : a_r[s];
                a_i[s] = mine ? vi : a_i[s];
            }
            // the group's later columns c: a[r][c] -= L[r][j] conj(L[c][j])
#pragma unroll
            for (int t = s + 1; t < 4; ++t) {
                const int c = 4 * G + t;
                const double cr_ = cb_readlane(a_r[s], c + CB * G), ci_ = cb_readlane(a_i[s], c + CB * G);
                const double lr = a_r[s], li = a_i[s];
                const double ur = a_r[t] - (lr * cr_ + li * ci_);
                const double ui = a_i[t] - (li * cr_ - lr * ci_);
                a_r[t] = mine ? ur : a_r[t];
                a_i[t] = mine ? ui : a_i[t];
            }
        }
        if (G == 3) break;
        if (mine)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                cre[r + CB * s] = a_r[s];
                cim[r + CB * s] = a_i[s];
            }
        cb_wave_sync();
        if (cg > G) {
            // rank-4 update of the later groups' columns c = 4 cg + t
            double lr[4], li[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                lr[s] = cre[r + CB * s];
                li[s] = cim[r + CB * s];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = 4 * cg + t;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double cr_ = cre[c + CB * s], ci_ = cim[c + CB * s];
                    a_r[t] -= lr[s] * cr_ + li[s] * ci_;
                    a_i[t] -= li[s] * cr_ - lr[s] * ci_;
                }
            }
        }
        cb_wave_sync();
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        br[r + CB * (4 * cg + s)] = a_r[s];
        bi[r + CB * (4 * cg + s)] = a_i[s];
    }
}

// X = L^{-1} of the lower block (lr_, li_) (LDS) by one wave, into global
// (xr, xi) with leading dimension ld; ds: dinv; cs: 32 doubles scratch.
__device__ inline void cb_inv_diag(const double* lr_, const double* li_, const double* ds, double* xr, double* xi,
                                   int64_t ld, double* cs, int lane) {
    const int r = lane & 15, cg = lane >> 4;
    double x_r[4], x_i[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        x_r[s] = (r == 4 * cg + s) ? 1.0 : 0.0;
        x_i[s] = 0.0;
    }
    double* rowr = cs;
    double* rowi = cs + CB;
#pragma unroll
    for (int k = 0; k < CB; ++k) {
        if (r == k) {
            const double dk = ds[k];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                x_r[s] *= dk;
                x_i[s] *= dk;
                rowr[4 * cg + s] = x_r[s];
                rowi[4 * cg + s] = x_i[s];
            }
        }
        cb_wave_sync();
        if (r > k) {
            const double l_r = lr_[r + CB * k], l_i = li_[r + CB * k];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double xr_ = rowr[4 * cg + s], xi_ = rowi[4 * cg + s];
                x_r[s] -= l_r * xr_ - l_i * xi_;
                x_i[s] -= l_r * xi_ + l_i * xr_;
            }
        }
        cb_wave_sync();
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        xr[r + ld * (4 * cg + s)] = x_r[s];
        xi[r + ld * (4 * cg + s)] = x_i[s];
    }
}

// G (D x D Hermitian, planar, column-major) = L L^H; Linv = L^{-1} (lower),
// R = L^H (upper).  work: 2 Dp^2 doubles (Dp = 16 ceil(D / 16)), untouched
// when D is a multiple of 16.
__global__ __launch_bounds__(CB_THREADS) void k_chol_blk(const double* G, int D, double* Linv, double* R,
                                                         double* work, StepDev* st) {
    __shared__ double s_re[CB_NBLK * 256], s_im[CB_NBLK * 256];
    __shared__ double s_cs[CB_WAVES * 64];
    __shared__ double s_col[8 * CB];   // the diagonal factorization's four published columns
    __shared__ double s_dinv[CB_MAXNB * CB];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NB = (D + CB - 1) / CB, Dp = NB * CB;
    const int64_t DD = (int64_t)D * D, P2 = (int64_t)Dp * Dp;
    // the inverse is built in place in Linv when D is a whole number of
    // blocks (no padding), else in the padded work array and copied out
    const bool direct = Dp == D;
    double* Xr = direct ? Linv : work;   // Dp x Dp column-major
    double* Xi = direct ? Linv + DD : work + P2;
    double* dall = s_dinv;            // 1 / L_jj of every diagonal block, 16 per block
    double* csw = s_cs + 64 * wave;   // per-wave scratch (32 used)
    if (tid == 0) s_bad = 0;
    const int nbl = NB * (NB + 1) / 2;
    {
        // lower blocks of G into LDS (packed by cb_bidx): every load of a
        // thread is issued before its first LDS store
        constexpr int LQ = CB_NBLK * 256 / CB_THREADS;
        static_assert(LQ * CB_THREADS == CB_NBLK * 256, "blocks must split evenly over the threads");
        if (nbl == 1) {   // D <= 16: one block, one entry per thread
            if (tid < 256) {
                const int gi = tid & 15, gj = tid >> 4;
                const bool in = gi < D && gj < D;
                s_re[tid] = in ? G[gi + (int64_t)D * gj] : (gi == gj ? 1.0 : 0.0);
                s_im[tid] = in ? G[DD + gi + (int64_t)D * gj] : 0.0;
            }
        } else {
            double gr[LQ], gim[LQ];
#pragma unroll
            for (int q = 0; q < LQ; ++q) {
                const int e = tid + CB_THREADS * q, b = e >> 8, rc = e & 255;
                // block row of packed block b: the largest I with I (I + 1) / 2 <= b,
                // floor((sqrt(8 b + 1) - 1) / 2); for b < 36 the value stays at
                // least 0.11 below the next integer, so the 0.05 guard absorbs any
                // rounding of the root at the perfect squares
                const int I = (int)((sqrtf((float)(8 * b + 1)) - 1.0f) * 0.5f + 0.05f);
                const int J = b - I * (I + 1) / 2;
                const int gi = CB * I + (rc & 15), gj = CB * J + (rc >> 4);
                const bool in = b < nbl && gi < D && gj < D;
                gr[q] = in ? G[gi + (int64_t)D * gj] : (gi == gj ? 1.0 : 0.0);
                gim[q] = in ? G[DD + gi + (int64_t)D * gj] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < LQ; ++q) {
                const int e = tid + CB_THREADS * q;
                if ((e >> 8) < nbl) {
                    s_re[e] = gr[q];
                    s_im[e] = gim[q];
                }
            }
        }
    }
    __syncthreads();
    int bad = 0;
    if (wave == 0) cb_chol_diag(s_re, s_im, dall, s_col, lane, bad);
    __syncthreads();
    for (int K = 0; K < NB; ++K) {
        const double* Lkr = s_re + 256 * cb_bidx(K, K);
        const double* Lki = s_im + 256 * cb_bidx(K, K);
        const double* dsum = dall + CB * K;
        // panel: rows of A_IK (I > K) solve L_IK L_KK^H = A_IK by substitution,
        // column-oriented: once x_k is known it is taken out of every later
        // column at once, so the dependent chain is one product per column
        // (the subtractions of each column still run in the order k = 0, 1, ..)
        const int nrows = CB * (NB - K - 1);
        if (tid < nrows) {
            const int I = K + 1 + tid / CB, r = tid % CB;
            double* ar = s_re + 256 * cb_bidx(I, K);
            double* ai = s_im + 256 * cb_bidx(I, K);
            double xr[CB], xi[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                xr[c] = ar[r + CB * c];
                xi[c] = ai[r + CB * c];
            }
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const double dk = dsum[k];
                xr[k] *= dk;
                xi[k] *= dk;
#pragma unroll
                for (int c = k + 1; c < CB; ++c) {   // - x_k conj(L[c][k])
                    const double l_r = Lkr[c + CB * k], l_i = -Lki[c + CB * k];
                    xr[c] -= xr[k] * l_r - xi[k] * l_i;
                    xi[c] -= xr[k] * l_i + xi[k] * l_r;
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                ar[r + CB * c] = xr[c];
                ai[r + CB * c] = xi[c];
            }
        }
        __syncthreads();
        // trailing update A_IJ -= L_IK L_JK^H (K < J <= I); wave 0 first updates
        // the next diagonal block and factors it (look-ahead).  Wave 4, which
        // shares wave 0's SIMD, takes no update blocks, so the factorization's
        // serial chain has that SIMD to itself (it clears the upper blocks of
        // the output once, global stores only); waves 1-3 and 5-7 share the rest
        const int m = NB - K - 1, nt = m * (m + 1) / 2;
        constexpr int UPD = CB_WAVES - 2;
        const int uw = wave < 4 ? wave - 1 : wave - 2;
        if (wave == 0) {
            if (m > 0) {
                const int b1 = cb_bidx(K + 1, K + 1), bk = cb_bidx(K + 1, K);
                cb_sub_abh_mfma(s_re + 256 * bk, s_im + 256 * bk, s_re + 256 * bk, s_im + 256 * bk,
                                s_re + 256 * b1, s_im + 256 * b1, lane);
                cb_wave_sync();
                cb_chol_diag(s_re + 256 * b1, s_im + 256 * b1, dall + CB * (K + 1), s_col, lane, bad);
            }
        } else if (wave == 4) {
            // meanwhile: the blocks (I, J), I < J, of an in-place inverse are
            // zero; the NB (NB - 1) / 2 of them, in order J, then I, are spread
            // over the iterations, ceil(that / NB) per iteration (lane l: row
            // l % 16 of columns 4 s + l / 16, four 128-byte segments a store)
            if (direct) {
                const int nup = NB * (NB - 1) / 2, per = (nup + NB - 1) / NB;
                for (int u = K * per; u < nup && u < (K + 1) * per; ++u) {
                    int J = 1;
                    while (J * (J + 1) / 2 <= u) ++J;
                    const int I = u - J * (J - 1) / 2;
                    const int i = CB * I + (lane & 15);
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int j = CB * J + 4 * s4 + (lane >> 4);
                        Linv[i + (int64_t)D * j] = 0.0;
                        Linv[DD + i + (int64_t)D * j] = 0.0;
                    }
                }
            }
        } else {
            for (int t = uw; t < nt; t += UPD) {
                int ii = 0;
                while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
                const int jj = t - ii * (ii + 1) / 2;
                if (ii == 0 && jj == 0) continue;   // the next diagonal block (wave 0)
                const int I = K + 1 + ii, J = K + 1 + jj;
                const int bi_ = cb_bidx(I, K), bj = cb_bidx(J, K), bo = cb_bidx(I, J);
                cb_sub_abh_mfma(s_re + 256 * bi_, s_im + 256 * bi_, s_re + 256 * bj, s_im + 256 * bj,
                                s_re + 256 * bo, s_im + 256 * bo, lane);
            }
        }
        __syncthreads();
    }
    if (bad && lane == 0) atomicOr(&s_bad, 1);
    // inverses of the diagonal blocks, one wave each
    if (wave < NB)
        cb_inv_diag(s_re + 256 * cb_bidx(wave, wave), s_im + 256 * cb_bidx(wave, wave), dall + CB * wave,
                    Xr + CB * wave + (int64_t)Dp * CB * wave, Xi + CB * wave + (int64_t)Dp * CB * wave, Dp, csw, lane);
    // R = L^H (upper): R[k, a] = conj(L[a, k]); lanes over k, so that a
    // store writes 512 contiguous bytes of a column of R (reading by 16 x 16
    // blocks instead, conflict-free in LDS but with 32-byte store segments,
    // measured slower)
    for (int a = wave; a < D; a += CB_WAVES)
        for (int k = lane; k < D; k += 64) {
            double vr = 0.0, vi = 0.0;
            if (a >= k) {
                const int q = 256 * cb_bidx(a >> 4, k >> 4) + (a & 15) + CB * (k & 15);
                vr = s_re[q];
                vi = -s_im[q];
            }
            R[k + (int64_t)D * a] = vr;
            R[DD + k + (int64_t)D * a] = vi;
        }
    __threadfence_block();
    __syncthreads();
    // inverse by block columns: X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ for
    // I = J + 1 ..; each wave owns one column J (columns 0-3 on waves 0-3 and
    // 7-4 on waves 4-7, so that the two waves sharing a SIMD share the work
    // evenly) and keeps the column's blocks X_KJ as B fragments in registers
    // (the output layout of one product is the B fragment layout of the
    // next), so the waves need no barrier between blocks; only the diagonal
    // inverses X_II, written before the last barrier, come from memory
    static_assert(CB_WAVES == 8 && CB_MAXNB == 8, "one wave per block column");
    {
        const int J = wave < 4 ? wave : 11 - wave;
        const int m = lane & 15, q = lane >> 4;
        double xb_r[4 * CB_MAXNB], xb_i[4 * CB_MAXNB];   // X_{J+t, J}, fragment j of block t
#pragma unroll
        for (int j = 0; j < 4 * CB_MAXNB; ++j) {
            xb_r[j] = 0.0;
            xb_i[j] = 0.0;
        }
        if (J < NB) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t g = (CB * J + 4 * j + q) + (int64_t)Dp * (CB * J + m);
                xb_r[j] = Xr[g];
                xb_i[j] = Xi[g];
            }
        }
#pragma unroll
        for (int dl = 1; dl < CB_MAXNB; ++dl) {
            const int I = J + dl;
            if (I < NB) {
                double xa_r[4], xa_i[4];   // A fragments of X_II[m][kk + q]
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t g = (CB * I + m) + (int64_t)Dp * (CB * I + 4 * j + q);
                    xa_r[j] = Xr[g];
                    xa_i[j] = Xi[g];
                }
                // T = sum_t L_{I,J+t} X_{J+t,J}, three real products per complex
                // product (Gauss): P1 = Lr Xr, P2 = Li Xi, P3 = (Lr + Li)(Xr + Xi),
                // Re T = P1 - P2, Im T = P3 - P1 - P2
                cb_d4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < dl; ++t) {
                    const double* Lr = s_re + 256 * cb_bidx(I, J + t);
                    const double* Li = s_im + 256 * cb_bidx(I, J + t);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int ia = m + CB * (4 * j + q);
                        const double lr = Lr[ia], li = Li[ia], br = xb_r[4 * t + j], bi = xb_i[4 * t + j];
                        p1 = cb_mfma(lr, br, p1);
                        p2 = cb_mfma(li, bi, p2);
                        p3 = cb_mfma(lr + li, br + bi, p3);
                    }
                }
                const cb_d4 tr = p1 - p2, ti = p3 - p1 - p2;
                // X_IJ = - X_II T, the same three-product form
                cb_d4 q1 = {0, 0, 0, 0}, q2 = {0, 0, 0, 0}, q3 = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    q1 = cb_mfma(xa_r[j], tr[j], q1);
                    q2 = cb_mfma(xa_i[j], ti[j], q2);
                    q3 = cb_mfma(xa_r[j] + xa_i[j], tr[j] + ti[j], q3);
                }
                const cb_d4 orr = q2 - q1, oi = q1 + q2 - q3;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t g = (CB * I + q + 4 * r) + (int64_t)Dp * (CB * J + m);
                    Xr[g] = orr[r];
                    Xi[g] = oi[r];
                    xb_r[4 * dl + r] = orr[r];
                    xb_i[4 * dl + r] = oi[r];
                }
            }
        }
    }
    __threadfence_block();
    __syncthreads();
    if (!direct)
        for (int j = wave; j < D; j += CB_WAVES)
            for (int i = lane; i < D; i += 64) {
                const bool lo = i >= j;
                const int64_t g = i + (int64_t)Dp * j;
                Linv[i + (int64_t)D * j] = lo ? Xr[g] : 0.0;
                Linv[DD + i + (int64_t)D * j] = lo ? Xi[g] : 0.0;
            }
    __syncthreads();
    if (tid == 0 && s_bad) atomicExch(&st->bad, 1);
}

}  // namespace

void chol_inv(const double* G, int D, double* Linv, double* R, const double* Rprev, double* work,
              StepDev* st, hipStream_t s) {
    if (g_dry_run) return;
    if (D <= CB * CB_MAXNB && !Rprev)
        hipLaunchKernelGGL(k_chol_blk, dim3(1), dim3(CB_THREADS), 0, s, G, D, Linv, R, work, st);
    else
        hipLaunchKernelGGL((k_chol_inv<false, 4, 8>), dim3(1), dim3(CHOL_THREADS), 0, s, G, D, Linv, R, Rprev,
                           work, st);
}

namespace {
// Smallest real diagonal entry of the D x D (planar, column-major) R of a
// gauge move, folded into the step's minimum (positive doubles order like
// their bit patterns).  One wave.
__global__ __launch_bounds__(64) void k_rdiag_min(const double* R, int D, StepDev* st) {
    double mn = 1e308;
    for (int k = threadIdx.x; k < D; k += 64) {
        const double v = R[k + (int64_t)D * k];
        mn = v < mn ? v : mn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(mn, o, 64);
        mn = t < mn ? t : mn;
    }
    if (threadIdx.x == 0 && mn > 0)
        atomicMin(&st->min_rdiag_bits, (unsigned long long)__double_as_longlong(mn));
}
}  // namespace

void rdiag_min(const double* R, int D, StepDev* st, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_rdiag_min, dim3(1), dim3(64), 0, s, R, D, st);
}

// ---------------------------------------------------------------------------
// Hermitian eigendecomposition (cyclic Jacobi) for the two-site split
// ---------------------------------------------------------------------------
namespace {
constexpr int JAC_THREADS = 1024;

// Eigenvalues and eigenvectors of a Hermitian n x n matrix A (planar complex,
// column-major; overwritten) by the cyclic Jacobi method with the round-robin
// ordering: each of the n' - 1 rounds of a sweep (n' = n rounded up to even,
// the extra index a zero row and column) rotates n' / 2 disjoint index pairs
// at once, all rotations taken from the matrix before the round.  Pair
// (p, q), b = A[p, q] = |b| e^{i phi}: J = diag(1, e^{-i phi}) R with the real
// Jacobi rotation R = [[c, s], [-s, c]] that diagonalises
// [[A_pp, |b|], [|b|, A_qq]] (t = sgn(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = (A_qq - A_pp) / (2 |b|), c = 1 / sqrt(1 + t^2), s = t c), applied as
// A <- J^H A J and V <- V J.  A pair is skipped when
// |b| <= tol sqrt(|A_pp A_qq|) (relative accuracy for positive definite
// matrices) or |b| <= 4 eps sum_i |A_ii| (the rounding level of the matrix,
// which pairs of numerically zero eigenvalues cannot get below); the
// iteration stops after a sweep without a rotation, or after max_sweeps
// (then st->bad is set).  Outputs: w[k] the k-th largest
// eigenvalue, order[k] its column in V.
__global__ __launch_bounds__(JAC_THREADS) void k_herm_jacobi(double* A, int n, double* V, double* w, int* order,
                                                             int max_sweeps, double tol, StepDev* st) {
    __shared__ double rc[JAC_NMAX / 2], rs[JAC_NMAX / 2], rer[JAC_NMAX / 2], rei[JAC_NMAX / 2];
    __shared__ int rp[JAC_NMAX / 2], rq[JAC_NMAX / 2];
    __shared__ int s_rot, s_done;
    __shared__ double sh[32];
    const int tid = threadIdx.x;
    const int np = n + (n & 1), half = np / 2;
    const int64_t nn = (int64_t)n * n;
    double* Ai = A + nn;
    double* Vi = V + nn;
    double tr = 0.0;
    for (int64_t e = tid; e < nn; e += JAC_THREADS) {
        const int i = (int)(e % n), j = (int)(e / n);
        V[e] = i == j ? 1.0 : 0.0;
        Vi[e] = 0.0;
        if (i == j) tr += fabs(A[e]);
    }
    // off-diagonal entries at the rounding level of the whole matrix cannot
    // be reduced further: a pair is also left alone below 4 eps sum |A_ii|
    const double abs_floor = 4.0 * 2.220446049250313e-16 * block_sum_all(tr, sh);
    if (tid == 0) s_done = 0;
    __syncthreads();
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            if (tid < half) {
                // circle method: slot 0 holds index 0, slots 1.. rotate
                auto player = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + r) % (np - 1); };
                int p = player(tid), q = player(np - 1 - tid);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
                if (q < n) {
                    const double a = A[p + (int64_t)n * p], d = A[q + (int64_t)n * q];
                    const double br = A[p + (int64_t)n * q], bi = Ai[p + (int64_t)n * q];
                    const double ab = sqrt(br * br + bi * bi);
                    if (ab > abs_floor && ab > tol * sqrt(fabs(a * d))) {
                        const double tau = (d - a) / (2.0 * ab);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        er = br / ab;   // e^{-i phi} = conj(b) / |b|
                        ei = -bi / ab;
                        s_rot = 1;
                    }
                }
                rc[tid] = c;
                rs[tid] = sn;
                rer[tid] = er;
                rei[tid] = ei;
                rp[tid] = p;
                rq[tid] = q;
            }
            __syncthreads();
            // A <- J^H A J, one 2 x 2 block (pair P rows, pair Q columns) per item
            for (int e = tid; e < half * half; e += JAC_THREADS) {
                const int P = e % half, Q = e / half;
                const int p0 = rp[P], q0 = rq[P], p1 = rp[Q], q1 = rq[Q];
                const bool rowq = q0 < n, colq = q1 < n;
                // block entries x[row][col], rows (p0, q0), columns (p1, q1)
                double xr[2][2], xi[2][2];
                const int rows[2] = {p0, q0}, cols[2] = {p1, q1};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const bool ok = (a == 0 || rowq) && (b == 0 || colq);
                        const int64_t o = rows[a] + (int64_t)n * cols[b];
                        xr[a][b] = ok ? A[o] : 0.0;
                        xi[a][b] = ok ? Ai[o] : 0.0;
                    }
                // rows: r_p = c x_p - s conj(e) x_q,  r_q = s x_p + c conj(e) x_q
                {
                    const double c = rc[P], sn = rs[P], er = rer[P], ei = -rei[P];   // conj(e)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const double qr = er * xr[1][b] - ei * xi[1][b], qi = er * xi[1][b] + ei * xr[1][b];
                        const double pr = xr[0][b], pi = xi[0][b];
                        xr[0][b] = c * pr - sn * qr;
                        xi[0][b] = c * pi - sn * qi;
                        xr[1][b] = sn * pr + c * qr;
                        xi[1][b] = sn * pi + c * qi;
                    }
                }
                // columns: k_p = c x_p - s e x_q,  k_q = s x_p + c e x_q
                {
                    const double c = rc[Q], sn = rs[Q], er = rer[Q], ei = rei[Q];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const double qr = er * xr[a][1] - ei * xi[a][1], qi = er * xi[a][1] + ei * xr[a][1];
                        const double pr = xr[a][0], pi = xi[a][0];
                        xr[a][0] = c * pr - sn * qr;
                        xi[a][0] = c * pi - sn * qi;
                        xr[a][1] = sn * pr + c * qr;
                        xi[a][1] = sn * pi + c * qi;
                    }
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        if (!((a == 0 || rowq) && (b == 0 || colq))) continue;
                        const int64_t o = rows[a] + (int64_t)n * cols[b];
                        A[o] = xr[a][b];
                        Ai[o] = xi[a][b];
                    }
            }
            // V <- V J on the columns of every pair
            for (int e = tid; e < n * half; e += JAC_THREADS) {
                const int i = e % n, Q = e / n;
                const int p1 = rp[Q], q1 = rq[Q];
                if (q1 >= n) continue;
                const double c = rc[Q], sn = rs[Q], er = rer[Q], ei = rei[Q];
                const int64_t op = i + (int64_t)n * p1, oq = i + (int64_t)n * q1;
                const double pr = V[op], pi = Vi[op], xr = V[oq], xi = Vi[oq];
                const double qr = er * xr - ei * xi, qi = er * xi + ei * xr;
                V[op] = c * pr - sn * qr;
                Vi[op] = c * pi - sn * qi;
                V[oq] = sn * pr + c * qr;
                Vi[oq] = sn * pi + c * qi;
            }
            __syncthreads();
        }
        const int rotated = s_rot;
        __syncthreads();   // every thread has read s_rot before it is reset
        if (!rotated) {
            if (tid == 0) s_done = 1;
            break;
        }
    }
    __syncthreads();
    // order[k]: the column of the k-th largest eigenvalue (ties by index)
    for (int i = tid; i < n; i += JAC_THREADS) {
        const double wi = A[i + (int64_t)n * i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double wj = A[j + (int64_t)n * j];
            rank += (wj > wi || (wj == wi && j < i)) ? 1 : 0;
        }
        order[rank] = i;
        w[rank] = wi;
    }
    if (tid == 0 && !s_done) atomicExch(&st->bad, 1);
}
}  // namespace

namespace {
// dst[c dc + s ds + p dp] = src[c sc + s ss + p sp] (conjugated if conj), for
// c < K, s < S, p < P; planar complex with the given plane distances.
__global__ void k_copy3(const double* src, int64_t src_plane, int64_t sc, int64_t ss, int64_t sp, double* dst,
                        int64_t dst_plane, int64_t dc, int64_t ds, int64_t dp, int K, int S, int P, int conj) {
    const int64_t total = (int64_t)K * S * P;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % K);
        const int64_t r = e / K;
        const int sidx = (int)(r % S), pidx = (int)(r / S);
        const int64_t i = c * sc + sidx * ss + pidx * sp, o = c * dc + sidx * ds + pidx * dp;
        dst[o] = src[i];
        dst[o + dst_plane] = conj ? -src[i + src_plane] : src[i + src_plane];
    }
}

// out[:, c] = V[:, order[c]] for c < k (n x n planar V, n x k planar out)
__global__ void k_gather_cols(const double* V, int n, const int* order, int k, double* out) {
    const int64_t total = (int64_t)n * k, nn = (int64_t)n * n, nk = (int64_t)n * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), c = (int)(e / n);
        const int64_t src = i + (int64_t)n * order[c];
        out[e] = V[src];
        out[e + nk] = V[src + nn];
    }
}

// The kept weight of a truncated split, from the descending eigenvalues w
// of its Gram matrix: kept = w_0 + .. + w_{k-1}, total = the sum of all n.
// Scales the centre tensor x (count complex entries) by sqrt(total / kept),
// restoring the norm of the untruncated tensor, and folds the discarded
// weight 1 - kept / total into the step's maximum.
__global__ void k_split_finish(const double* w, int n, int k, double* x, int64_t count, StepDev* st) {
    __shared__ double sh[8];
    double kept = 0, total = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        total += w[i];
        if (i < k) kept += w[i];
    }
    kept = block_sum_all(kept, sh);
    total = block_sum_all(total, sh);
    const double f = kept > 0.0 ? sqrt(total / kept) : 1.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        x[e] *= f;
        x[e + count] *= f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double disc = total > 0.0 ? 1.0 - kept / total : 0.0;
        if (disc < 0.0) disc = 0.0;
        if (!(kept > 0.0) || !(disc == disc)) atomicExch(&st->bad, 1);
        atomicMax(&st->max_disc_bits, (unsigned long long)__double_as_longlong(disc));
    }
}
}  // namespace

void copy3(const double* src, int64_t src_plane, int64_t sc, int64_t ss, int64_t sp, double* dst, int64_t dst_plane,
           int64_t dc, int64_t ds, int64_t dp, int K, int S, int P, bool conj, hipStream_t s) {
    if (g_dry_run) return;
    const int64_t total = (int64_t)K * S * P;
    hipLaunchKernelGGL(k_copy3, dim3(grid_for(total)), dim3(256), 0, s, src, src_plane, sc, ss, sp, dst, dst_plane, dc,
                       ds, dp, K, S, P, conj ? 1 : 0);
}

void gather_cols(const double* V, int n, const int* order, int k, double* out, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_gather_cols, dim3(grid_for((int64_t)n * k)), dim3(256), 0, s, V, n, order, k, out);
}

void split_finish(const double* w, int n, int k, double* x, int64_t count, StepDev* st, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_split_finish, dim3(grid_for(count)), dim3(256), 0, s, w, n, k, x, count, st);
}

void herm_eig(double* A, int n, double* V, double* w, int* order, StepDev* st, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_herm_jacobi, dim3(1), dim3(JAC_THREADS), 0, s, A, n, V, w, order, 60, 1e-15, st);
}

// ---------------------------------------------------------------------------
// leaf operator blocks and product-state contractions
// ---------------------------------------------------------------------------
namespace {
__global__ void k_contract_node_vec(const double* T, int DL, int DR, int DP, const double* a,
                                    const double* b, double* out) {
    __shared__ double sh[16];
    const int p = blockIdx.x;
    const int64_t n = (int64_t)DL * DR * DP;
    const int64_t LR = (int64_t)DL * DR;
    double re = 0, im = 0;
    for (int64_t e = threadIdx.x; e < LR; e += blockDim.x) {
        const int l = (int)(e % DL), r = (int)(e / DL);
        const double ar = a[l], ai = a[l + DL], br = b[r], bi = b[r + DR];
        const double abr = ar * br - ai * bi, abi = ar * bi + ai * br;
        const double tr = T[e + LR * p], ti = T[n + e + LR * p];
        re += abr * tr - abi * ti;
        im += abr * ti + abi * tr;
    }
    const double sr = block_sum(re, sh);
    const double si = block_sum(im, sh);
    if (threadIdx.x == 0) {
        out[p] = sr;
        out[p + DP] = si;
    }
}
}  // namespace

void contract_node_vec(const double* T, int DL, int DR, int DP, const double* a, const double* b,
                       double* out, hipStream_t s) {
    if (g_dry_run) return;
    hipLaunchKernelGGL(k_contract_node_vec, dim3(DP), dim3(256), 0, s, T, DL, DR, DP, a, b, out);
}

}  // namespace ttn
