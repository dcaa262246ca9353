// Complex contraction (GEMM) kernels of the TDVP library for gfx950: a tiled
// VALU fallback, the MFMA kernel and the split-K reduction, with the host-side
// dispatch cgemm().
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <initializer_list>

#include "ttn_internal.h"

namespace ttn {

namespace {

constexpr int GEMM_THREADS = 256;

template <typename R, int BM, int BN, int BK>
__global__ __launch_bounds__(GEMM_THREADS) void k_cgemm(Gemm<R> g, int tilesM, int tilesN,
                                                        int splits, int kchunk, R* partial,
                                                        int a_mfast, int b_nfast) {
    if (g.skip && *g.skip) return;
    constexpr int TM = BM / 16, TN = BN / 16;
    __shared__ R As[2][BK][BM + 1];
    __shared__ R Bs[2][BK][BN + 1];
    int64_t bid = blockIdx.x;
    const int tm = bid % tilesM;
    bid /= tilesM;
    const int tn = bid % tilesN;
    bid /= tilesN;
    const int sp = bid % splits;
    bid /= splits;
    const int b = (int)bid;
    const int b1 = b % g.B1, b2 = b / g.B1;
    const R* A = g.A + b1 * g.sab1 + b2 * g.sab2;
    const R* B = g.B + b1 * g.sbb1 + b2 * g.sbb2;
    const int m0 = tm * BM, n0 = tn * BN;
    const int K = g.Kin * g.Kout;
    const int kb = sp * kchunk;
    const int ke = min(K, kb + kchunk);
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    R acc_re[TM][TN], acc_im[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            acc_re[i][j] = 0;
            acc_im[i][j] = 0;
        }
    const R sa = g.conjA ? R(-1) : R(1);
    const R sb = g.conjB ? R(-1) : R(1);
    for (int k0 = kb; k0 < ke; k0 += BK) {
        for (int e = tid; e < BM * BK; e += GEMM_THREADS) {
            int mm, kk;
            if (a_mfast) {
                mm = e % BM;
                kk = e / BM;
            } else {
                kk = e % BK;
                mm = e / BK;
            }
            const int m = m0 + mm, k = k0 + kk;
            R re = 0, im = 0;
            if (m < g.M && k < ke) {
                const int kin = k % g.Kin, kout = k / g.Kin;
                const int64_t off = (int64_t)m * g.sam + (int64_t)kin * g.sak + (int64_t)kout * g.sako;
                re = A[off];
                im = sa * A[off + g.a_plane];
            }
            As[0][kk][mm] = re;
            As[1][kk][mm] = im;
        }
        for (int e = tid; e < BN * BK; e += GEMM_THREADS) {
            int nn, kk;
            if (b_nfast) {
                nn = e % BN;
                kk = e / BN;
            } else {
                kk = e % BK;
                nn = e / BK;
            }
            const int n = n0 + nn, k = k0 + kk;
            R re = 0, im = 0;
            if (n < g.N && k < ke) {
                const int kin = k % g.Kin, kout = k / g.Kin;
                const int64_t off = (int64_t)n * g.sbn + (int64_t)kin * g.sbk + (int64_t)kout * g.sbko;
                re = B[off];
                im = sb * B[off + g.b_plane];
            }
            Bs[0][kk][nn] = re;
            Bs[1][kk][nn] = im;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            R ar[TM], ai[TM], br[TN], bi[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                ar[i] = As[0][kk][tx + 16 * i];
                ai[i] = As[1][kk][tx + 16 * i];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                br[j] = Bs[0][kk][ty + 16 * j];
                bi[j] = Bs[1][kk][ty + 16 * j];
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    acc_re[i][j] = fma(ar[i], br[j], acc_re[i][j]);
                    acc_re[i][j] = fma(-ai[i], bi[j], acc_re[i][j]);
                    acc_im[i][j] = fma(ar[i], bi[j], acc_im[i][j]);
                    acc_im[i][j] = fma(ai[i], br[j], acc_im[i][j]);
                }
        }
        __syncthreads();
    }
    if (splits == 1) {
        R* C = g.C + b1 * g.scb1 + b2 * g.scb2;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = m0 + tx + 16 * i;
            if (m >= g.M) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + ty + 16 * j;
                if (n >= g.N) continue;
                const int64_t off = (int64_t)m * g.scm + (int64_t)n * g.scn;
                R re = g.alpha * acc_re[i][j], im = g.alpha * acc_im[i][j];
                if (g.beta) {
                    re += C[off];
                    im += C[off + g.c_plane];
                }
                C[off] = re;
                C[off + g.c_plane] = im;
            }
        }
    } else {
        const int64_t MN = (int64_t)g.M * g.N;
        const int nbatch = g.B1 * g.B2;
        R* P = partial + ((int64_t)sp * nbatch + b) * 2 * MN;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int m = m0 + tx + 16 * i;
            if (m >= g.M) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = n0 + ty + 16 * j;
                if (n >= g.N) continue;
                P[m + (int64_t)g.M * n] = acc_re[i][j];
                P[MN + m + (int64_t)g.M * n] = acc_im[i][j];
            }
        }
    }
}

// Sum of the split-K partials into C (alpha, beta applied).  G threads share
// an element (G a power of two dividing 256): thread group q sums splits q,
// q + G, ... with four loads in flight, and the G group sums meet in LDS in a
// fixed order, so the result does not depend on timing.  Blocks walk
// (batch, chunk of 256 / G elements) pairs; element indices are 32-bit
// (the host checks M N < 2^31).
template <typename R>
__global__ __launch_bounds__(256) void k_splitk_reduce(Gemm<R> g, int splits, const R* partial, int G) {
    if (g.skip && *g.skip) return;
    __shared__ R sre[256], sim[256];
    const int MN = g.M * g.N;
    const int nbatch = g.B1 * g.B2;
    const int epb = 256 / G;
    const int el = threadIdx.x % epb, grp = threadIdx.x / epb;
    const int chunks = (MN + epb - 1) / epb;
    const int64_t sstride = (int64_t)nbatch * 2 * MN;
    const bool contig = g.scm == 1 && g.scn == g.M;
    for (int64_t blk = blockIdx.x; blk < (int64_t)chunks * nbatch; blk += gridDim.x) {
        const int b = (int)(blk / chunks);
        const int mn = (int)(blk % chunks) * epb + el;
        R re = 0, im = 0;
        if (mn < MN) {
            const R* P = partial + (int64_t)b * 2 * MN + mn;
            R r4[4] = {0, 0, 0, 0}, i4[4] = {0, 0, 0, 0};
            int sp = grp;
            for (; sp + 3 * G < splits; sp += 4 * G) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    r4[u] += P[(int64_t)(sp + u * G) * sstride];
                    i4[u] += P[(int64_t)(sp + u * G) * sstride + MN];
                }
            }
            for (; sp < splits; sp += G) {
                r4[0] += P[(int64_t)sp * sstride];
                i4[0] += P[(int64_t)sp * sstride + MN];
            }
            re = (r4[0] + r4[1]) + (r4[2] + r4[3]);
            im = (i4[0] + i4[1]) + (i4[2] + i4[3]);
        }
        if (G > 1) {
            sre[threadIdx.x] = re;
            sim[threadIdx.x] = im;
            __syncthreads();
            if (grp == 0)
                for (int q = 1; q < G; ++q) {
                    re += sre[q * epb + el];
                    im += sim[q * epb + el];
                }
            __syncthreads();
        }
        if (grp == 0 && mn < MN) {
            const int b1 = b % g.B1, b2 = b / g.B1;
            R* C = g.C + b1 * g.scb1 + b2 * g.scb2;
            const int64_t off = contig ? (int64_t)mn : (int64_t)(mn % g.M) * g.scm + (int64_t)(mn / g.M) * g.scn;
            re *= g.alpha;
            im *= g.alpha;
            if (g.beta) {
                re += C[off];
                im += C[off + g.c_plane];
            }
            C[off] = re;
            C[off + g.c_plane] = im;
        }
    }
}

// k_splitk_reduce for a contiguous, 16-byte aligned output with few splits:
// each thread sums one 16-byte vector of W consecutive elements of every
// split (in split order, as the scalar kernel does with one thread per
// element) and stores it whole.
template <typename R>
__global__ __launch_bounds__(256) void k_splitk_reduce_vec(Gemm<R> g, int splits, const R* partial) {
    if (g.skip && *g.skip) return;
    constexpr int W = 16 / sizeof(R);
    typedef R V __attribute__((ext_vector_type(W)));
    const int MN = g.M * g.N, nbatch = g.B1 * g.B2;
    const int nv = MN / W;
    const int64_t sstride = (int64_t)nbatch * 2 * MN;
    const int total = nv * nbatch;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int b = e / nv, q = e - b * nv;
        const R* P = partial + (int64_t)b * 2 * MN + (int64_t)q * W;
        V re = *(const V*)P, im = *(const V*)(P + MN);
        for (int sp = 1; sp < splits; ++sp) {
            re += *(const V*)(P + sp * sstride);
            im += *(const V*)(P + sp * sstride + MN);
        }
        const int b1 = b % g.B1, b2 = b / g.B1;
        R* C = g.C + b1 * g.scb1 + b2 * g.scb2 + (int64_t)q * W;
        re *= g.alpha;
        im *= g.alpha;
        if (g.beta) {
            re += *(const V*)C;
            im += *(const V*)(C + g.c_plane);
        }
        *(V*)C = re;
        *(V*)(C + g.c_plane) = im;
    }
}

// Launch of the split-K reduction: the vector kernel for contiguous aligned
// outputs and fewer than four splits, else k_splitk_reduce with up to eight
// threads per element when the splits are many and the elements few.
template <typename R>
void splitk_reduce(const Gemm<R>& g, int splits, const R* partial, hipStream_t s) {
    const int64_t MN = (int64_t)g.M * g.N, nbatch = (int64_t)g.B1 * g.B2;
    constexpr int W = 16 / sizeof(R);
    const bool contig = g.scm == 1 && g.scn == g.M;
    if (splits < 4 && contig && MN % W == 0 && MN * nbatch / W < (1LL << 31) && (uintptr_t)g.C % 16 == 0 &&
        (uintptr_t)partial % 16 == 0 && g.c_plane % W == 0 && g.scb1 % W == 0 && g.scb2 % W == 0) {
        const int nb = (int)std::min<int64_t>((MN * nbatch / W + 255) / 256, 8192);
        hipLaunchKernelGGL((k_splitk_reduce_vec<R>), dim3(nb), dim3(256), 0, s, g, splits, partial);
        return;
    }
    int G = 1;
    while (G < 8 && splits >= 8 * 2 * G && MN * nbatch * 2 * G <= 256LL * 1024) G *= 2;
    const int64_t blocks = (MN + 256 / G - 1) / (256 / G) * nbatch;
    const int nb = (int)std::min<int64_t>(blocks, 8192);
    hipLaunchKernelGGL((k_splitk_reduce<R>), dim3(nb), dim3(256), 0, s, g, splits, partial, G);
}

// ---------------------------------------------------------------------------
// MFMA contraction kernel (gfx950).  Complex C = A B with three real
// products per complex product (Gauss): P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi), then Re C = P1 - P2 and Im C = P3 - P1 - P2 -- a
// quarter fewer matrix-core operations than the four-product form, for a
// third accumulator per output tile.  The matrix-core operands are fed
// transposed (B^T as the first, A^T as the second) so that the output lanes
// of each 16x16x4 tile run along m, the contiguous index of C.  Tiles of A
// (BM x BK) and B (BK x BN) are staged through double-buffered LDS; the next
// k-tile is fetched into registers while the current one is multiplied.  A
// k-tile never crosses a boundary of the outer contraction index
// (Kin % BK == 0).  The block holds WGM x WGN waves of (BM/WGM) x (BN/WGN)
// outputs each.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename R>
struct MfmaT;
template <>
struct MfmaT<float> {
    typedef f32x4 acc_t;
    static __device__ inline acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of register r of lane l inside the 16x16 output tile
    static __device__ inline int row(int l, int r) { return 4 * (l / 16) + r; }
    static constexpr int PAD = 16;
};
template <>
struct MfmaT<double> {
    typedef f64x4 acc_t;
    static __device__ inline acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int l, int r) { return (l / 16) + 4 * r; }
    static constexpr int PAD = 8;
};

template <typename R, int BM, int BN, int WGM, int WGN, int MINB, int BK, bool AK, bool BKF>
__global__ __launch_bounds__(64 * WGM * WGN, MINB) void k_cgemm_mfma(Gemm<R> g, int tilesM, int tilesN,
                                                                    int splits, int kchunk, R* partial) {
    if (g.skip && *g.skip) return;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TI = WM / 16, TJ = WN / 16;
    static_assert(TI >= 1 && TJ >= 1, "wave tile below 16 x 16");
    constexpr int PAD = MfmaT<R>::PAD;
    constexpr int QA = BM * BK / NT, QB = BN * BK / NT;
    static_assert(QA >= 1 && QB >= 1, "tile smaller than the block");
    typedef typename MfmaT<R>::acc_t acc_t;
    // LDS tiles [buffer][plane][row][col]: an operand whose global layout is
    // contiguous along k is staged k-contiguous with a row stride of BK + 1
    // (BK + 2 for 32-wide FP32 k-tiles: a fragment read takes rows r = 0..15
    // at k + q, q = 0..3, and 34 r + q, unlike 33 r + q, spreads over 64
    // distinct banks), so that both the coalesced stash and the MFMA fragment
    // reads hit distinct banks; the others are staged [k][index] with a pad.
    constexpr int KS = BK + ((sizeof(R) == 4 && BK == 32) ? 2 : 1);
    constexpr int AR = AK ? BM : BK, AC = AK ? KS : BM + PAD;
    constexpr int BR = BKF ? BN : BK, BC = BKF ? KS : BN + PAD;
    __shared__ R As[2][2][AR][AC];
    __shared__ R Bs[2][2][BR][BC];
    int64_t bid = blockIdx.x;
    const int tm = bid % tilesM;
    bid /= tilesM;
    const int tn = bid % tilesN;
    bid /= tilesN;
    const int sp = bid % splits;
    bid /= splits;
    const int b = (int)bid;
    const int b1 = b % g.B1, b2 = b / g.B1;
    const int m0 = tm * BM, n0 = tn * BN;
    const R* A = g.A + b1 * g.sab1 + b2 * g.sab2 + (int64_t)m0 * g.sam;
    const R* B = g.B + b1 * g.sbb1 + b2 * g.sbb2 + (int64_t)n0 * g.sbn;
    const int K = g.Kin * g.Kout;
    const int kb = sp * kchunk;
    const int ke = min(K, kb + kchunk);
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm0 = (wave % WGM) * WM, wn0 = (wave / WGM) * WN;
    const R sa = g.conjA ? R(-1) : R(1), sb = g.conjB ? R(-1) : R(1);
    const int mlim = g.M - m0, nlim = g.N - n0;

    int offA[QA], offB[QB];
    R mA[QA], mB[QB];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        const int e = tid + NT * q;
        const int mm = AK ? e / BK : e % BM, kk = AK ? e % BK : e / BM;
        const bool ok = mm < mlim;
        mA[q] = ok ? R(1) : R(0);
        offA[q] = (ok ? mm : 0) * (int)g.sam + kk * (int)g.sak;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int e = tid + NT * q;
        const int nn = BKF ? e / BK : e % BN, kk = BKF ? e % BK : e / BN;
        const bool ok = nn < nlim;
        mB[q] = ok ? R(1) : R(0);
        offB[q] = (ok ? nn : 0) * (int)g.sbn + kk * (int)g.sbk;
    }
    R pa[2][QA], pb[2][QB];
    auto fetch = [&](int k0) {
        const int kin = k0 % g.Kin, kout = k0 / g.Kin;
        const R* Ab = A + (int64_t)kin * g.sak + (int64_t)kout * g.sako;
        const R* Bb = B + (int64_t)kin * g.sbk + (int64_t)kout * g.sbko;
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            pa[0][q] = mA[q] * Ab[offA[q]];
            pa[1][q] = (sa * mA[q]) * Ab[offA[q] + g.a_plane];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            pb[0][q] = mB[q] * Bb[offB[q]];
            pb[1][q] = (sb * mB[q]) * Bb[offB[q] + g.b_plane];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const int mm = AK ? e / BK : e % BM, kk = AK ? e % BK : e / BM;
            As[buf][0][AK ? mm : kk][AK ? kk : mm] = pa[0][q];
            As[buf][1][AK ? mm : kk][AK ? kk : mm] = pa[1][q];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            const int nn = BKF ? e / BK : e % BN, kk = BKF ? e % BK : e / BN;
            Bs[buf][0][BKF ? nn : kk][BKF ? kk : nn] = pb[0][q];
            Bs[buf][1][BKF ? nn : kk][BKF ? kk : nn] = pb[1][q];
        }
    };
    acc_t c1[TI][TJ], c2[TI][TJ], c3[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            c1[i][j] = acc_t{0, 0, 0, 0};
            c2[i][j] = acc_t{0, 0, 0, 0};
            c3[i][j] = acc_t{0, 0, 0, 0};
        }
    const int nt = (ke - kb) / BK;
    if (nt > 0) {
        fetch(kb);
        stash(0);
        if (nt > 1) fetch(kb + BK);
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
        const int cur = t & 1;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + lane / 16, c16 = lane % 16;
            R br[TJ], bi[TJ], bs[TJ], ar[TI], ai[TI], as[TI];
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int bn = wn0 + 16 * j + c16;
                br[j] = BKF ? Bs[cur][0][bn][kr] : Bs[cur][0][kr][bn];
                bi[j] = BKF ? Bs[cur][1][bn][kr] : Bs[cur][1][kr][bn];
                bs[j] = br[j] + bi[j];
            }
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int am = wm0 + 16 * i + c16;
                ar[i] = AK ? As[cur][0][am][kr] : As[cur][0][kr][am];
                ai[i] = AK ? As[cur][1][am][kr] : As[cur][1][kr][am];
                as[i] = ar[i] + ai[i];
            }
            // the three products of one tile are independent: back-to-back
            // MFMAs never share an accumulator
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j) {
                    c1[i][j] = MfmaT<R>::mfma(br[j], ar[i], c1[i][j]);
                    c2[i][j] = MfmaT<R>::mfma(bi[j], ai[i], c2[i][j]);
                    c3[i][j] = MfmaT<R>::mfma(bs[j], as[i], c3[i][j]);
                }
        }
        if (t + 1 < nt) {
            stash(cur ^ 1);
            if (t + 2 < nt) fetch(kb + (t + 2) * BK);
        }
        __syncthreads();
    }
    const int64_t MN = (int64_t)g.M * g.N;
    const int nbatch = g.B1 * g.B2;
    R* C = g.C + b1 * g.scb1 + b2 * g.scb2;
    R* P = partial + ((int64_t)sp * nbatch + b) * 2 * MN;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm0 + 16 * i + lane % 16;
                const int n = n0 + wn0 + 16 * j + MfmaT<R>::row(lane, r);
                if (m >= g.M || n >= g.N) continue;
                const R vre = c1[i][j][r] - c2[i][j][r];
                const R vim = c3[i][j][r] - c1[i][j][r] - c2[i][j][r];
                if (splits == 1) {
                    const int64_t off = (int64_t)m * g.scm + (int64_t)n * g.scn;
                    R re = g.alpha * vre, im = g.alpha * vim;
                    if (g.beta) {
                        re += C[off];
                        im += C[off + g.c_plane];
                    }
                    C[off] = re;
                    C[off + g.c_plane] = im;
                } else {
                    P[m + (int64_t)g.M * n] = vre;
                    P[MN + m + (int64_t)g.M * n] = vim;
                }
            }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// BF16-split contraction (precision mode BF16x3): FP32 operands, every real
// product from bf16 pieces x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) as
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32 accumulation
// (about 16 bits of each operand; relative error near 2^-16 per product).
// The complex product takes the four real products (Re Re, Im Im, Re Im,
// Im Re): each operand is staged as four bf16 planes (Re hi, Re lo, Im hi,
// Im lo), so a matrix-core operation needs a third fewer LDS fragment bytes
// than the three-product form, whose Re + Im sums add two more planes (that
// form measured 4-13% slower on the 128^3 stages, and its sums cost accuracy:
// relative error 1e-5 against 5e-6).  Operand lane layout of the 16x16x32
// instruction: lane l holds k = 8 (l / 16) .. +7 of row (A) or column (B)
// l % 16; the output layout is that of 16x16x4.  A 128 x 128 block tile
// over WGM x WGN waves.  LDS rows are 32 bf16 (64 bytes) with the four 16-byte
// k-chunks of a row permuted by (row / 4) mod 4, so that the 16 rows of a
// fragment read fall on distinct banks; two buffers of 64 KB let the next
// k-tile be stashed while the current one is multiplied (one barrier per
// k-tile).
// ---------------------------------------------------------------------------
template <int WGM, int WGN, bool AK, bool BKF>
__global__ __launch_bounds__(64 * WGM * WGN, 1) void k_cgemm_bf16x3(Gemm<float> g, int tilesM, int tilesN,
                                                                    int splits, int kchunk, float* partial, int vec) {
    if (g.skip && *g.skip) return;
    constexpr int BM = 128, BN = 128, NT = 64 * WGM * WGN, BK = 32;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TI = WM / 16, TJ = WN / 16;
    constexpr int QA = BM * BK / (4 * NT), QB = BN * BK / (4 * NT);
    static_assert(QA >= 1 && QB >= 1, "tile smaller than the block");
    typedef f32x4 acc_t;
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) __bf16 As[2][4][BM][BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][4][BN][BK];
    int64_t bid = blockIdx.x;
    const int tm = bid % tilesM;
    bid /= tilesM;
    const int tn = bid % tilesN;
    bid /= tilesN;
    const int sp = bid % splits;
    bid /= splits;
    const int b = (int)bid;
    const int b1 = b % g.B1, b2 = b / g.B1;
    const int m0 = tm * BM, n0 = tn * BN;
    const float* A = g.A + b1 * g.sab1 + b2 * g.sab2 + (int64_t)m0 * g.sam;
    const float* B = g.B + b1 * g.sbb1 + b2 * g.sbb2 + (int64_t)n0 * g.sbn;
    const int K = g.Kin * g.Kout;
    const int kb = sp * kchunk;
    const int ke = min(K, kb + kchunk);
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm0 = (wave % WGM) * WM, wn0 = (wave / WGM) * WN;
    const float sa = g.conjA ? -1.0f : 1.0f, sb = g.conjB ? -1.0f : 1.0f;
    const int mlim = g.M - m0, nlim = g.N - n0;
    // slot e (< 1024) of a 128-row tile -> row and k-quad (k = 4 kq .. 4 kq +
    // 3): a k-fast operand takes eight consecutive slots per row (one row =
    // 128 contiguous bytes); an index-fast one takes 32 consecutive rows per
    // k pair
    auto slot = [&](int e, bool kfast, int& row, int& kq) {
        if (kfast) {
            row = e / (BK / 4);
            kq = e % (BK / 4);
        } else {
            row = e % 32 + 32 * ((e / 64) % 4);
            kq = (e / 32) % 2 + 2 * (e / 256);
        }
    };
    // element offset of (row, k) inside a [rows][32] plane: the 16-byte chunk
    // k / 8 moves to chunk (k / 8) ^ ((row / 4) % 4)
    auto lds_off = [](int row, int k) { return row * BK + ((((k >> 3) ^ (row >> 2)) & 3) << 3) + (k & 7); };
    int offA[QA], offB[QB];
    float mA[QA], mB[QB];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        int mm, kq;
        slot(tid + NT * q, AK, mm, kq);
        const bool ok = mm < mlim;
        mA[q] = ok ? 1.0f : 0.0f;
        offA[q] = (ok ? mm : 0) * (int)g.sam + 4 * kq * (int)g.sak;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        int nn, kq;
        slot(tid + NT * q, BKF, nn, kq);
        const bool ok = nn < nlim;
        mB[q] = ok ? 1.0f : 0.0f;
        offB[q] = (ok ? nn : 0) * (int)g.sbn + 4 * kq * (int)g.sbk;
    }
    float pa[8][QA], pb[8][QB];   // [re k .. k+3, im k .. k+3]
    auto fetch = [&](int k0) {
        const int kin = k0 % g.Kin, kout = k0 / g.Kin;
        const float* Ab = A + (int64_t)kin * g.sak + (int64_t)kout * g.sako;
        const float* Bb = B + (int64_t)kin * g.sbk + (int64_t)kout * g.sbko;
        const int ka = (int)g.sak, kbs = (int)g.sbk;
        const bool va = AK && (vec & 1), vb = BKF && (vec & 2);
#pragma unroll
        for (int q = 0; q < QA; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float* src = Ab + offA[q] + (h ? g.a_plane : 0);
                const float sc = h ? sa * mA[q] : mA[q];
                if (va) {
                    const float4 t4 = *(const float4*)src;
                    pa[4 * h][q] = sc * t4.x;
                    pa[4 * h + 1][q] = sc * t4.y;
                    pa[4 * h + 2][q] = sc * t4.z;
                    pa[4 * h + 3][q] = sc * t4.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) pa[4 * h + j][q] = sc * src[j * ka];
                }
            }
#pragma unroll
        for (int q = 0; q < QB; ++q)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float* src = Bb + offB[q] + (h ? g.b_plane : 0);
                const float sc = h ? sb * mB[q] : mB[q];
                if (vb) {
                    const float4 t4 = *(const float4*)src;
                    pb[4 * h][q] = sc * t4.x;
                    pb[4 * h + 1][q] = sc * t4.y;
                    pb[4 * h + 2][q] = sc * t4.z;
                    pb[4 * h + 3][q] = sc * t4.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) pb[4 * h + j][q] = sc * src[j * kbs];
                }
            }
    };
    auto put = [](__bf16* hi_dst, __bf16* lo_dst, float x0, float x1, float x2, float x3) {
        const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1, h2 = (__bf16)x2, h3 = (__bf16)x3;
        *(bf16x4*)hi_dst = bf16x4{h0, h1, h2, h3};
        *(bf16x4*)lo_dst = bf16x4{(__bf16)(x0 - (float)h0), (__bf16)(x1 - (float)h1), (__bf16)(x2 - (float)h2),
                                  (__bf16)(x3 - (float)h3)};
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            int mm, kq;
            slot(tid + NT * q, AK, mm, kq);
            const int o = lds_off(mm, 4 * kq);
            put(&As[buf][0][0][0] + o, &As[buf][1][0][0] + o, pa[0][q], pa[1][q], pa[2][q], pa[3][q]);
            put(&As[buf][2][0][0] + o, &As[buf][3][0][0] + o, pa[4][q], pa[5][q], pa[6][q], pa[7][q]);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            int nn, kq;
            slot(tid + NT * q, BKF, nn, kq);
            const int o = lds_off(nn, 4 * kq);
            put(&Bs[buf][0][0][0] + o, &Bs[buf][1][0][0] + o, pb[0][q], pb[1][q], pb[2][q], pb[3][q]);
            put(&Bs[buf][2][0][0] + o, &Bs[buf][3][0][0] + o, pb[4][q], pb[5][q], pb[6][q], pb[7][q]);
        }
    };
    acc_t crr[TI][TJ], cii[TI][TJ], cim[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            crr[i][j] = acc_t{0, 0, 0, 0};
            cii[i][j] = acc_t{0, 0, 0, 0};
            cim[i][j] = acc_t{0, 0, 0, 0};
        }
    const int nt = (ke - kb) / BK;
    const int kg = 8 * (lane / 16), c16 = lane % 16;
    if (nt > 0) {
        fetch(kb);
        stash(0);
        if (nt > 1) fetch(kb + BK);
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
        const int cur = t & 1;
        bf16x8 bf[TJ][4];
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int o = lds_off(wn0 + 16 * j + c16, kg);
#pragma unroll
            for (int p = 0; p < 4; ++p) bf[j][p] = *(const bf16x8*)(&Bs[cur][p][0][0] + o);
        }
#pragma unroll
        for (int i = 0; i < TI; ++i) {
            bf16x8 af[4];
            const int o = lds_off(wm0 + 16 * i + c16, kg);
#pragma unroll
            for (int p = 0; p < 4; ++p) af[p] = *(const bf16x8*)(&As[cur][p][0][0] + o);
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                // planes: 0 Re hi, 1 Re lo, 2 Im hi, 3 Im lo; each real product
                // hi*hi + lo*hi + hi*lo
                crr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][0], af[0], crr[i][j], 0, 0, 0);
                cii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][2], af[2], cii[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][2], af[0], cim[i][j], 0, 0, 0);
                crr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][1], af[0], crr[i][j], 0, 0, 0);
                cii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][3], af[2], cii[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][3], af[0], cim[i][j], 0, 0, 0);
                crr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][0], af[1], crr[i][j], 0, 0, 0);
                cii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][2], af[3], cii[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][2], af[1], cim[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][0], af[2], cim[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][1], af[2], cim[i][j], 0, 0, 0);
                cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j][0], af[3], cim[i][j], 0, 0, 0);
            }
        }
        if (t + 1 < nt) {
            stash(cur ^ 1);
            if (t + 2 < nt) fetch(kb + (t + 2) * BK);
        }
        __syncthreads();
    }
    const int64_t MN = (int64_t)g.M * g.N;
    const int nbatch = g.B1 * g.B2;
    float* C = g.C + b1 * g.scb1 + b2 * g.scb2;
    float* P = partial + ((int64_t)sp * nbatch + b) * 2 * MN;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm0 + 16 * i + c16;
                const int n = n0 + wn0 + 16 * j + 4 * (lane / 16) + r;
                if (m >= g.M || n >= g.N) continue;
                const float vre = crr[i][j][r] - cii[i][j][r];
                const float vim = cim[i][j][r];
                if (splits == 1) {
                    const int64_t off = (int64_t)m * g.scm + (int64_t)n * g.scn;
                    float re = g.alpha * vre, im = g.alpha * vim;
                    if (g.beta) {
                        re += C[off];
                        im += C[off + g.c_plane];
                    }
                    C[off] = re;
                    C[off + g.c_plane] = im;
                } else {
                    P[m + (int64_t)g.M * n] = vre;
                    P[MN + m + (int64_t)g.M * n] = vim;
                }
            }
}

// Largest element offset an operand can touch (all strides are >= 0).
inline bool inside(const GemmScratch& ws, const void* base, int64_t max_off, int64_t plane, int esz) {
    if (!ws.regions) return true;
    const uintptr_t p = (uintptr_t)base;
    int lo = 0, hi = ws.n_regions - 1, f = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) / 2;
        if (ws.regions[mid].lo <= p) {
            f = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    if (f < 0) return false;
    const uintptr_t end = p + (uintptr_t)(max_off + plane + 1) * esz;
    return p >= ws.regions[f].lo && end <= ws.regions[f].hi;
}

}  // namespace

bool g_dry_run = false;

template <typename R>
bool cgemm(const Gemm<R>& g, const GemmScratch& ws, hipStream_t s, char* why, int whylen, hipEvent_t ev0,
           hipEvent_t ev1, CgemmInfo* info) {
    if (info) *info = CgemmInfo{};
    if (g.M <= 0 || g.N <= 0 || g.B1 * g.B2 <= 0) return true;
    {
        const int64_t km = g.Kin > 0 ? g.Kin - 1 : 0, ko = g.Kout > 0 ? g.Kout - 1 : 0;
        const int64_t b1 = g.B1 - 1, b2 = g.B2 - 1;
        const int64_t amax = (g.M - 1) * g.sam + km * g.sak + ko * g.sako + b1 * g.sab1 + b2 * g.sab2;
        const int64_t bmax = (g.N - 1) * g.sbn + km * g.sbk + ko * g.sbko + b1 * g.sbb1 + b2 * g.sbb2;
        const int64_t cmax = (g.M - 1) * g.scm + (g.N - 1) * g.scn + b1 * g.scb1 + b2 * g.scb2;
        const bool neg = g.sam < 0 || g.sak < 0 || g.sako < 0 || g.sab1 < 0 || g.sab2 < 0 || g.sbn < 0 ||
                         g.sbk < 0 || g.sbko < 0 || g.sbb1 < 0 || g.sbb2 < 0 || g.scm < 0 || g.scn < 0 ||
                         g.scb1 < 0 || g.scb2 < 0 || g.a_plane < 0 || g.b_plane < 0 || g.c_plane < 0;
        const char* bad = neg ? "negative stride"
                          : !inside(ws, g.A, amax, g.a_plane, sizeof(R)) ? "operand A out of its region"
                          : !inside(ws, g.B, bmax, g.b_plane, sizeof(R)) ? "operand B out of its region"
                          : !inside(ws, g.C, cmax, g.c_plane, sizeof(R)) ? "operand C out of its region"
                                                                         : nullptr;
        if (bad) {
            if (why)
                snprintf(why, whylen, "%s (M=%d N=%d Kin=%d Kout=%d B=%dx%d)", bad, g.M, g.N, g.Kin, g.Kout,
                         g.B1, g.B2);
            return false;
        }
    }
    if (g_dry_run) return true;
    const int K = g.Kin * g.Kout;
    const int64_t nbatch = (int64_t)g.B1 * g.B2;
    const bool a_k = g.sak == 1 && g.sam != 1, b_k = g.sbk == 1 && g.sbn != 1;
    // per-element offsets inside a tile are 32-bit in the MFMA kernel
    const bool off32 = (int64_t)128 * (g.sam + g.sbn) + 32 * (g.sak + g.sbk) + g.a_plane + g.b_plane < (1LL << 31);
    const bool mfma_ok = K >= 16 && g.Kin % 16 == 0 && g.M >= 16 && g.N >= 16 && (g.sam == 1 || g.sak == 1) &&
                         (g.sbn == 1 || g.sbk == 1) && off32;
    if (mfma_ok) {
        // tile choice: the large tiles, unless their grid (after split-K) would
        // leave more than half of the 256 CUs idle; then the small tiles, whose
        // grid is four times larger and whose splits may be finer
        struct Plan {
            bool large;
            int bm, bn, kq, tilesM, tilesN, splits;
            int64_t tiles;
        };
        auto plan = [&](bool large) {
            Plan p;
            p.large = large;
            p.bm = large ? 128 : 64;
            p.bn = large ? (sizeof(R) == 4 ? 128 : 64) : 64;
            // FP32 large tiles take 32-wide k-tiles (half the barriers) where
            // the inner contraction extent allows them
            p.kq = (sizeof(R) == 4 && large && g.Kin % 32 == 0) ? 32 : 16;
            p.tilesM = (g.M + p.bm - 1) / p.bm;
            p.tilesN = (g.N + p.bn - 1) / p.bn;
            p.tiles = (int64_t)p.tilesM * p.tilesN * nbatch;
            p.splits = 1;
            const int ktiles = K / 16;
            // split K until the grid covers the chip once: 256 workgroups of the
            // large tiles (one resident per CU), 512 of the small ones (two per
            // CU); a split keeps at least four 16-wide k-tiles (large) or two
            const int64_t target = large ? 256 : 512;
            const int minkt = large ? 4 : 2;
            if (p.tiles < 256 && ktiles >= 2 * minkt && (int64_t)g.M * g.N < (1LL << 31)) {
                p.splits = (int)std::min<int64_t>((target + p.tiles - 1) / p.tiles, ktiles / minkt);
                const int64_t per = 2 * (int64_t)g.M * g.N * nbatch * (int64_t)sizeof(R);
                const int64_t cap = per > 0 ? ws.bytes / per : 1;
                if (p.splits > cap) p.splits = (int)cap;
                if (p.splits < 1) p.splits = 1;
            }
            return p;
        };
        Plan pl = plan(g.M >= 128 && g.N >= (sizeof(R) == 4 ? 128 : 64));
        if (pl.large && pl.tiles * pl.splits < 128) pl = plan(false);
        const bool big = pl.large;
        const int BM = pl.bm, kq = pl.kq, tilesM = pl.tilesM, tilesN = pl.tilesN;
        const int64_t tiles = pl.tiles;
        int splits = pl.splits;
        const bool bf16 = sizeof(R) == 4 && g.split && big && kq == 32;
        int kchunk = K;
        if (splits > 1) {
            kchunk = ((K / kq + splits - 1) / splits) * kq;
            splits = (K + kchunk - 1) / kchunk;
        }
        const dim3 grid((unsigned)(tiles * splits));
        R* part = (R*)ws.partial;
        if (info) *info = CgemmInfo{bf16 ? 3 : 2, splits};
        // BF16 path: k-fast operands whose k quads are 16-byte aligned load
        // them as one vector (k tiles start at multiples of 32 in Kin)
        auto quads = [](const void* p, std::initializer_list<int64_t> strides) {
            if ((uintptr_t)p % 16) return false;
            for (int64_t st : strides)
                if (st % 4) return false;
            return true;
        };
        const int vec = (a_k && quads(g.A, {g.sam, g.sako, g.sab1, g.sab2, g.a_plane}) ? 1 : 0) |
                        (b_k && quads(g.B, {g.sbn, g.sbko, g.sbb1, g.sbb2, g.b_plane}) ? 2 : 0);
        if (ev0) (void)hipEventRecord(ev0, s);
#define TTN_MFMA_LAUNCH(bm, bn, wgm, wgn, minb, bk)                                                        \
    do {                                                                                                   \
        const dim3 blk(64 * wgm * wgn);                                                                    \
        if (a_k && b_k)                                                                                    \
            hipLaunchKernelGGL((k_cgemm_mfma<R, bm, bn, wgm, wgn, minb, bk, true, true>), grid, blk, 0, s,   \
                               g, tilesM, tilesN, splits, kchunk, part);                                   \
        else if (a_k)                                                                                      \
            hipLaunchKernelGGL((k_cgemm_mfma<R, bm, bn, wgm, wgn, minb, bk, true, false>), grid, blk, 0, s,  \
                               g, tilesM, tilesN, splits, kchunk, part);                                   \
        else if (b_k)                                                                                      \
            hipLaunchKernelGGL((k_cgemm_mfma<R, bm, bn, wgm, wgn, minb, bk, false, true>), grid, blk, 0, s,  \
                               g, tilesM, tilesN, splits, kchunk, part);                                   \
        else                                                                                               \
            hipLaunchKernelGGL((k_cgemm_mfma<R, bm, bn, wgm, wgn, minb, bk, false, false>), grid, blk, 0, s, \
                               g, tilesM, tilesN, splits, kchunk, part);                                   \
    } while (0)
        // large tiles: 16 waves (4 x 4) per block, one block per CU (FP32 waves
        // own 32 x 32 outputs, FP64 waves 32 x 16); small tiles: 4 waves
        // (2 x 2), two blocks per CU
        if constexpr (sizeof(R) == 4) {
            // BF16x3 mode: the large tiles with 32-wide k-tiles take the split
            // products; the small shapes stay FP32
            if (bf16) {
                // 8 waves (2 x 4) of 64 x 32 outputs
                const dim3 blk(512);
                if (a_k && b_k)
                    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 4, true, true>), grid, blk, 0, s, g, tilesM, tilesN,
                                       splits, kchunk, part, vec);
                else if (a_k)
                    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 4, true, false>), grid, blk, 0, s, g, tilesM, tilesN,
                                       splits, kchunk, part, vec);
                else if (b_k)
                    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 4, false, true>), grid, blk, 0, s, g, tilesM, tilesN,
                                       splits, kchunk, part, vec);
                else
                    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 4, false, false>), grid, blk, 0, s, g, tilesM, tilesN,
                                       splits, kchunk, part, vec);
            }
            else if (BM == 128 && kq == 32)
                TTN_MFMA_LAUNCH(128, 128, 4, 4, 1, 32);
            else if (BM == 128)
                TTN_MFMA_LAUNCH(128, 128, 4, 4, 1, 16);
            else
                TTN_MFMA_LAUNCH(64, 64, 2, 2, 2, 16);
        } else {
            if (BM == 128)
                TTN_MFMA_LAUNCH(128, 64, 4, 4, 1, 16);
            else
                TTN_MFMA_LAUNCH(64, 64, 2, 2, 2, 16);
        }
#undef TTN_MFMA_LAUNCH
        if (splits > 1) {
            splitk_reduce(g, splits, (const R*)ws.partial, s);
        }
        // the timing window closes after the split-K reduction: a launch's
        // time is the main kernel plus its reduction
        if (ev1) (void)hipEventRecord(ev1, s);
        return true;
    }
    constexpr int BM = 64, BN = 64, BK = 16;
    const int tilesM = (g.M + BM - 1) / BM, tilesN = (g.N + BN - 1) / BN;
    const int64_t tiles = (int64_t)tilesM * tilesN * nbatch;
    int splits = 1;
    if (K > 0 && tiles < 256 && K > 8 * BK && (int64_t)g.M * g.N < (1LL << 31)) {
        splits = (int)std::min<int64_t>((512 + tiles - 1) / tiles, K / (4 * BK));
        const int64_t per = 2 * (int64_t)g.M * g.N * nbatch * (int64_t)sizeof(R);
        const int64_t cap = per > 0 ? ws.bytes / per : 1;
        if (splits > cap) splits = (int)cap;
        if (splits < 1) splits = 1;
    }
    int kchunk = K;
    if (splits > 1) {
        kchunk = ((K + splits - 1) / splits + BK - 1) / BK * BK;
        splits = (K + kchunk - 1) / kchunk;
    }
    if (K == 0) kchunk = 0;
    const int a_mfast = (g.sam == 1 || g.sak != 1) ? 1 : 0;
    const int b_nfast = (g.sbn == 1 || g.sbk != 1) ? 1 : 0;
    const int64_t blocks = tiles * splits;
    if (info) *info = CgemmInfo{1, splits};
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL((k_cgemm<R, BM, BN, BK>), dim3((unsigned)blocks), dim3(GEMM_THREADS), 0, s, g,
                       tilesM, tilesN, splits, kchunk, (R*)ws.partial, a_mfast, b_nfast);
    if (splits > 1) {
        splitk_reduce(g, splits, (const R*)ws.partial, s);
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    return true;
}

template bool cgemm<double>(const Gemm<double>&, const GemmScratch&, hipStream_t, char*, int, hipEvent_t,
                            hipEvent_t, CgemmInfo*);
template bool cgemm<float>(const Gemm<float>&, const GemmScratch&, hipStream_t, char*, int, hipEvent_t,
                           hipEvent_t, CgemmInfo*);

}  // namespace ttn
