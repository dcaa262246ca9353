// Internal interfaces of the TTN/TDVP device library (gfx950).
//
// Storage convention: a complex array of n elements is n real parts followed
// by n imaginary parts ("planar"); stacks of such arrays are concatenated,
// so slot k of a stack of n-element arrays starts at 2*n*k.
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>

#include <cstdint>

namespace ttn {

constexpr int KRYLOV_MAX = 16;

// Strided, batched, planar-complex GEMM:
//   C[m, n] = alpha * sum_k opA[m, k] opB[k, n] + beta * C[m, n]
// with k = k_in + Kin * k_out (two-level contraction index) and batch
// b = b1 + B1 * b2.  Offsets are in real elements; *_plane is the distance
// from a real part to its imaginary part.
template <typename R>
struct Gemm {
    int M = 0, N = 0, Kin = 1, Kout = 1, B1 = 1, B2 = 1;
    const R* A = nullptr;
    int64_t a_plane = 0, sam = 0, sak = 0, sako = 0, sab1 = 0, sab2 = 0;
    bool conjA = false;
    const R* B = nullptr;
    int64_t b_plane = 0, sbk = 0, sbko = 0, sbn = 0, sbb1 = 0, sbb2 = 0;
    bool conjB = false;
    R* C = nullptr;
    int64_t c_plane = 0, scm = 0, scn = 0, scb1 = 0, scb2 = 0;
    R alpha = 1;
    int beta = 0;                 // 0 overwrite, 1 accumulate
    const int* skip = nullptr;    // device flag: launch is a no-op when set
    int split = 0;                // FP32 only: products from bf16 hi/lo splits (BF16x3)
};

// A device allocation [lo, hi) of the workspace, for launch extent checks.
struct Region {
    uintptr_t lo, hi;
};

// Scratch for split-K partial sums (real elements) owned by the engine, and
// the table of workspace regions every GEMM operand must stay inside.
struct GemmScratch {
    void* partial = nullptr;
    int64_t bytes = 0;
    const Region* regions = nullptr;   // sorted by lo
    int n_regions = 0;
};

// What a cgemm call launched: the kernel (1 the VALU tile kernel k_cgemm,
// 2 the MFMA kernel k_cgemm_mfma, 3 the BF16x3 kernel k_cgemm_bf16x3) and
// the split-K factor (> 1: a k_splitk_reduce* launch follows).
struct CgemmInfo {
    int kernel = 0;
    int splits = 0;
};

// Validates every operand extent against the region table and launches.
// Returns false (and launches nothing) when an operand would leave its
// region; `why` receives a description.  ev_begin / ev_end (optional) are
// recorded before the main kernel and after its split-K reduction.
template <typename R>
bool cgemm(const Gemm<R>& g, const GemmScratch& ws, hipStream_t s, char* why, int whylen,
           hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr, CgemmInfo* info = nullptr);

// When set, launchers validate but enqueue nothing (plan checking without a
// device).
extern bool g_dry_run;

// Lanczos state kept on the device so that no host round trip is needed.
struct LanczosDev {
    double beta0;
    double alpha[KRYLOV_MAX];
    double beta[KRYLOV_MAX];
    double c[2 * KRYLOV_MAX];
    double y[2 * KRYLOV_MAX];
    int m_eff;
    int done;
    int zero;
    int nonherm;     // Arnoldi: keep the whole Hessenberg projection in hs
    // hs[2 (j KRYLOV_MAX + i)] = H[i][j] (re, im) for i <= j (Arnoldi only;
    // the subdiagonal is beta)
    double hs[2 * KRYLOV_MAX * KRYLOV_MAX];
};

// Step-level device flags and statistics.
struct StepDev {
    int bad;                 // non-zero after a failed Cholesky pivot / NaN
    int min_krylov;
    unsigned long long min_rdiag_bits;   // positive double as ordered bits
    unsigned long long max_disc_bits;    // non-negative double as ordered bits
    double scratch[8];
};

// Krylov bases of the general Lanczos path are stored in chunks of KCH
// elements: element i of slot k, plane p (0 re, 1 im) at
// (i / KCH) S + (2 k + p) KCH + i % KCH, with chunk stride S = 2 KCH (slots);
// a projection pass then reads one contiguous stretch per chunk rather than
// 2 (k + 1) separate streams (measured 6.0 against 4.7 TB/s on 12 vectors of
// 2^21 elements).  S = 0 marks a planar vector (slot stride 2 n).
constexpr int KCH = 256;
__host__ __device__ inline int64_t kch_ofs(int64_t i, int64_t S) { return (i / KCH) * S + (i % KCH); }
// element e < 2 n of a planar vector (e >= n: imaginary part) in a chunked slot
__host__ __device__ inline int64_t kch_elem(int64_t e, int64_t n, int64_t S) {
    const int64_t p = e >= n ? 1 : 0;
    return kch_ofs(e - p * n, S) + p * KCH;
}
inline int64_t kch_pad(int64_t n) { return (n + KCH - 1) / KCH * KCH; }
// planar copy of the first `slots` vectors of a chunked basis
void krylov_unchunk(const double* V, int64_t S, int64_t n, int slots, double* out, const int* skip, hipStream_t s);

// reductions / vector kernels (double master vectors)
// nonherm != 0 starts an Arnoldi basis (non-Hermitian operator): the
// projections of both Gram-Schmidt passes are kept as Hessenberg columns and
// lz_expm exponentiates the Hessenberg matrix instead of the tridiagonal one
// v0f != nullptr also receives v0 in FP32 (the next mixed matvec's input)
// v0 planar (S == 0) or slot 0 of a chunked basis
void lz_start(const double* x, int64_t n, double* v0, int64_t S, LanczosDev* lz, double* partial, int nb,
              hipStream_t s, int nonherm = 0, float* v0f = nullptr);
// Reductions over at most LZ_FUSE_NB blocks may take their totals inside the
// next kernel of the iteration (every block sums the block partials itself),
// which saves the one-block total kernels; their partials alternate between
// `partial` and partial + LZ_PARTIAL_HALF (the reduction buffer holds both).
constexpr int LZ_FUSE_NB = 256;
constexpr int64_t LZ_PARTIAL_HALF = (int64_t)LZ_FUSE_NB * 2 * KRYLOV_MAX;
// wf != nullptr: w is first written from the FP32 matvec output wf (widened);
// total = false leaves the projections as block partials for a fused
// lz_subtract_project
// V: chunked basis (chunk stride S) or planar vectors (S == 0); vnext: a slot of V
void lz_project(const double* V, int64_t S, int kcount, const double* w, int64_t n, double* partial, int nb,
                LanczosDev* lz, int alpha_index, hipStream_t s, const float* wf = nullptr, bool total = true);
// w -= V c, then c <- V^H w (second Gram-Schmidt pass), fused
void lz_subtract_project(const double* V, int64_t S, int kcount, double* w, int64_t n, double* partial, int nb,
                         LanczosDev* lz, hipStream_t s, bool fuse = false);
// w -= V c, then beta_j = ||w||, breakdown test, v_{j+1} = w / beta_j
void lz_subtract_next(const double* V, int64_t S, int kcount, double* w, int64_t n, double* vnext, LanczosDev* lz,
                      int j, double* partial, int nb, double tol, hipStream_t s, float* vnextf = nullptr,
                      bool fuse = false);
// a whole iteration after the matvec (projection, two Gram-Schmidt passes,
// beta_j and breakdown, v_{j+1}) in one block, for n <= LZ_SMALL_N
constexpr int64_t LZ_SMALL_N = 1024;
void lz_iter_small(double* V, int j, int m, double* w, int64_t n, LanczosDev* lz, double tol, hipStream_t s);
void lz_expm(LanczosDev* lz, double tau, StepDev* st, hipStream_t s);
// x <- exp(-i tau Op) x in one workgroup for small operators (the four
// matvec stages, Krylov recursion with two Gram-Schmidt passes, exponential
// and recombination, all in LDS, FP64): usable when n = DL DR DP <=
// SMALL_EVOLVE_N and small_evolve_doubles(...) <= SMALL_EVOLVE_POOL.
// L: [1 + sL] left stack; R: right stack (only its N_j slots are read, and
// only when W != nullptr); B: [1 + sL] right-leg stack or nullptr; W:
// [1 + sL + sR] parent-leg stack or nullptr (the root).
constexpr int64_t SMALL_EVOLVE_N = 1024;
constexpr int SMALL_EVOLVE_POOL = 16384;   // doubles of LDS for vectors and stacks
int64_t small_evolve_doubles(int DL, int DR, int DP, int sL, int sR, int m, bool hasB, bool hasW);
void small_evolve(const double* L, const double* R, const double* B, const double* W, int DL, int DR, int DP,
                  int sL, int sR, int m, double tau, double tol, bool nonherm, double* x, StepDev* st,
                  hipStream_t s);
// V planar (S == 0, the small path) or chunked with stride S
void lz_combine(const double* V, int64_t S, int64_t n, double* out, LanczosDev* lz, hipStream_t s);

// conversions and copies
void convert_d2f(const double* x, float* y, int64_t count, const int* skip, hipStream_t s);
// several FP64 -> FP32 conversions in one launch (null or empty items
// skipped); an item with eye = D > 0 writes the planar D x D identity
// (count 2 D^2) instead of converting x
struct D2FItem {
    const double* x;
    float* y;
    int64_t count;
    int eye = 0;
};
constexpr int D2F_MAX = 10;
struct D2FBatch {
    const double* x[D2F_MAX];
    float* y[D2F_MAX];
    int64_t c[D2F_MAX];
    int eye[D2F_MAX];
    int n;
};
void convert_d2f_many(std::initializer_list<D2FItem> items, const int* skip, hipStream_t s);
void convert_f2d(const float* x, double* y, int64_t count, const int* skip, hipStream_t s);
void copy_d(const double* x, double* y, int64_t count, const int* skip, hipStream_t s);
void transpose_c(const double* x, double* y, int rows, int cols, hipStream_t s);
void fill_zero_d(double* y, int64_t count, hipStream_t s);
// out_k = (in_k + in_k^H) / 2 for `count` planar D x D FP32 matrices, into FP64;
// with raw_first the first matrix is converted unchanged (a non-Hermitian block)
void herm_f2d(const float* in, double* out, int D, int count, hipStream_t s, bool raw_first = false);
// dst = sum_{k < count} src_k for planar D x D FP64 matrices stored one after another
void sum_mats(const double* src, int D, int count, double* dst, hipStream_t s);

// Eigenvalues (descending, w[k]) and eigenvectors (columns order[k] of V) of
// a Hermitian n x n matrix A (planar, column-major; destroyed), n <= JAC_NMAX,
// by cyclic Jacobi in one workgroup; st->bad when it does not converge.
constexpr int JAC_NMAX = 256;
void herm_eig(double* A, int n, double* V, double* w, int* order, StepDev* st, hipStream_t s);
// dst[c dc + s ds + p dp] = (conj) src[c sc + s ss + p sp], c < K, s < S, p < P
void copy3(const double* src, int64_t src_plane, int64_t sc, int64_t ss, int64_t sp, double* dst, int64_t dst_plane,
           int64_t dc, int64_t ds, int64_t dp, int K, int S, int P, bool conj, hipStream_t s);
// out[:, c] = V[:, order[c]], c < k
void gather_cols(const double* V, int n, const int* order, int k, double* out, hipStream_t s);
// scales the centre x (count complex) of a split by sqrt(total / kept) of the
// descending Gram eigenvalues w (n of them, k kept); records the discarded
// weight 1 - kept / total in st->max_disc_bits
void split_finish(const double* w, int n, int k, double* x, int64_t count, StepDev* st, hipStream_t s);

// min over k of Re R[k][k] into st->min_rdiag_bits (R: D x D planar)
void rdiag_min(const double* R, int D, StepDev* st, hipStream_t s);
// Cholesky of a Hermitian D x D Gram matrix G (planar, column-major):
// G = L L^H.  Writes Linv (lower, L^{-1}) and R = L^H (upper), or R = L^H * Rprev
// when Rprev != nullptr (D > 128 only).  Sets st->bad on a non-positive pivot.
// work: 2 Dp^2 doubles (Dp = 16 ceil(D / 16)) for D <= 128, else
// D (D + 1) + 32 D.
void chol_inv(const double* G, int D, double* Linv, double* R, const double* Rprev, double* work,
              StepDev* st, hipStream_t s);

// out[p] = sum_{l,r} a[l] b[r] T[l, r, p] (planar complex vectors); used for
// overlaps with product states.
void contract_node_vec(const double* T, int DL, int DR, int DP, const double* a, const double* b,
                       double* out, hipStream_t s);

}  // namespace ttn
