// Host orchestration of single-site TDVP on a binary tree tensor network
// (arXiv 2210.03763, Sec. "Tensor network simulations") and the C ABI of
// include/ttn.h.  Every arithmetic step on the state runs in the device
// kernels of kernels.hip; the host only walks the tree and enqueues work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ttn.h"
#include "ttn_internal.h"

using namespace ttn;

namespace {

constexpr double LANCZOS_TOL = 1e-12;     // beta_{j+1} <= tol (|alpha_j| + beta_j)
constexpr double COMPLETION_TOL = 1e-8;   // Gram-Schmidt acceptance for initial isometries
// workgroups of the Lanczos reductions over long vectors (four per CU): on
// 2^21-element vectors 1024 measured a little faster than 1536 or 2048 (the
// single-workgroup final sums shrink), 4096 and 8192 slower
constexpr int RED_BLOCKS = 1024;

struct StatusError {
    int code;
    std::string msg;
};

#define HIPCHECK(x)                                                                       \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess)                                                             \
            throw StatusError{TTN_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures.
struct Bump {
    char* base;
    size_t off = 0, cap;
    std::vector<Region>* regions;
    Bump(void* b, size_t c, std::vector<Region>* r = nullptr) : base((char*)b), cap(c), regions(r) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        if (regions && base) regions->push_back(Region{(uintptr_t)p, (uintptr_t)p + count * sizeof(T)});
        off += count * sizeof(T);
        if (base && off > cap) throw StatusError{TTN_ENOMEM, "workspace too small"};
        return p;
    }
};

struct AdjState;   // reverse-mode state (adjoint.inc)

struct Event {
    int step, site;
    double* U;   // device, d x d planar column-major
    bool applied;
};

}  // namespace

struct ttn_handle {
    // configuration
    int N = 0, d = 0, chi = 0, m = 0, prec = 0;
    double c6 = 1, rcut = 0, leak = 0;
    double gamma = 0;       // Rydberg decay rate (open system); > 0 selects Arnoldi
    bool split_bf16 = false; // BF16x3 products in the FP32 contractions
    bool nonherm = false;
    bool two_site = false;   // two-tensor TDVP update with truncated splits
    hipStream_t stream = nullptr;
    std::string err;
    bool poisoned = false;
    // tree
    int K = 0, n_nodes = 0, root = 0;
    std::vector<int> level, idx, parent, ch0, ch1, DL, DR, DP, sfirst, scount;
    std::vector<int> leaf_site;
    std::vector<double> V;   // N x N
    // device state
    std::vector<double*> T, up, dn, vLR, vRL;
    double* leafblk = nullptr;
    int* d_leaf_site = nullptr;
    // scratch
    int64_t nmax = 0, stack_max = 0, env_max = 0;
    int max_sites = 0, Dmax = 0;
    double *X = nullptr, *W = nullptr, *Vk = nullptr, *Qtmp = nullptr, *Ttmp = nullptr;
    float *Xf = nullptr, *Yf = nullptr;
    double *Bstk = nullptr, *Astk = nullptr;
    float *Lf = nullptr, *Rf = nullptr, *Bf = nullptr, *Wf = nullptr, *Ef = nullptr;
    // FP32 stacks of the fused-left matvec: [N_i (S_L), H_L] and
    // [H_P, W_i (S_L), identity, W_j (S_R)]
    float *Lf2 = nullptr, *Wf2 = nullptr;
    double *G = nullptr, *Linv = nullptr, *R1 = nullptr, *R2 = nullptr, *Rq = nullptr, *Cb = nullptr,
           *cholwork = nullptr;
    double* red = nullptr;
    LanczosDev *lz = nullptr, *lz_obs = nullptr;
    StepDev* st = nullptr;
    GemmScratch gs;
    double *ov_vec = nullptr, *ov_leaf = nullptr, *ov_M = nullptr, *ov_Y1 = nullptr, *ov_Y2 = nullptr;
    double* opbuf = nullptr;
    // two-site update: merged tensor, Gram matrix, its eigenvectors and
    // eigenvalues (descending) with their column order, split factors
    int64_t n2max = 0, ngmax = 0, mkmax = 0;
    double *Th = nullptr, *G2 = nullptr, *EV = nullptr, *ew = nullptr, *MV = nullptr, *Cm = nullptr;
    int* eorder = nullptr;
    // program
    int n_seg = 0;
    std::vector<double> edges;
    double *d_omega = nullptr, *d_delta = nullptr;
    double *d_omx = nullptr, *d_omz = nullptr;   // single-qubit channels (both or neither)
    double* d_evU = nullptr;
    std::vector<Event> events;
    int64_t step_count = 0;
    double dt = 0;
    bool dt_set = false;
    int cur_seg = -2;
    size_t ws_bytes = 0;
    // host staging for asynchronous copies
    LanczosDev h_lzinit{}, h_lzout{};
    StepDev h_stepinit{}, h_stepout{};
    // workspace regions for launch extent checks (sorted by address)
    std::vector<Region> regions;
    bool dry = false;
    // profiling window: event pairs around GEMM kernel launches
    bool prof = false;
    bool in_heff = false;
    bool prof_timed = true;   // false: launches are recorded, no events
    std::vector<hipEvent_t> ev_pool;
    int ev_used = 0;
    struct MatvecRec {
        int ev;          // event pair around every contraction launch of one matvec
        double flops;
    };
    std::vector<MatvecRec> mv_recs;
    struct ProfRec {
        int ev;          // begin event (end: ev + 1), -1 when timed per matvec
        int prec;        // 0 fp64, 1 fp32
        double flops;    // algorithmic real flops (8 per complex multiply-add)
        bool heff;
        int kernel = 0;  // CgemmInfo::kernel
        int splits = 0;
        int matvec = -1;
    };
    std::vector<ProfRec> prof_recs;
    std::vector<ttn_launch_rec> prof_last;   // launches of the last closed window
    struct VecRec {
        int ev;
        double bytes;    // bytes the Lanczos vector kernels of the call read and write
        int64_t n;       // complex elements per vector
    };
    std::vector<VecRec> vec_recs;
    int64_t prof_matvecs = 0;
    // reverse mode (checkpoints, tape, adjoints); null until recording starts
    AdjState* adj = nullptr;
    // the step body (environment rebuild and both sweeps) replayed as a HIP graph
    bool use_graphs = true, graph_failed = false;
    hipGraphExec_t step_graph = nullptr;
    hipStream_t cap_stream = nullptr;
    double graph_dt = 0;
};

namespace {

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
int64_t capped_pow(int d, int e, int64_t cap) {
    int64_t v = 1;
    for (int i = 0; i < e; ++i) {
        v *= d;
        if (v >= cap) return cap;
    }
    return v;
}

int link_dim(const ttn_handle* h, int s) {
    if (s >= h->N) return 1;
    int64_t a = capped_pow(h->d, s, h->chi + 1), b = capped_pow(h->d, h->N - s, h->chi + 1);
    return (int)std::min<int64_t>({(int64_t)h->chi, a, b});
}

void build_tree(ttn_handle* h) {
    int K = 0;
    while ((1 << K) < h->N) ++K;
    h->K = K;
    std::vector<int> off(K);
    int o = 0;
    for (int l = 0; l < K; ++l) {
        off[l] = o;
        o += h->N >> (l + 1);
    }
    h->n_nodes = o;
    h->root = o - 1;
    for (int l = 0; l < K; ++l)
        for (int j = 0; j < (h->N >> (l + 1)); ++j) {
            h->level.push_back(l);
            h->idx.push_back(j);
            h->parent.push_back(l + 1 < K ? off[l + 1] + j / 2 : -1);
            h->ch0.push_back(l == 0 ? -1 : off[l - 1] + 2 * j);
            h->ch1.push_back(l == 0 ? -1 : off[l - 1] + 2 * j + 1);
            const int dc = l == 0 ? h->d : link_dim(h, 1 << l);
            h->DL.push_back(dc);
            h->DR.push_back(dc);
            h->DP.push_back(link_dim(h, 1 << (l + 1)));
            const int w = 1 << (l + 1);
            h->sfirst.push_back(j * w);
            h->scount.push_back(w);
        }
    for (int v = 0; v < h->n_nodes; ++v)
        if ((int64_t)h->DP[v] > (int64_t)h->DL[v] * h->DR[v])
            throw StatusError{TTN_EINVAL, "inconsistent link dimensions"};
}

inline int64_t nsize(const ttn_handle* h, int v) { return (int64_t)h->DL[v] * h->DR[v] * h->DP[v]; }
inline bool is_bottom(const ttn_handle* h, int v) { return h->level[v] == 0; }
inline int leg_in_parent(const ttn_handle* h, int v) { return h->idx[v] & 1; }
inline int sites_left(const ttn_handle* h, int v) { return h->scount[v] / 2; }

// The edge between v and its parent u, as the two-site update sees it: the
// merged tensor Theta[l, r, s, p] (l, r the legs of v's children, s the leg
// of v's sibling in u, p u's parent leg), matricised as (l r) x (s p), m x n,
// split back with k = the link dimension of the edge.
struct Edge2 {
    int u, leg, sib;
    int DL, DR, DS, DP, k;
    int sL, sR, sS;     // sites below v's left child, right child, the sibling
    int64_t m, n;
};
Edge2 edge2(const ttn_handle* h, int v) {
    Edge2 e;
    e.u = h->parent[v];
    e.leg = leg_in_parent(h, v);
    e.sib = e.leg == 0 ? h->ch1[e.u] : h->ch0[e.u];
    e.DL = h->DL[v];
    e.DR = h->DR[v];
    e.k = h->DP[v];
    e.DS = e.leg == 0 ? h->DR[e.u] : h->DL[e.u];
    e.DP = h->DP[e.u];
    e.sL = e.sR = sites_left(h, v);
    e.sS = h->scount[v];
    e.m = (int64_t)e.DL * e.DR;
    e.n = (int64_t)e.DS * e.DP;
    return e;
}

// plan every buffer; with ws == nullptr only sizes are accumulated
void plan(ttn_handle* h, Bump& b) {
    const int nn = h->n_nodes;
    h->T.assign(nn, nullptr);
    h->up.assign(nn, nullptr);
    h->dn.assign(nn, nullptr);
    h->vLR.assign(nn, nullptr);
    h->vRL.assign(nn, nullptr);
    h->nmax = 0;
    h->stack_max = 0;
    h->Dmax = h->d;
    h->max_sites = 0;
    h->env_max = 0;
    for (int v = 0; v < nn; ++v) {
        const int64_t n = nsize(h, v);
        h->nmax = std::max(h->nmax, n);
        // matvec stack [X, U_i (S_L), H_L X, Z_j (S_R)]
        h->stack_max = std::max(h->stack_max, (int64_t)(2 + h->scount[v]) * n);
        h->Dmax = std::max({h->Dmax, h->DL[v], h->DR[v], h->DP[v]});
        h->max_sites = std::max(h->max_sites, h->scount[v]);
        h->T[v] = b.take<double>(2 * n);
        const int64_t e = (int64_t)(1 + h->scount[v]) * h->DP[v] * h->DP[v];
        h->env_max = std::max(h->env_max, e);
        if (v != h->root) {
            h->up[v] = b.take<double>(2 * e);
            h->dn[v] = b.take<double>(2 * e);
        }
        const int sL = sites_left(h, v);
        h->vLR[v] = b.take<double>(2 * (int64_t)sL * sL);
        h->vRL[v] = b.take<double>(2 * (int64_t)sL * sL);
    }
    // bond stacks (sites below v, size DP^2) are bounded by stack_max as well
    for (int v = 0; v < nn; ++v)
        h->stack_max = std::max(h->stack_max, (int64_t)(2 + h->scount[v]) * h->DP[v] * h->DP[v]);
    // two-site: merged tensors of every edge, their matvec stacks
    // [X, U_i, Z_j, V_k] and the split factors
    h->n2max = h->ngmax = h->mkmax = 0;
    if (h->two_site)
        for (int v = 0; v < nn; ++v) {
            if (v == h->root) continue;
            const Edge2 e = edge2(h, v);
            h->n2max = std::max(h->n2max, e.m * e.n);
            h->ngmax = std::max(h->ngmax, std::min(e.m, e.n));
            h->mkmax = std::max(h->mkmax, std::max(e.m, e.n) * e.k);
            h->stack_max = std::max(h->stack_max, (int64_t)(1 + e.sL + e.sR + e.sS) * e.m * e.n);
        }
    const int64_t nvec = std::max(h->nmax, h->n2max);   // Krylov vectors: nodes and merged tensors
    const int64_t nqr = std::max(h->nmax, h->mkmax);     // QR scratch: nodes and split factors
    const int64_t D2 = (int64_t)h->Dmax * h->Dmax;
    const int64_t smax = h->max_sites + 1;
    h->leafblk = b.take<double>((int64_t)h->N * 4 * h->d * h->d);
    h->d_leaf_site = b.take<int>(h->N);
    h->X = b.take<double>(2 * h->stack_max);
    h->W = b.take<double>(2 * nvec);
    // planar bases (small path, n <= LZ_SMALL_N) or chunked ones: padded to whole chunks
    h->Vk = b.take<double>(2 * kch_pad(nvec) * (h->m + 1));
    h->Qtmp = b.take<double>(2 * nqr);
    h->Ttmp = b.take<double>(2 * h->nmax);
    if (h->two_site) {
        h->Th = b.take<double>(2 * h->n2max);
        h->G2 = b.take<double>(2 * h->ngmax * h->ngmax);
        h->EV = b.take<double>(2 * h->ngmax * h->ngmax);
        h->ew = b.take<double>(h->ngmax);
        h->eorder = b.take<int>(h->ngmax);
        h->MV = b.take<double>(2 * h->mkmax);
        h->Cm = b.take<double>(2 * h->mkmax);
    }
    if (h->prec == TTN_PREC_FP32) {
        h->Xf = b.take<float>(2 * h->stack_max);
        h->Yf = b.take<float>(2 * h->nmax);
        h->Lf = b.take<float>(2 * smax * D2);
        h->Rf = b.take<float>(2 * smax * D2);
        h->Bf = b.take<float>(2 * smax * D2);
        h->Wf = b.take<float>(2 * smax * D2);
        h->Lf2 = b.take<float>(2 * smax * D2);
        h->Wf2 = b.take<float>(2 * (smax + 1) * D2);
        h->Ef = b.take<float>(2 * h->env_max);
    }
    h->Bstk = b.take<double>(2 * smax * D2);
    h->Astk = b.take<double>(2 * smax * D2);
    h->G = b.take<double>(2 * D2);
    h->Linv = b.take<double>(2 * D2);
    h->R1 = b.take<double>(2 * D2);
    h->R2 = b.take<double>(2 * D2);
    h->Rq = b.take<double>(2 * D2);
    h->Cb = b.take<double>(2 * D2);
    // Cholesky work: the padded inverse of the blocked kernel (2 Dp^2, Dp = 16
    // ceil(D / 16)) for D <= 128, the panel buffers of the larger kernel above
    const int64_t Dp = 16 * ((std::min(h->Dmax, 128) + 15) / 16);
    h->cholwork = b.take<double>(std::max(2 * D2 + 2 * (int64_t)h->Dmax * 16, 2 * Dp * Dp) + 64);
    h->red = b.take<double>((int64_t)RED_BLOCKS * KRYLOV_MAX * 2 + 64);
    h->lz = b.take<LanczosDev>(1);
    h->lz_obs = b.take<LanczosDev>(1);
    h->st = b.take<StepDev>(1);
    // split-K partials: at most 1024 tiles worth of 64x64 complex outputs
    h->gs.bytes = (int64_t)2 * 64 * 64 * 1024 * sizeof(double) * 2;
    h->gs.partial = b.take<char>(h->gs.bytes);
    int64_t sumDP = 0;
    for (int v = 0; v < nn; ++v) sumDP += h->DP[v];
    h->ov_vec = b.take<double>(2 * sumDP + 2 * 64);
    h->ov_leaf = b.take<double>((int64_t)2 * h->N * h->d);
    h->ov_M = b.take<double>(2 * (int64_t)nn * h->Dmax * h->Dmax);
    h->ov_Y1 = b.take<double>(2 * h->nmax);
    h->ov_Y2 = b.take<double>(2 * h->nmax);
    h->opbuf = b.take<double>(2 * h->d * h->d);
}

// ---------------------------------------------------------------------------
// GEMM helpers on node tensors T[l, r, p] (l fastest), planar complex
// ---------------------------------------------------------------------------
// k consecutive events of the profiling pool (created on first use); returns
// the index of the first.  The pool restarts at every profiling window.
int take_events(ttn_handle* h, int k) {
    const int idx = h->ev_used;
    h->ev_used += k;
    while ((int)h->ev_pool.size() < h->ev_used) {
        hipEvent_t e;
        HIPCHECK(hipEventCreate(&e));
        h->ev_pool.push_back(e);
    }
    return idx;
}

template <typename R>
struct Ctx {
    ttn_handle* h;
    const int* skip;
    double flops_less = 0;   // flops of the next launches that are not algorithmic (padding terms)
    void run(const Gemm<R>& g) {
        char why[256];
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool rec = h->prof && !h->dry && g.M > 0 && g.N > 0;
        if (rec) {
            // launches inside an H_eff / K_eff matvec are timed per matvec
            // (one event pair around all its launches), the others one by one
            int idx = -1;
            if (h->prof_timed && !h->in_heff) {
                idx = take_events(h, 2);
                e0 = h->ev_pool[idx];
                e1 = h->ev_pool[idx + 1];
            }
            const double fl = 8.0 * g.M * g.N * (double)g.Kin * g.Kout * (double)g.B1 * g.B2 - flops_less;
            h->prof_recs.push_back({idx, sizeof(R) == 4 ? 1 : 0, fl, h->in_heff, 0, 0,
                                    h->in_heff ? (int)h->prof_matvecs - 1 : -1});
        }
        Gemm<R> gg = g;
        if (sizeof(R) == 4 && h->split_bf16) gg.split = 1;
        CgemmInfo info;
        if (!cgemm<R>(gg, h->gs, h->stream, why, sizeof(why), e0, e1, &info))
            throw StatusError{TTN_EINVAL, std::string("launch extent check failed: ") + why};
        if (rec) {
            h->prof_recs.back().kernel = info.kernel;
            h->prof_recs.back().splits = info.splits;
        }
    }
};

// Event pair around one Lanczos vector-kernel call inside a profiling
// window, with the bytes those kernels read and write by construction.
struct VecTimer {
    ttn_handle* h;
    int idx = -1;
    VecTimer(ttn_handle* hh, double bytes, int64_t n) : h(hh) {
        if (!h->prof || !h->prof_timed || h->dry) return;
        idx = take_events(h, 2);
        h->vec_recs.push_back({idx, bytes, n});
        (void)hipEventRecord(h->ev_pool[idx], h->stream);
    }
    ~VecTimer() {
        if (idx >= 0) (void)hipEventRecord(h->ev_pool[idx + 1], h->stream);
    }
};

// extent check for non-GEMM launches: [p, p + count) must lie in one region
void chk(const ttn_handle* h, const void* p, int64_t count_doubles, const char* what) {
    const uintptr_t a = (uintptr_t)p, e = a + (uintptr_t)count_doubles * sizeof(double);
    for (const Region& r : h->regions)
        if (a >= r.lo && e <= r.hi) return;
    throw StatusError{TTN_EINVAL, std::string("launch extent check failed: ") + what};
}

void sort_regions(ttn_handle* h) {
    std::sort(h->regions.begin(), h->regions.end(), [](const Region& a, const Region& b) { return a.lo < b.lo; });
    h->gs.regions = h->regions.data();
    h->gs.n_regions = (int)h->regions.size();
}

void h2d(ttn_handle* h, void* dst, const void* src, size_t bytes) {
    if (h->dry) return;
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
}
void d2h(ttn_handle* h, void* dst, const void* src, size_t bytes) {
    if (h->dry) {
        std::memset(dst, 0, bytes);
        return;
    }
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
}
void sync(ttn_handle* h) {
    if (h->dry) return;
    HIPCHECK(hipStreamSynchronize(h->stream));
}

// Y[.., a, ..] (+)= sum_b Op[a, b] X[.., b, ..] on leg `leg` of a (DL, DR, DP)
// tensor; nops operators (slot stride so) act on nops tensors (stride sx, or
// 0 for a shared X) writing nops outputs (stride sy).  trans: use Op^T;
// conj: use conj(Op).
template <typename R>
void leg_apply(Ctx<R>& c, int leg, const R* Op, int64_t so, const R* X, int64_t sx, R* Y, int64_t sy,
               int DL, int DR, int DP, int nops, int beta, bool conj = false, bool trans = false) {
    const int64_t n = (int64_t)DL * DR * DP;
    Gemm<R> g;
    g.beta = beta;
    g.skip = c.skip;
    if (leg == 0) {
        const int D = DL;
        g.M = D;
        g.N = DR * DP;
        g.Kin = D;
        g.A = Op;
        g.a_plane = (int64_t)D * D;
        g.sam = trans ? D : 1;
        g.sak = trans ? 1 : D;
        g.sab1 = so;
        g.conjA = conj;
        g.B = X;
        g.b_plane = n;
        g.sbk = 1;
        g.sbn = DL;
        g.sbb1 = sx;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = DL;
        g.scb1 = sy;
        g.B1 = nops;
    } else if (leg == 1) {
        const int D = DR;
        g.M = DL;
        g.N = D;
        g.Kin = D;
        g.B1 = DP;
        g.B2 = nops;
        g.A = X;
        g.a_plane = n;
        g.sam = 1;
        g.sak = DL;
        g.sab1 = (int64_t)DL * DR;
        g.sab2 = sx;
        g.B = Op;
        g.b_plane = (int64_t)D * D;
        g.sbk = trans ? 1 : D;
        g.sbn = trans ? D : 1;
        g.sbb2 = so;
        g.conjB = conj;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = DL;
        g.scb1 = (int64_t)DL * DR;
        g.scb2 = sy;
    } else {
        const int D = DP;
        g.M = DL * DR;
        g.N = D;
        g.Kin = D;
        g.A = X;
        g.a_plane = n;
        g.sam = 1;
        g.sak = (int64_t)DL * DR;
        g.sab1 = sx;
        g.B = Op;
        g.b_plane = (int64_t)D * D;
        g.sbk = trans ? 1 : D;
        g.sbn = trans ? D : 1;
        g.sbb1 = so;
        g.conjB = conj;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = (int64_t)DL * DR;
        g.scb1 = sy;
        g.B1 = nops;
    }
    c.run(g);
}

// Y (+)= sum_{k<cnt} Op_k on leg of X_k (operator slots stride so, tensor slots
// stride sx) -- one GEMM with a two-level contraction index.
template <typename R>
void leg_apply_sum(Ctx<R>& c, int leg, const R* Op, int64_t so, const R* X, int64_t sx, R* Y, int DL,
                   int DR, int DP, int cnt, int beta, bool conj = false, bool trans = false) {
    if (cnt <= 0) return;
    const int64_t n = (int64_t)DL * DR * DP;
    Gemm<R> g;
    g.beta = beta;
    g.skip = c.skip;
    g.Kout = cnt;
    if (leg == 1) {
        const int D = DR;
        g.M = DL;
        g.N = D;
        g.Kin = D;
        g.B1 = DP;
        g.A = X;
        g.a_plane = n;
        g.sam = 1;
        g.sak = DL;
        g.sako = sx;
        g.sab1 = (int64_t)DL * DR;
        g.B = Op;
        g.b_plane = (int64_t)D * D;
        g.sbk = trans ? 1 : D;
        g.sbn = trans ? D : 1;
        g.sbko = so;
        g.conjB = conj;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = DL;
        g.scb1 = (int64_t)DL * DR;
    } else if (leg == 2) {
        const int D = DP;
        g.M = DL * DR;
        g.N = D;
        g.Kin = D;
        g.A = X;
        g.a_plane = n;
        g.sam = 1;
        g.sak = (int64_t)DL * DR;
        g.sako = sx;
        g.B = Op;
        g.b_plane = (int64_t)D * D;
        g.sbk = trans ? 1 : D;
        g.sbn = trans ? D : 1;
        g.sbko = so;
        g.conjB = conj;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = (int64_t)DL * DR;
    } else {
        // L leg: Y[a, .] = sum_k sum_b Op_k[a, b] X_k[b, .]
        const int D = DL;
        g.M = D;
        g.N = DR * DP;
        g.Kin = D;
        g.A = Op;
        g.a_plane = (int64_t)D * D;
        g.sam = trans ? D : 1;
        g.sak = trans ? 1 : D;
        g.sako = so;
        g.conjA = conj;
        g.B = X;
        g.b_plane = n;
        g.sbk = 1;
        g.sbko = sx;
        g.sbn = DL;
        g.C = Y;
        g.c_plane = n;
        g.scm = 1;
        g.scn = DL;
    }
    c.run(g);
}

// E_k[a, b] = alpha sum over the other legs of opA(A_k[.., a, ..]) opB(B_k[.., b, ..])
// (+ E_k if beta) for nb pairs (A stride sa, B stride sb: 0 for a shared
// tensor); opX conjugates when conjX.  Outputs D x D column-major, stride se.
template <typename R>
void leg_gram_gen(Ctx<R>& c, int leg, const R* A, int64_t sa, bool conjA, const R* B, int64_t sb, bool conjB,
                  R* E, int64_t se, int DL, int DR, int DP, int nb, int beta = 0, R alpha = 1) {
    const int64_t n = (int64_t)DL * DR * DP;
    Gemm<R> g;
    g.skip = c.skip;
    g.alpha = alpha;
    g.beta = beta;
    g.conjA = conjA;
    g.conjB = conjB;
    g.A = A;
    g.a_plane = n;
    g.sab1 = sa;
    g.B = B;
    g.b_plane = n;
    g.sbb1 = sb;
    g.C = E;
    g.scm = 1;
    g.scb1 = se;
    g.B1 = nb;
    if (leg == 2) {
        const int D = DP;
        g.M = g.N = D;
        g.Kin = DL * DR;
        g.sam = (int64_t)DL * DR;
        g.sak = 1;
        g.sbk = 1;
        g.sbn = (int64_t)DL * DR;
        g.c_plane = (int64_t)D * D;
        g.scn = D;
    } else if (leg == 0) {
        const int D = DL;
        g.M = g.N = D;
        g.Kin = DR * DP;
        g.sam = 1;
        g.sak = DL;
        g.sbk = DL;
        g.sbn = 1;
        g.c_plane = (int64_t)D * D;
        g.scn = D;
    } else {
        const int D = DR;
        g.M = g.N = D;
        g.Kin = DL;
        g.Kout = DP;
        g.sam = DL;
        g.sak = 1;
        g.sako = (int64_t)DL * DR;
        g.sbk = 1;
        g.sbko = (int64_t)DL * DR;
        g.sbn = DL;
        g.c_plane = (int64_t)D * D;
        g.scn = D;
    }
    c.run(g);
}

// E_k[a, b] = sum over the other legs of conj(Q[.., a, ..]) X_k[.., b, ..]
// for nx tensors X_k (stride sx); outputs D x D column-major (stride se).
template <typename R>
void leg_gram(Ctx<R>& c, int leg, const R* Q, const R* X, int64_t sx, R* E, int64_t se, int DL, int DR, int DP,
              int nx) {
    leg_gram_gen<R>(c, leg, Q, 0, true, X, sx, false, E, se, DL, DR, DP, nx);
}

// A stack: out slot i = sum_j V[i][j] N_j for the operator stack Nstk (slots
// 1..ns of a [H, N_1..] stack with matrices D x D), V given as a planar
// (ni x ns) matrix in column-major j + ns*i (i.e. V^T col-major).
void vsum_stack(Ctx<double>& c, const double* Nstk, int D, int ns, const double* Vt, int ni,
                double* out_slot1, int beta = 0) {
    if (ni <= 0 || ns <= 0) return;
    const int64_t D2 = (int64_t)D * D;
    Gemm<double> g;
    g.skip = c.skip;
    g.beta = beta;
    g.M = (int)D2;
    g.N = ni;
    g.Kin = ns;
    g.A = Nstk + 2 * D2;   // slot 1
    g.a_plane = D2;
    g.sam = 1;
    g.sak = 2 * D2;
    g.B = Vt;
    g.b_plane = (int64_t)ns * ni;
    g.sbk = 1;
    g.sbn = ns;
    g.C = out_slot1;
    g.c_plane = D2;
    g.scm = 1;
    g.scn = 2 * D2;
    c.run(g);
}

// ---------------------------------------------------------------------------
// environments and effective Hamiltonians
// ---------------------------------------------------------------------------
const double* child_block(ttn_handle* h, int v, int side) {
    if (is_bottom(h, v)) {
        const int leaf = 2 * h->idx[v] + side;
        return h->leafblk + (int64_t)leaf * 4 * h->d * h->d;
    }
    return h->up[side == 0 ? h->ch0[v] : h->ch1[v]];
}

// Two-site effective Hamiltonian of the edge (v, u) on Theta[l, r, s, p]
// (Edge2), from the environments of the four outer links: the block
// Hamiltonians H_L, H_R, H_S, H_P on their legs, and every coupling V_ij
// n_i n_j between sites below different outer links: pairs across l and r,
// l or r and s (through A'_i = sum_{k below s} V_ik N_k, i below v), and
// every site below u with the rest of the lattice (W_i on p).
struct Op2 {
    Edge2 e;
    const double* Lb;   // [H_L, N_i (i below l)]
    const double* Rb;   // [H_R, N_j (j below r)]
    const double* Bv;   // [H_R, A_i (i below l)], A_i = sum_{j below r} V_ij N_j
    const double* Sb;   // [H_S, N_k (k below s)]
    const double* Sa;   // [H_S, A'_i (i below v)], A'_i = sum_{k below s} V_ik N_k
    const double* Wu;   // [H_P, W_i (i below u, leaf order)], nullptr when u is the root
};

// Operator description of H_eff at node v (or K_eff at the link above v);
// with e2 the two-site H_eff of an edge (DL DR DP = the merged tensor size).
struct OpDesc {
    int DL, DR, DP, sL, sR;
    const double* Lb;   // [H_L, N_i (i in S_L)]      DL x DL each
    const double* Rb;   // [H_R, N_j (j in S_R)]      DR x DR
    const double* Bb;   // [H_R, A_i (i in S_L)]      DR x DR, A_i = sum_j V_ij N_j
    const double* Wb;   // [H_P, W_i (S_L), W_j (S_R)] DP x DP, nullptr at the root
    const Op2* e2 = nullptr;
};

// Bstk = [H_R, A_1..A_sL] for node v
void prepare_B(ttn_handle* h, Ctx<double>& c, int v, const double* Rb, int DR, int sL, int sR) {
    const int64_t D2 = (int64_t)DR * DR;
    copy_d(Rb, h->Bstk, 2 * D2, c.skip, h->stream);
    vsum_stack(c, Rb, DR, sR, h->vRL[v], sL, h->Bstk + 2 * D2);
}

OpDesc node_op(ttn_handle* h, Ctx<double>& c, int v) {
    OpDesc o;
    o.DL = h->DL[v];
    o.DR = h->DR[v];
    o.DP = h->DP[v];
    o.sL = o.sR = sites_left(h, v);
    o.Lb = child_block(h, v, 0);
    o.Rb = child_block(h, v, 1);
    prepare_B(h, c, v, o.Rb, o.DR, o.sL, o.sR);
    o.Bb = h->Bstk;
    o.Wb = v == h->root ? nullptr : h->dn[v];
    return o;
}

// K_eff on the link above v as an operator on a (D_below, 1, D_above) tensor
OpDesc bond_op(ttn_handle* h, int v) {
    OpDesc o;
    o.DL = h->DP[v];
    o.DR = 1;
    o.DP = h->DP[v];
    o.sL = h->scount[v];
    o.sR = 0;
    o.Lb = h->up[v];
    o.Rb = nullptr;
    o.Bb = nullptr;
    o.Wb = h->dn[v];
    return o;
}

// Y = H X with X in slot 0 of the stack Xs (slot stride 2n).
template <typename R>
void apply_op(Ctx<R>& c, const OpDesc& o, const R* Lb, const R* Rb, const R* Bb, const R* Wb, R* Xs,
              R* Y) {
    const int DL = o.DL, DR = o.DR, DP = o.DP, sL = o.sL, sR = o.sR;
    const int64_t n = (int64_t)DL * DR * DP, sx = 2 * n;
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    // stage A: Y = H_L X, U_i = N_i X on the left leg
    leg_apply<R>(c, 0, Lb, 0, Xs, 0, Y, 0, DL, DR, DP, 1, 0);
    if (sL > 0) leg_apply<R>(c, 0, Lb + 2 * L2, 2 * L2, Xs, 0, Xs + sx, sx, DL, DR, DP, sL, 0);
    // stage B: Z_j = N_j X on the right leg (needed by the parent-leg terms)
    if (Wb && sR > 0) leg_apply<R>(c, 1, Rb + 2 * R2, 2 * R2, Xs, 0, Xs + sx * (1 + sL), sx, DL, DR, DP, sR, 0);
    // stage C: Y += H_R X + sum_i A_i U_i on the right leg
    if (Bb) leg_apply_sum<R>(c, 1, Bb, 2 * R2, Xs, sx, Y, DL, DR, DP, 1 + sL, 1);
    // stage D: Y += H_P X + sum_i W_i U_i + sum_j W_j Z_j on the parent leg
    if (Wb) leg_apply_sum<R>(c, 2, Wb, 2 * P2, Xs, sx, Y, DL, DR, DP, 1 + sL + sR, 1);
}

// Y = H_eff2 X for the merged tensor X[l, r, s, p] (slot 0 of the stack Xs,
// slot stride 2 m n); the other slots receive U_i = N_i on l, Z_j = N_j on r
// and V_k = N_k on s.  Slot order [X, U, Z, V] when v is u's left child,
// [X, V, U, Z] when it is the right one, so that the parent-leg operators
// of u (leaf order: left subtree of u first) meet their tensors in order.
// Every leg operation is a leg contraction of a three-leg view:
// l, r on (DL, DR, DS DP); s, p on (DL DR, DS, DP).
void apply_op2(Ctx<double>& c, const Op2& o, double* Xs, double* Y) {
    const Edge2& e = o.e;
    const int DL = e.DL, DR = e.DR, DS = e.DS, DP = e.DP, sL = e.sL, sR = e.sR, sS = e.sS;
    const int64_t sx = 2 * e.m * e.n;
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, S2 = (int64_t)DS * DS, P2 = (int64_t)DP * DP;
    const bool hasP = o.Wu != nullptr;
    const int oV = e.leg == 0 ? 1 + sL + sR : 1;
    const int oU = e.leg == 0 ? 1 : 1 + sS;
    const int oZ = oU + sL;
    const int DSP = DS * DP, DLR = DL * DR;
    // l leg: Y = H_L X, U_i = N_i X
    leg_apply<double>(c, 0, o.Lb, 0, Xs, 0, Y, 0, DL, DR, DSP, 1, 0);
    leg_apply<double>(c, 0, o.Lb + 2 * L2, 2 * L2, Xs, 0, Xs + oU * sx, sx, DL, DR, DSP, sL, 0);
    // r leg: Z_j = N_j X
    leg_apply<double>(c, 1, o.Rb + 2 * R2, 2 * R2, Xs, 0, Xs + oZ * sx, sx, DL, DR, DSP, sR, 0);
    // s leg: V_k = N_k X (they only feed the parent-leg terms)
    if (hasP) leg_apply<double>(c, 1, o.Sb + 2 * S2, 2 * S2, Xs, 0, Xs + oV * sx, sx, DLR, DS, DP, sS, 0);
    // r leg sums: H_R X + sum_i A_i U_i
    if (oU == 1) {
        leg_apply_sum<double>(c, 1, o.Bv, 2 * R2, Xs, sx, Y, DL, DR, DSP, 1 + sL, 1);
    } else {
        leg_apply_sum<double>(c, 1, o.Bv, 2 * R2, Xs, sx, Y, DL, DR, DSP, 1, 1);
        leg_apply_sum<double>(c, 1, o.Bv + 2 * R2, 2 * R2, Xs + oU * sx, sx, Y, DL, DR, DSP, sL, 1);
    }
    // s leg sums: H_S X + sum_{i below v} A'_i (U_i or Z_i)
    if (oU == 1) {
        leg_apply_sum<double>(c, 1, o.Sa, 2 * S2, Xs, sx, Y, DLR, DS, DP, 1 + sL + sR, 1);
    } else {
        leg_apply_sum<double>(c, 1, o.Sa, 2 * S2, Xs, sx, Y, DLR, DS, DP, 1, 1);
        leg_apply_sum<double>(c, 1, o.Sa + 2 * S2, 2 * S2, Xs + oU * sx, sx, Y, DLR, DS, DP, sL + sR, 1);
    }
    // p leg sums: H_P X + sum over every site below u of W_i on its tensor
    if (hasP) leg_apply_sum<double>(c, 2, o.Wu, 2 * P2, Xs, sx, Y, DLR, DS, DP, 1 + sL + sR + sS, 1);
}

// FP32 copies of an operator's stacks for the mixed-precision matvec
void stage_f32(ttn_handle* h, const OpDesc& o, const int* skip) {
    const int64_t L2 = (int64_t)o.DL * o.DL, R2 = (int64_t)o.DR * o.DR, P2 = (int64_t)o.DP * o.DP;
    chk(h, o.Lb, 2 * (1 + o.sL) * L2, "L stack");
    chk(h, h->Lf, (1 + o.sL) * L2, "L stack fp32");
    if (o.Rb) chk(h, o.Rb, 2 * (1 + o.sR) * R2, "R stack");
    if (o.Bb) chk(h, o.Bb, 2 * (1 + o.sL) * R2, "B stack");
    if (o.Wb) {
        chk(h, o.Wb, 2 * (1 + o.sL + o.sR) * P2, "W stack");
        chk(h, h->Wf, (1 + o.sL + o.sR) * P2, "W stack fp32");
    }
    const int64_t wl = 2 * (1 + o.sL) * P2;   // [H_P, W_i (S_L)]
    if (o.Wb) {
        chk(h, h->Lf2, (1 + o.sL) * L2, "fused-left L stack fp32");
        chk(h, h->Wf2, (2 + o.sL + o.sR) * P2, "fused-left W stack fp32");
    }
    convert_d2f_many({{o.Lb, h->Lf, 2 * (1 + o.sL) * L2},
                      {o.Rb, h->Rf, 2 * (1 + o.sR) * R2},
                      {o.Bb, h->Bf, 2 * (1 + o.sL) * R2},
                      {o.Wb, h->Wf, 2 * (1 + o.sL + o.sR) * P2},
                      // the fused-left matvec's stacks (nodes below the root)
                      {o.Wb ? o.Lb + 2 * L2 : nullptr, h->Lf2, 2 * o.sL * L2},
                      {o.Wb ? o.Lb : nullptr, h->Lf2 + 2 * o.sL * L2, 2 * L2},
                      {o.Wb, h->Wf2, wl},
                      {nullptr, h->Wf2 + wl, 2 * P2, o.Wb ? o.DP : 0},
                      {o.Wb ? o.Wb + wl : nullptr, h->Wf2 + wl + 2 * P2, 2 * o.sR * P2}},
                     skip, h->stream);
}

// Y = H X for operators with a parent leg (FP32 stacks from stage_f32), in
// four launches instead of five: the left block Hamiltonian rides with the
// left-site operators (stack [N_i, H_L], outputs [U_i, T = H_L X] in slots
// 1 .. 1 + sL) and T enters the parent-leg sum through an identity operator
// (stack [H_P, W_i, I, W_j] over [X, U_i, T, Z_j]).  The identity term costs
// D_P more rows of K in the parent-leg GEMM and saves a launch (with its
// split-K reduction) per matvec; its flops are left out of the algorithmic
// count.
void apply_op_fused_left(Ctx<float>& c, const OpDesc& o, const float* Lf2, const float* Rf, const float* Bf,
                         const float* Wf2, float* Xs, float* Y) {
    const int DL = o.DL, DR = o.DR, DP = o.DP, sL = o.sL, sR = o.sR;
    const int64_t n = (int64_t)DL * DR * DP, sx = 2 * n;
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    // stage A: U_i = N_i X and T = H_L X on the left leg
    leg_apply<float>(c, 0, Lf2, 2 * L2, Xs, 0, Xs + sx, sx, DL, DR, DP, 1 + sL, 0);
    // stage B: Z_j = N_j X on the right leg, after T
    if (sR > 0) leg_apply<float>(c, 1, Rf + 2 * R2, 2 * R2, Xs, 0, Xs + sx * (2 + sL), sx, DL, DR, DP, sR, 0);
    // stage C: Y = H_R X + sum_i A_i U_i on the right leg
    if (Bf) leg_apply_sum<float>(c, 1, Bf, 2 * R2, Xs, sx, Y, DL, DR, DP, 1 + sL, 0);
    // stage D: Y (+)= H_P X + sum_i W_i U_i + T + sum_j W_j Z_j on the parent leg
    c.flops_less = 8.0 * (double)n * DP;
    leg_apply_sum<float>(c, 2, Wf2, 2 * P2, Xs, sx, Y, DL, DR, DP, 2 + sL + sR, Bf ? 1 : 0);
    c.flops_less = 0;
}

// staged: the mixed-precision matvec whose input is already in the FP32 slot
// (h->Xf) and whose output stays in h->Yf (the Lanczos kernels convert).
// xS != 0: x is a slot of a chunked Krylov basis with that chunk stride.
void apply_op_prec(ttn_handle* h, const OpDesc& o, const double* x, double* y, const int* skip,
                   bool force_fp64 = false, bool staged = false, int64_t xS = 0) {
    const int64_t n = (int64_t)o.DL * o.DR * o.DP;
    // marks the contraction launches of one matvec; in a timed profiling
    // window one event pair brackets them (no events between its launches)
    struct HeffMark {
        ttn_handle* h;
        int idx = -1;
        size_t first = 0;
        explicit HeffMark(ttn_handle* hh) : h(hh) {
            if (h->prof) h->prof_matvecs += 1;
            if (h->prof && h->prof_timed && !h->dry) {
                idx = take_events(h, 2);
                first = h->prof_recs.size();
                (void)hipEventRecord(h->ev_pool[idx], h->stream);
            }
            h->in_heff = true;
        }
        ~HeffMark() {
            h->in_heff = false;
            if (idx >= 0) {
                (void)hipEventRecord(h->ev_pool[idx + 1], h->stream);
                double fl = 0;
                for (size_t i = first; i < h->prof_recs.size(); ++i) fl += h->prof_recs[i].flops;
                h->mv_recs.push_back({idx, fl});
            }
        }
    };
    // the FP64 input slot: a copy of x, or its planar image when x is chunked
    auto to_slot0 = [&]() {
        if (xS)
            krylov_unchunk(x, xS, n, 1, h->X, skip, h->stream);
        else
            copy_d(x, h->X, 2 * n, skip, h->stream);
    };
    if (o.e2) {   // two-site update: FP64
        Ctx<double> c{h, skip};
        to_slot0();
        HeffMark mark(h);
        apply_op2(c, *o.e2, h->X, y);
        return;
    }
    if (h->prec == TTN_PREC_FP32 && !force_fp64) {
        Ctx<float> c{h, skip};
        if (!staged) {
            if (xS) throw StatusError{TTN_ENOTSUP, "unstaged mixed matvec on a chunked basis slot"};
            convert_d2f(x, h->Xf, 2 * n, skip, h->stream);
        }
        {
            HeffMark mark(h);
            if (o.Wb)
                apply_op_fused_left(c, o, h->Lf2, h->Rf, o.Bb ? h->Bf : nullptr, h->Wf2, h->Xf, h->Yf);
            else
                apply_op<float>(c, o, h->Lf, o.Rb ? h->Rf : nullptr, o.Bb ? h->Bf : nullptr, nullptr, h->Xf,
                                h->Yf);
        }
        if (!staged) convert_f2d(h->Yf, y, 2 * n, skip, h->stream);
    } else {
        Ctx<double> c{h, skip};
        to_slot0();
        HeffMark mark(h);
        apply_op<double>(c, o, o.Lb, o.Rb, o.Bb, o.Wb, h->X, y);
    }
}

// chunk stride of the Krylov basis of an operator of n entries: the general
// path stores it in chunks (0: the planar basis of the small path)
int64_t krylov_stride(const ttn_handle* h, int64_t n) {
    return n > LZ_SMALL_N ? 2 * (int64_t)KCH * (h->m + 1) : 0;
}

// x <- exp(-i tau Op) x by Lanczos (full re-orthogonalisation, device scalars)
// Krylov basis of Op from x (full re-orthogonalisation, device scalars):
// h->Vk holds the basis, h->lz the tridiagonal projection and ||x||.
void lanczos_basis(ttn_handle* h, const OpDesc& o, const double* x) {
    const int64_t n = (int64_t)o.DL * o.DR * o.DP;
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, (n + 255) / 256);
    hipStream_t s = h->stream;
    LanczosDev* lz = h->lz;
    const int64_t S = krylov_stride(h, n);
    chk(h, x, 2 * n, "krylov input");
    chk(h, h->Vk, 2 * (S ? kch_pad(n) : n) * (h->m + 1), "krylov basis");
    chk(h, h->W, 2 * n, "krylov work vector");
    chk(h, h->X, 2 * n, "stack slot 0");
    if (h->prec == TTN_PREC_FP32) {
        chk(h, h->Xf, n, "fp32 stack slot 0");
        chk(h, h->Yf, n, "fp32 output");
        stage_f32(h, o, nullptr);
    }
    // mixed precision: the Lanczos kernels write the FP32 input of the next
    // matvec and widen its FP32 output themselves
    float* xf = (h->prec == TTN_PREC_FP32 && n > LZ_SMALL_N) ? h->Xf : nullptr;
    // bytes per call: 16 per complex FP64 element, 8 per FP32 element
    const double E = 16.0 * (double)n, Ef = xf ? 8.0 * (double)n : 0.0;
    {
        VecTimer t(h, 3 * E + Ef, n);   // norm of x, then v0 = x / |x| (+ its FP32 copy)
        lz_start(x, n, h->Vk, S, lz, h->red, nb, s, h->nonherm ? 1 : 0, xf);
    }
    if (n <= LZ_SMALL_N) {
        for (int j = 0; j < h->m; ++j) {
            apply_op_prec(h, o, h->Vk + 2 * n * j, h->W, &lz->done);
            lz_iter_small(h->Vk, j, h->m, h->W, n, lz, LANCZOS_TOL, s);
        }
        return;
    }
    // operators of at most LZ_FUSE_NB reduction blocks take the totals of each
    // pass inside the following kernel
    const bool fuse = nb <= LZ_FUSE_NB;
    static_assert((int64_t)RED_BLOCKS * KRYLOV_MAX * 2 >= 2 * LZ_PARTIAL_HALF, "reduction buffer too small");
    for (int j = 0; j < h->m; ++j) {
        double* vj = h->Vk + 2 * KCH * j;
        apply_op_prec(h, o, vj, h->W, &lz->done, false, xf != nullptr, S);
        // classical Gram-Schmidt, two passes: the first projection also gives alpha_j
        const bool last = j == h->m - 1;
        const double kc = j + 1;
        {
            // V^H w over j + 1 vectors; w read, or widened from the FP32 matvec output
            VecTimer t(h, kc * E + (xf ? 0.5 * E + E : E), n);
            lz_project(h->Vk, S, j + 1, h->W, n, h->red, nb, lz, j, s, xf ? h->Yf : nullptr, last || !fuse);
        }
        if (last) break;
        {
            VecTimer t(h, kc * E + 2 * E, n);   // w -= V c and V^H w in one pass (w read and written)
            lz_subtract_project(h->Vk, S, j + 1, h->W, n, h->red, nb, lz, s, fuse);
        }
        {
            // w -= V c' with |w|^2, then v_{j+1} = w / beta_j (+ its FP32 copy)
            VecTimer t(h, kc * E + 2 * E + 2 * E + Ef, n);
            lz_subtract_next(h->Vk, S, j + 1, h->W, n, h->Vk + 2 * KCH * (j + 1), lz, j, h->red, nb, LANCZOS_TOL,
                             s, xf, fuse);
        }
    }
}

// Whether an operator of these dimensions evolves in the fused one-workgroup
// kernel (no Krylov basis is left in h->Vk then).
bool evolve_fused(const ttn_handle* h, int DL, int DR, int DP, int sL, int sR, bool hasB, bool hasW) {
    return (int64_t)DL * DR * DP <= SMALL_EVOLVE_N &&
           small_evolve_doubles(DL, DR, DP, sL, sR, h->m, hasB, hasW) <= SMALL_EVOLVE_POOL;
}
bool node_evolve_fused(const ttn_handle* h, int v) {
    const int s = sites_left(h, v);
    return evolve_fused(h, h->DL[v], h->DR[v], h->DP[v], s, s, true, v != h->root);
}
bool bond_evolve_fused(const ttn_handle* h, int v) {
    return evolve_fused(h, h->DP[v], 1, h->DP[v], h->scount[v], 0, false, true);
}

// x <- exp(-i tau Op) x by Lanczos (Arnoldi for the open system).  Small
// operators run the whole evolution in one workgroup (FP64 in both modes).
void lanczos_expm(ttn_handle* h, const OpDesc& o, double* x, double tau) {
    const int64_t n = (int64_t)o.DL * o.DR * o.DP;
    if (!o.e2 && evolve_fused(h, o.DL, o.DR, o.DP, o.sL, o.sR, o.Bb != nullptr, o.Wb != nullptr)) {
        const int64_t L2 = (int64_t)o.DL * o.DL, R2 = (int64_t)o.DR * o.DR, P2 = (int64_t)o.DP * o.DP;
        chk(h, x, 2 * n, "krylov input");
        chk(h, o.Lb, 2 * (1 + o.sL) * L2, "L stack");
        if (o.Wb && o.sR > 0) chk(h, o.Rb, 2 * (1 + o.sR) * R2, "R stack");
        if (o.Bb) chk(h, o.Bb, 2 * (1 + o.sL) * R2, "B stack");
        if (o.Wb) chk(h, o.Wb, 2 * (1 + o.sL + o.sR) * P2, "W stack");
        small_evolve(o.Lb, o.Rb, o.Bb, o.Wb, o.DL, o.DR, o.DP, o.sL, o.sR, h->m, tau, LANCZOS_TOL, h->nonherm, x,
                     h->st, h->stream);
        return;
    }
    lanczos_basis(h, o, x);
    lz_expm(h->lz, tau, h->st, h->stream);
    VecTimer t(h, 16.0 * (double)n * (h->m + 1), n);   // x = |x| V y: m basis vectors read, x written
    lz_combine(h->Vk, krylov_stride(h, n), n, x, h->lz, h->stream);
}

// ---------------------------------------------------------------------------
// QR gauge move (CholeskyQR2): T[.., a, ..] = sum_k Q[.., k, ..] R[k, a]
// with R upper triangular, real positive diagonal; Q overwrites T, R -> Rout.
// ---------------------------------------------------------------------------
// With rinvh != nullptr also writes R^{-H} = L2^{-1} L1^{-1} (for the adjoint),
// keeping L1^{-1} in l1inv (D x D scratch).
void qr_toward(ttn_handle* h, int DL, int DR, int DP, double* Tv, int leg, double* Rout,
               double* rinvh = nullptr, double* l1inv = nullptr) {
    Ctx<double> c{h, nullptr};
    const int D = leg == 0 ? DL : (leg == 1 ? DR : DP);
    const int64_t n = (int64_t)DL * DR * DP;
    chk(h, Tv, 2 * n, "qr tensor");
    chk(h, h->Qtmp, 2 * n, "qr scratch");
    chk(h, h->G, 2 * (int64_t)D * D, "gram");
    chk(h, h->Linv, 2 * (int64_t)D * D, "Linv");
    chk(h, h->R1, 2 * (int64_t)D * D, "R1");
    chk(h, h->R2, 2 * (int64_t)D * D, "R2");
    chk(h, Rout, 2 * (int64_t)D * D, "R out");
    const int64_t Dpad = 16 * (int64_t)((D + 15) / 16);
    chk(h, h->cholwork, D <= 128 ? 2 * Dpad * Dpad : (int64_t)D * (D + 1) + 2 * (int64_t)D * 16, "cholesky work");
    leg_gram(c, leg, Tv, Tv, 0, h->G, 0, DL, DR, DP, 1);
    chol_inv(h->G, D, h->Linv, h->R1, nullptr, h->cholwork, h->st, h->stream);
    if (rinvh) {
        chk(h, l1inv, 2 * (int64_t)D * D, "L1 inverse");
        copy_d(h->Linv, l1inv, 2 * (int64_t)D * D, nullptr, h->stream);
    }
    leg_apply<double>(c, leg, h->Linv, 0, Tv, 0, h->Qtmp, 0, DL, DR, DP, 1, 0, true, false);
    leg_gram(c, leg, h->Qtmp, h->Qtmp, 0, h->G, 0, DL, DR, DP, 1);
    chol_inv(h->G, D, h->Linv, h->R2, nullptr, h->cholwork, h->st, h->stream);
    leg_apply<double>(c, leg, h->Linv, 0, h->Qtmp, 0, Tv, 0, DL, DR, DP, 1, 0, true, false);
    if (rinvh) {
        chk(h, rinvh, 2 * (int64_t)D * D, "R^-H");
        Gemm<double> gi;
        gi.M = gi.N = D;
        gi.Kin = D;
        gi.A = h->Linv;
        gi.a_plane = (int64_t)D * D;
        gi.sam = 1;
        gi.sak = D;
        gi.B = l1inv;
        gi.b_plane = (int64_t)D * D;
        gi.sbk = 1;
        gi.sbn = D;
        gi.C = rinvh;
        gi.c_plane = (int64_t)D * D;
        gi.scm = 1;
        gi.scn = D;
        c.run(gi);
    }
    // R = R2 R1 (both upper triangular, D x D column-major)
    Gemm<double> g;
    g.M = g.N = D;
    g.Kin = D;
    g.A = h->R2;
    g.a_plane = (int64_t)D * D;
    g.sam = 1;
    g.sak = D;
    g.B = h->R1;
    g.b_plane = (int64_t)D * D;
    g.sbk = 1;
    g.sbn = D;
    g.C = Rout;
    g.c_plane = (int64_t)D * D;
    g.scm = 1;
    g.scn = D;
    c.run(g);
    rdiag_min(Rout, D, h->st, h->stream);
    (void)n;
}

// T (tensor of node v) <- Op on leg (via a temporary)
void absorb(ttn_handle* h, int v, int leg, const double* Op, bool trans) {
    Ctx<double> c{h, nullptr};
    const int64_t n = nsize(h, v);
    chk(h, h->Ttmp, 2 * n, "absorb scratch");
    leg_apply<double>(c, leg, Op, 0, h->T[v], 0, h->Ttmp, 0, h->DL[v], h->DR[v], h->DP[v], 1, 0, false,
                      trans);
    copy_d(h->Ttmp, h->T[v], 2 * n, nullptr, h->stream);
}

// Up environment of the link above v from its isometry Q: block
// Q^dag (H_L + H_R + sum_{i in L} n_i A_i) Q and Q^dag n_i Q for every site
// below, written as the stack E = [H, N_(S_L), N_(S_R)].
template <typename R>
void build_up_core(Ctx<R>& c, int DL, int DR, int DP, int sL, int sR, const R* Q, const R* Lb, const R* Rb,
                   const R* Bb, R* Xs, R* Y, R* E) {
    const int64_t n = (int64_t)DL * DR * DP, sx = 2 * n;
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    leg_apply<R>(c, 0, Lb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 0);
    leg_apply<R>(c, 0, Lb + 2 * L2, 2 * L2, Q, 0, Xs + sx, sx, DL, DR, DP, sL, 0);
    leg_apply<R>(c, 1, Rb + 2 * R2, 2 * R2, Q, 0, Xs + sx * (1 + sL), sx, DL, DR, DP, sR, 0);
    leg_apply<R>(c, 1, Bb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 1);
    leg_apply_sum<R>(c, 1, Bb + 2 * R2, 2 * R2, Xs + sx, sx, Y, DL, DR, DP, sL, 1);
    leg_gram<R>(c, 2, Q, Y, 0, E, 0, DL, DR, DP, 1);
    leg_gram<R>(c, 2, Q, Xs + sx, sx, E + 2 * P2, 2 * P2, DL, DR, DP, sL + sR);
}

// Down environment of the link above child c (leg `leg` of its parent u,
// whose tensor Q is canonical toward c): block Hamiltonian of everything
// outside the subtree of c and W_i = sum_{j outside} V_ij n_j for the sites
// below c, as the stack E = [H, W_(sites of c)].  Ab: for leg 0 the stack
// [H_R, A_i] (A_i = sum_{j in R} V_ij n_j), for leg 1 the slots A''_j =
// sum_{k in L} V_jk n_k at slot 1...
template <typename R>
void build_down_core(Ctx<R>& c, int leg, int DL, int DR, int DP, int sL, int sR, const R* Q, const R* Lb,
                     const R* Rb, const R* Wb, const R* Ab, R* Xs, R* Y, R* E) {
    const int64_t n = (int64_t)DL * DR * DP, sx = 2 * n;
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    const int Dc = leg == 0 ? DL : DR;
    const int64_t C2 = (int64_t)Dc * Dc;
    if (leg == 0) {
        // block: H_R + H_P + sum_{j in R} N_j W_j ; fields W_i (i in L): A_i on R + W_i on P
        leg_apply<R>(c, 1, Rb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 0);
        if (Wb) {
            leg_apply<R>(c, 2, Wb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 1);
            leg_apply<R>(c, 1, Rb + 2 * R2, 2 * R2, Q, 0, Xs + sx * (1 + sL), sx, DL, DR, DP, sR, 0);
            leg_apply_sum<R>(c, 2, Wb + 2 * P2 * (1 + sL), 2 * P2, Xs + sx * (1 + sL), sx, Y, DL, DR, DP, sR, 1);
        }
        leg_gram<R>(c, 0, Q, Y, 0, E, 0, DL, DR, DP, 1);
        leg_apply<R>(c, 1, Ab + 2 * R2, 2 * R2, Q, 0, Xs + sx, sx, DL, DR, DP, sL, 0);
        if (Wb) leg_apply<R>(c, 2, Wb + 2 * P2, 2 * P2, Q, 0, Xs + sx, sx, DL, DR, DP, sL, 1);
        leg_gram<R>(c, 0, Q, Xs + sx, sx, E + 2 * C2, 2 * C2, DL, DR, DP, sL);
    } else {
        leg_apply<R>(c, 0, Lb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 0);
        if (Wb) {
            leg_apply<R>(c, 2, Wb, 0, Q, 0, Y, 0, DL, DR, DP, 1, 1);
            leg_apply<R>(c, 0, Lb + 2 * L2, 2 * L2, Q, 0, Xs + sx, sx, DL, DR, DP, sL, 0);
            leg_apply_sum<R>(c, 2, Wb + 2 * P2, 2 * P2, Xs + sx, sx, Y, DL, DR, DP, sL, 1);
        }
        leg_gram<R>(c, 1, Q, Y, 0, E, 0, DL, DR, DP, 1);
        leg_apply<R>(c, 0, Ab + 2 * L2, 2 * L2, Q, 0, Xs + sx * (1 + sL), sx, DL, DR, DP, sR, 0);
        if (Wb)
            leg_apply<R>(c, 2, Wb + 2 * P2 * (1 + sL), 2 * P2, Q, 0, Xs + sx * (1 + sL), sx, DL, DR, DP, sR, 1);
        leg_gram<R>(c, 1, Q, Xs + sx * (1 + sL), sx, E + 2 * C2, 2 * C2, DL, DR, DP, sR);
    }
}

// In the mixed path the environment contractions run in complex FP32 on
// FP32 copies of their operands; the FP32 results are made exactly
// Hermitian while converted back into the FP64 environment store (all but
// the block Hamiltonian of an open system, which is not Hermitian).
void build_up(ttn_handle* h, int v) {
    Ctx<double> c{h, nullptr};
    const int DL = h->DL[v], DR = h->DR[v], DP = h->DP[v];
    const int sL = sites_left(h, v), sR = sL;
    const int64_t n = nsize(h, v);
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    const double* Lb = child_block(h, v, 0);
    const double* Rb = child_block(h, v, 1);
    prepare_B(h, c, v, Rb, DR, sL, sR);
    if (h->prec == TTN_PREC_FP32) {
        Ctx<float> cf{h, nullptr};
        float* Qf = h->Xf;   // slot 0 of the FP32 stack is free during an environment build
        chk(h, h->Ef, (1 + sL + sR) * P2, "fp32 environment staging");
        convert_d2f_many({{h->T[v], Qf, 2 * n},
                          {Lb, h->Lf, 2 * (1 + sL) * L2},
                          {Rb, h->Rf, 2 * (1 + sR) * R2},
                          {h->Bstk, h->Bf, 2 * (1 + sL) * R2}},
                         nullptr, h->stream);
        build_up_core<float>(cf, DL, DR, DP, sL, sR, Qf, h->Lf, h->Rf, h->Bf, h->Xf, h->Yf, h->Ef);
        herm_f2d(h->Ef, h->up[v], DP, 1 + sL + sR, h->stream, h->nonherm);
    } else {
        build_up_core<double>(c, DL, DR, DP, sL, sR, h->T[v], Lb, Rb, h->Bstk, h->X, h->W, h->up[v]);
    }
}

void build_down(ttn_handle* h, int cnode) {
    Ctx<double> c{h, nullptr};
    const int u = h->parent[cnode];
    const int leg = leg_in_parent(h, cnode);
    const int DL = h->DL[u], DR = h->DR[u], DP = h->DP[u];
    const int sL = sites_left(h, u), sR = sL;
    const int64_t n = nsize(h, u);
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR, P2 = (int64_t)DP * DP;
    const double* Lb = child_block(h, u, 0);
    const double* Rb = child_block(h, u, 1);
    const double* Wb = u == h->root ? nullptr : h->dn[u];
    const int Dc = leg == 0 ? DL : DR;
    const int64_t C2 = (int64_t)Dc * Dc;
    const double* Ab;
    int64_t Alen;
    if (leg == 0) {
        prepare_B(h, c, u, Rb, DR, sL, sR);   // [H_R, A_i = sum_{j in R} V_ij N_j]
        Ab = h->Bstk;
        Alen = (1 + sL) * R2;
    } else {
        // A''_j = sum_{k in L} V_jk N_k (left operators), j in R, at slots 1..
        vsum_stack(c, Lb, DL, sL, h->vLR[u], sR, h->Astk + 2 * L2);
        Ab = h->Astk;
        Alen = (1 + sR) * L2;
    }
    if (h->prec == TTN_PREC_FP32) {
        Ctx<float> cf{h, nullptr};
        float* Qf = h->Xf;
        chk(h, h->Ef, (1 + (leg == 0 ? sL : sR)) * C2, "fp32 environment staging");
        convert_d2f_many({{h->T[u], Qf, 2 * n},
                          {Lb, h->Lf, 2 * (1 + sL) * L2},
                          {Rb, h->Rf, 2 * (1 + sR) * R2},
                          {Wb, h->Wf, 2 * (1 + sL + sR) * P2},
                          leg == 0 ? D2FItem{Ab, h->Bf, 2 * Alen}
                                   : D2FItem{Ab + 2 * L2, h->Bf + 2 * L2, 2 * (Alen - L2)}},
                         nullptr, h->stream);
        build_down_core<float>(cf, leg, DL, DR, DP, sL, sR, Qf, h->Lf, h->Rf, Wb ? h->Wf : nullptr, h->Bf, h->Xf,
                               h->Yf, h->Ef);
        herm_f2d(h->Ef, h->dn[cnode], Dc, 1 + (leg == 0 ? sL : sR), h->stream, h->nonherm);
    } else {
        build_down_core<double>(c, leg, DL, DR, DP, sL, sR, h->T[u], Lb, Rb, Wb, Ab, h->X, h->W, h->dn[cnode]);
    }
}

void evolve_node(ttn_handle* h, int v, double tau) {
    Ctx<double> c{h, nullptr};
    OpDesc o = node_op(h, c, v);
    lanczos_expm(h, o, h->T[v], tau);
}

void evolve_bond(ttn_handle* h, int v, double* C, double tau) {
    OpDesc o = bond_op(h, v);
    lanczos_expm(h, o, C, -tau);
}

// ---------------------------------------------------------------------------
// sweeps
// ---------------------------------------------------------------------------
void visit_fwd(ttn_handle* h, int v, double tau) {
    const int u = h->parent[v], leg = leg_in_parent(h, v);
    qr_toward(h, h->DL[u], h->DR[u], h->DP[u], h->T[u], leg, h->Rq);
    absorb(h, v, 2, h->Rq, false);                 // T_v[.., k] = sum_a R[k, a] T_v[.., a]
    build_down(h, v);
    if (!is_bottom(h, v)) {
        visit_fwd(h, h->ch0[v], tau);
        visit_fwd(h, h->ch1[v], tau);
    }
    evolve_node(h, v, tau);
    qr_toward(h, h->DL[v], h->DR[v], h->DP[v], h->T[v], 2, h->Cb);
    build_up(h, v);
    evolve_bond(h, v, h->Cb, tau);
    absorb(h, u, leg, h->Cb, false);               // T_u[k at leg] = sum_p C[k, p] T_u[p at leg]
}

void visit_bwd(ttn_handle* h, int v, double tau) {
    const int u = h->parent[v], leg = leg_in_parent(h, v);
    const int D = h->DP[v];
    chk(h, h->Cb, 2 * (int64_t)D * D, "bond buffer");
    qr_toward(h, h->DL[u], h->DR[u], h->DP[u], h->T[u], leg, h->Rq);
    build_down(h, v);
    transpose_c(h->Rq, h->Cb, D, D, h->stream);    // C[below, above] = R^T
    evolve_bond(h, v, h->Cb, tau);
    absorb(h, v, 2, h->Cb, true);                  // T_v[.., k] = sum_a T_v[.., a] C[a, k]
    evolve_node(h, v, tau);
    if (!is_bottom(h, v)) {
        visit_bwd(h, h->ch1[v], tau);
        visit_bwd(h, h->ch0[v], tau);
    }
    qr_toward(h, h->DL[v], h->DR[v], h->DP[v], h->T[v], 2, h->Rq);
    build_up(h, v);
    absorb(h, u, leg, h->Rq, false);
}

void sweep_fwd(ttn_handle* h, double tau) {
    if (!is_bottom(h, h->root)) {
        visit_fwd(h, h->ch0[h->root], tau);
        visit_fwd(h, h->ch1[h->root], tau);
    }
    evolve_node(h, h->root, tau);
}

void sweep_bwd(ttn_handle* h, double tau) {
    evolve_node(h, h->root, tau);
    if (!is_bottom(h, h->root)) {
        visit_bwd(h, h->ch1[h->root], tau);
        visit_bwd(h, h->ch0[h->root], tau);
    }
}

// ---------------------------------------------------------------------------
// two-site (two-tensor) update
// ---------------------------------------------------------------------------
// C (M x N, leading dimension ldc) = op(A) op(B) in planar complex FP64:
// op(A) is A (M x K, ld lda) or, with ta, the conjugate transpose of A (K x M,
// ld lda); op(B) likewise (tb: B is N x K).
void zgemm(Ctx<double>& c, int M, int N, int K, const double* A, int64_t lda, int64_t ap, bool ta,
           const double* B, int64_t ldb, int64_t bp, bool tb, double* C, int64_t ldc, int64_t cp) {
    Gemm<double> g;
    g.M = M;
    g.N = N;
    g.Kin = K;
    g.A = A;
    g.a_plane = ap;
    g.sam = ta ? lda : 1;
    g.sak = ta ? 1 : lda;
    g.conjA = ta;
    g.B = B;
    g.b_plane = bp;
    g.sbk = tb ? ldb : 1;
    g.sbn = tb ? 1 : ldb;
    g.conjB = tb;
    g.C = C;
    g.c_plane = cp;
    g.scm = 1;
    g.scn = ldc;
    c.run(g);
}

// Writes the k x n matrix X (X[c, j] at X[c sc + j sj], j = s + DS p,
// conjugated if conj) into the tensor of u in the layout of the edge's leg:
// leg 0: T_u[c, s, p]; leg 1: T_u[s, c, p].
void put_u(ttn_handle* h, const Edge2& e, const double* X, int64_t xplane, int64_t sc, int64_t sj, bool conj) {
    const int64_t k = e.k, DS = e.DS;
    const int64_t dc = e.leg == 0 ? 1 : DS, ds = e.leg == 0 ? k : 1;
    chk(h, h->T[e.u], 2 * k * e.n, "split factor of the parent");
    copy3(X, xplane, sc, sj, sj * DS, h->T[e.u], k * e.n, dc, ds, k * DS, (int)k, (int)DS, e.DP, conj, h->stream);
}

// Forward two-site update of the edge (v, parent u):
// Theta <- exp(-i tau H_eff2) Theta, then the split back into T_v and T_u
// truncated to the edge's link dimension k: the kept subspace is spanned by
// the eigenvectors of the k largest eigenvalues of the smaller Gram matrix
// (Theta^H Theta or Theta Theta^H, i.e. the k largest singular values), the
// other factor is the projection of Theta on it, rescaled to the norm of the
// untruncated Theta (the kept and discarded weights are the eigenvalue sums).
// centre_up: T_v an isometry toward its parent, T_u the centre; else T_u an
// isometry toward v and T_v the centre.  Rebuilds the environment of the
// link on the isometry's side.
void update_edge2(ttn_handle* h, int v, double tau, bool centre_up) {
    Ctx<double> c{h, nullptr};
    const Edge2 e = edge2(h, v);
    const int u = e.u;
    const int64_t m = e.m, n = e.n, k = e.k, mn = m * n;
    chk(h, h->Th, 2 * mn, "merged tensor");
    chk(h, h->T[v], 2 * m * k, "node tensor");
    chk(h, h->Cm, 2 * k * n, "split factor");
    chk(h, h->MV, 2 * m * k, "split factor");
    // Theta = T_v (m x k) times T_u as a k x n matrix
    const double* Tu = h->T[u];
    if (e.leg == 1) {   // T_u[s, c, p] -> Cm[c, s + DS p]
        chk(h, h->T[u], 2 * k * n, "parent tensor");
        copy3(h->T[u], k * n, e.DS, 1, (int64_t)e.DS * k, h->Cm, k * n, 1, k, k * e.DS, (int)k, e.DS, e.DP, false,
              h->stream);
        Tu = h->Cm;
    }
    zgemm(c, (int)m, (int)n, (int)k, h->T[v], m, m * k, false, Tu, k, k * n, false, h->Th, m, mn);
    // the two-site effective Hamiltonian of the edge
    Op2 o2;
    o2.e = e;
    o2.Lb = child_block(h, v, 0);
    o2.Rb = child_block(h, v, 1);
    prepare_B(h, c, v, o2.Rb, e.DR, e.sL, e.sR);
    o2.Bv = h->Bstk;
    o2.Sb = h->up[e.sib];
    const int64_t S2 = (int64_t)e.DS * e.DS;
    chk(h, h->Astk, 2 * (1 + e.sL + e.sR) * S2, "sibling coupling stack");
    copy_d(o2.Sb, h->Astk, 2 * S2, nullptr, h->stream);
    vsum_stack(c, o2.Sb, e.DS, e.sS, e.leg == 0 ? h->vRL[u] : h->vLR[u], e.sL + e.sR, h->Astk + 2 * S2);
    o2.Sa = h->Astk;
    o2.Wu = u == h->root ? nullptr : h->dn[u];
    OpDesc o{};
    o.DL = (int)m;
    o.DR = e.DS;
    o.DP = e.DP;
    o.e2 = &o2;
    lanczos_expm(h, o, h->Th, tau);
    // the split
    const int64_t ng = std::min(m, n);
    chk(h, h->G2, 2 * ng * ng, "Gram matrix");
    chk(h, h->EV, 2 * ng * ng, "eigenvectors");
    chk(h, h->ew, ng, "eigenvalues");
    if (n <= m) {
        zgemm(c, (int)n, (int)n, (int)m, h->Th, m, mn, true, h->Th, m, mn, false, h->G2, n, n * n);   // Theta^H Theta
        herm_eig(h->G2, (int)n, h->EV, h->ew, h->eorder, h->st, h->stream);
        gather_cols(h->EV, (int)n, h->eorder, (int)k, h->Cm, h->stream);   // V_k (n x k)
        if (centre_up) {
            zgemm(c, (int)m, (int)k, (int)n, h->Th, m, mn, false, h->Cm, n, n * k, false, h->MV, m, m * k);
            qr_toward(h, (int)m, 1, (int)k, h->MV, 2, h->Rq);   // T_v = orth(Theta V_k)
            copy_d(h->MV, h->T[v], 2 * m * k, nullptr, h->stream);
            zgemm(c, (int)k, (int)n, (int)m, h->MV, m, m * k, true, h->Th, m, mn, false, h->Ttmp, k, k * n);
            chk(h, h->Ttmp, 2 * k * n, "split factor");
            put_u(h, e, h->Ttmp, k * n, 1, k, false);                  // T_u = T_v^H Theta
            split_finish(h->ew, (int)n, (int)k, h->T[u], k * n, h->st, h->stream);
        } else {
            zgemm(c, (int)m, (int)k, (int)n, h->Th, m, mn, false, h->Cm, n, n * k, false, h->T[v], m, m * k);
            put_u(h, e, h->Cm, n * k, n, 1, true);                     // T_u = V_k^H
            split_finish(h->ew, (int)n, (int)k, h->T[v], m * k, h->st, h->stream);
        }
    } else {
        zgemm(c, (int)m, (int)m, (int)n, h->Th, m, mn, false, h->Th, m, mn, true, h->G2, m, m * m);   // Theta Theta^H
        herm_eig(h->G2, (int)m, h->EV, h->ew, h->eorder, h->st, h->stream);
        gather_cols(h->EV, (int)m, h->eorder, (int)k, h->MV, h->stream);   // U_k (m x k)
        if (centre_up) {
            copy_d(h->MV, h->T[v], 2 * m * k, nullptr, h->stream);
            zgemm(c, (int)k, (int)n, (int)m, h->MV, m, m * k, true, h->Th, m, mn, false, h->Ttmp, k, k * n);
            chk(h, h->Ttmp, 2 * k * n, "split factor");
            put_u(h, e, h->Ttmp, k * n, 1, k, false);                  // T_u = U_k^H Theta
            split_finish(h->ew, (int)m, (int)k, h->T[u], k * n, h->st, h->stream);
        } else {
            zgemm(c, (int)n, (int)k, (int)m, h->Th, m, mn, true, h->MV, m, m * k, false, h->Cm, n, n * k);
            qr_toward(h, (int)n, 1, (int)k, h->Cm, 2, h->Rq);        // Q = orth(Theta^H U_k)
            zgemm(c, (int)m, (int)k, (int)n, h->Th, m, mn, false, h->Cm, n, n * k, false, h->T[v], m, m * k);
            put_u(h, e, h->Cm, n * k, n, 1, true);                     // T_u = Q^H
            split_finish(h->ew, (int)m, (int)k, h->T[v], m * k, h->st, h->stream);
        }
    }
    if (centre_up)
        build_up(h, v);
    else
        build_down(h, v);
}

// Half-step of the two-site integrator below v (centre at v's parent on
// entry and exit): every edge of the subtree and the edge above v is
// updated forward once; v itself, between the updates of the edges that
// meet there, is evolved backward (after each child edge).
void visit2_fwd(ttn_handle* h, int v, double tau) {
    const int u = h->parent[v], leg = leg_in_parent(h, v);
    if (!is_bottom(h, v)) {
        qr_toward(h, h->DL[u], h->DR[u], h->DP[u], h->T[u], leg, h->Rq);   // centre down to v
        absorb(h, v, 2, h->Rq, false);
        build_down(h, v);
        visit2_fwd(h, h->ch0[v], tau);
        evolve_node(h, v, -tau);
        visit2_fwd(h, h->ch1[v], tau);
        evolve_node(h, v, -tau);
    }
    update_edge2(h, v, tau, true);
}

// The exact reverse of visit2_fwd.
void visit2_bwd(ttn_handle* h, int v, double tau) {
    const int u = h->parent[v], leg = leg_in_parent(h, v);
    if (is_bottom(h, v)) {
        update_edge2(h, v, tau, true);
        return;
    }
    update_edge2(h, v, tau, false);
    evolve_node(h, v, -tau);
    visit2_bwd(h, h->ch1[v], tau);
    evolve_node(h, v, -tau);
    visit2_bwd(h, h->ch0[v], tau);
    qr_toward(h, h->DL[v], h->DR[v], h->DP[v], h->T[v], 2, h->Rq);         // centre back up to u
    build_up(h, v);
    absorb(h, u, leg, h->Rq, false);
}

void sweep2_fwd(ttn_handle* h, double tau) {
    visit2_fwd(h, h->ch0[h->root], tau);
    evolve_node(h, h->root, -tau);
    visit2_fwd(h, h->ch1[h->root], tau);
}

void sweep2_bwd(ttn_handle* h, double tau) {
    visit2_bwd(h, h->ch1[h->root], tau);
    evolve_node(h, h->root, -tau);
    visit2_bwd(h, h->ch0[h->root], tau);
}

void step_body(ttn_handle* h, double tau);

void postorder(const ttn_handle* h, int v, std::vector<int>& out) {
    if (!is_bottom(h, v)) {
        postorder(h, h->ch0[v], out);
        postorder(h, h->ch1[v], out);
    }
    out.push_back(v);
}

int segment_at(const ttn_handle* h, double t) {
    for (int s = 0; s < h->n_seg; ++s)
        if (h->edges[s] <= t && t < h->edges[s + 1]) return s;
    return -1;
}

__global__ void k_leaf_blocks_seg(double* blk, const int* leaf_site, const double* om,
                                  const double* de, const double* omx, const double* omz, int n_seg, int seg,
                                  int n_leaves, int d, double leak, double gamma) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_leaves) return;
    const int s = leaf_site[k];
    const int dd = d * d;
    double* hh = blk + (int64_t)k * 4 * dd;
    double* nn = hh + 2 * dd;
    for (int e = 0; e < 2 * dd; ++e) {
        hh[e] = 0.0;
        nn[e] = 0.0;
    }
    const double o2 = seg >= 0 ? 0.5 * om[(int64_t)s * n_seg + seg] : 0.0;
    const double dl = seg >= 0 ? de[(int64_t)s * n_seg + seg] : 0.0;
    hh[1 + d * 2] += o2;   // Omega/2 (|1><r| + |r><1|), r = level 2
    hh[2 + d * 1] += o2;
    if (d >= 4) {           // leak_ratio Omega/2 (|leak><r| + h.c.), leak = level 3
        hh[3 + d * 2] += leak * o2;
        hh[2 + d * 3] += leak * o2;
    }
    hh[2 + d * 2] -= dl;   // -Delta |r><r|
    hh[dd + 2 + d * 2] -= gamma;   // open system: -i gamma |r><r| (imaginary plane)
    if (omx && seg >= 0) {         // Omega^x sigma^x + Omega^z sigma^z on {|0>, |1>}
        const double ox = omx[(int64_t)s * n_seg + seg], oz = omz[(int64_t)s * n_seg + seg];
        hh[0 + d * 1] += ox;
        hh[1 + d * 0] += ox;
        hh[0 + d * 0] += oz;
        hh[1 + d * 1] -= oz;
    }
    nn[2 + d * 2] = 1.0;
}

void set_hamiltonian(ttn_handle* h, int seg) {
    h->cur_seg = seg;
    if (h->dry) return;
    hipLaunchKernelGGL(k_leaf_blocks_seg, dim3((h->N + 63) / 64), dim3(64), 0, h->stream, h->leafblk,
                       h->d_leaf_site, h->d_omega, h->d_delta, h->d_omx, h->d_omz, h->n_seg, seg, h->N, h->d,
                       h->leak, h->gamma);
    h->cur_seg = seg;
}

void rebuild_up(ttn_handle* h) {
    std::vector<int> po;
    postorder(h, h->root, po);
    for (int v : po)
        if (v != h->root) build_up(h, v);
}

void step_body(ttn_handle* h, double tau) {
    rebuild_up(h);
    if (h->two_site) {
        sweep2_fwd(h, tau);
        sweep2_bwd(h, tau);
        return;
    }
    sweep_fwd(h, tau);
    sweep_bwd(h, tau);
}

// Device time of one individually timed contraction launch (its main kernel
// and split-K reduction between two events); -1 for launches timed per matvec.
double launch_ms(const ttn_handle::ProfRec& r, const std::vector<hipEvent_t>& pool) {
    if (r.ev < 0) return -1.0;
    float a = 0.f;
    HIPCHECK(hipEventElapsedTime(&a, pool[r.ev], pool[r.ev + 1]));
    return (double)a;
}

// Adds the launches, flops and device times of a window to `out`: launches
// outside H_eff / K_eff matvecs carry their own event time; the matvec
// launches are timed together, per matvec.
void accumulate_prof(const ttn_handle* h, ttn_profile* out) {
    for (const auto& r : h->prof_recs) {
        const double ms = r.ev >= 0 ? launch_ms(r, h->ev_pool) : 0.0;
        ttn_kernel_prof& k = r.prec ? out->gemm_f32 : out->gemm_f64;
        k.launches += 1;
        k.ms += ms;
        k.flops += r.flops;
        if (r.kernel == 3) {
            out->gemm_bf16x3.launches += 1;
            out->gemm_bf16x3.ms += ms;
            out->gemm_bf16x3.flops += r.flops;
        }
        if (r.heff) {
            out->heff.launches += 1;
            out->heff.flops += r.flops;
        }
    }
    for (const auto& m : h->mv_recs) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, h->ev_pool[m.ev], h->ev_pool[m.ev + 1]));
        out->heff.ms += ms;
        // the matvec launches' share of their precision class
        (h->prec == TTN_PREC_FP64 ? out->gemm_f64 : out->gemm_f32).ms += ms;
    }
}

// Captures step_body on a private stream into *exec (nullptr on failure).
void capture_step(ttn_handle* h, double tau, hipGraphExec_t* exec) {
    if (!h->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const hipStream_t saved = h->stream;
    h->stream = h->cap_stream;
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    try {
        step_body(h, tau);
    } catch (...) {
        (void)hipStreamEndCapture(h->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        h->stream = saved;
        throw;
    }
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    h->stream = saved;
    if (e == hipSuccess && g) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *exec = nullptr;
    }
}

// The step body is the same launch sequence every step (the Hamiltonian of
// the step lives in the leaf blocks, set before it), so it is captured once
// on a private stream and replayed on the handle's stream.  Profiling windows
// run it eagerly (timing events recorded inside graph replays cannot be read
// back on this runtime); a failed capture falls back to eager launches.
void run_step_body(ttn_handle* h) {
    const double tau = h->dt / 2;
    if (h->dry || h->prof || !h->use_graphs || h->graph_failed) {
        step_body(h, tau);
        return;
    }
    if (!h->step_graph || h->graph_dt != h->dt) {
        if (h->step_graph) HIPCHECK(hipGraphExecDestroy(h->step_graph));
        h->step_graph = nullptr;
        capture_step(h, tau, &h->step_graph);
        if (!h->step_graph) {
            h->graph_failed = true;
            step_body(h, tau);
            return;
        }
        h->graph_dt = h->dt;
    }
    HIPCHECK(hipGraphLaunch(h->step_graph, h->stream));
}

void apply_events_at(ttn_handle* h, int64_t step) {
    for (auto& e : h->events) {
        if (e.step != step || e.applied) continue;
        e.applied = true;
        int k = 0;
        while (h->leaf_site[k] != e.site) ++k;
        const int b = k / 2, side = k & 1;
        absorb(h, b, side, e.U, false);
    }
}

void canonicalise(ttn_handle* h) {
    std::vector<int> po;
    postorder(h, h->root, po);
    for (int v : po) {
        if (v == h->root) break;
        qr_toward(h, h->DL[v], h->DR[v], h->DP[v], h->T[v], 2, h->Rq);
        absorb(h, h->parent[v], leg_in_parent(h, v), h->Rq, false);
    }
    const int r = h->root;
    const int64_t n = nsize(h, r);
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, (n + 255) / 256);
    lz_start(h->T[r], n, h->T[r], 0, h->lz_obs, h->red, nb, h->stream);
}

void reset_step_dev(ttn_handle* h) {
    StepDev& s = h->h_stepinit;
    s = StepDev{};
    s.bad = 0;
    s.min_krylov = 1 << 30;
    const double big = 1e308;
    std::memcpy(&s.min_rdiag_bits, &big, sizeof(double));
    h2d(h, h->st, &s, sizeof(s));
}

// <x|y> into *out (complex) using the observation Lanczos scratch
void dot_c(ttn_handle* h, const double* x, const double* y, int64_t n, double out[2]) {
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, (n + 255) / 256);
    chk(h, x, 2 * n, "dot x");
    chk(h, y, 2 * n, "dot y");
    h2d(h, h->lz_obs, &h->h_lzinit, sizeof(LanczosDev));
    lz_project(x, 0, 1, y, n, h->red, nb, h->lz_obs, -1, h->stream);
    d2h(h, &h->h_lzout, h->lz_obs, sizeof(LanczosDev));
    sync(h);
    out[0] = h->h_lzout.c[0];
    out[1] = h->h_lzout.c[1];
}

// ||psi||^2 and <psi|H|psi> with the centre at the root (FP64 matvec)
void observables(ttn_handle* h, double* norm2, double* energy) {
    const int r = h->root;
    const int64_t n = nsize(h, r);
    Ctx<double> c{h, nullptr};
    OpDesc o = node_op(h, c, r);
    apply_op_prec(h, o, h->T[r], h->W, nullptr, true);
    double a[2], b[2];
    dot_c(h, h->T[r], h->T[r], n, a);
    dot_c(h, h->T[r], h->W, n, b);
    *norm2 = a[0];
    *energy = b[0];
}

// sum_i <psi|n_i|psi> with the centre at the root: the n_i of the sites below
// each child link of the root are slots 1.. of that link's operator stack
// (the leaf blocks when the root is a bottom node)
void rydberg_population(ttn_handle* h, double* pop) {
    const int r = h->root;
    const int DL = h->DL[r], DR = h->DR[r], DP = h->DP[r];
    const int sL = sites_left(h, r), sR = sL;
    const int64_t n = nsize(h, r);
    const int64_t L2 = (int64_t)DL * DL, R2 = (int64_t)DR * DR;
    const double* Lb = child_block(h, r, 0);
    const double* Rb = child_block(h, r, 1);
    chk(h, h->Rq, 2 * L2, "left number operator");
    chk(h, h->Cb, 2 * R2, "right number operator");
    chk(h, h->W, 2 * n, "number operator image");
    sum_mats(Lb + 2 * L2, DL, sL, h->Rq, h->stream);
    sum_mats(Rb + 2 * R2, DR, sR, h->Cb, h->stream);
    Ctx<double> c{h, nullptr};
    leg_apply<double>(c, 0, h->Rq, 0, h->T[r], 0, h->W, 0, DL, DR, DP, 1, 0);
    leg_apply<double>(c, 1, h->Cb, 0, h->T[r], 0, h->W, 0, DL, DR, DP, 1, 1);
    double a[2];
    dot_c(h, h->T[r], h->W, n, a);
    *pop = a[0];
}

// product-state overlap <phi|psi>, phi given per leaf (planar d-vectors, already conjugated)
void product_overlap(ttn_handle* h, const std::vector<double>& leafvec, double out[2]) {
    chk(h, h->ov_leaf, (int64_t)leafvec.size(), "leaf vectors");
    h2d(h, h->ov_leaf, leafvec.data(), leafvec.size() * sizeof(double));
    std::vector<int64_t> voff(h->n_nodes);
    int64_t o = 0;
    for (int v = 0; v < h->n_nodes; ++v) {
        voff[v] = o;
        o += 2 * h->DP[v];
    }
    for (int v = 0; v < h->n_nodes; ++v) {
        const double *a, *b;
        if (is_bottom(h, v)) {
            a = h->ov_leaf + (int64_t)2 * h->d * (2 * h->idx[v]);
            b = h->ov_leaf + (int64_t)2 * h->d * (2 * h->idx[v] + 1);
        } else {
            a = h->ov_vec + voff[h->ch0[v]];
            b = h->ov_vec + voff[h->ch1[v]];
        }
        chk(h, a, 2 * h->DL[v], "overlap a");
        chk(h, b, 2 * h->DR[v], "overlap b");
        chk(h, h->ov_vec + voff[v], 2 * h->DP[v], "overlap out");
        contract_node_vec(h->T[v], h->DL[v], h->DR[v], h->DP[v], a, b, h->ov_vec + voff[v], h->stream);
    }
    double res[2];
    d2h(h, res, h->ov_vec + voff[h->root], 2 * sizeof(double));
    sync(h);
    out[0] = res[0];
    out[1] = res[1];
}

// <a|b> by bottom-up contraction; node `mod` of b optionally replaced by modT
void ttn_contract(ttn_handle* a, ttn_handle* b, int mod, const double* modT, double out[2]) {
    ttn_handle* h = a;
    Ctx<double> c{h, nullptr};
    const int64_t Dm2 = (int64_t)h->Dmax * h->Dmax;
    for (int v = 0; v < h->n_nodes; ++v) {
        const int DL = h->DL[v], DR = h->DR[v], DP = h->DP[v];
        const double* TB = (v == mod) ? modT : b->T[v];
        double* M = h->ov_M + 2 * Dm2 * v;
        if (is_bottom(h, v)) {
            leg_gram(c, 2, a->T[v], TB, 0, M, 0, DL, DR, DP, 1);
        } else {
            const double* ML = h->ov_M + 2 * Dm2 * h->ch0[v];
            const double* MR = h->ov_M + 2 * Dm2 * h->ch1[v];
            leg_apply<double>(c, 0, ML, 0, TB, 0, h->ov_Y1, 0, DL, DR, DP, 1, 0);
            leg_apply<double>(c, 1, MR, 0, h->ov_Y1, 0, h->ov_Y2, 0, DL, DR, DP, 1, 0);
            leg_gram(c, 2, a->T[v], h->ov_Y2, 0, M, 0, DL, DR, DP, 1);
        }
    }
    double res[2];
    const double* Mr = h->ov_M + 2 * Dm2 * h->root;
    d2h(h, &res[0], Mr, sizeof(double));
    d2h(h, &res[1], Mr + 1, sizeof(double));
    sync(h);
    out[0] = res[0];
    out[1] = res[1];
}

// host-side initial isometries (product state, Gram-Schmidt completion, dressing)
void initial_tensors(ttn_handle* h, const ttn_config* cfg) {
    int64_t noff = 0;
    for (int v = 0; v < h->n_nodes; ++v) {
        const int DL = h->DL[v], DR = h->DR[v], DP = h->DP[v];
        const int64_t LR = (int64_t)DL * DR, n = LR * DP;
        std::vector<double> re(n, 0.0), im(n, 0.0);
        std::vector<std::vector<double>> cr, ci;   // accepted columns
        std::vector<double> c0r(LR, 0.0), c0i(LR, 0.0);
        if (is_bottom(h, v)) {
            const int a = h->leaf_site[2 * h->idx[v]], b = h->leaf_site[2 * h->idx[v] + 1];
            const double* pa = cfg->init_product + 2 * h->d * a;
            const double* pb = cfg->init_product + 2 * h->d * b;
            for (int r = 0; r < DR; ++r)
                for (int l = 0; l < DL; ++l) {
                    c0r[l + DL * r] = pa[2 * l] * pb[2 * r] - pa[2 * l + 1] * pb[2 * r + 1];
                    c0i[l + DL * r] = pa[2 * l] * pb[2 * r + 1] + pa[2 * l + 1] * pb[2 * r];
                }
        } else {
            c0r[0] = 1.0;
        }
        cr.push_back(c0r);
        ci.push_back(c0i);
        for (int64_t k = 0; k < LR && (int)cr.size() < DP; ++k) {
            // candidate e_k; modified Gram-Schmidt against the accepted columns.
            // While e is still the unit vector, <c_q, e> = conj(c_q[k]) and a
            // zero coefficient leaves e unchanged, so most columns of large
            // nodes cost O(1).
            std::vector<double> er(LR, 0.0), ei(LR, 0.0);
            er[k] = 1.0;
            bool unit = true;
            for (size_t q = 0; q < cr.size(); ++q) {
                double dr = 0, di = 0;   // <c_q, e>
                if (unit) {
                    dr = cr[q][k];
                    di = -ci[q][k];
                } else {
                    for (int64_t i = 0; i < LR; ++i) {
                        dr += cr[q][i] * er[i] + ci[q][i] * ei[i];
                        di += cr[q][i] * ei[i] - ci[q][i] * er[i];
                    }
                }
                if (dr == 0.0 && di == 0.0) continue;
                unit = false;
                for (int64_t i = 0; i < LR; ++i) {
                    er[i] -= dr * cr[q][i] - di * ci[q][i];
                    ei[i] -= dr * ci[q][i] + di * cr[q][i];
                }
            }
            double nrm = 0;
            for (int64_t i = 0; i < LR; ++i) nrm += er[i] * er[i] + ei[i] * ei[i];
            nrm = std::sqrt(nrm);
            if (nrm > COMPLETION_TOL) {
                for (int64_t i = 0; i < LR; ++i) {
                    er[i] /= nrm;
                    ei[i] /= nrm;
                }
                cr.push_back(er);
                ci.push_back(ei);
            }
        }
        if ((int)cr.size() != DP) throw StatusError{TTN_EINVAL, "isometry completion failed"};
        for (int p = 0; p < DP; ++p)
            for (int64_t i = 0; i < LR; ++i) {
                re[i + LR * p] = cr[p][i];
                im[i + LR * p] = ci[p][i];
            }
        if (cfg->dress_eps > 0) {
            if (!cfg->dress_noise || noff + n > cfg->dress_noise_len)
                throw StatusError{TTN_EINVAL, "dressing noise stream too short"};
            const double sc = cfg->dress_eps / std::sqrt((double)LR);
            for (int64_t i = 0; i < n; ++i) {
                re[i] += sc * cfg->dress_noise[2 * (noff + i)];
                im[i] += sc * cfg->dress_noise[2 * (noff + i) + 1];
            }
        }
        noff += n;
        h2d(h, h->T[v], re.data(), n * sizeof(double));
        h2d(h, h->T[v] + n, im.data(), n * sizeof(double));
        sync(h);
    }
}

void validate(const ttn_config* c) {
    if (!c) throw StatusError{TTN_EINVAL, "null config"};
    if (c->n_sites < 2 || c->n_sites > 1024 || (c->n_sites & (c->n_sites - 1)))
        throw StatusError{TTN_EINVAL, "n_sites must be a power of two in [2, 1024]"};
    if (c->d < 3 || c->d > 4) throw StatusError{TTN_EINVAL, "d must be 3 or 4"};
    if (c->chi < 1 || c->chi > 256) throw StatusError{TTN_EINVAL, "chi must be in [1, 256]"};
    if (c->krylov_dim < 1 || c->krylov_dim > KRYLOV_MAX)
        throw StatusError{TTN_EINVAL, "krylov_dim must be in [1, 16]"};
    if (c->precision != TTN_PREC_FP64 && c->precision != TTN_PREC_FP32 && c->precision != TTN_PREC_BF16X3)
        throw StatusError{TTN_EINVAL, "unknown precision"};
    if (!c->pos_xy || !c->leaf_order || !c->init_product)
        throw StatusError{TTN_EINVAL, "missing positions, leaf order or initial product state"};
    std::vector<char> seen(c->n_sites, 0);
    for (int k = 0; k < c->n_sites; ++k) {
        const int s = c->leaf_order[k];
        if (s < 0 || s >= c->n_sites || seen[s]) throw StatusError{TTN_EINVAL, "leaf order is not a permutation"};
        seen[s] = 1;
    }
    if (!(c->dress_eps >= 0) || !std::isfinite(c->c6) || !std::isfinite(c->leak_ratio) ||
        !(c->gamma >= 0) || !std::isfinite(c->gamma))
        throw StatusError{TTN_EINVAL, "bad scalar parameter"};
    if (c->update != TTN_UPDATE_ONE_SITE && c->update != TTN_UPDATE_TWO_SITE)
        throw StatusError{TTN_EINVAL, "unknown update"};
    if (c->update == TTN_UPDATE_TWO_SITE) {
        if (c->precision != TTN_PREC_FP64) throw StatusError{TTN_ENOTSUP, "the two-site update runs in FP64 only"};
        if (c->gamma != 0.0) throw StatusError{TTN_ENOTSUP, "the two-site update needs a closed system"};
        if (c->n_sites < 4) throw StatusError{TTN_ENOTSUP, "the two-site update needs at least four sites"};
    }
    for (int i = 0; i < c->n_sites; ++i)
        for (int j = 0; j < i; ++j)
            if (c->pos_xy[2 * i] == c->pos_xy[2 * j] && c->pos_xy[2 * i + 1] == c->pos_xy[2 * j + 1])
                throw StatusError{TTN_EINVAL, "two sites share a position"};
}

void setup_config(ttn_handle* h, const ttn_config* c) {
    h->N = c->n_sites;
    h->d = c->d;
    h->chi = c->chi;
    h->m = c->krylov_dim;
    // BF16x3 runs the mixed path with split-product contractions
    h->prec = c->precision == TTN_PREC_BF16X3 ? TTN_PREC_FP32 : c->precision;
    h->split_bf16 = c->precision == TTN_PREC_BF16X3;
    h->c6 = c->c6;
    h->rcut = c->r_cut;
    h->leak = c->leak_ratio;
    h->gamma = c->gamma;
    h->nonherm = c->gamma != 0.0;
    h->leaf_site.assign(c->leaf_order, c->leaf_order + c->n_sites);
    h->two_site = c->update == TTN_UPDATE_TWO_SITE;
    build_tree(h);
    if (h->two_site)
        for (int v = 0; v < h->n_nodes; ++v) {
            if (v == h->root) continue;
            const Edge2 e = edge2(h, v);
            if (std::min(e.m, e.n) > JAC_NMAX)
                throw StatusError{TTN_ENOTSUP, "two-site split wider than the eigensolver (smaller side of a merged "
                                               "tensor above 256)"};
        }
}

// van der Waals couplings V_ij = C6 / d_ij^6 (Eq. c6, positive, i != j, cutoff)
void build_couplings(ttn_handle* h, const double* pos) {
    h->V.assign((size_t)h->N * h->N, 0.0);
    for (int i = 0; i < h->N; ++i)
        for (int j = 0; j < h->N; ++j) {
            if (i == j) continue;
            const double dx = pos[2 * i] - pos[2 * j], dy = pos[2 * i + 1] - pos[2 * j + 1];
            const double dist = std::sqrt(dx * dx + dy * dy);
            if (h->rcut > 0 && dist > h->rcut) continue;
            h->V[(size_t)i * h->N + j] = h->c6 / std::pow(dist, 6);
        }
    for (int v = 0; v < h->n_nodes; ++v) {
        const int sL = sites_left(h, v), f = h->sfirst[v];
        std::vector<double> lr(2 * (size_t)sL * sL, 0.0), rl(2 * (size_t)sL * sL, 0.0);
        for (int i = 0; i < sL; ++i)
            for (int j = 0; j < sL; ++j) {
                const int si = h->leaf_site[f + i], sj = h->leaf_site[f + sL + j];
                const double val = h->V[(size_t)si * h->N + sj];
                lr[i + (size_t)sL * j] = val;   // V[i in L][j in R], column-major i + sL j
                rl[j + (size_t)sL * i] = val;   // V[j in R][i in L] transposed layout
            }
        h2d(h, h->vLR[v], lr.data(), lr.size() * sizeof(double));
        h2d(h, h->vRL[v], rl.data(), rl.size() * sizeof(double));
        sync(h);
    }
}

thread_local std::string g_init_error;

int fail(ttn_handle* h, const StatusError& e) {
    if (h) {
        h->err = e.msg;
        if (e.code == TTN_ENUMERIC || e.code == TTN_EDEVICE) h->poisoned = true;
    }
    return e.code;
}

void check_step_flags(ttn_handle* h, StepDev* out) {
    StepDev& s = h->h_stepout;
    d2h(h, &s, h->st, sizeof(s));
    sync(h);
    if (h->dry) {
        s.min_krylov = h->m;
        const double one = 1.0;
        std::memcpy(&s.min_rdiag_bits, &one, sizeof(double));
    }
    if (out) *out = s;
    if (s.bad) throw StatusError{TTN_ENUMERIC, "non-positive pivot in a QR gauge move (rank-deficient node)"};
}

#include "adjoint.inc"
#include "sampling.inc"

// A device-free handle for plan checks: workspace carved at a fake address,
// the initial network built and a one-segment program with a gate on every site.
ttn_handle* make_dry_handle(const ttn_config* cfg, size_t bytes);

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int ttn_workspace_query(const ttn_config* cfg, size_t* device_bytes) {
    try {
        validate(cfg);
        if (!device_bytes) return TTN_EINVAL;
        ttn_handle h;
        setup_config(&h, cfg);
        Bump b(nullptr, 0);
        plan(&h, b);
        *device_bytes = b.off + 256;
        return TTN_OK;
    } catch (const StatusError& e) {
        return e.code;
    } catch (...) {
        return TTN_EINVAL;
    }
}

int ttn_init(const ttn_config* cfg, void* d_workspace, size_t bytes, void* hip_stream, ttn_handle** out) {
    if (!out) return TTN_EINVAL;
    *out = nullptr;
    ttn_handle* h = nullptr;
    try {
        validate(cfg);
        if (!d_workspace) return TTN_EINVAL;
        h = new ttn_handle();
        h->stream = (hipStream_t)hip_stream;
        setup_config(h, cfg);
        Bump b(d_workspace, bytes, &h->regions);
        plan(h, b);
        sort_regions(h);
        h->ws_bytes = bytes;
        h2d(h, h->d_leaf_site, h->leaf_site.data(), h->N * sizeof(int));
        build_couplings(h, cfg->pos_xy);
        initial_tensors(h, cfg);
        reset_step_dev(h);
        if (!h->dry) HIPCHECK(hipGetLastError());
        canonicalise(h);
        if (!h->dry) HIPCHECK(hipGetLastError());
        StepDev s;
        check_step_flags(h, &s);
        *out = h;
        return TTN_OK;
    } catch (const StatusError& e) {
        g_init_error = e.msg;
        delete h;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_init_error = "host allocation failed";
        delete h;
        return TTN_ENOMEM;
    } catch (...) {
        g_init_error = "unexpected exception";
        delete h;
        return TTN_EINVAL;
    }
}

int ttn_set_pulses(ttn_handle* h, int32_t n_seg, const double* seg_edges, const double* omega,
                   const double* delta, int32_t n_events, const int32_t* ev_step, const int32_t* ev_site,
                   const double* ev_u) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    if (h->adj) h->adj->active = false;   // a recording is tied to one pulse table
    try {
        if (n_seg < 0 || (n_seg > 0 && (!seg_edges || !omega || !delta)) || n_events < 0 ||
            (n_events > 0 && (!ev_step || !ev_site || !ev_u)))
            throw StatusError{TTN_EINVAL, "bad pulse arguments"};
        for (int s = 0; s < n_seg; ++s)
            if (!(seg_edges[s + 1] > seg_edges[s])) throw StatusError{TTN_EINVAL, "segment edges must ascend"};
        for (int64_t i = 0; i < (int64_t)h->N * n_seg; ++i)
            if (!std::isfinite(omega[i]) || !std::isfinite(delta[i]))
                throw StatusError{TTN_EINVAL, "non-finite pulse value"};
        for (int e = 0; e < n_events; ++e) {
            if (ev_site[e] < 0 || ev_site[e] >= h->N || ev_step[e] < 0)
                throw StatusError{TTN_EINVAL, "bad gate event"};
            for (int k = 0; k < 2 * h->d * h->d; ++k)
                if (!std::isfinite(ev_u[(int64_t)e * 2 * h->d * h->d + k]))
                    throw StatusError{TTN_EINVAL, "non-finite gate"};
        }
        // device copies of the program (small; allocated here, outside the workspace)
        auto drop_region = [h](const void* p) {
            h->regions.erase(std::remove_if(h->regions.begin(), h->regions.end(),
                                            [p](const Region& r) { return r.lo == (uintptr_t)p; }),
                             h->regions.end());
        };
        for (double** pp : {&h->d_omega, &h->d_delta, &h->d_evU, &h->d_omx, &h->d_omz}) {
            if (*pp) {
                drop_region(*pp);
                if (!h->dry) HIPCHECK(hipFree(*pp));
                *pp = nullptr;
            }
        }
        const int dd = h->d * h->d;
        const int64_t ns = std::max<int64_t>(1, (int64_t)h->N * n_seg);
        const int64_t nu = std::max<int64_t>(1, (int64_t)n_events * 2 * dd);
        if (h->dry) {
            // distinct fake addresses far above the workspace, never dereferenced
            const uintptr_t top = (h->regions.empty() ? 0 : h->regions.back().hi) + (uintptr_t(1) << 32);
            h->d_omega = (double*)top;
            h->d_delta = (double*)(top + (uintptr_t(1) << 30));
            h->d_evU = (double*)(top + (uintptr_t(2) << 30));
        } else {
            HIPCHECK(hipMalloc(&h->d_omega, ns * sizeof(double)));
            HIPCHECK(hipMalloc(&h->d_delta, ns * sizeof(double)));
            HIPCHECK(hipMalloc(&h->d_evU, nu * sizeof(double)));
            if (n_seg > 0) {
                HIPCHECK(hipMemcpy(h->d_omega, omega, (int64_t)h->N * n_seg * sizeof(double), hipMemcpyHostToDevice));
                HIPCHECK(hipMemcpy(h->d_delta, delta, (int64_t)h->N * n_seg * sizeof(double), hipMemcpyHostToDevice));
            }
        }
        h->regions.push_back(Region{(uintptr_t)h->d_omega, (uintptr_t)h->d_omega + ns * sizeof(double)});
        h->regions.push_back(Region{(uintptr_t)h->d_delta, (uintptr_t)h->d_delta + ns * sizeof(double)});
        h->regions.push_back(Region{(uintptr_t)h->d_evU, (uintptr_t)h->d_evU + nu * sizeof(double)});
        sort_regions(h);
        h->n_seg = n_seg;
        h->edges.assign(seg_edges, seg_edges + (n_seg > 0 ? n_seg + 1 : 0));
        h->events.clear();
        if (n_events > 0) {
            std::vector<double> planar((int64_t)n_events * 2 * dd);
            for (int e = 0; e < n_events; ++e)
                for (int a = 0; a < h->d; ++a)
                    for (int b2 = 0; b2 < h->d; ++b2) {
                        const double* src = ev_u + (int64_t)e * 2 * dd + 2 * (a * h->d + b2);
                        planar[(int64_t)e * 2 * dd + a + h->d * b2] = src[0];
                        planar[(int64_t)e * 2 * dd + dd + a + h->d * b2] = src[1];
                    }
            if (!h->dry)
                HIPCHECK(hipMemcpy(h->d_evU, planar.data(), planar.size() * sizeof(double), hipMemcpyHostToDevice));
            for (int e = 0; e < n_events; ++e)
                if (ev_step[e] >= h->step_count)
                    h->events.push_back(Event{ev_step[e], ev_site[e], h->d_evU + (int64_t)e * 2 * dd, false});
        }
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_set_qubit_pulses(ttn_handle* h, const double* omega_x, const double* omega_z) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (!h->d_omega) throw StatusError{TTN_ESTATE, "ttn_set_pulses must be called first"};
        const int64_t cnt = (int64_t)h->N * h->n_seg;
        for (const double* a : {omega_x, omega_z})
            if (a)
                for (int64_t i = 0; i < cnt; ++i)
                    if (!std::isfinite(a[i])) throw StatusError{TTN_EINVAL, "non-finite pulse value"};
        if (h->adj) h->adj->active = false;   // a recording is tied to one pulse table
        for (double** pp : {&h->d_omx, &h->d_omz}) {
            if (*pp) {
                const uintptr_t lo = (uintptr_t)*pp;
                h->regions.erase(std::remove_if(h->regions.begin(), h->regions.end(),
                                                [lo](const Region& r) { return r.lo == lo; }),
                                 h->regions.end());
                if (!h->dry) HIPCHECK(hipFree(*pp));
                *pp = nullptr;
            }
        }
        if (!omega_x && !omega_z) return TTN_OK;
        const int64_t ns = std::max<int64_t>(1, cnt);
        std::vector<double> zero;
        if (!omega_x || !omega_z) zero.assign(ns, 0.0);
        const double* src[2] = {omega_x ? omega_x : zero.data(), omega_z ? omega_z : zero.data()};
        double** dst[2] = {&h->d_omx, &h->d_omz};
        for (int k = 0; k < 2; ++k) {
            if (h->dry) {
                const uintptr_t top = (h->regions.empty() ? 0 : h->regions.back().hi) + (uintptr_t(1) << 32);
                *dst[k] = (double*)top;
            } else {
                HIPCHECK(hipMalloc(dst[k], ns * sizeof(double)));
                if (cnt > 0) HIPCHECK(hipMemcpy(*dst[k], src[k], cnt * sizeof(double), hipMemcpyHostToDevice));
            }
            h->regions.push_back(Region{(uintptr_t)*dst[k], (uintptr_t)*dst[k] + ns * sizeof(double)});
            sort_regions(h);
        }
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_tdvp_step(ttn_handle* h, double dt, int32_t n_steps, ttn_step_stats* stats) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (!(dt > 0) || !std::isfinite(dt) || n_steps < 0) throw StatusError{TTN_EINVAL, "bad dt or n_steps"};
        if (h->dt_set && dt != h->dt) throw StatusError{TTN_EINVAL, "dt must not change between calls"};
        if (!h->d_omega) throw StatusError{TTN_ESTATE, "ttn_set_pulses must be called first"};
        h->dt = dt;
        h->dt_set = true;
        for (int i = 0; i < n_steps; ++i) {
            reset_step_dev(h);
            apply_events_at(h, h->step_count);
            record_step_start(h);
            const double t = ((double)h->step_count + 0.5) * dt;
            set_hamiltonian(h, segment_at(h, t));
            run_step_body(h);
            record_step_end(h);
            h->step_count += 1;
            if (stats) {
                StepDev s;
                check_step_flags(h, &s);
                ttn_step_stats& o = stats[i];
                observables(h, &o.norm2, &o.energy);
                std::memcpy(&o.min_r_diag, &s.min_rdiag_bits, sizeof(double));
                std::memcpy(&o.max_discarded, &s.max_disc_bits, sizeof(double));
                o.min_krylov = s.min_krylov;
                o.reserved = 0;
                // closed system: the norm is conserved; open system: it may only decay
                const bool drift = h->nonherm ? o.norm2 > 1.0 + 1e-6 : std::fabs(o.norm2 - 1.0) > 1e-6;
                if (!h->dry && (!std::isfinite(o.norm2) || drift))
                    throw StatusError{TTN_ENUMERIC, "norm drift beyond 1e-6"};
            }
        }
        apply_events_at(h, h->step_count);
        check_step_flags(h, nullptr);
        if (!h->dry) HIPCHECK(hipGetLastError());
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_fidelity(ttn_handle* h, int32_t n_target, const int32_t* target_sites, double* F, double overlap[2]) {
    if (!h || !F) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (n_target < 0 || (n_target > 0 && !target_sites)) throw StatusError{TTN_EINVAL, "bad target"};
        std::vector<char> in(h->N, 0);
        for (int i = 0; i < n_target; ++i) {
            if (target_sites[i] < 0 || target_sites[i] >= h->N) throw StatusError{TTN_EINVAL, "bad target site"};
            in[target_sites[i]] = 1;
        }
        const int d = h->d;
        std::vector<double> zero((size_t)2 * h->N * d, 0.0), one((size_t)2 * h->N * d, 0.0);
        for (int k = 0; k < h->N; ++k) {
            zero[(size_t)2 * d * k + 0] = 1.0;
            one[(size_t)2 * d * k + (in[h->leaf_site[k]] ? 1 : 0)] = 1.0;
        }
        double o0[2], o1[2];
        product_overlap(h, zero, o0);
        product_overlap(h, one, o1);
        const double s = 1.0 / std::sqrt(2.0);
        const double re = s * (o0[0] + o1[0]), im = s * (o0[1] + o1[1]);
        *F = re * re + im * im;
        if (overlap) {
            overlap[0] = re;
            overlap[1] = im;
        }
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_observables(ttn_handle* h, double* norm2, double* energy) {
    if (!h || !norm2 || !energy) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (h->cur_seg == -2) {
            set_hamiltonian(h, h->d_omega ? segment_at(h, 0.0) : -1);
            if (!h->d_omega) h->cur_seg = -1;
            rebuild_up(h);
        }
        observables(h, norm2, energy);
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_rydberg_population(ttn_handle* h, double* pop) {
    if (!h || !pop) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (h->cur_seg == -2) {
            set_hamiltonian(h, h->d_omega ? segment_at(h, 0.0) : -1);
            if (!h->d_omega) h->cur_seg = -1;
            rebuild_up(h);
        }
        rydberg_population(h, pop);
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_local_expectation(ttn_handle* h, int32_t site, const double* op, double out[2]) {
    if (!h || !op || !out) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (site < 0 || site >= h->N) throw StatusError{TTN_EINVAL, "bad site"};
        const int d = h->d, dd = d * d;
        std::vector<double> planar(2 * dd);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                planar[a + d * b] = op[2 * (a * d + b)];
                planar[dd + a + d * b] = op[2 * (a * d + b) + 1];
            }
        h2d(h, h->opbuf, planar.data(), planar.size() * sizeof(double));
        int k = 0;
        while (h->leaf_site[k] != site) ++k;
        const int b = k / 2, side = k & 1;
        Ctx<double> c{h, nullptr};
        leg_apply<double>(c, side, h->opbuf, 0, h->T[b], 0, h->Ttmp, 0, h->DL[b], h->DR[b], h->DP[b], 1, 0);
        ttn_contract(h, h, b, h->Ttmp, out);
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_overlap(ttn_handle* a, ttn_handle* b, double out[2]) {
    if (!a || !b || !out) return TTN_EINVAL;
    if (a->poisoned || b->poisoned) return TTN_ESTATE;
    try {
        if (a->N != b->N || a->d != b->d || a->chi != b->chi || a->leaf_site != b->leaf_site)
            throw StatusError{TTN_EINVAL, "handles differ in shape"};
        sync(b);
        std::vector<Region> own = a->regions;
        a->regions.insert(a->regions.end(), b->regions.begin(), b->regions.end());
        sort_regions(a);
        try {
            ttn_contract(a, b, -1, nullptr, out);
        } catch (...) {
            a->regions = own;
            sort_regions(a);
            throw;
        }
        a->regions = own;
        sort_regions(a);
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(a, e);
    }
}

int64_t ttn_export_state(ttn_handle* h, double* host, int64_t len) {
    if (!h) return TTN_EINVAL;
    int64_t total = 0;
    for (int v = 0; v < h->n_nodes; ++v) total += nsize(h, v);
    if (!host) return total;
    if (h->poisoned) return TTN_ESTATE;
    if (len < total) return TTN_EINVAL;
    try {
        int64_t o = 0;
        std::vector<double> buf;
        for (int v = 0; v < h->n_nodes; ++v) {
            const int64_t n = nsize(h, v);
            buf.resize(2 * n);
            d2h(h, buf.data(), h->T[v], 2 * n * sizeof(double));
            sync(h);
            for (int64_t i = 0; i < n; ++i) {
                host[2 * (o + i)] = buf[i];
                host[2 * (o + i) + 1] = buf[n + i];
            }
            o += n;
        }
        return total;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

namespace {

// Checks the arguments of a leg contraction and enqueues it on `stream`, with
// `partial` (bytes) as split-K scratch.  Throws StatusError.
void leg_contract_enqueue(int32_t precision, int32_t leg, int32_t DL, int32_t DR, int32_t DP, int32_t n_ops,
                          const void* d_ops, const void* d_x, int32_t x_per_op, void* d_y, int32_t sum_ops,
                          int32_t accumulate, hipStream_t stream, void* partial, int64_t bytes) {
    if (precision != TTN_PREC_FP64 && precision != TTN_PREC_FP32 && precision != TTN_PREC_BF16X3)
        throw StatusError{TTN_EINVAL, "bad precision"};
    if (leg < 0 || leg > 2 || DL < 1 || DR < 1 || DP < 1 || n_ops < 1 || !d_ops || !d_x || !d_y)
        throw StatusError{TTN_EINVAL, "bad leg, dimensions or pointers"};
    if (sum_ops && !x_per_op) throw StatusError{TTN_EINVAL, "sum_ops requires x_per_op"};
    const int D = leg == 0 ? DL : (leg == 1 ? DR : DP);
    const int64_t n = (int64_t)DL * DR * DP, D2 = (int64_t)D * D;
    const size_t esz = precision == TTN_PREC_FP64 ? 8 : 4;
    ttn_handle h;
    h.stream = stream;
    h.split_bf16 = precision == TTN_PREC_BF16X3;
    // operand regions come from the argument sizes
    const int nx = x_per_op ? n_ops : 1, ny = sum_ops ? 1 : n_ops;
    h.regions.push_back(Region{(uintptr_t)d_ops, (uintptr_t)d_ops + 2 * D2 * n_ops * esz});
    h.regions.push_back(Region{(uintptr_t)d_x, (uintptr_t)d_x + 2 * n * nx * esz});
    h.regions.push_back(Region{(uintptr_t)d_y, (uintptr_t)d_y + 2 * n * ny * esz});
    h.gs.partial = partial;
    h.gs.bytes = bytes;
    sort_regions(&h);
    if (precision != TTN_PREC_FP64) {
        Ctx<float> c{&h, nullptr};
        if (sum_ops)
            leg_apply_sum<float>(c, leg, (const float*)d_ops, 2 * D2, (const float*)d_x, 2 * n, (float*)d_y, DL, DR,
                                 DP, n_ops, accumulate ? 1 : 0);
        else
            leg_apply<float>(c, leg, (const float*)d_ops, 2 * D2, (const float*)d_x, x_per_op ? 2 * n : 0,
                             (float*)d_y, 2 * n, DL, DR, DP, n_ops, accumulate ? 1 : 0);
    } else {
        Ctx<double> c{&h, nullptr};
        if (sum_ops)
            leg_apply_sum<double>(c, leg, (const double*)d_ops, 2 * D2, (const double*)d_x, 2 * n, (double*)d_y,
                                  DL, DR, DP, n_ops, accumulate ? 1 : 0);
        else
            leg_apply<double>(c, leg, (const double*)d_ops, 2 * D2, (const double*)d_x, x_per_op ? 2 * n : 0,
                              (double*)d_y, 2 * n, DL, DR, DP, n_ops, accumulate ? 1 : 0);
    }
    HIPCHECK(hipGetLastError());
}

// Split-K scratch of the allocating entry point, and the size of the
// file-scope array of the no-allocation one: the same size, so that both
// choose the same split factors and give the same bits.
constexpr int64_t LEG_SCRATCH_BYTES = (int64_t)64 << 20;

// Split-K scratch of ttn_leg_contract_noalloc: every GPU the library runs on
// holds one copy until the process ends.  Host code never uses this name as
// an address; it uses the per-device pointer from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[LEG_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up once per device with
// that device current.
void* scratch_for_current_device() {
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) throw StatusError{TTN_EDEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw StatusError{TTN_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

int ttn_leg_contract(int32_t precision, int32_t leg, int32_t DL, int32_t DR, int32_t DP, int32_t n_ops,
                     const void* d_ops, const void* d_x, int32_t x_per_op, void* d_y, int32_t sum_ops,
                     int32_t accumulate, void* hip_stream) {
    void* partial = nullptr;
    try {
        const hipStream_t st = (hipStream_t)hip_stream;
        HIPCHECK(hipMalloc(&partial, LEG_SCRATCH_BYTES));
        leg_contract_enqueue(precision, leg, DL, DR, DP, n_ops, d_ops, d_x, x_per_op, d_y, sum_ops, accumulate, st,
                             partial, LEG_SCRATCH_BYTES);
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipFree(partial));
        return TTN_OK;
    } catch (const StatusError& e) {
        if (partial) {
            (void)hipStreamSynchronize((hipStream_t)hip_stream);
            (void)hipFree(partial);
        }
        g_init_error = e.msg;
        return e.code;
    }
}

int ttn_leg_contract_noalloc(int32_t precision, int32_t leg, int32_t DL, int32_t DR, int32_t DP, int32_t n_ops,
                             const void* d_ops, const void* d_x, int32_t x_per_op, void* d_y, int32_t sum_ops,
                             int32_t accumulate, void* hip_stream) {
    try {
        void* partial = scratch_for_current_device();
        leg_contract_enqueue(precision, leg, DL, DR, DP, n_ops, d_ops, d_x, x_per_op, d_y, sum_ops, accumulate,
                             (hipStream_t)hip_stream, partial, LEG_SCRATCH_BYTES);
        return TTN_OK;
    } catch (const StatusError& e) {
        g_init_error = e.msg;
        return e.code;
    }
}

int ttn_herm_eig(int32_t n, void* d_a, void* d_v, void* d_w, void* d_order, void* hip_stream) {
    StepDev* st = nullptr;
    const hipStream_t s = (hipStream_t)hip_stream;
    try {
        if (n < 1 || n > JAC_NMAX || !d_a || !d_v || !d_w || !d_order)
            throw StatusError{TTN_EINVAL, "bad size or pointer"};
        HIPCHECK(hipMalloc(&st, sizeof(StepDev)));
        HIPCHECK(hipMemsetAsync(st, 0, sizeof(StepDev), s));
        herm_eig((double*)d_a, n, (double*)d_v, (double*)d_w, (int*)d_order, st, s);
        StepDev hs;
        HIPCHECK(hipMemcpyAsync(&hs, st, sizeof(StepDev), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        HIPCHECK(hipFree(st));
        st = nullptr;
        if (hs.bad) throw StatusError{TTN_ENUMERIC, "Jacobi iteration did not converge"};
        return TTN_OK;
    } catch (const StatusError& e) {
        if (st) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(st);
        }
        g_init_error = e.msg;
        return e.code;
    }
}

int ttn_profile_begin(ttn_handle* h) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    h->prof = true;
    h->prof_timed = true;
    h->prof_recs.clear();
    h->vec_recs.clear();
    h->mv_recs.clear();
    h->ev_used = 0;
    h->prof_matvecs = 0;
    return TTN_OK;
}

int ttn_profile_begin_untimed(ttn_handle* h) {
    const int rc = ttn_profile_begin(h);
    if (rc == TTN_OK) h->prof_timed = false;
    return rc;
}

int ttn_profile_end(ttn_handle* h, ttn_profile* out) {
    if (!h || !out) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        sync(h);
        std::memset(out, 0, sizeof(*out));
        accumulate_prof(h, out);
        out->matvecs = h->prof_matvecs;
        h->prof_last.clear();
        for (const auto& r : h->prof_recs)
            h->prof_last.push_back(ttn_launch_rec{r.kernel, r.prec, r.heff ? 1 : 0, r.splits, r.matvec, 0, r.flops,
                                                  launch_ms(r, h->ev_pool)});
        for (const auto& r : h->vec_recs) {
            float ms = 0.f;
            HIPCHECK(hipEventElapsedTime(&ms, h->ev_pool[r.ev], h->ev_pool[r.ev + 1]));
            for (ttn_vec_prof* p : {&out->lanczos, r.n >= (1 << 20) ? &out->lanczos_large : nullptr}) {
                if (!p) continue;
                p->calls += 1;
                p->ms += ms;
                p->bytes += r.bytes;
            }
        }
        h->prof = false;
        h->prof_recs.clear();
        h->vec_recs.clear();
        h->mv_recs.clear();
        return TTN_OK;
    } catch (const StatusError& e) {
        h->prof = false;
        h->vec_recs.clear();
        h->mv_recs.clear();
        return fail(h, e);
    }
}

int64_t ttn_profile_launches(const ttn_handle* h, ttn_launch_rec* out, int64_t max) {
    if (!h || max < 0) return TTN_EINVAL;
    const int64_t n = (int64_t)h->prof_last.size();
    if (out)
        for (int64_t i = 0; i < std::min(n, max); ++i) out[i] = h->prof_last[i];
    return n;
}

int ttn_validate_plan(const ttn_config* cfg, int32_t n_steps, char* msg, int32_t msg_len) {
    ttn_handle* h = nullptr;
    auto report = [&](const std::string& m) {
        if (msg && msg_len > 0) snprintf(msg, msg_len, "%s", m.c_str());
    };
    try {
        validate(cfg);
        size_t bytes = 0;
        int rc = ttn_workspace_query(cfg, &bytes);
        if (rc != TTN_OK) return rc;
        g_dry_run = true;
        h = make_dry_handle(cfg, bytes);
        const int N = h->N, d = h->d;
        // record the steps for the adjoint, then walk the backward pass too
        // (closed systems only: the adjoint rejects an open system)
        const bool adj = !h->nonherm && !h->two_site;
        const int32_t k = std::max(1, n_steps / 2);
        {   // single-qubit channels on every site
            std::vector<double> ones((size_t)N * h->n_seg, 1.0);
            rc = ttn_set_qubit_pulses(h, ones.data(), ones.data());
            if (rc != TTN_OK) throw StatusError{rc, h->err};
        }
        if (adj) {
            const size_t abytes = adjoint_bytes(h, n_steps, k);
            void* afake = (void*)(uintptr_t(1) << 45);
            rc = ttn_record_begin(h, n_steps, k, afake, abytes);
            if (rc != TTN_OK) throw StatusError{rc, h->err};
        }
        std::vector<ttn_step_stats> stats(std::max(1, n_steps));
        rc = ttn_tdvp_step(h, 0.01, n_steps, stats.data());
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        double F, ov[2];
        std::vector<int32_t> all(N);
        for (int i = 0; i < N; ++i) all[i] = i;
        rc = ttn_fidelity(h, N, all.data(), &F, ov);
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        std::vector<double> op((size_t)2 * d * d, 0.0);
        rc = ttn_local_expectation(h, N - 1, op.data(), ov);
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        rc = ttn_overlap(h, h, ov);
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        rc = ttn_rydberg_population(h, ov);
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        if (adj) {
            std::vector<double> go((size_t)N * h->n_seg), gd((size_t)N * h->n_seg);
            rc = ttn_backward(h, N, all.data(), 1.0, go.data(), gd.data());
            if (rc != TTN_OK) throw StatusError{rc, h->err};
        }
        size_t sbytes = 0;
        rc = ttn_sample_query(h, 3, &sbytes);
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        std::vector<uint8_t> cfgs(7 * (size_t)N);
        std::vector<double> amp(14);
        rc = ttn_sample(h, 7, 1, 0, (void*)(uintptr_t(1) << 47), sbytes, cfgs.data(), amp.data());
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        g_dry_run = false;
        report("ok");
        ttn_destroy(h);
        return TTN_OK;
    } catch (const StatusError& e) {
        g_dry_run = false;
        report(e.msg);
        if (h) ttn_destroy(h);
        return e.code;
    } catch (...) {
        g_dry_run = false;
        report("unexpected exception");
        if (h) ttn_destroy(h);
        return TTN_EINVAL;
    }
}

int ttn_sample_query(ttn_handle* h, int32_t batch, size_t* device_bytes) {
    if (!h || !device_bytes || batch < 1) return TTN_EINVAL;
    SampleBufs probe;
    *device_bytes = sample_carve(h, batch, nullptr, 0, &probe) + 256;
    return TTN_OK;
}

int ttn_sample(ttn_handle* h, int64_t n_shots, uint64_t seed, int64_t shot0, void* d_buf, size_t bytes,
               uint8_t* configs, double* amps) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (n_shots < 0 || shot0 < 0 || !d_buf) throw StatusError{TTN_EINVAL, "bad shot count or buffer"};
        if (h->d > 8) throw StatusError{TTN_ENOTSUP, "sampling supports d <= 8"};
        sample_shots(h, n_shots, seed, shot0, (char*)d_buf, bytes, configs, amps);
        if (!h->dry) HIPCHECK(hipGetLastError());
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_set_graphs(ttn_handle* h, int32_t enabled) {
    if (!h) return TTN_EINVAL;
    h->use_graphs = enabled != 0;
    return TTN_OK;
}

int ttn_adjoint_query(const ttn_config* cfg, int32_t n_steps, int32_t ckpt_every, size_t* device_bytes) {
    if (!cfg || !device_bytes || n_steps < 0 || ckpt_every < 1) return TTN_EINVAL;
    ttn_handle* h = nullptr;
    try {
        validate(cfg);
        size_t bytes = 0;
        int rc = ttn_workspace_query(cfg, &bytes);
        if (rc != TTN_OK) return rc;
        g_dry_run = true;
        h = make_dry_handle(cfg, bytes);
        *device_bytes = adjoint_bytes(h, n_steps, ckpt_every);
        g_dry_run = false;
        ttn_destroy(h);
        return TTN_OK;
    } catch (const StatusError& e) {
        g_dry_run = false;
        g_init_error = e.msg;
        if (h) ttn_destroy(h);
        return e.code;
    } catch (...) {
        g_dry_run = false;
        g_init_error = "unexpected exception";
        if (h) ttn_destroy(h);
        return TTN_EINVAL;
    }
}

int ttn_record_begin(ttn_handle* h, int32_t n_steps, int32_t ckpt_every, void* d_buf, size_t bytes) {
    if (!h) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (!h->d_omega && !h->dry) throw StatusError{TTN_ESTATE, "ttn_set_pulses must be called first"};
        if (h->nonherm) throw StatusError{TTN_EINVAL, "the adjoint needs a Hermitian Hamiltonian (gamma = 0)"};
        if (h->two_site) throw StatusError{TTN_ENOTSUP, "the adjoint covers the single-site update only"};
        record_begin(h, n_steps, ckpt_every, d_buf, bytes);
        if (!h->dry) HIPCHECK(hipGetLastError());
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_backward(ttn_handle* h, int32_t n_target, const int32_t* target_sites, double dF, double* grad_omega,
                 double* grad_delta) {
    if (!h || !grad_omega || !grad_delta) return TTN_EINVAL;
    if (h->poisoned) return TTN_ESTATE;
    try {
        if (!h->adj || !h->adj->active) throw StatusError{TTN_ESTATE, "no recording (call ttn_record_begin)"};
        if (h->adj->overflow) throw StatusError{TTN_ESTATE, "more steps taken than the recording declared"};
        if (n_target < 0 || (n_target > 0 && !target_sites)) throw StatusError{TTN_EINVAL, "bad target"};
        std::vector<char> in(h->N, 0);
        for (int i = 0; i < n_target; ++i) {
            if (target_sites[i] < 0 || target_sites[i] >= h->N) throw StatusError{TTN_EINVAL, "bad target site"};
            in[target_sites[i]] = 1;
        }
        reset_step_dev(h);
        backward(h, in, dF, grad_omega, grad_delta);
        check_step_flags(h, nullptr);
        if (!h->dry) HIPCHECK(hipGetLastError());
        return TTN_OK;
    } catch (const StatusError& e) {
        return fail(h, e);
    }
}

int ttn_destroy(ttn_handle* h) {
    if (!h) return TTN_EINVAL;
    delete h->adj;
    if (!h->dry) {
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        if (h->step_graph) (void)hipGraphExecDestroy(h->step_graph);
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
        if (h->d_omega) (void)hipFree(h->d_omega);
        if (h->d_delta) (void)hipFree(h->d_delta);
        if (h->d_evU) (void)hipFree(h->d_evU);
        if (h->d_omx) (void)hipFree(h->d_omx);
        if (h->d_omz) (void)hipFree(h->d_omz);
    }
    delete h;
    return TTN_OK;
}

const char* ttn_last_error(const ttn_handle* h) {
    if (!h) return g_init_error.c_str();
    return h->err.c_str();
}

}  // extern "C"

namespace {

ttn_handle* make_dry_handle(const ttn_config* cfg, size_t bytes) {
    ttn_handle* h = new ttn_handle();
    try {
        h->dry = true;
        setup_config(h, cfg);
        void* fake = (void*)(uintptr_t(1) << 44);
        Bump b(fake, bytes, &h->regions);
        plan(h, b);
        sort_regions(h);
        build_couplings(h, cfg->pos_xy);
        initial_tensors(h, cfg);
        canonicalise(h);
        const int N = h->N, d = h->d;
        std::vector<double> edges = {0.0, 1e9}, om(N, 1.0), de(N, 0.5), u((size_t)N * 2 * d * d, 0.0);
        std::vector<int32_t> st(N, 0), site(N);
        for (int i = 0; i < N; ++i) {
            site[i] = i;
            for (int a = 0; a < d; ++a) u[(size_t)i * 2 * d * d + 2 * (a * d + a)] = 1.0;
        }
        const int rc = ttn_set_pulses(h, 1, edges.data(), om.data(), de.data(), N, st.data(), site.data(), u.data());
        if (rc != TTN_OK) throw StatusError{rc, h->err};
        return h;
    } catch (...) {
        ttn_destroy(h);
        throw;
    }
}

}  // namespace

