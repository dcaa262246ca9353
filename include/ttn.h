/*
 * ttn.h -- C ABI of the MI355X (gfx950) tree-tensor-network TDVP library.
 *
 * The library time-evolves a binary tree tensor network (TTN) under the
 * time-dependent Rydberg Hamiltonian of arXiv 2210.03763 with single-site
 * TDVP, entirely on one GPU.  Paper anchors:
 *   - Hamiltonian: Eq. (eq:ham) with the van der Waals coupling Eq. (eq:c6),
 *     Sec. "Modeling 88Sr quantum computers on two-dimensional grids".  Read
 *     here as   H(t) = sum_i [Omega_i(t)/2 (|1><r| + h.c.) - Delta_i(t) |r><r|
 *                   + leak_ratio Omega_i(t)/2 (|leak><r| + h.c.)]
 *                   + sum_{i<j} C6 / |x_i - x_j|^6 n_i n_j ,  n = |r><r| ;
 *   - TTN with Hilbert-curve leaf order, tensor product operator with all
 *     two-body terms, TDVP time evolution, bond dimension chi, interaction
 *     cut-off radius: Sec. "Tensor network simulations";
 *   - fidelity F = |<psi(tau)|psi_GHZ>|^2: Sec. on GHZ state preparation;
 *   - per-layer piecewise pulses, idle atoms undriven: Sec. "Tensor network
 *     simulations".
 *
 * Conventions shared by every entry point
 *   - Complex numbers in host arrays are interleaved (re, im) doubles.
 *   - Sites are numbered s = 0..N-1; the caller gives their positions.  The
 *     tree has N = 2^K leaves; leaf k holds site leaf_order[k]; bottom nodes
 *     own leaves (2j, 2j+1); link dimension above a subtree of s sites is
 *     min(chi, d^s, d^(N-s)).  Node tensors T[l, r, p] (left child, right
 *     child, parent), l fastest; nodes numbered level by level from the
 *     bottom (level 0) to the root.
 *   - Step n (counted from ttn_init) applies the gate events scheduled at n,
 *     freezes H at t = (n + 1/2) dt, and performs S(dt/2) followed by its
 *     exact reverse; events scheduled at the step count reached at the end of
 *     a ttn_tdvp_step call are applied before it returns.
 *   - Every call enqueues work on the stream given to ttn_init and returns
 *     after the stream is synchronised (calls return host values).
 *   - Errors: a negative status.  No C++ exception crosses this boundary.
 *     TTN_EINVAL leaves the handle unchanged.  TTN_ENUMERIC (NaN/Inf, a
 *     non-positive Cholesky pivot in a QR gauge move, norm drift) poisons the
 *     handle: every later call except ttn_last_error/ttn_destroy returns
 *     TTN_ESTATE.  ttn_last_error gives a text.  A handle is not thread
 *     safe; distinct handles are independent.
 */
#ifndef TTN_H
#define TTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTN_OK 0
#define TTN_EINVAL -1
#define TTN_ENOMEM -2
#define TTN_EDEVICE -3
#define TTN_ENUMERIC -4
#define TTN_ESTATE -5
#define TTN_ENOTSUP -6

/* Arithmetic of the tensor contractions.  TTN_PREC_FP64: everything in
 * complex FP64.  TTN_PREC_FP32 (mixed): the H_eff / K_eff matvecs, the
 * environment updates and the adjoint's exponential adjoints contract in
 * complex FP32 with FP32 accumulation (results stored in FP64);
 * TTN_PREC_BF16X3: as TTN_PREC_FP32, but the large contractions form every
 * real product from bf16 pieces (x = hi + lo; hi*hi + hi*lo + lo*hi, about
 * 2^-16 relative per product) on the bf16 matrix cores.  In every mode the
 * Lanczos scalars and re-orthogonalisation, the small exponential, the QR
 * gauge moves and the master node tensors are FP64. */
#define TTN_PREC_FP64 0
#define TTN_PREC_FP32 1
#define TTN_PREC_BF16X3 2

/* Update scheme of the sweep (Sec. "Tensor network simulations": TDVP with
 * a two-tensor update).  TTN_UPDATE_ONE_SITE: single-site TDVP at fixed bond
 * dimensions.  TTN_UPDATE_TWO_SITE: every edge (v, parent u) is evolved as
 * the merged tensor Theta[l, r, s, p] = sum_k T_v[l, r, k] T_u[k, s, p] under
 * its two-site effective Hamiltonian and split back, truncated to the edge's
 * link dimension by the largest singular values (computed from the smaller
 * Gram matrix Theta^H Theta or Theta Theta^H with a Jacobi eigensolver), the
 * kept values rescaled to the norm of Theta; nodes between the updates of the
 * edges that meet there are evolved backward.  FP64 only, closed systems
 * only, N >= 4, and the smaller side of every merged tensor (min(D_l D_r,
 * D_s D_p)) at most 256 (TTN_ENOTSUP otherwise); no adjoint. */
#define TTN_UPDATE_ONE_SITE 0
#define TTN_UPDATE_TWO_SITE 1

typedef struct ttn_handle ttn_handle;

typedef struct {
    int32_t n_sites;        /* N = 2^K, 2 <= N <= 1024                       */
    int32_t d;              /* local dimension: 3 {0,1,r} or 4 {0,1,r,leak}   */
    int32_t chi;            /* maximal bond dimension, 1 <= chi <= 256        */
    int32_t krylov_dim;     /* Lanczos dimension m, 1 <= m <= 16              */
    int32_t precision;      /* TTN_PREC_*                                     */
    int32_t update;         /* TTN_UPDATE_* (0: single-site)                  */
    double c6;              /* van der Waals coefficient (a = 1 units)         */
    double r_cut;           /* pairs farther than r_cut dropped; <= 0: all     */
    double leak_ratio;      /* |r>-|leak> coupling relative to Omega/2 (d = 4) */
    const double* pos_xy;   /* host [N][2] positions                          */
    const int32_t* leaf_order; /* host [N], a permutation of 0..N-1           */
    const double* init_product; /* host [N][d] complex: one local state per site */
    double dress_eps;       /* dressing amplitude epsilon (>= 0)               */
    const double* dress_noise;  /* host complex stream G, node blocks level by
                                   level, l fastest; may be NULL if eps == 0 */
    int64_t dress_noise_len;    /* complex elements in dress_noise           */
    double gamma;           /* Rydberg decay rate of the open system,
                               Eq. (eq:hoqs): every site's local term gains
                               -i gamma |r><r|, the state loses norm and the
                               local exponentials switch from Lanczos to
                               Arnoldi; 0 = closed system.  >= 0.          */
} ttn_config;

/* Per-step diagnostics, filled by ttn_tdvp_step when stats != NULL. */
typedef struct {
    double norm2;           /* ||psi||^2 after the step                       */
    double energy;          /* <psi|H(t_n + dt/2)|psi> after the step         */
    double min_r_diag;      /* smallest R_kk of every QR in the step           */
    int32_t min_krylov;     /* smallest Krylov dimension reached (breakdown)   */
    int32_t reserved;
    double max_discarded;   /* two-site update: largest discarded weight
                               (dropped share of |Theta|^2) of the step's
                               splits; 0 for the single-site update          */
} ttn_step_stats;

/* Device bytes the caller must provide to ttn_init for this configuration
 * (one allocation, 256-byte aligned).  Returns TTN_EINVAL for a bad config. */
int ttn_workspace_query(const ttn_config* cfg, size_t* device_bytes);

/* Builds the tree, the van der Waals matrix (Eq. c6) and the initial
 * state: isometries carrying the product state init_product, completed by
 * Gram-Schmidt of unit vectors in order and, if dress_eps > 0, dressed as
 * T += eps G / sqrt(D_l D_r); then QR-canonicalised toward the root and
 * normalised.  d_workspace is caller-owned device memory of at least the
 * queried size that must outlive the handle; hip_stream is a hipStream_t
 * (NULL: the null stream).  Host arrays are copied.  On success *out is a
 * library-owned handle released by ttn_destroy. */
int ttn_init(const ttn_config* cfg, void* d_workspace, size_t workspace_bytes,
             void* hip_stream, ttn_handle** out);

/* Piecewise-constant drive and exact local gate events.
 *   seg_edges [n_seg + 1] ascending times; segment s covers
 *   [seg_edges[s], seg_edges[s+1]); outside all segments the drive is zero.
 *   omega, delta [N][n_seg] (site-major).
 *   Event e applies the d x d unitary ev_u[e] (complex, row-major U[a][b])
 *   to site ev_site[e] at step ev_step[e].
 * Replaces any earlier program; events at steps already passed are ignored. */
int ttn_set_pulses(ttn_handle* h, int32_t n_seg, const double* seg_edges,
                   const double* omega, const double* delta, int32_t n_events,
                   const int32_t* ev_step, const int32_t* ev_site, const double* ev_u);

/* The single-qubit drive of Eq. (eq:ham): Omega^x_i(t) sigma^x_i +
 * Omega^z_i(t) sigma^z_i with sigma^x = |0><1| + |1><0| and sigma^z =
 * |0><0| - |1><1| (zero on |r> and |leak>), piecewise constant on the
 * segments of the last ttn_set_pulses call: omega_x, omega_z host
 * [N][n_seg] (site-major), either may be NULL (zero); both NULL removes the
 * channels.  Gates can then be driven as square pulses through the TDVP
 * instead of exact gate events.  ttn_set_pulses resets the channels to
 * zero; this call ends an adjoint recording (the adjoint differentiates
 * Omega and Delta only).  TTN_ESTATE before ttn_set_pulses, TTN_EINVAL for
 * non-finite values.  Allocates two small device arrays. */
int ttn_set_qubit_pulses(ttn_handle* h, const double* omega_x, const double* omega_z);

/* n_steps TDVP steps of size dt (dt must not change between calls).
 * stats: host array [n_steps] or NULL. */
int ttn_tdvp_step(ttn_handle* h, double dt, int32_t n_steps, ttn_step_stats* stats);

/* Fidelity with the GHZ-type target (|0..0> + |1_S 0_rest>)/sqrt 2 where S
 * are the n_target sites listed (S = all sites gives the GHZ state; the
 * centre atom plus its four neighbours gives the five-qubit repetition code
 * with the other atoms idle).  F = |<target|psi>|^2; overlap = <target|psi>. */
int ttn_fidelity(ttn_handle* h, int32_t n_target, const int32_t* target_sites,
                 double* F, double overlap[2]);

/* ||psi||^2 and <psi|H|psi> with H at the last step's midpoint. */
int ttn_observables(ttn_handle* h, double* norm2, double* energy);

/* Total Rydberg population sum_i <psi|n_i|psi> of the current state (not
 * normalised: with gamma > 0 it is the population of the surviving norm),
 * the integrand of the integrated time in the Rydberg state T_R and, at the
 * final time, the remaining population P_R (open-system section,
 * definitions of P_R and T_R).  Uses the environments of the root, which
 * every step leaves current.  Synchronises the stream. */
int ttn_rydberg_population(ttn_handle* h, double* pop);

/* <psi|O_site|psi> for a d x d complex operator (row-major O[a][b]). */
int ttn_local_expectation(ttn_handle* h, int32_t site, const double* op, double out[2]);

/* <psi_a|psi_b> for two handles of the same shape (same N, d, chi, leaf
 * order); used for the state infidelity C = 1 - |<a|b>|^2 (Tab. conv8x8). */
int ttn_overlap(ttn_handle* a, ttn_handle* b, double out[2]);

/* Copies every node tensor to host, complex interleaved, in the node order
 * and layout above; len = complex elements available.  Returns the number
 * of complex elements needed when host == NULL. */
int64_t ttn_export_state(ttn_handle* h, double* host, int64_t len);

/* Reverse mode (gradient of the fidelity with respect to the pulse table).
 * The paper optimises pulses by simulation but states no gradient method;
 * the gradient here is the exact derivative of the discrete map the forward
 * path computes, by reverse-mode differentiation of every operation of the
 * steps (gauge moves, environment builds, Lanczos exponentials with the
 * Frechet derivative of the exponential by Gauss-Legendre quadrature).
 *
 * ttn_adjoint_query: device bytes of the adjoint buffer for recording
 * n_steps steps with a checkpoint every ckpt_every (>= 1) steps:
 * ceil(n_steps / ckpt_every) + ckpt_every + 1 network states, the adjoint
 * scratch and the tape of one step.  TTN_EINVAL for a bad config. */
int ttn_adjoint_query(const ttn_config* cfg, int32_t n_steps, int32_t ckpt_every, size_t* device_bytes);

/* Starts recording at the current state: the gate events of the current
 * step count are applied now, and the next n_steps TDVP steps store
 * checkpoints in d_buf (caller-owned device memory of at least the queried
 * size, which must outlive the recording; TTN_ENOMEM if it is smaller).  A
 * later ttn_set_pulses ends the recording; steps beyond n_steps invalidate
 * it.  TTN_EINVAL for an open system (gamma > 0): the adjoint assumes a
 * Hermitian Hamiltonian. */
int ttn_record_begin(ttn_handle* h, int32_t n_steps, int32_t ckpt_every, void* d_buf, size_t bytes);

/* grad_omega, grad_delta (host [N][n_seg], overwritten) = dF * dF/dOmega,
 * dF * dF/dDelta for F = |<GHZ_S|psi>|^2 at the current state (S =
 * target_sites, as in ttn_fidelity), through every step recorded since
 * ttn_record_begin.  The steps are recomputed from the checkpoints with a
 * tape and reversed; the state is left as it was.  TTN_ESTATE without a
 * valid recording. */
int ttn_backward(ttn_handle* h, int32_t n_target, const int32_t* target_sites, double dF, double* grad_omega,
                 double* grad_delta);

/* Projective measurements of all sites (Sec. on parallel quantum algorithms:
 * the paper's measurement histograms come from a million shots drawn from
 * the TTN).  Each shot is drawn exactly from |psi(s)|^2 of the current
 * (root-canonical) state, top-down through the tree: a node's pure input
 * state u on its parent link gives B = Q u on its child links, the left
 * subtree is sampled from one column of B picked with the weights
 * ||B[:, r]||^2, the right subtree from its exact conditional state, bottom
 * nodes draw their two sites in turn.  Uniforms come from Philox4x32-10
 * with counter (shot low word, shot high word, draw index, 0) and key
 * (seed low word, seed high word); node v uses draw v, bottom node j draws
 * n_nodes + 2 j and n_nodes + 2 j + 1 (shot0 + b is the shot index of shot b,
 * so a run can be split over calls).
 *   configs: host [n_shots][N] (site-indexed values 0..d-1) or NULL;
 *   amps: host [n_shots] complex psi(s) of each drawn configuration, or NULL.
 * d_buf: caller-owned device scratch; shots are processed in batches as
 * large as it allows (ttn_sample_query gives the bytes for a batch size).
 * The state is not changed. */
int ttn_sample_query(ttn_handle* h, int32_t batch, size_t* device_bytes);
int ttn_sample(ttn_handle* h, int64_t n_shots, uint64_t seed, int64_t shot0, void* d_buf, size_t bytes,
               uint8_t* configs, double* amps);

/* The tensor-product-operator contraction on one leg of node tensors
 * (Sec. "Tensor network simulations": each term of the Hamiltonian acts on
 * a node through its environment operators), on caller device memory:
 *   sum_ops == 0:  y_k = Op_k (x) leg  x_k   for k < n_ops
 *   sum_ops != 0:  y   = sum_k Op_k (x) leg  x_k
 * where (Op (x) leg x)[.., a, ..] = sum_b Op[a, b] x[.., b, ..], leg 0/1/2 =
 * left/right/parent of a (DL, DR, DP) tensor with the left index fastest.
 * Every array is planar complex (all real parts, then all imaginary parts)
 * in FP64 or FP32 (precision: TTN_PREC_FP64, or TTN_PREC_FP32 / TTN_PREC_BF16X3
 * on FP32 arrays); Op_k are D x D column-major (D = dimension
 * of the leg), stored one after another (2 D^2 reals each); x_k likewise
 * (2 DL DR DP reals each) when x_per_op != 0, otherwise one x is shared
 * (sum_ops requires x_per_op).  accumulate != 0 adds into y.  Enqueued on
 * hip_stream and synchronised before returning; the arrays are borrowed.
 * Allocates and frees its own split-K scratch.  TTN_EINVAL for bad sizes;
 * ttn_last_error(NULL) gives the text. */
int ttn_leg_contract(int32_t precision, int32_t leg, int32_t DL, int32_t DR, int32_t DP, int32_t n_ops,
                     const void* d_ops, const void* d_x, int32_t x_per_op, void* d_y, int32_t sum_ops,
                     int32_t accumulate, void* hip_stream);

/* ttn_leg_contract without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks and result as
 * ttn_leg_contract (the same kernels and split factors, so the same bits),
 * but the split-K partial sums live in a file-scope device array of
 * 64 MiB that every GPU the library runs on holds until the process ends,
 * and the call only enqueues: it does not synchronise the stream (errors of
 * the kernels show at the caller's next synchronisation).  No input exceeds
 * the array: the split factor is capped so that the partial sums fit, and
 * split-free launches need none.  Every call on one GPU shares that GPU's
 * array, so calls that may overlap on one GPU (different streams without
 * ordering) race; calls on one stream are ordered.  The array's address is
 * looked up once per device, on the first call with that device current. */
int ttn_leg_contract_noalloc(int32_t precision, int32_t leg, int32_t DL, int32_t DR, int32_t DP,
                             int32_t n_ops, const void* d_ops, const void* d_x, int32_t x_per_op, void* d_y,
                             int32_t sum_ops, int32_t accumulate, void* hip_stream);

/* The eigensolver of the two-site split on caller memory (kernel unit
 * tests): eigenvalues and eigenvectors of the Hermitian n x n matrix d_a
 * (planar complex FP64, column-major; destroyed), 1 <= n <= 256, by the
 * cyclic Jacobi method with round-robin pair ordering in one workgroup.
 * d_w[k] receives the k-th largest eigenvalue, d_order[k] (int32) the
 * column of d_v (n x n planar) holding its eigenvector.  Synchronises
 * hip_stream; TTN_ENUMERIC if the iteration does not converge, TTN_EINVAL
 * for bad arguments.  Allocates a small status block. */
int ttn_herm_eig(int32_t n, void* d_a, void* d_v, void* d_w, void* d_order, void* hip_stream);

/* Device time of the contraction kernels inside a profiling window. */
typedef struct {
    int64_t launches;       /* kernel launches                                  */
    double ms;              /* summed device time between events around them    */
    double flops;           /* algorithmic real flops: 8 per complex multiply-add
                               of the contraction (M N K per launch)            */
} ttn_kernel_prof;

/* Device time of the Lanczos vector kernels (projections, Gram-Schmidt
 * subtractions, norms, scaling, recombination) of the general Krylov path. */
typedef struct {
    int64_t calls;          /* wrapper calls (each one to three kernel launches) */
    double ms;              /* summed device time between events around them     */
    double bytes;           /* bytes those kernels read and write by construction
                               (16 per complex FP64 element, 8 per FP32 one)     */
} ttn_vec_prof;

/* Launch counts and flops per class cover every contraction launch of the
 * window.  Times: the launches of one H_eff / K_eff matvec run back to back
 * between one pair of HIP events (heff.ms sums those matvec times, and they
 * count in the ms of their precision class); every other contraction launch
 * is bracketed by its own pair (before the main kernel, after its split-K
 * reduction).  gemm_bf16x3.ms holds only such individually timed launches. */
typedef struct {
    ttn_kernel_prof gemm_f32;   /* complex FP32 contraction kernel (incl. BF16x3) */
    ttn_kernel_prof gemm_f64;   /* complex FP64 contraction kernel               */
    ttn_kernel_prof heff;       /* the subset that applies H_eff / K_eff         */
    int64_t matvecs;            /* H_eff / K_eff applications                     */
    ttn_kernel_prof gemm_bf16x3; /* the FP32 launches that ran the BF16x3 kernel  */
    ttn_vec_prof lanczos;       /* Lanczos vector kernels, every operator size    */
    ttn_vec_prof lanczos_large; /* the subset on vectors of >= 2^20 elements      */
} ttn_profile;

/* One contraction launch of a profiling window, in launch order. */
typedef struct {
    int32_t kernel;   /* 1 VALU tile kernel (k_cgemm), 2 MFMA kernel
                         (k_cgemm_mfma), 3 BF16x3 kernel (k_cgemm_bf16x3)     */
    int32_t prec;     /* 0 FP64 operands, 1 FP32 operands                     */
    int32_t heff;     /* 1 when the launch applies H_eff / K_eff              */
    int32_t splits;   /* split-K factor; > 1: a k_splitk_reduce* launch follows
                         the main kernel                                      */
    int32_t matvec;   /* ordinal of the H_eff / K_eff matvec in the window the
                         launch belongs to, -1 for other launches             */
    int32_t reserved;
    double flops;     /* algorithmic real flops (8 M N K)                     */
    double ms;        /* event time of the main kernel and its reduction; -1
                         for H_eff / K_eff launches (timed per matvec) and in
                         untimed windows                                      */
} ttn_launch_rec;

/* Opens a profiling window: from now on contraction launches are recorded
 * and timed with HIP events on the handle's stream (see ttn_profile), and so
 * are the Lanczos vector kernels of the general Krylov path. */
int ttn_profile_begin(ttn_handle* h);

/* The same window without any event: launches are only recorded (class,
 * split factor, H_eff flag, flops) and ttn_profile's times stay 0.  For runs
 * under hardware-counter collection, which should see plain dispatches. */
int ttn_profile_begin_untimed(ttn_handle* h);

/* Closes the window (synchronises the stream) and sums the event times and
 * algorithmic flops per kernel class. */
int ttn_profile_end(ttn_handle* h, ttn_profile* out);

/* The launches of the last window closed by ttn_profile_end, in launch order
 * (for matching hardware-counter dispatches to launch classes): copies up to
 * max records into out (may be NULL) and returns how many the window had. */
int64_t ttn_profile_launches(const ttn_handle* h, ttn_launch_rec* out, int64_t max);

/* The environment rebuild and both sweeps of a step are the same launch
 * sequence every step; by default it is captured once as a HIP graph (on a
 * private stream) and replayed on the handle's stream.  enabled == 0 runs
 * every launch eagerly.  Profiling windows always run eagerly (their timing
 * events need individual launches). */
int ttn_set_graphs(ttn_handle* h, int32_t enabled);

/* Checks the launch plan of a configuration without a device: walks
 * initialisation, n_steps TDVP steps of a one-segment program with a gate on
 * every site (recorded for the adjoint when gamma = 0), the fidelity, a
 * local expectation, a self overlap, the Rydberg population, the backward
 * pass (gamma = 0) and a few sampled shots, and verifies that every kernel
 * operand stays inside its workspace or adjoint-buffer allocation.
 * No device memory is touched.  msg (may be NULL) receives "ok" or the first
 * violation.  Not thread safe with concurrent device calls of this library. */
int ttn_validate_plan(const ttn_config* cfg, int32_t n_steps, char* msg, int32_t msg_len);

int ttn_destroy(ttn_handle* h);
/* Text of the last error of h; with h == NULL, of the last failed ttn_init
 * on this thread. */
const char* ttn_last_error(const ttn_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* TTN_H */
