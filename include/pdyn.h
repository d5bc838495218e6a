/*
 * pdyn -- batched rigid-body dynamics of serial chains on AMD Instinct MI355X
 * (gfx950), after Yang, Wu & Pan, "Parallel Dynamics Computation using Prefix
 * Sum Operations" (arXiv:1609.04493).
 *
 * C ABI. Every array argument is a DEVICE pointer unless marked "host". The
 * caller owns every buffer; the library allocates no user-visible memory and
 * keeps no pointer after a call returns. Outputs are overwritten, never
 * accumulated. Calls are asynchronous on the given HIP stream (a hipStream_t
 * passed as void*, NULL = the null stream), perform no host synchronisation and
 * no allocation, and are re-entrant.
 *
 * Conventions (paper, Table I and Sec. II):
 *   twist V = (v, w), wrench F = (f, n), power V^T F.
 *   f_{i-1,i} = M_i exp(S_i q_i) maps link frame i to frame i-1 (eq. (1)).
 *   S_i (joint twist) and the link inertia are expressed in frame i.
 *   Links are numbered base (1) to tip (n); arrays are 0-based.
 *
 * Errors: 0 on success; a negative PDYN_E* code otherwise. Arguments are
 * checked on the host BEFORE any device work is queued, so a failing call
 * leaves outputs and device state untouched. Non-finite inputs or a
 * non-positive articulated pivot S^T Jhat S are not trapped: they propagate
 * as NaN/Inf in the outputs.
 */
#ifndef PDYN_H
#define PDYN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PDYN_OK = 0,
  PDYN_EINVAL = -1,        /* null required pointer, non-positive size, inconsistent sizes */
  PDYN_EALIGN = -2,        /* a pointer not aligned to its element size (workspace: 256 B) */
  PDYN_EWORKSPACE = -3,    /* workspace smaller than pdyn_workspace_bytes() */
  PDYN_ELAUNCH = -4,       /* the HIP runtime reported an error when queueing a kernel */
  PDYN_EUNSUPPORTED = -5   /* a size beyond the library's limits (see pdyn_max_links) */
};

/*
 * A set of serial chains (the robot model), CSR over links.
 *
 * n_chains == 1: one chain of n_links_max links, shared by every state.
 * n_chains  > 1: one chain per state (n_chains must equal the batch's
 *                n_states); chain c owns links link_ptr[c] .. link_ptr[c+1]-1.
 *
 * Per-link arrays, scalar = float for the plain entry points and double for
 * the _f64 ones, row-major, L = total link count:
 *   placement [L][7]  M_i: unit quaternion (w, x, y, z) of the rotation
 *                     (normalised by the library), then the translation.
 *   twist     [L][6]  S_i = (v, w) in frame i, w != 0 (revolute or helical
 *                     joint; the exponential is exact for any |w| > 0).
 *   inertia   [L][10] m, c_x, c_y, c_z, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz:
 *                     mass, centre of mass in frame i, and the rotational
 *                     inertia about the centre of mass in frame-i axes.
 */
typedef struct pdyn_model {
  int32_t n_chains;
  int32_t n_links_max;      /* host: links of the longest chain (the only chain if n_chains == 1) */
  int64_t n_links_total;    /* host: L */
  const int32_t* link_ptr;  /* [n_chains + 1], link_ptr[0] = 0; may be NULL when n_chains == 1 */
  const void* placement;
  const void* twist;
  const void* inertia;
  /* Derived per-link tables filled by pdyn_model_prepare for this model and
   * scalar type, or NULL: then every call derives them again inside its
   * workspace (one extra small kernel per call). */
  const void* prepared;
  /* One chain per state only: a permutation [n_chains] of the chains in the
   * order lanes take them (e.g. longest first, so that each wavefront holds
   * chains of similar length and the longest start first), or NULL for the
   * natural order. Results are written in the natural layout either way.
   * The derived tables are laid out for this order (each wavefront's link
   * records interleaved over its lanes), so a prepared model keeps the order
   * it was prepared with; a new order takes effect when it is prepared again. */
  const int32_t* order;
  /* Host copies of link_ptr and order, with the same contents. Required when
   * n_chains > 1 (link_ptr_host) and when order is set (order_host); ignored
   * otherwise. The library checks them on the host before any device work --
   * in pdyn_model_prepare, and in every call that is given no prepared tables
   * -- and returns PDYN_EINVAL unless link_ptr_host[0] == 0, every chain has
   * 1 .. n_links_max links, link_ptr_host[n_chains] == n_links_total and
   * order_host is a permutation of 0 .. n_chains-1. The device copies are
   * read only by the table derivation, which clamps every chain to
   * n_links_max links inside 0 .. n_links_total and every order entry to a
   * valid chain, so device copies that differ from the checked host copies
   * give wrong results for the chains concerned but no access outside the
   * caller's arrays. The library keeps neither pointer after a call. */
  const int32_t* link_ptr_host;
  const int32_t* order_host;
} pdyn_model;

/*
 * A batch of states. n_states == 0 is a valid empty batch (the call returns
 * PDYN_OK and queues nothing) when the chain is shared.
 *
 * Joint arrays (q, qd, qdd, tau and their adjoints): with a shared chain,
 * [n_states][n] row-major; with one chain per state, ragged: state s owns
 * entries link_ptr[s] .. link_ptr[s+1]-1.
 *
 * base_vel, base_acc (host): V_0 and dV_0 of eqs. (3)-(4), uniform over the
 * batch. A uniform gravity field g enters as dV_0 = (-g, 0), e.g.
 * (0, 0, 9.81, 0, 0, 0) for gravity -9.81 z.
 * tip_wrench: F_{n+1} of eqs. (2)-(4) per state, [n_states][6], expressed in
 * the frame of the last link (the wrench the last link exerts on its
 * environment), or NULL for zero.
 */
typedef struct pdyn_batch {
  int32_t n_states;
  double base_vel[6];
  double base_acc[6];
  const void* tip_wrench;
  /* Launch shape (0 = library default): threads per workgroup for the
   * inverse/forward dynamics and rollout kernels (a multiple of 64, at most
   * 256; the adjoint kernels always use 64), and an upper bound on the number
   * of workgroups -- fewer than the work needs makes the launch persistent,
   * each workgroup striding over the remaining work in a fixed order. */
  int32_t block_threads;
  int32_t max_blocks;
  /* Kernel variant; 0 = library default: 2 for the adjoints, and for inverse
   * dynamics, forward dynamics and ID+FD 2 up to 128 states per compute unit,
   * else 1. Inverse dynamics: 1 = one wavefront per 64 states; 2 = one
   * wavefront forms the joint transforms (eq. 1) and hands them to another
   * that runs the two Newton-Euler sweeps (eqs. 1, 2).
   * Forward dynamics and fused ID+FD: 1 = one wavefront runs every recursion
   * of its 64 states; 2 = role split -- per group of 64 states one wavefront
   * runs the articulated-body inertia recursion (7) while others run the
   * Newton-Euler passes (and, for ID+FD, the inverse dynamics), then the
   * z-hat / lambda recursions of (8). Adjoints (pdyn_*_vjp): 1 = one
   * wavefront per 64 states; 2 = role split -- one wavefront runs the
   * cotangent recursions (for FD first the articulated-body solve), another
   * the Newton-Euler sweeps, then the inertia-parameter terms and the
   * tip-to-base adjoint sweep run side by side. 3 = the plain form: for the
   * forward operations the sweeps of variant 1 as separate launches, one per
   * recursion sweep; for the adjoints the passes of the role split (cotangent
   * recursion or articulated-body solve, Newton-Euler sweep, wrench sweep,
   * inertia-parameter terms, tip-to-base adjoint sweep) as separate launches;
   * either way with the per-link intermediates in the workspace (HBM) between
   * them. 4 (the adjoints take it as 1) = the paper's serial-parallel hybrid:
   * each chain is cut into `segments` consecutive segments handled by as many
   * lanes; every lane folds its segment's scan operands (eqs. (12)-(13) for
   * the velocities and accelerations, eq. (16) for the wrenches), the lanes of
   * a chain combine their aggregates with an inclusive scan across lanes, and
   * each lane then runs its segment from the value at its start. Forward
   * dynamics and ID+FD take the bias forces (and the inverse dynamics) this
   * way, while one wavefront runs the articulated-body recursion (7), which is
   * not a linear recursion, serially per chain beside them, and another the
   * two recursions of eq. (8) behind it. block_threads and max_blocks apply to
   * variants 1 and 3. Every variant gives the same results to rounding. */
  int32_t variant;
  /* Lanes per chain, a power of two; 0 = library default. Variant 4 of the
   * inverse dynamics: 1 .. 64; of forward dynamics and ID+FD: 1 .. 16 (32 and
   * 64 give PDYN_EUNSUPPORTED); default the largest power of two within that
   * bound that leaves at least 8 links per segment. pdyn_articulated_inertia
   * and pdyn_aba_fd_scan: lanes per state 1 .. 128, default described there.
   * Other values: PDYN_EINVAL. Ignored by the other operations and variants. */
  int32_t segments;
} pdyn_batch;

/* Status word. The first 256 bytes of every workspace hold a 32-bit word into
 * which the kernels OR these bits when a fault occurs (the call itself still
 * returns PDYN_OK; faulty values propagate as NaN/inf):
 *   PDYN_STATUS_NONFINITE  an output (tau, qdd, q_bar, u = tau_bar) is not finite;
 *   PDYN_STATUS_PIVOT      an articulated-body pivot D_i = S_i^T Jhat_i S_i (Sec. II-B,
 *                          eq. (7)) is not positive: the inertia parameters are not
 *                          physical for this configuration;
 *   PDYN_STATUS_WAIT       a wavefront of a multi-wavefront kernel gave up waiting for
 *                          another wavefront of its workgroup after its spin bound
 *                          (~30 ms): the hand-off it waited for never came, and the
 *                          outputs of that workgroup's states are not to be trusted.
 *                          A correct kernel never sets it.
 * A new workspace must start with this word zero; pdyn_read_status clears it. */
#define PDYN_STATUS_NONFINITE 1u
#define PDYN_STATUS_PIVOT 2u
#define PDYN_STATUS_WAIT 4u

/* Operation selector for pdyn_workspace_bytes. */
enum {
  PDYN_OP_RNEA_ID = 0,
  PDYN_OP_ABA_FD = 1,
  PDYN_OP_ID_FD = 2,
  PDYN_OP_RNEA_ID_VJP = 3,
  PDYN_OP_ABA_FD_VJP = 4,
  PDYN_OP_JSIIA_FD = 5,
  PDYN_OP_MASS_MATRIX = 6,
  PDYN_OP_RNEA_ID_JACOBIAN = 7,
  PDYN_OP_ABA_FD_JACOBIAN = 8,
  PDYN_OP_RNEA_ID_HESSIAN = 9,
  PDYN_OP_ARTICULATED_INERTIA = 10,
  PDYN_OP_ABA_FD_SCAN = 11
};

/* Bytes of device workspace that operation op needs for this model and batch
 * with the given scalar size (4 or 8); 0 on invalid arguments. It includes
 * room for the derived tables unless model->prepared is set. The workspace
 * must be 256-byte aligned; its contents on entry are ignored. */
size_t pdyn_workspace_bytes(int op, const pdyn_model* model, const pdyn_batch* batch, int scalar_bytes);

/* Bytes of the derived per-link tables of a model (scalar_bytes 4 or 8); 0 on
 * invalid arguments. One shared chain: 32 words per link in the scalar type
 * and 32 in double. One chain per state: as much per record slot, with
 * n_links_max slots for each group of 64 chains (chains shorter than the
 * longest of their group leave slots unused), plus the lane order. */
size_t pdyn_model_prepared_bytes(const pdyn_model* model, int scalar_bytes);

/* Derive the per-link tables (rotation of each placement, twist norms, first
 * moments and inertias about the joint frame) into `prepared` (device, 256-byte
 * aligned, pdyn_model_prepared_bytes long), asynchronously on `stream`. The
 * model's own `prepared` field is ignored. Valid until the model's arrays
 * change. */
int pdyn_model_prepare(const pdyn_model* model, int scalar_bytes, void* prepared, size_t prepared_bytes,
                       void* stream);

/* Longest chain the kernels accept. */
int pdyn_max_links(void);

/*
 * Installs a launch tuning table (host text, NUL-terminated), as written by the
 * project's autotuner:
 *   {"entries": [{"op": 2, "scalar": 4, "shared": 0, "n_max": 100, "n_states": 4096,
 *                 "block": 0, "max_blocks": 0, "variant": 2, "segments": 0}, ...]}
 * op is a PDYN_OP_* value, scalar 4 or 8, shared 1 for a shared chain and 0
 * for one chain per state; block, max_blocks, variant and segments (optional,
 * 0 by default) follow the rules of pdyn_batch's launch fields. A later call
 * that leaves all four launch fields
 * of its batch at 0 takes them from the entry of its operation, scalar size
 * and model kind whose n_max and n_states are nearest in log scale, provided
 * both lie within a factor of 2; without such an entry the library defaults
 * apply. Every variant gives the same results to rounding, so a table changes
 * speed only. NULL or "" removes the table. Returns PDYN_EINVAL (and keeps the
 * previous table) for text outside this form or an invalid value. Thread-safe;
 * calls already running keep the table they started with.
 */
int pdyn_load_tuning(const char* json);

/* The launch fields (block_threads, max_blocks, variant, segments; host
 * outputs) that a call of operation op with this model and batch would run
 * with: the batch's own if any is non-zero, else the installed tuning table's
 * entry for it, else zeros (the library defaults). For variant 4, segments is
 * the resolved lane count per chain. Host only: no device work. */
int pdyn_launch_choice(int op, const pdyn_model* model, const pdyn_batch* batch, int scalar_bytes,
                       int32_t* block_threads, int32_t* max_blocks, int32_t* variant, int32_t* segments);

/* Human-readable text for a status code (static storage). */
const char* pdyn_strerror(int status);

/* Reads the status word of workspace ws (the same pointer passed to the
 * operations) into *bits after all work queued on stream (0 = default stream)
 * has finished, and clears it. Synchronises the stream, so it is not for use
 * inside a captured graph. Returns PDYN_EINVAL for a null pointer,
 * PDYN_EALIGN if ws is not 256-byte aligned, PDYN_ELAUNCH if a HIP call fails. */
int pdyn_read_status(void* ws, void* stream, uint32_t* bits);

/*
 * Inverse dynamics, eq. (3): tau = ID(q, qd, qdd, V_0, dV_0, F_{n+1}) by the
 * recursive Newton-Euler recursions (1)-(2): link transforms, the forward
 * velocity/acceleration scan (12)-(13), the bias wrench, the backward wrench
 * scan (16) and tau_i = S_i^T F_i.
 */
int pdyn_rnea_id(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                 const float* qdd, float* tau, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_rnea_id_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                     const double* qdd, double* tau, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward dynamics, eq. (4): qdd = FD(q, qd, tau, V_0, dV_0, F_{n+1}) by the
 * articulated-body recursions (Sec. II-B and III-E): the bias torques
 * tau_bias = ID(q, qd, 0, ...) of eq. (5), the articulated-body inertia
 * recursion (7) (run serially: it is not a linear recursion), then the
 * backward z-hat / c-hat recursion and the forward lambda / qdd recursion of
 * eq. (8) (the scans (18)-(19)).
 */
int pdyn_aba_fd(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                const float* tau, float* qdd, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_aba_fd_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                    const double* tau, double* qdd, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Inverse and forward dynamics of the same states in one pass:
 *   tau_out = ID(q, qd, qdd_in, ...)  and  qdd_out = FD(q, qd, tau_in, ...).
 * The link transforms and velocities are shared between the two.
 */
int pdyn_id_fd(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
               const float* qdd_in, const float* tau_in, float* tau_out, float* qdd_out,
               void* workspace, size_t workspace_bytes, void* stream);
int pdyn_id_fd_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                   const double* qdd_in, const double* tau_in, double* tau_out, double* qdd_out,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * Joint-space inertia M(q) of eq. (17), the matrix with tau = M(q) qdd + tau_bias
 * (eqs. (5)-(6)): M[s] is written whole (both triangles), [n_states][n][n]
 * row-major. Column j of M is the inverse dynamics of a unit acceleration of
 * joint j with no velocity, base motion or gravity (eq. (17)); the kernel
 * forms it from the composite bodies of the chain, n(n+1)/2 wrench transforms
 * per state, computed in double whatever the scalar type of q and M.
 * Shared chain only (model->n_chains == 1; PDYN_EUNSUPPORTED otherwise).
 * block_threads and max_blocks of the batch apply; variant and segments are
 * ignored. Workspace: pdyn_workspace_bytes(PDYN_OP_MASS_MATRIX, ...).
 */
int pdyn_mass_matrix(const pdyn_model* model, const pdyn_batch* batch, const float* q, float* M, void* workspace,
                     size_t workspace_bytes, void* stream);
int pdyn_mass_matrix_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, double* M,
                         void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward dynamics by the joint-space inertia inversion algorithm (JSIIA,
 * Sec. II-B, eq. (6)): qdd = M(q)^-1 (tau - tau_bias) with
 * tau_bias = ID(q, qd, 0, V_0, dV_0, F_{n+1}) (eq. (5)), M(q) as for
 * pdyn_mass_matrix, factored as L L^T (Cholesky) and solved by two triangular
 * substitutions. Same arguments and results as pdyn_aba_fd (the two differ by
 * rounding only). All arithmetic after the joint angles' (sin, cos) runs in
 * double: forming and factoring M amplify rounding by its condition number.
 * A pivot of the factorisation that is not positive sets PDYN_STATUS_PIVOT.
 * Shared chain only (PDYN_EUNSUPPORTED otherwise); launch fields as for
 * pdyn_mass_matrix. Workspace: pdyn_workspace_bytes(PDYN_OP_JSIIA_FD, ...),
 * (13 n + max(6 n, n (n + 1) / 2)) doubles per state plus the tables.
 */
int pdyn_jsiia_fd(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                  const float* tau, float* qdd, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_jsiia_fd_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                      const double* tau, double* qdd, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Full Jacobians of the dynamics of a shared chain (model->n_chains == 1;
 * PDYN_EUNSUPPORTED otherwise), the paper's stated future work (Sec. VI), each
 * [n_states][n][n] row-major with J[s][i][k] = d y_i / d x_k for state s:
 *   pdyn_rnea_id_jacobian: y = tau = ID(q, qd, qdd, ...) (eq. (3)); J_q, J_qd and
 *     J_qdd = d tau / d qdd = M(q), the joint-space inertia of eq. (17);
 *   pdyn_aba_fd_jacobian: y = qdd = FD(q, qd, tau, ...) (eq. (4)), taken at the
 *     forward output `qdd` (pass pdyn_aba_fd's result); J_q, J_qd and
 *     J_tau = d qdd / d tau = M(q)^-1.
 * Row i of each is the adjoint (pdyn_rnea_id_vjp / pdyn_aba_fd_vjp) with the
 * one-hot cotangent e_i: the call expands chunks of states into n rows each in
 * its workspace and runs the adjoint kernels over them, so J is exactly what n
 * adjoint calls with e_0 .. e_{n-1} would give. Workspace:
 * pdyn_workspace_bytes(PDYN_OP_RNEA_ID_JACOBIAN or PDYN_OP_ABA_FD_JACOBIAN, ...)
 * (at most 2^17 expanded rows per chunk); the batch's launch fields apply to
 * the adjoint launches, and its status word is the adjoint's.
 */
int pdyn_rnea_id_jacobian(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                          const float* qdd, float* J_q, float* J_qd, float* J_qdd, void* workspace,
                          size_t workspace_bytes, void* stream);
int pdyn_rnea_id_jacobian_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                              const double* qdd, double* J_q, double* J_qd, double* J_qdd, void* workspace,
                              size_t workspace_bytes, void* stream);
int pdyn_aba_fd_jacobian(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                         const float* qdd, float* J_q, float* J_qd, float* J_tau, void* workspace,
                         size_t workspace_bytes, void* stream);
int pdyn_aba_fd_jacobian_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                             const double* qdd, double* J_q, double* J_qd, double* J_tau, void* workspace,
                             size_t workspace_bytes, void* stream);

/*
 * Second derivatives of the inverse dynamics tau = ID(q, qd, qdd, ...) (eqs.
 * (1)-(3)) of a shared chain (model->n_chains == 1; PDYN_EUNSUPPORTED
 * otherwise), the Hessians that Sec. VI names as future work. Four blocks,
 * each [n_states][n][n][n] row-major:
 *   H_qq[s][i][j][k]   = d^2 tau_i / dq_j dq_k     (symmetric in j, k)
 *   H_qqd[s][i][j][k]  = d^2 tau_i / dq_j dqd_k
 *   H_qdqd[s][i][j][k] = d^2 tau_i / dqd_j dqd_k   (symmetric in j, k; no qd or qdd dependence)
 *   H_qqdd[s][i][j][k] = d^2 tau_i / dq_j dqdd_k = dM_ik / dq_j
 * (tau is linear in qdd, so no other block is nonzero). Any output may be NULL
 * and is then not computed; at least one must be given (PDYN_EINVAL). Base
 * motion and the tip wrench (held fixed) come from the batch. Exact up to
 * rounding: the recursions run on hyper-dual numbers, one thread per (state,
 * block, j, k), with j <= k only in the two symmetric blocks (each such thread
 * writes both halves). A non-finite entry sets PDYN_STATUS_NONFINITE in the
 * workspace's status word. Workspace: pdyn_workspace_bytes(PDYN_OP_RNEA_ID_HESSIAN,
 * ...); the batch's launch fields are ignored.
 */
int pdyn_rnea_id_hessian(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                         const float* qdd, float* H_qq, float* H_qqd, float* H_qdqd, float* H_qqdd, void* workspace,
                         size_t workspace_bytes, void* stream);
int pdyn_rnea_id_hessian_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                             const double* qdd, double* H_qq, double* H_qqd, double* H_qdqd, double* H_qqdd,
                             void* workspace, size_t workspace_bytes, void* stream);

/*
 * Articulated-body inertias Jhat_1 .. Jhat_n of eq. (7) (Sec. II-B) for every
 * state of a shared chain (model->n_chains == 1; PDYN_EUNSUPPORTED otherwise),
 * computed by an associative scan instead of the serial tip-to-base recursion.
 * Sec. II-B treats eq. (7) as unscannable because its step is not linear in
 * Jhat_{i+1}; the step is, however, the limit of a Riccati (linear-fractional)
 * map E(P) = Q + A^T P (I + C P)^-1 A with C = infinity * S_{i+1} S_{i+1}^T, and
 * such maps compose in closed form, so the recursion becomes a prefix scan of
 * 84-number elements.
 *
 * batch->segments: lanes per state P, a power of two 1 .. 128 (PDYN_EINVAL
 * otherwise; P = 128 spans two wavefronts of one workgroup); 0 = library
 * default (the smallest P that gives the batch 16384 lanes, at most 128,
 * keeping at least 4 links per segment). P = 1 is the
 * serial recursion, one lane per state; with P > 1 each lane folds a
 * consecutive segment of links into one element, the lanes combine them with
 * log2(P) scan steps, and each lane reruns its segment from the result. Both
 * give Jhat to rounding; the scan shortens the per-state latency of long
 * chains (O(n / P + log P) steps instead of O(n)). The other launch fields are
 * ignored.
 *
 * q: [n_states][n]. Jhat: [n_states][n][6][6] row-major, Jhat[s][i] the
 * articulated inertia of link i+1 in its own frame, mapping a twist (v, w) to
 * a wrench (f, n). Everything after the joint angles' (sin, cos) runs in
 * double; the FP32 entry rounds the result. A pivot S^T Jhat S (or a pivot of
 * the scan's combines) that is not positive sets PDYN_STATUS_PIVOT, a
 * non-finite entry PDYN_STATUS_NONFINITE. Workspace:
 * pdyn_workspace_bytes(PDYN_OP_ARTICULATED_INERTIA, ...).
 */
int pdyn_articulated_inertia(const pdyn_model* model, const pdyn_batch* batch, const float* q, float* Jhat,
                             void* workspace, size_t workspace_bytes, void* stream);
int pdyn_articulated_inertia_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, double* Jhat,
                                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * Forward dynamics qdd = ABA(q, qd, tau) (Sec. II-B, eqs. (5), (7), (8)) of a
 * shared chain (model->n_chains == 1; PDYN_EUNSUPPORTED otherwise) with every
 * recursion evaluated as a prefix scan over a team of batch->segments lanes
 * per state (P, a power of two 1 .. 128, PDYN_EINVAL otherwise; 0 = library
 * default: the smallest P that gives the batch 32768 lanes, at most 128,
 * keeping at least 4 links per segment):
 *   1. velocities and bias accelerations of tau_bias (eq. (5)), base to tip,
 *      scan operand of eqs. (12)-(13);
 *   2. the articulated-body inertias (eq. (7)) by the Riccati scan of
 *      pdyn_articulated_inertia;
 *   3. the bias wrench and z-hat / c-hat (eqs. (2), (8); operand eq. (18) with
 *      the bias wrench carried in the same recursion), tip to base, a scan of
 *      6x6 affine maps;
 *   4. lambda and qdd (eq. (8), operand eq. (19)), base to tip, likewise.
 * Each phase folds each lane's segment, combines the team's aggregates in
 * log2(P) steps and reruns the segment from the result, so a state's latency
 * is O(n / P + log P) steps instead of the serial recursions' O(n): this is
 * the form for long chains with few states. P = 1 runs the same phases
 * serially. batch->variant: 0 or 1 (default) runs phase 3 as one scan of
 * the merged recursion; 2 runs it as two scans, the bias wrench (eq. (2),
 * giving tau-hat of eq. (5)) and then z-hat (operand eq. (18)), the split
 * form the merged one is measured against; other values PDYN_EINVAL. Same
 * arguments and results as pdyn_aba_fd (base motion and tip wrench from the
 * batch; the other launch fields are ignored); everything
 * after the joint angles' (sin, cos) runs in double. A pivot D_i = S_i^T
 * Jhat_i S_i (or a pivot of the Riccati combines) that is not positive sets
 * PDYN_STATUS_PIVOT, a non-finite qdd PDYN_STATUS_NONFINITE. Workspace:
 * pdyn_workspace_bytes(PDYN_OP_ABA_FD_SCAN, ...), 208 bytes per link and
 * state beyond the status word and tables.
 */
int pdyn_aba_fd_scan(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                     const float* tau, float* qdd, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_aba_fd_scan_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                         const double* tau, double* qdd, void* workspace, size_t workspace_bytes, void* stream);

/*
 * pdyn_id_fd without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the call allocates nothing, on the device or through
 * any library routine. Its scratch is a static device array of
 * PDYN_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends; the caller still passes inputs and outputs.
 *
 * Same arguments, results and rules as pdyn_id_fd (the same kernels run), except:
 *  - PDYN_EWORKSPACE when pdyn_workspace_bytes(PDYN_OP_ID_FD, model, batch, 4)
 *    exceeds PDYN_NOALLOC_SCRATCH_BYTES (64 MiB: e.g. 32 links x 16384 states
 *    with prepared tables needs 50 MiB), checked before any device work;
 *  - the call zeroes the array's status word first; status_out (device, one
 *    32-bit word, or NULL) then receives the PDYN_STATUS_* bits of this call.
 *    For an empty batch nothing is queued and *status_out is not written.
 * All calls on one device share that device's array: calls that overlap in
 * time on one device (several host threads, or several streams) race and give
 * undefined results. Serialise them, e.g. on one stream.
 */
#define PDYN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pdyn_id_fd_noalloc(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                       const float* qdd_in, const float* tau_in, float* tau_out, float* qdd_out, uint32_t* status_out,
                       void* stream);

/*
 * Adjoint of the inverse dynamics (vector-Jacobian product). Gradients of the
 * dynamics are the paper's stated future work (Sec. VI); this is reverse-mode
 * differentiation of the recursions (1)-(2):
 *   (q_bar, qd_bar, qdd_bar, inertia_bar) = (d tau / d(q, qd, qdd, pi))^T tau_bar
 * at tau = ID(q, qd, qdd, V_0, dV_0, F_{n+1}). V_0, dV_0, F_{n+1} and the
 * joint geometry are held constant. inertia_bar is [n][10] summed over the
 * states for a shared chain, [L][10] (one row per link) with one chain per
 * state, in the order of the model's inertia parameters; pass NULL to skip it.
 * The sum over states is deterministic (fixed reduction order).
 */
int pdyn_rnea_id_vjp(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                     const float* qdd, const float* tau_bar, float* q_bar, float* qd_bar, float* qdd_bar,
                     float* inertia_bar, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_rnea_id_vjp_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                         const double* qdd, const double* tau_bar, double* q_bar, double* qd_bar, double* qdd_bar,
                         double* inertia_bar, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Adjoint of the forward dynamics at the solution qdd = FD(q, qd, tau, ...)
 * (pass the forward output as `qdd`). Since ID(q, qd, FD(q, qd, tau)) = tau
 * (eq. (5)), with u = M(q)^-1 qdd_bar:
 *   tau_bar = u,   (q_bar, qd_bar, inertia_bar) = -(d tau/d(q, qd, pi))^T u,
 * the derivative of ID taken at (q, qd, qdd). u is computed by the
 * articulated-body recursions of eq. (8) with tau-hat := qdd_bar; inertia_bar
 * as for pdyn_rnea_id_vjp (NULL to skip).
 */
int pdyn_aba_fd_vjp(const pdyn_model* model, const pdyn_batch* batch, const float* q, const float* qd,
                    const float* qdd, const float* qdd_bar, float* q_bar, float* qd_bar, float* tau_bar,
                    float* inertia_bar, void* workspace, size_t workspace_bytes, void* stream);
int pdyn_aba_fd_vjp_f64(const pdyn_model* model, const pdyn_batch* batch, const double* q, const double* qd,
                        const double* qdd, const double* qdd_bar, double* q_bar, double* qd_bar, double* tau_bar,
                        double* inertia_bar, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Rollouts: `steps` steps of semi-implicit Euler driven by the forward
 * dynamics (eq. (4) is "numerically integrated" to produce trajectories),
 *   qdd_t = FD(q_t, qd_t, tau_t), qd_{t+1} = qd_t + dt qdd_t, q_{t+1} = q_t + dt qd_{t+1},
 * all steps in one launch. q and qd (joint layout) hold the initial state on
 * entry and the final state on return. tau_seq is [steps][joint layout].
 * Checkpoints of (q_t, qd_t) at t = 0, k, 2k, ... (k = ckpt_every) are written
 * to ckpt_q, ckpt_qd, each [ceil(steps / k)][joint layout]. No tip wrench
 * (batch->tip_wrench must be NULL: PDYN_EUNSUPPORTED otherwise).
 */
int pdyn_rollout(const pdyn_model* model, const pdyn_batch* batch, int steps, double dt, int ckpt_every,
                 const float* tau_seq, float* q, float* qd, float* ckpt_q, float* ckpt_qd, void* workspace,
                 size_t workspace_bytes, void* stream);
int pdyn_rollout_f64(const pdyn_model* model, const pdyn_batch* batch, int steps, double dt, int ckpt_every,
                     const double* tau_seq, double* q, double* qd, double* ckpt_q, double* ckpt_qd, void* workspace,
                     size_t workspace_bytes, void* stream);

/*
 * Adjoint of a rollout: given the checkpoints written by pdyn_rollout (same
 * steps, dt, ckpt_every, tau_seq) and the cotangents qT_bar, qdT_bar of the
 * final state, returns dL/dq_0 (q0_bar), dL/dqd_0 (qd0_bar), dL/dtau_t for
 * every step (tau_bar_seq, [steps][joint layout]) and, unless NULL, dL/dpi
 * (inertia_bar, as for pdyn_rnea_id_vjp, summed over steps and states). Each
 * k-step segment is recomputed from its checkpoint, then run backwards with
 * the forward-dynamics adjoint. One launch for the whole reverse pass.
 */
int pdyn_rollout_vjp(const pdyn_model* model, const pdyn_batch* batch, int steps, double dt, int ckpt_every,
                     const float* tau_seq, const float* ckpt_q, const float* ckpt_qd, const float* qT_bar,
                     const float* qdT_bar, float* q0_bar, float* qd0_bar, float* tau_bar_seq, float* inertia_bar,
                     void* workspace, size_t workspace_bytes, void* stream);
int pdyn_rollout_vjp_f64(const pdyn_model* model, const pdyn_batch* batch, int steps, double dt, int ckpt_every,
                         const double* tau_seq, const double* ckpt_q, const double* ckpt_qd, const double* qT_bar,
                         const double* qdT_bar, double* q0_bar, double* qd0_bar, double* tau_bar_seq,
                         double* inertia_bar, void* workspace, size_t workspace_bytes, void* stream);

/*
 * One step of the rollouts' integrator (semi-implicit Euler, the plain
 * per-step form of pdyn_rollout), in place over n joint values:
 *   qd <- qd + dt qdd,  then  q <- q + dt qd  (with the updated qd).
 * n == 0 is a no-op; PDYN_EINVAL for n < 0, a NaN dt or a null array.
 */
int pdyn_euler_step(int64_t n, double dt, float* q, float* qd, const float* qdd, void* stream);
int pdyn_euler_step_f64(int64_t n, double dt, double* q, double* qd, const double* qdd, void* stream);

/*
 * Adjoint of pdyn_euler_step, for a reverse pass over the steps that
 * alternates it with pdyn_aba_fd_vjp. On entry (q_bar, qd_bar) are the
 * cotangents of the state after the step, (q_{t+1}, qd_{t+1}); they are updated
 * in place (an explicit exception to "outputs are overwritten"):
 *  1. if q_bar_fd is not NULL (then qd_bar_fd must not be either), the
 *     forward-dynamics adjoint of the later step is added first:
 *     q_bar += q_bar_fd, qd_bar += qd_bar_fd; if pi_bar_fd is not NULL,
 *     pi_bar[0 .. n_pi) += pi_bar_fd (inertia cotangents summed over steps);
 *  2. if qdd_bar is not NULL, the step's own adjoint:
 *     qd_bar <- qd_bar + dt q_bar (the cotangent of qd_t through the update),
 *     qdd_bar = dt qd_bar (the cotangent of qdd_t = FD(q_t, qd_t, tau_t), to be
 *     passed to pdyn_aba_fd_vjp); q_bar passes through unchanged.
 * Calling it with qdd_bar == NULL after the first step's forward-dynamics
 * adjoint leaves (q_bar, qd_bar) = dL/d(q_0, qd_0).
 */
int pdyn_euler_step_vjp(int64_t n, double dt, float* q_bar, float* qd_bar, const float* q_bar_fd,
                        const float* qd_bar_fd, float* qdd_bar, int64_t n_pi, float* pi_bar, const float* pi_bar_fd,
                        void* stream);
int pdyn_euler_step_vjp_f64(int64_t n, double dt, double* q_bar, double* qd_bar, const double* q_bar_fd,
                            const double* qd_bar_fd, double* qdd_bar, int64_t n_pi, double* pi_bar,
                            const double* pi_bar_fd, void* stream);

/* Workspace bytes of pdyn_rollout (with_grad = 0) or pdyn_rollout_vjp (1). */
size_t pdyn_rollout_workspace_bytes(int with_grad, const pdyn_model* model, const pdyn_batch* batch, int ckpt_every,
                                    int scalar_bytes);

#ifdef __cplusplus
}
#endif

#endif /* PDYN_H */
