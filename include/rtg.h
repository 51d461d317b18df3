/*
 * rtg.h -- C ABI of the MI355X (gfx950) RTG-GMRES library (librtg.so).
 *
 * RTG-GMRES solves  min || Phi(X) - C ||_F  (eq. (1)) for third-order tensors
 * X, C in R^{I1 x I2 x J} with the operator of eq. (2),
 *
 *     Phi(X) = A *_2 X *_1 B,     a[i1,i2,k1,k2] = A1[i1,k1] A2[i2,k2],
 *
 * i.e. Phi(X) = X x_1 A1 x_2 A2 x_3 B^T, by the sketched tensor global
 * Arnoldi process (Sec. 4.3) whose inner products are the sketched Einstein
 * inner products <X,Y>_Theta = <S(X), S(Y)>_F with the mode-wise sketch
 * S(X) = X x_1 Om1 x_2 Om2 x_3 Om3 (Sec. 3.1), followed by the projected
 * Tikhonov problem  min ||beta e1 - H y||^2 + mu ||y||^2  (eqs. (12)-(13)),
 * mu fixed or chosen by the discrepancy principle or by GCV (Sec. 3), and
 * X = X0 + sum_j y_j V_j (algorithm "Block GMRES via Sketched Einstein
 * Product", Sec. 4.4).  Also: sketched Block Golub-Kahan in place of the
 * Arnoldi process (Sec. 4.5; rtg_params.method), a general non-separable PSF
 * in place of A1 (x) A2 (eqs. (56)-(57); rtg_setup_operator_psf), restarted
 * RTG-GMRES (rtg_params.restarts), the identity sketch (unsketched global
 * GMRES), batches of uneven problems and a learned warm start.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Tensors are device arrays of I1*I2*J elements in column-major order,
 *   i1 fastest: offset(i1,i2,j) = i1 + I1*(i2 + I2*j) (the ivec order of
 *   Sec. 4.1).  I1 must be a multiple of 8 and device pointers 16-byte
 *   aligned.
 * - A banded factor M (I x I, half-bandwidth r) is a HOST array of
 *   I*(2r+1) floats, row-major: band[i*(2r+1) + d + r] = M[i, i+d] for
 *   -r <= d <= r; entries whose column leaves [0, I) are ignored (zero
 *   boundary conditions, Sec. 5.1).
 * - Sketch factors Om_k are HOST arrays, row-major l_k x I_k; NULL means the
 *   identity (then l_k must equal I_k).
 * - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *   Compute calls only enqueue work; they return after argument checks.
 * - Return codes (synchronous, host-side): RTG_OK or a negative RTG_E_*.
 *   Numerical outcomes are reported in device-resident rtg_info.flags.
 * - Ownership: all tensors and workspaces are caller-owned device memory.
 *   Handles own small device copies of the bands (and of their transposes,
 *   the adjoint operator of Golub-Kahan) and sketch factors and are
 *   immutable after setup: one handle may be used concurrently on several
 *   streams with separate workspaces.  Compute calls never allocate.
 */
#ifndef RTG_H
#define RTG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtg_op_s* rtg_op;
typedef struct rtg_sk_s* rtg_sk;

/* element types of tensors the library reads (X inputs, the Krylov basis);
 * RTG_F32_BF16 (basis only): the basis is stored in float32 and the sketch
 * contractions take bfloat16 MFMA operands with float32 accumulation (each
 * new basis tensor rounded to bfloat16 for the products; Om1 rounded to
 * bfloat16, its composition with A1 kept in two bfloat16 terms) */
enum { RTG_F32 = 0, RTG_BF16 = 1, RTG_F32_BF16 = 2 };

/* return codes */
enum {
    RTG_OK = 0,
    RTG_E_ARG = -1,        /* null pointer, bad enum, misaligned pointer  */
    RTG_E_SHAPE = -2,      /* inconsistent or unsupported sizes           */
    RTG_E_HIP = -3,        /* a HIP runtime call failed                   */
    RTG_E_NOMEM = -4,      /* device allocation in a setup call failed    */
    RTG_E_WORKSPACE = -5   /* workspace smaller than required             */
};

/* numerical outcome flags (rtg_info.flags, device side) */
enum {
    RTG_F_BREAKDOWN = 1,           /* h_{j+1,j} <= bd_tol ||S(Phi(V_j))||: solved at j
                                      (Golub-Kahan: beta_{k+1} or alpha_{k+1} below
                                      bd_tol times the sketched norm of Phi(V_k) or
                                      Phi^T(U_{k+1}); solved with the complete columns) */
    RTG_F_DISCREP_UNREACHABLE = 2, /* LS residual already above eta*delta: mu = 0      */
    RTG_F_MU_INF = 4,              /* eta*delta >= beta: y = 0, X = X0                  */
    RTG_F_NONFINITE = 8,           /* NaN/Inf met in a coefficient                     */
    RTG_F_NOT_CONVERGED = 16,      /* stop_res requested and not reached within m      */
    RTG_F_FALLBACK = 32,           /* rtg_solve_batched_fallback: the result is the
                                      plain solver's re-solve of this problem          */
    RTG_F_TIMEOUT = 64             /* the persistent batched launch was abandoned (a
                                      wait between its workgroups exceeded the limit
                                      of rtg_set_wait_limit): no steps, X = X0         */
};

/* Solver parameters. */
typedef struct {
    int m;            /* maximum number of Arnoldi steps (Golub-Kahan: columns),
                         1 <= m <= 96                                            */
    int basis_dtype;  /* RTG_F32, RTG_BF16 (storage of V_j and MFMA precision) or
                         RTG_F32_BF16 (float32 storage, bfloat16 sketch products;
                         RTG-GMRES only)                                         */
    double mu;        /* >= 0: fixed Tikhonov parameter; < 0: chosen by mu_rule    */
    double delta;     /* absolute noise-norm estimate ||E||_F (discrepancy)       */
    double eta;       /* discrepancy safety factor (1.01 is customary)            */
    double stop_res;  /* > 0: stop at the first j whose projected LS residual is
                         <= stop_res; <= 0: run m steps                          */
    double bd_tol;    /* breakdown threshold relative to ||S(Phi(V_j))||          */
    int mu_rule;      /* when mu < 0: RTG_MU_DISCREPANCY (root of the projected
                         residual at eta*delta) or RTG_MU_GCV (minimiser of the
                         GCV function of the projected problem, Sec. 3; delta
                         and eta unused)                                        */
    int method;       /* RTG_METHOD_GMRES: RTG-GMRES (Sec. 4.4);
                         RTG_METHOD_GOLUB_KAHAN: sketched Block Golub-Kahan
                         (Sec. 4.5), m columns of the lower bidiagonal matrix
                         in place of the Hessenberg matrix, the same projected
                         Tikhonov problem and mu rules                        */
    int restarts;     /* restarted RTG-GMRES: while ||C - Phi(X)||_Theta >= eps
                         (eps = stop_res > 0, required) after a solve, start
                         another from X0 = X, at most `restarts` times (0 =
                         none; RTG-GMRES only).  rtg_info then reports the
                         last solve, with iters summed over all of them      */
} rtg_params;

enum { RTG_MU_DISCREPANCY = 0, RTG_MU_GCV = 1 };
enum { RTG_METHOD_GMRES = 0, RTG_METHOD_GOLUB_KAHAN = 1 };

/* Result summary, written by the device at the end of a solve. */
typedef struct {
    int iters;        /* number of Arnoldi steps (Golub-Kahan: bidiagonal
                         columns) taken (m_eff)                                   */
    int flags;        /* RTG_F_* bits                                            */
    double mu;        /* Tikhonov parameter used (inf if RTG_F_MU_INF)            */
    double beta;      /* ||R0||_Theta                                            */
    double res_proj;  /* ||beta e1 - H y||_2, which is ||S(C - Phi(X))||_F for
                         RTG-GMRES (Theta-orthonormal basis, Sec. 4.4); for
                         Golub-Kahan the same norm with the bidiagonal matrix */
    double res_ls;    /* least-squares residual of the projected problem (11S)    */
} rtg_info;

/* One problem of a batch (rtg_solve_batched). */
typedef struct {
    rtg_op op;
    rtg_sk sk;
    const float* C;   /* device, observation                                      */
    const float* X0;  /* device initial guess, or NULL for X0 = 0                 */
    float* X;         /* device output                                            */
    rtg_params params;
    rtg_info* info;   /* device pointer                                           */
} rtg_problem;

/* ---- operator (eq. (2); Sec. 5.1-5.2) ------------------------------------
 * Phi(X) = X x_1 A1 x_2 A2 x_3 B^T.  b_band is the band of B as it appears in
 * X *_1 B, (X *_1 B)[:,:,j] = sum_k X[:,:,k] B[k,j]; the library applies B^T
 * along mode 3 itself.  Requires 0 <= r1 < I1, 0 <= r2 < I2 (r <= 12),
 * 0 <= rB < J (rB <= 8).  Copies the bands to the device. */
int rtg_setup_operator(int I1, int I2, int J,
                       const float* a1_band, int r1,
                       const float* a2_band, int r2,
                       const float* b_band, int rB, rtg_op* out);
/* General (non-separable) PSF (eqs. (56)-(57)): Phi(X) = (A *_2 X) *_1 B with
 * A built from a (2r+1) x (2r+1) PSF, every channel convolved with zero
 * boundary conditions, (A *_2 X)[i1,i2,k] = sum_{a,b} P[r-a][r-b] X[i1+a,i2+b,k]
 * for |a|, |b| <= r.  psf is a HOST array, row-major P[r + a][r + b] with the
 * row index along i1 (centre at [r][r]); b_band as above.  Requires
 * 0 <= r <= 12, r < I1, r < I2 (or I2 = 1), 0 <= rB < J (rB <= 8).  Solves
 * with such an operator sketch each W = Phi(V_j) after forming it (the
 * composed sketch matrices need separable factors), so a step costs one more
 * pass over W; one kind of operator per batch (RTG_E_ARG otherwise), and
 * Golub-Kahan is refused for it (RTG_E_ARG). */
int rtg_setup_operator_psf(int I1, int I2, int J, const float* psf, int r,
                           const float* b_band, int rB, rtg_op* out);
/* Y = Phi(X)  (C == NULL)  or  Y = C - Phi(X)  (C != NULL); X of x_dtype. */
int rtg_apply_operator(rtg_op op, int x_dtype, const void* X, const float* C,
                       float* Y, void* stream);
int rtg_destroy_operator(rtg_op op);

/* ---- sketch (Sec. 3.1, global tensor sketching operator) ------------------
 * S(X) = X x_1 Om1 x_2 Om2 x_3 Om3 with Om_k in R^{l_k x I_k}.  Requires
 * 1 <= l1 <= min(I1, 128), 1 <= l2 <= min(I2, 128), 1 <= l3 <= min(J, 16)
 * when Om3 is given, and I1, I2 below 2^20.  The device keeps float32 copies and a
 * bfloat16 copy of Om1 (used by the BF16 path), plus copies of Om1 in the
 * tile order of the matrix-core contractions. */
int rtg_setup_sketch(int I1, int I2, int J, int l1, int l2, int l3,
                     const float* om1, const float* om2, const float* om3,
                     rtg_sk* out);
size_t rtg_sketch_workspace_bytes(rtg_sk sk);
/* SX = S(X), L = l1*l2*l3 floats in column-major order (a fastest):
 * SX[a + l1*(b + l2*c)].  x_dtype RTG_F32 uses float32 MFMA; RTG_BF16 reads a
 * bfloat16 X and uses bfloat16 MFMA with float32 accumulation. */
int rtg_sketch(rtg_sk sk, int x_dtype, const void* X, float* SX,
               void* ws, size_t ws_bytes, void* stream);
/* rtg_sketch without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  The descriptor and the partial sketches live in
 * a device array of RTG_SKETCH_NOALLOC_MAX_BYTES that the library keeps on
 * every GPU it runs on until the process ends; the call allocates nothing.
 * RTG_E_WORKSPACE when rtg_sketch_workspace_bytes(sk) exceeds that size
 * (J * ceil(I2 / 32) * l1 * l2 * 4 bytes plus a few hundred, e.g. 0.8 MB for
 * a 512x512x3 tensor with a 64x64x3 sketch); other argument errors as
 * rtg_sketch.  All calls on one GPU share its array: calls that overlap in
 * time on one GPU (several streams, several host threads) race and must be
 * serialised by the caller.  Results are identical to rtg_sketch's. */
#define RTG_SKETCH_NOALLOC_MAX_BYTES (8u << 20)
int rtg_sketch_noalloc(rtg_sk sk, int x_dtype, const void* X, float* SX, void* stream);
int rtg_destroy_sketch(rtg_sk sk);

/* ---- Arnoldi and solve ----------------------------------------------------- */
/* Workspace of one problem with at most m steps and the given basis type
 * (RTG-GMRES, also with restarts). */
size_t rtg_workspace_bytes(rtg_op op, rtg_sk sk, int m, int basis_dtype);

/* m steps of the sketched global Arnoldi process from R0 (Sec. 4.3):
 * beta = ||R0||_Theta, V1 = R0/beta, h_ij = <V_i, Phi(V_j)>_Theta (classical
 * Gram-Schmidt with one reorthogonalisation, evaluated in sketch space),
 * h_{j+1,j} = ||.||_Theta.  Outputs (device): H, (m+1) x m column-major
 * float64 (zero below the computed part); *beta; *m_done (< m after a
 * breakdown).  The basis stays in ws (see rtg_workspace_layout). */
int rtg_arnoldi(rtg_op op, rtg_sk sk, const float* R0, int m, int basis_dtype,
                double bd_tol, void* ws, size_t ws_bytes,
                double* H, double* beta, int* m_done, void* stream);

/* Offsets (bytes from ws) of the basis V_1..V_{m+1} (consecutive tensors of
 * basis_dtype) and of the sketched basis S(V_1)..S(V_{m+1}) (consecutive
 * float32 vectors of L entries, internal order (a*l2 + b)*l3 + c). */
int rtg_workspace_layout(rtg_op op, rtg_sk sk, int m, int basis_dtype,
                         size_t* v_offset, size_t* sv_offset);

/* Workspace of one sketched Block Golub-Kahan solve (params.method =
 * RTG_METHOD_GOLUB_KAHAN) with at most m columns: a second basis
 * U_1..U_{m+1} with its sketches and the composed sketch matrices of the
 * adjoint operator on top of rtg_workspace_bytes. */
size_t rtg_gk_workspace_bytes(rtg_op op, rtg_sk sk, int m, int basis_dtype);

/* m columns of the sketched Block Golub-Kahan bidiagonalisation from R0
 * (Sec. 4.5, recurrences as for rtg_solve below).  Outputs (device): B,
 * (m+1) x m column-major float64 lower bidiagonal (alpha_k on the diagonal,
 * beta_{k+1} below it; zero past the computed part); *beta = beta_1;
 * *m_done (< m after a breakdown: beta_{k+1} <= bd_tol ||S(Phi(V_k))|| or
 * alpha_{k+1} <= bd_tol ||S(Phi^T(U_{k+1}))||).  The bases U_1..U_{m+1} and
 * V_1..V_m stay in ws (rtg_gk_workspace_layout); ws_bytes >=
 * rtg_gk_workspace_bytes.  Needs a sketch with at least one Om_k given and
 * a banded operator (RTG_E_ARG otherwise: a general PSF has no adjoint here). */
int rtg_golub_kahan(rtg_op op, rtg_sk sk, const float* R0, int m, int basis_dtype,
                    double bd_tol, void* ws, size_t ws_bytes,
                    double* B, double* beta, int* m_done, void* stream);

/* Offsets (bytes from ws) of V_1..V_{m+1} and U_1..U_{m+1} (consecutive
 * tensors of basis_dtype) in the workspace of rtg_golub_kahan. */
int rtg_gk_workspace_layout(rtg_op op, rtg_sk sk, int m, int basis_dtype,
                            size_t* v_offset, size_t* u_offset);

/* Full solve of one problem, RTG-GMRES or (params->method) sketched Block
 * Golub-Kahan; info is a device pointer.
 * Golub-Kahan (Sec. 4.5): beta_1 = ||R0||_Theta, U_1 = R0/beta_1,
 * alpha_1 V_1 = Phi^T(U_1), then beta_{k+1} U_{k+1} = Phi(V_k) - alpha_k U_k
 * and alpha_{k+1} V_{k+1} = Phi^T(U_{k+1}) - beta_{k+1} V_k with Theta-norms
 * (Phi^T the Frobenius adjoint, X x_1 A1^T x_2 A2^T x_3 B); X = X0 + sum
 * y_k V_k with y from min ||beta_1 e1 - B y||^2 + mu ||y||^2.  It needs a
 * sketch with at least one Om_k given (RTG_E_ARG for the all-identity
 * sketch) and a workspace of rtg_gk_workspace_bytes. */
int rtg_solve(rtg_op op, rtg_sk sk, const float* C, const float* X0,
              const rtg_params* params, void* ws, size_t ws_bytes,
              float* X, rtg_info* info, void* stream);

/* Many independent problems (uneven sizes allowed) solved together: every
 * stage is one launch over the tiles of all problems.  probs is a HOST array.
 * One basis type, one method and one kind of operator (banded or general
 * PSF) per batch (RTG_E_ARG otherwise). */
size_t rtg_batch_workspace_bytes(int count, const rtg_problem* probs);
int rtg_solve_batched(int count, const rtg_problem* probs, void* ws,
                      size_t ws_bytes, void* stream);

/* The plain solver as the fallback of warm-started (or otherwise shortened)
 * solves.  The batch is solved as by rtg_solve_batched; then every problem
 * whose flags meet fail_mask (a set of RTG_F_* bits, typically
 * RTG_F_NOT_CONVERGED | RTG_F_NONFINITE: a solve stopped at stop_res that did
 * not reach it within m steps, or met a non-finite value) is solved again by
 * the plain solver: RTG-GMRES (Sec. 4.4) from X0 = 0 with fb_m steps and
 * basis type fb_basis, the problem's own mu rule, delta, eta and bd_tol, no
 * stop_res and no restarts.  That result replaces X and info, and its flags
 * carry RTG_F_FALLBACK.  SYNCHRONOUS: the flags are read back to the host
 * (one small copy) before the re-solves are enqueued, and the call returns
 * once they are enqueued.  *n_fallback receives the number of re-solved
 * problems.  ws_bytes >= rtg_fallback_workspace_bytes(count, probs, fb_m,
 * fb_basis), which covers the batch and the largest single re-solve; the
 * re-solves run as many at a time as ws_bytes holds.  Argument errors as
 * rtg_solve_batched, RTG_E_ARG for fail_mask bits outside RTG_F_BREAKDOWN ..
 * RTG_F_NOT_CONVERGED or a bad fb_basis, RTG_E_SHAPE for an fb_m the
 * problems' sketches cannot take (0 from the size query). */
size_t rtg_fallback_workspace_bytes(int count, const rtg_problem* probs,
                                    int fb_m, int fb_basis);
int rtg_solve_batched_fallback(int count, const rtg_problem* probs, int fb_m,
                               int fb_basis, int fail_mask, void* ws,
                               size_t ws_bytes, int* n_fallback, void* stream);

/* The same fallback in two calls, so that the stream can take other work
 * (the next batch's warm start, say) while the flags travel: the host waits
 * only for the flag copy, not for what was queued after it.
 * rtg_solve_batched_fallback_begin solves the batch as rtg_solve_batched
 * does and queues the copy of every problem's flags to flags_host (count
 * ints of caller-owned host memory, page-locked for the copy to run
 * asynchronously; it must not be touched before the matching _end);
 * asynchronous.  rtg_solve_batched_fallback_end, called with the same
 * arguments and the same flags_host, waits for that copy, re-solves the
 * problems whose flags meet fail_mask exactly as rtg_solve_batched_fallback
 * does, and returns once the re-solves are queued; *n_fallback receives their
 * number.  Errors as rtg_solve_batched_fallback; _end without a pending
 * _begin for flags_host returns RTG_E_ARG.  Calls for different flags_host
 * buffers may be in flight together. */
int rtg_solve_batched_fallback_begin(int count, const rtg_problem* probs,
                                     int fb_m, int fb_basis, int fail_mask,
                                     void* ws, size_t ws_bytes,
                                     int* flags_host, void* stream);
int rtg_solve_batched_fallback_end(int count, const rtg_problem* probs,
                                   int fb_m, int fb_basis, int fail_mask,
                                   void* ws, size_t ws_bytes,
                                   const int* flags_host, int* n_fallback,
                                   void* stream);

/* ---- tile autotuner (the batching form's launch shapes) --------------------
 * The launch shapes of a batch: every combination that the fields allow is
 * a correct solve of the same problems (they change which thread computes
 * what, not the arithmetic), so the choice is a matter of speed.  A process-
 * wide table (host memory, guarded by a mutex) maps a batch's shape key --
 * count, method, basis type and, per problem, the sizes, band half-widths,
 * sketch sizes, operator kind, m and whether X0 is given -- to a choice;
 * rtg_solve_batched and rtg_solve use the table's entry for their key, and
 * the library defaults (every field -1) when there is none.
 * Fields (-1: the default for that batch):
 *   phi_jt        operator kernel: output channels per tile, 4 or 8
 *   phi_slab      operator slab staging: 0 single-word loads, 1 16-byte loads
 *                 (float32 inputs under 2^31 bytes), 2 asynchronous
 *                 global-to-LDS loads (general PSF with J <= 3)
 *   phi_toeplitz  1: the taps of Toeplitz bands in registers (separable
 *                 operators whose bands are all Toeplitz, phi_slab >= 1);
 *                 0: band rows streamed through LDS
 *   tile_rows     tile kernel: 16-row sketch tiles per wave, 2 (used where
 *                 the stacked sketch rows fit, else 4) or 4
 *   step_rows     fused bfloat16 Arnoldi step: the same, 2 or 4
 *   step_toeplitz fused step: 1 Toeplitz taps (all bands Toeplitz), 0 band rows
 *   gram_pairs    sketched inner products: (a, b) sketch pairs per workgroup,
 *                 256, 512 or 1024 (capped at 4096 / l3 finished values; never
 *                 below the library's own choice for the problem)
 *   persist       1: the Arnoldi process of the whole batch (the start and
 *                 every step of every problem) as one persistent launch whose
 *                 workgroups take the stages' tiles in order from a device-side
 *                 counter, each stage of a problem waiting only for that
 *                 problem's earlier stages (RTG-GMRES with a sketch, a
 *                 separable operator, a float32 basis in either product form,
 *                 J <= 4 and inputs under 2^31 bytes); 0: one launch per stage
 *                 over all problems */
typedef struct {
    int phi_jt;
    int phi_slab;
    int phi_toeplitz;
    int tile_rows;
    int step_rows;
    int step_toeplitz;
    int gram_pairs;
    int persist;
} rtg_tune;           /* 32 bytes */

/* Time the batch's solve (the Arnoldi or Golub-Kahan loop; no projected
 * solve, no assembly, the outputs X and info untouched) under candidate
 * shapes -- the operator fields first, then the tile rows, the Gram pairs,
 * then the fused step's fields, each group with the others at their best so
 * far -- on
 * stream, the minimum over reps >= 1 runs of each candidate (hipEvents),
 * and record the fastest in the table.  Synchronous.  *chosen receives the
 * choice with every field resolved (no -1), *best_ms (may be NULL) its
 * time.  The workspace is that of rtg_batch_workspace_bytes; its contents
 * are overwritten.  Argument errors as rtg_solve_batched. */
int rtg_autotune_batched(int count, const rtg_problem* probs, void* ws,
                         size_t ws_bytes, int reps, rtg_tune* chosen,
                         double* best_ms, void* stream);
/* Record a choice for the batch's key (RTG_E_ARG for a field outside the
 * values above or one the batch cannot use: phi_slab 1 or 2 for inputs of
 * 2^31 bytes or more, phi_slab 2 for a separable operator or J > 3,
 * toeplitz fields for non-Toeplitz bands or a general PSF, persist 1 for a
 * batch that cannot take it or with phi_jt 8 or phi_slab 0). */
int rtg_tune_set(int count, const rtg_problem* probs, const rtg_tune* tune);
/* The choice a solve of this batch would use, every field resolved. */
int rtg_tune_get(int count, const rtg_problem* probs, rtg_tune* tune);
/* Forget every recorded choice. */
int rtg_tune_clear(void);

/* Bound on every wait between workgroups of the persistent launch
 * (rtg_tune.persist = 1): a workgroup that finds a dependency unmet after
 * this many polls (about a microsecond each) abandons the launch; every
 * workgroup then stops taking work, and every problem of the batch ends
 * with RTG_F_TIMEOUT in its info flags, no steps and X = X0 (zero when X0
 * is NULL).  Process-wide, read at each launch; polls >= 0 (RTG_E_ARG
 * otherwise), default 4194304.  A limit that low waits never pass is what
 * tests of the failure path use. */
int rtg_set_wait_limit(int polls);

/* ---- learned warm start ----------------------------------------------------
 * X0 = C + f(C), f = six 3x3 zero-padded convolutions 3 -> 32 -> 32 -> 32 ->
 * 32 -> 32 -> 3 with biases and ReLU after the first five (38,755
 * parameters), computed with bfloat16 MFMA and float32 accumulation; float32
 * master weights and Adam moments.  The warm start only changes X0: the
 * RTG-GMRES solve that follows is the method itself and corrects it.
 * Parameters cross the ABI as one HOST float array, layer after layer, each
 * layer w[co][t1][t2][ci] (t1, t2 in 0..2: offsets -1..+1 along i1 and i2)
 * followed by b[co].  Images are device arrays [N][3][I2][I1] (each the
 * column-major tensor layout above).  state is a caller-owned device buffer
 * of rtg_cnn_state_bytes(); ws of rtg_cnn_workspace_bytes(N, I1, I2). */
size_t rtg_cnn_state_bytes(void);
size_t rtg_cnn_workspace_bytes(int N, int I1, int I2);
/* copy the parameters in, zero the moments (synchronous on stream) */
int rtg_cnn_init(void* state, const float* params, void* stream);
/* copy the float32 master parameters out (synchronous) */
int rtg_cnn_export(const void* state, float* params, void* stream);
/* X0 = C + f(C).  N * I1 * I2 below 2^25 pixels per call (32-bit byte
 * offsets into the 32-channel activations); larger batches are split by the
 * caller. */
int rtg_cnn_forward(const void* state, const float* C, int N, int I1, int I2,
                    float* X0, void* ws, size_t ws_bytes, void* stream);
/* gradients of sum((X0 - Y)^2) / (3 N I1 I2) w.r.t. every parameter, kept
 * in state; *loss (device float) receives the sum of squared errors */
int rtg_cnn_gradients(void* state, const float* C, const float* Y, int N, int I1,
                      int I2, void* ws, size_t ws_bytes, float* loss, void* stream);
/* the gradients of the last rtg_cnn_gradients call, parameter layout (synchronous) */
int rtg_cnn_read_gradients(const void* state, float* grads, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction for step >= 1) */
int rtg_cnn_adam(void* state, float lr, int step, void* stream);

/* ---- measurement ----------------------------------------------------------
 * When enabled, every launch of the selected kernel kinds made by the solver
 * calls (bit k of kind_mask: 0 operator Phi, 1 multi-AXPY + sketch tile,
 * 2 sketched Gram / Hessenberg update, 3 projected Tikhonov solve, 4 Arnoldi
 * step with the operator applied on the fly, 5 the persistent launch of the
 * Arnoldi process) is
 * bracketed by two hipEvents recorded on the launch stream.
 * rtg_event_timing_read waits for those events and returns, per kind, the
 * summed duration in milliseconds and the number of launches, then clears
 * the record.  Host-side state shared by the process (not thread-safe); a
 * kind_mask of 0 disables recording. */
int rtg_event_timing_enable(int kind_mask);
int rtg_event_timing_read(double* ms, long long* launches, int nkinds);

const char* rtg_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* RTG_H */
