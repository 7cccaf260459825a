/*
 * ptebd.h -- C ABI of libptebd, the MI355X (gfx950) pTEBD layer library.
 *
 * The library evolves matrix-product states (MPS) in the Vidal form {Gamma, Lambda}
 * (Sec. II.B, Eq. (mps_cano_decomp)) under layers of non-overlapping two-qubit gates
 * (Sec. IV, Eq. (circ_decomp)) with the parallel TEBD algorithm of Algorithm 1:
 * every gate of a layer is applied at once by the TEBD procedure of Sec. II.C, every
 * updated bond is truncated by the projector compression of Sec. III.B, its Schmidt
 * values are rescaled by the norm-stabilization factor nu_i = (1 - eps_i)^(-1/2) of
 * Sec. III.C.2 (Eq. (lren)), and, when the layer had to be compressed, g parallel
 * trivial-simple-update (PtSU) steps of Sec. III.D follow (IPMC, Sec. III.E).
 *
 * Conventions used by every call:
 *   - Sites q = 0..N-1, bonds i = 0..N.  Lambda[i] sits between sites i-1 and i,
 *     Lambda[0] = Lambda[N] = (1); it is real, positive, descending and held in FP64.
 *     Gamma[q] has shape (chi_q, 2, chi_{q+1}) with chi_i = len(Lambda[i]).
 *   - A gate "at q" acts on sites (q, q+1): it rewrites Lambda[q+1], Gamma[q], Gamma[q+1]
 *     and reads Lambda[q], Lambda[q+2].
 *   - A gate is 16 complex128 numbers, interleaved (re, im), row-major 4x4
 *     U[(s' t'), (s t)] with the left site's index s as the high bit.
 *   - Host complex arrays are complex128 interleaved (re, im).  Gamma[q] in host
 *     arrays is C-ordered (a, s, m), i.e. element (a, s, m) at ((a*2 + s)*chi_{q+1} + m).
 *   - Every call returns an int status: 0 = OK, negative = error, positive = warning.
 *     After an error the state is unchanged if the error was detected before any
 *     device work was enqueued (all argument validation happens first).
 *     ptebd_last_error() returns a thread-local message for the last non-zero status.
 *   - No C++ exception crosses this interface.
 *
 * Ownership: the caller owns every host array it passes; the library copies what it
 * needs before returning, so the caller may free or reuse them at once.  The library
 * owns all device memory it allocates; device pointers never leave it.  The handle is
 * bound to the HIP device current at create time and to the stream given there.
 * Calls on one handle must not run concurrently from several host threads.
 */
#ifndef PTEBD_H
#define PTEBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define PTEBD_OK 0
#define PTEBD_EINVAL (-1)        /* bad argument: N, d, chi, cutoff < 0, q out of range, NaN/Inf gate */
#define PTEBD_EOVERLAP (-2)      /* two gates of one layer share a site of the same state */
#define PTEBD_ENOMEM (-3)        /* device or pinned host allocation failed */
#define PTEBD_EDEVICE (-4)       /* a HIP runtime call failed */
#define PTEBD_ENONFINITE (-5)    /* a non-finite Lambda or singular value was produced */
#define PTEBD_EANNIHILATED (-6)  /* a two-site wavefunction vanished or eps_i >= 1 */
#define PTEBD_WNOCONV 1          /* some SVD reached the sweep cap; result usable */

/* ------------------------------------------------------------------ precisions */
#define PTEBD_FP64 0  /* Gamma, theta and every product in FP64 (FP64 MFMA) */
#define PTEBD_FP32 1  /* Gamma, theta, Jacobi column updates in FP32 (FP32 MFMA); the
                         Jacobi rotation angles, singular values, eps, nu, Lambda and
                         the Lambda^{-1} divisions in FP64 */
#define PTEBD_BF16X3 2 /* contractions on bf16 MFMA with each FP32 operand split into
                          hi = bf16(x), lo = bf16(x - hi) and the products hi hi + hi lo + lo hi
                          accumulated in FP32.  Not built in this library: every call that
                          takes a precision returns PTEBD_EINVAL for it.  The split keeps
                          ~16 mantissa bits, so the Jacobi column updates could not use it
                          at a 1e-6 fidelity budget, and the theta contraction it would speed
                          up is a few per cent of a layer. */

/* On the FP32 path every truncation (gates and tSU) drops the singular values
 * sigma <= max(cutoff, PTEBD_FP32_CUTOFF_FLOOR) sigma_1.  The exact zeros of a rank-deficient
 * theta (CZ, SWAP, product gates) come out of FP32 arithmetic as rounding residues: the SVD
 * stops rotating a column once its norm is below 16 u (u = 2^-24) times its partner's, so a
 * residue can keep up to 2^-20 sigma_1; keeping it would put a noise direction, divided by
 * Lambda, into Gamma.  The floor is twice that level, 2^-19; the weight it drops is below
 * 3.7e-12 sigma_1^2 per value. */
#define PTEBD_FP32_CUTOFF_FLOOR 1.9073486328125e-06

/* ------------------------------------------------------------------ layer flags */
#define PTEBD_FLAG_NO_STABILIZE 1  /* nu_i = 1 (norm-stabilization ablation: the norm decay of
                                      Sec. III.C.1 without the remedy of Sec. III.C.2) */
#define PTEBD_FLAG_RELATIVE_EPS 2  /* eps_i = discarded sigma^2 / sum sigma^2 (keeps each bond's
                                      local norm); default: the literal discarded sigma^2 */
#define PTEBD_FLAG_COMPLEMENT_EPS 4 /* eps_i = 1 - kept sigma^2, so that nu_i rescales the kept
                                      values to unit norm.  All three readings of Theorem 1's
                                      local error agree on a normalized canonical input; this
                                      one keeps the stabilized norm near 1 over long circuits
                                      (the norm-vs-depth result of Sec. IV.B, numerical
                                      stability), the literal one lets it grow under heavy
                                      truncation.  Not combinable with RELATIVE_EPS. */

typedef struct ptebd_mps* ptebd_mps_t;

/* Per-layer statistics.  The array pointers are caller-owned outputs of length
 * n_gates (any may be NULL); the scalars are filled by the library. */
typedef struct {
  int32_t* k;       /* kept bond dimension of each gate's bond */
  int32_t* rank;    /* r = #{sigma > cutoff * sigma_1} */
  double* eps;      /* local truncation error eps_i of Theorem 1 under the chosen reading
                       (default: the sum of the dropped sigma^2) */
  double* nu;       /* stabilization factor applied to Lambda[q+1]: (1 - eps_i)^(-1/2) when
                       the layer was compressed and stabilization is on, else exactly 1 */
  int32_t* sweeps;  /* Jacobi sweeps used by the gate's SVD */
  int32_t triggered;      /* 1 if some gate had r > chi_max (the layer was compressed) */
  int32_t ptsu_done;      /* PtSU steps executed after the gates */
  int32_t max_sweeps;     /* max Jacobi sweeps over all SVDs of the layer, PtSU included */
  int32_t n_unconverged;  /* SVDs that hit the sweep cap */
  double device_ms;       /* device time of the layer, from HIP events on the stream */
} ptebd_layer_stats;

/* Library version string. */
const char* ptebd_version(void);

/* Thread-local text of the last non-zero status returned on this thread. */
const char* ptebd_last_error(void);

/*
 * Create a batch of n_states MPS, each in |0...0> (chi_0 = 1, Sec. IV.A: Gamma[q] = e_0,
 * every Lambda = (1)).
 *   n_sites[s]  >= 2, number of qubits of state s;
 *   chi_cap[s]  in [1, 512], largest bond dimension state s may reach (sizes its device slots:
 *               N * 2 * chi_cap^2 complex numbers of the chosen precision);
 *   d           local dimension, must be 2;
 *   precision   PTEBD_FP64 or PTEBD_FP32 (PTEBD_BF16X3: EINVAL, not built);
 *   hip_stream  hipStream_t every device operation of the handle is ordered on
 *               (NULL = the null stream); the library does not own it.
 * Errors: EINVAL, ENOMEM, EDEVICE.  *out is NULL on error.
 */
int ptebd_mps_create(int n_states, const int32_t* n_sites, const int32_t* chi_cap, int d,
                     int precision, void* hip_stream, ptebd_mps_t* out);

/* Free the handle and all its device memory.  NULL is accepted. */
int ptebd_mps_destroy(ptebd_mps_t h);

/* Controls of the batched one-sided block Jacobi SVD of a handle. */
typedef struct {
  int max_sweeps;       /* >= 1, default 30 */
  double tol_factor;    /* > 0, default 1 for FP32 and 4 for FP64: a pair of columns counts
                           as orthogonal when |x^H y| <= max(tol_factor sqrt(rows), 8) eps
                           |x| |y|, eps the unit roundoff of the precision (the floor: a short
                           pair's cosine is not computed more accurately than that) */
  int inner_sweeps;     /* in [1, 64]: at most this many cyclic sweeps over each 32x32 block
                           pair's Gram matrix (default 2 for FP32, 1 for FP64) */
  double inner_repeat;  /* >= 0: a further inner sweep runs only while the previous one rotated
                           a pair whose cosine |g| / sqrt(a b) exceeded it (0: while it rotated
                           at all); default 1e-2 for FP32, 0 for FP64 */
  int sort_pairs;       /* 0/1, default 1: order each pair's new columns by norm */
  int precondition;     /* 0/1, FP32 handles only, default 1: sort theta's columns by norm,
                           factor their FP64 Gram matrix G = R^H R (Cholesky) and run the
                           Jacobi on R^H, whose columns start nearly orthogonal, with the left
                           vectors recovered as theta Y / S (about half the sweeps on saturated
                           Haar bonds, and no right-vector accumulation).  FP64 handles ignore
                           it: the Gram matrix would square the condition number and cost the
                           relative accuracy of the FP64 path. */
  int streams;          /* 1 or 2, default 2: with 2, a batch of at least 64 bond updates is
                           split into two halves, each run end to end (theta, preconditioning,
                           Jacobi sweeps, finalize, write-back) on its own HIP stream (the
                           second one is the library's own, default priority); each half
                           sweeps until its own gates have converged, so one half's work
                           fills the GPU while the other's launches drain.  The call returns
                           once both streams have drained.  Results are the same bit for
                           bit as with 1. */
  int block_cols;       /* 16 (default) or 32, FP32 handles only: columns per Jacobi block.
                           A round pairs blocks of this width; 32-column blocks take fewer
                           sweeps and move half the bytes per sweep, with a 64 x 64 inner
                           problem per pair.  Results differ from 16 in the rounding only. */
  int graphs;           /* 0/1, default 1: each Jacobi sweep (its rounds and convergence check)
                           runs as one launch of a captured HIP graph, instantiated once per
                           batch shape and cached in the handle.  Either way the sweeps are
                           device-driven: the next sweep is queued before the host reads the
                           previous sweep's count of unconverged SVDs, and its launches return
                           at once when that count was zero.  Results are the same bit for bit
                           with 0. */
} ptebd_svd_params;

/* Read (get) or replace (set) the SVD controls of a handle.  set validates every field
 * (EINVAL, nothing changed).  Both return EINVAL on a NULL pointer. */
int ptebd_get_svd_params(ptebd_mps_t h, ptebd_svd_params* out);
/* Replace the controls (validated first; on EINVAL nothing changes). */
int ptebd_set_svd_params(ptebd_mps_t h, const ptebd_svd_params* params);

/*
 * Apply one circuit layer (one step of Algorithm 1) to states of the batch.
 *   n_gates      number of gates (>= 0);
 *   state_idx    [n_gates] state of each gate, or NULL when the handle holds one state;
 *   bonds        [n_gates] left site q of each gate, 0 <= q <= N-2;
 *   gates        [n_gates * 32] doubles: 16 complex128 per gate (see conventions);
 *   chi_max      bond-dimension bound chi, in [1, the state's chi_cap]; or 0: every gate
 *                is bounded by its own state's chi_cap (states of different caps, one launch);
 *   cutoff       >= 0: singular values sigma <= cutoff * sigma_1 are always dropped
 *                (their weight counts in eps_i); on the FP32 path the cutoff is at least
 *                PTEBD_FP32_CUTOFF_FLOOR;
 *   ptsu_steps   g >= 0 PtSU steps run when some gate of the layer had r > chi_max;
 *   flags        0 or an OR of PTEBD_FLAG_NO_STABILIZE and one of PTEBD_FLAG_RELATIVE_EPS,
 *                PTEBD_FLAG_COMPLEMENT_EPS (both eps flags: EINVAL);
 *   stats        optional per-layer statistics (see ptebd_layer_stats).
 * The gates of one state must act on disjoint sites (else EOVERLAP).  As in Algorithm 1,
 * the layer counts as compressed for a state when some gate of that state had r > chi_max
 * ("if chi~ > chi"); only then are that state's new Schmidt values multiplied by nu_i and
 * the PtSU steps run (IPMC, Sec. III.E).  On a layer that needed no compression every
 * nu_i is 1 and Lambda[q+1] is the kept singular values as they are.  The call enqueues
 * the layer on the handle's stream and returns after it has completed (the new bond
 * dimensions are read back to size the next layer).
 * Errors: EINVAL, EOVERLAP, ENOMEM, EDEVICE, ENONFINITE, EANNIHILATED; warning WNOCONV.
 * The gate layer and each PtSU half-step after it are batches that commit as a whole: the
 * host checks every gate's ENONFINITE / EANNIHILATED flag before anything of the state is
 * written, so a batch that fails leaves Gamma, Lambda, the bond dimensions and the norm and
 * fidelity estimates as they were before it (an error in the layer leaves the state as it
 * was before the call; one in a PtSU half-step leaves the layer and the earlier half-steps
 * applied).  EINVAL and EOVERLAP are found before any device work.
 */
int ptebd_apply_layer(ptebd_mps_t h, int n_gates, const int32_t* state_idx,
                      const int32_t* bonds, const double* gates, int chi_max, double cutoff,
                      int ptsu_steps, int flags, ptebd_layer_stats* stats);

/* Restore the canonical form of state s: the Canonicalize step of Algorithm 1, done before
 * measuring or sampling.  tSU steps (as in ptebd_ptsu: identity gate skipped, cutoff
 * only, nu = 1) sweep from both ends to the middle bond m = (N-2)/2 -- the pairs (0,1),
 * (1,2), .. up to m and (N-2,N-1), (N-3,N-2), .. down to m, two per batch -- then one tSU at
 * m, then sweeps from the middle back out to both ends; then the normalization
 * Lambda[i] /= n on the inner bonds and Gamma[q] *= n on the inner sites, n the norm
 * (n^2 = sum Lambda[1]^2 once canonical).
 * Afterwards the state has unit norm and satisfies the canonical conditions of Eq.
 * (l_r_cano); bond dimensions can only shrink (values <= cutoff * sigma_1 are dropped; the
 * FP32 floor applies).  norm_out (may be NULL) receives n.  The 2N-3 bond updates run in
 * about N sequential batches: the cost is sequential in N, unlike a layer.  The norm and
 * fidelity estimates are left unchanged.  Its SVDs use one inner Jacobi sweep per pair
 * whatever ptebd_set_svd_params set (each step is a batch of one or two SVDs, whose rounds
 * are latency-bound); the outer convergence test is the handle's.
 * Errors: EINVAL, ENOMEM, EDEVICE, ENONFINITE, EANNIHILATED; warning WNOCONV.  Each batch
 * of tSU steps commits as a whole (see ptebd_apply_layer); after an error the state holds the
 * batches done so far, which change its gauge but not the wavefunction beyond the cutoff. */
int ptebd_canonicalize(ptebd_mps_t h, int s, double cutoff, double* norm_out);

/* Perfect sampling of n_samples bit strings from state s, which must be in canonical form
 * (call ptebd_canonicalize first; on any other state the draws do not follow |Psi|^2).
 * Site by site, for every sample at once: with the prefix vector v (v = (1) at site 0) and
 * the right-isometric B[q] = Gamma[q] Lambda[q+1], w_p = v B[q]_p (p = 0, 1),
 * p_p = |w_p|^2, bit q = (u < p_0 / (p_0 + p_1)) ? 0 : 1, v = w_bit / sqrt(p_bit) (the method
 * of Ferris and Vidal that Algorithm 1 cites for sampling).  The products run on MFMA in the
 * handle's precision; p_0, p_1 and the decision are FP64.
 *   uniforms  [n_samples * N] caller-owned doubles in [0, 1): uniforms[i * N + q] decides bit
 *             q of sample i (the random numbers are an input, so runs are reproducible);
 *   bits      [n_samples * N] caller-owned output, 0 or 1, same layout.
 * Errors: EINVAL (n_samples < 0, NULL buffers, a uniform outside [0, 1)), ENOMEM, EDEVICE,
 * ENONFINITE (a conditional probability vanished: the state was not canonical). */
int ptebd_sample(ptebd_mps_t h, int s, int n_samples, const double* uniforms, uint8_t* bits);

/* Run g parallel trivial-simple-update (PtSU) steps on state s, the canonical-form recovery
 * of Sec. III.D (Theorem 4: N/2 steps restore the exact canonical form for even N): each step
 * is a tSU on all pairs (0,1),(2,3),..., then on (1,2),(3,4),...; a tSU is the TEBD procedure
 * of Sec. II.C with the identity gate skipped (the shortcut noted in Sec. III.D), cutoff only
 * (no chi bound), nu = 1.  It leaves the state unchanged up to rounding and the cutoff.
 * steps >= 0, cutoff in [0, 1).  Errors: EINVAL, ENOMEM, EDEVICE, ENONFINITE, EANNIHILATED;
 * warning WNOCONV.  Each half-step commits as a whole (see ptebd_apply_layer). */
int ptebd_ptsu(ptebd_mps_t h, int s, int steps, double cutoff);

/* Exact norm n = sqrt(<Psi|Psi>) of state s (the quantity whose decay Sec. III.C.1 studies)
 * in FP64, by the left-to-right transfer sweep of the quantum-map recursion Eq. (recu) with
 * no projector inserted.  The cost is sequential in N (O(N chi^3)).  out: one double.
 * Errors: EINVAL (bad handle or state, NULL out), ENOMEM, EDEVICE. */
int ptebd_norm(ptebd_mps_t h, int s, double* out);

/* Exact overlap <Psi_a|Psi_b> in FP64, the quantity in the fidelities of Eq. (F_2) and
 * Eq. (F), by a transfer sweep over both chains.  The states may live in different handles
 * (of the same device), differ in precision and bond dimensions, but must have the same
 * number of sites.  Everything runs on ha's stream after hb's pending work has completed.
 * re, im: one double each.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ptebd_overlap(ptebd_mps_t ha, int sa, ptebd_mps_t hb, int sb, double* re, double* im);

/* <Z_q> / <Psi|Psi> for every site q of state s (out: N doubles), from FP64 left and right
 * environments (the L and R partial contractions of Eqs. (llid)-(rrid), without assuming
 * they are identities): the "measurements" step of Algorithm 1, exact for any state, so it
 * needs no Canonicalize first.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ptebd_expect_z(ptebd_mps_t h, int s, double* out);

/* Distance to the canonical form, Eq. (dist_to_cano), of state s scaled to norm 1
 * (every inner Lambda multiplied by n^(-1/(N-1))). */
int ptebd_canon_distance(ptebd_mps_t h, int s, double* out);

/* n*_upper = prod of every nu_i applied to state s since create/import (Eq. (n_up) of
 * Theorem 3).  out: one double.  Errors: EINVAL. */
int ptebd_norm_estimate(ptebd_mps_t h, int s, double* out);

/* Fidelity estimate: the product over every applied truncation since create/import of
 * (1 - eps_i), eps_i the local error of Theorem 1 (on a normalized canonical input the
 * fidelity of one bond's truncation is 1 - eps_i).  The paper defines no fidelity estimator
 * for a whole pTEBD run; this is the product of the per-bond values.  Under the complement
 * reading eps_i also absorbs the deviation of a non-normalized bond from unit weight, so the
 * product is then a diagnostic, not a fidelity.  out: one double.  Errors: EINVAL. */
int ptebd_fidelity_estimate(ptebd_mps_t h, int s, double* out);

/* Bond dimensions chi_0..chi_N of state s into out[0..N] (cap >= N+1). */
int ptebd_bond_dims(ptebd_mps_t h, int s, int32_t* out, int cap);

/* Lambda[bond] of state s into out (cap doubles); *len receives chi_bond. */
int ptebd_get_lambda(ptebd_mps_t h, int s, int bond, double* out, int cap, int* len);

/*
 * Export state s: gamma receives the concatenation over q of Gamma[q] in C order
 * (a, s, m) as complex128 (gamma_cap counts doubles, >= 2 * sum_q 2 chi_q chi_{q+1});
 * lambda receives the concatenation of Lambda[0..N] (lambda_cap >= sum_i chi_i).
 */
int ptebd_export(ptebd_mps_t h, int s, double* gamma, size_t gamma_cap, double* lambda,
                 size_t lambda_cap);

/* Export only Gamma[q] of state s (C order (a, s, m), complex128, gamma_cap doubles
 * >= 4 chi_q chi_{q+1}); *dims_out (optional, 2 ints) receives chi_q, chi_{q+1}. */
int ptebd_export_site(ptebd_mps_t h, int s, int q, double* gamma, size_t gamma_cap,
                      int32_t* dims_out);

/* Import state s from host data in the export format; dims = chi_0..chi_N
 * (chi_0 = chi_N = 1, every chi_i <= chi_cap).  Resets the nu / eps products to 1. */
int ptebd_import(ptebd_mps_t h, int s, const int32_t* dims, const double* gamma,
                 const double* lambda);

/*
 * Build the two-site wavefunction of a gate at q of state s on the device (the
 * contraction of Sec. II.C, with the gate applied; gate may be NULL for the identity)
 * and copy it to out as a complex128 row-major (2 chi_q) x (2 chi_{q+2}) matrix with
 * rows (a, s') and columns (t', c).  For kernel-level parity checks.
 */
int ptebd_debug_theta(ptebd_mps_t h, int s, int q, const double* gate, double* out);

/*
 * Batched truncated-SVD primitive on the device (the Jacobi SVD used by apply_layer):
 * for each of `batch` complex128 row-major m x n matrices a[b], compute the singular
 * values (descending, min(m,n) of them) and the left / right singular vectors:
 *   s  [batch * kmin] doubles,
 *   u  [batch * m * kmin * 2] doubles, row-major m x kmin complex (may be NULL),
 *   vh [batch * kmin * n * 2] doubles, row-major kmin x n complex (may be NULL),
 * with kmin = min(m, n) <= 1024.  sweeps (optional, [batch]) receives the sweeps used.
 * precision as in ptebd_mps_create.  Runs on hip_stream and returns when done.
 */
int ptebd_svd_batched(int precision, int batch, int m, int n, const double* a, double* s,
                      double* u, double* vh, int32_t* sweeps, int max_sweeps,
                      double tol_factor, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the batched SVD of ptebd_svd_batched, with the same
 * arguments, results and errors, that allocates nothing.  Every device buffer it needs (work
 * and rotation matrices, descriptors, per-matrix outputs, input and output staging) lies in
 * one fixed array of PTEBD_NOALLOC_SCRATCH_BYTES per device, which the library holds until the
 * process ends; the host arrays are the caller's and are copied directly.  The need grows
 * with batch * (16 m n + 16 min(m,n) (m + n) + e min(m,n) max(m,n) + e min(m,n)^2) bytes
 * (e = 16 for FP64, 8 for FP32) plus small per-matrix outputs; a batch that does not fit is
 * rejected with EINVAL (the message gives the bytes it would need) before any device work.
 * Example: one 512 x 512 matrix needs about 20 MiB in FP64 and 16 MiB in FP32.  All calls on
 * one device share its array: calls that overlap in time on one device race (serialize them).
 * Each call writes everything it reads first, so no state carries over between calls.
 */
#define PTEBD_NOALLOC_SCRATCH_BYTES (32u << 20)
int ptebd_svd_batched_noalloc(int precision, int batch, int m, int n, const double* a,
                              double* s, double* u, double* vh, int32_t* sweeps, int max_sweeps,
                              double tol_factor, void* hip_stream);

/* ------------------------------------------------------------------ kernel timing
 * When profiling is on, every hot-path kernel launch of the handle is bracketed by HIP
 * events on the handle's stream, and per kernel class the library accumulates the device
 * time, the number of launches and the algorithmic flops and bytes of those launches:
 *   THETA      32 chi_q chi_{q+1} chi_{q+2} (+ 128 chi_q chi_{q+2} for the gate mix) flops;
 *              reads both Gammas, writes theta (complex elements of the precision).
 *   JACOBI     one block-Jacobi round; per 16+16-column pair: 6144 R flops for the three
 *              16x16 complex Gram tiles over R rows, plus 8192 (R + C) flops when the pair
 *              is rotated (32x32 complex update of W's and V's 32 columns); bytes: the 32
 *              columns of W read once, and those of W and V read and written when rotated.
 *   FINALIZE   column norms: reads W (R C complex elements); no MFMA flops counted.
 *   WRITEBACK  reads the k kept columns, writes both Gammas (2 k (chi_q + chi_{q+2})
 *              complex elements each way).
 * When a batch runs as two halves on two streams (ptebd_svd_params.streams), a class's time
 * is the union of its intervals on both streams, each half's launch counting as half a
 * launch, so that time and launches stand for the work over all gates.
 * ptebd_set_profiling(h, 1) enables and resets; ptebd_get_kernel_stats reads a class. */
#define PTEBD_KERNEL_THETA 0
#define PTEBD_KERNEL_JACOBI 1
#define PTEBD_KERNEL_FINALIZE 2
#define PTEBD_KERNEL_WRITEBACK 3
#define PTEBD_KERNEL_SAMPLE 4   /* ptebd_sample: one launch per site */
#define PTEBD_KERNEL_PRECOND 5  /* FP32 preconditioning: column sort, FP64 Gram, Cholesky,
                                   X = R^H, and the recovery of the singular vectors */
#define PTEBD_KERNEL_COUNT 6

typedef struct {
  double total_ms;   /* summed event-measured duration of the launches */
  int64_t launches;  /* number of launches */
  double flops;      /* algorithmic flops of those launches */
  double bytes;      /* algorithmic HBM bytes of those launches */
} ptebd_kernel_stats;

/* enable != 0: start timing the handle's kernels (every class reset to zero); 0: stop.
 * Waits for the handle's stream first.  Errors: EINVAL (bad handle), EDEVICE. */
int ptebd_set_profiling(ptebd_mps_t h, int enable);
/* The accumulated timing of kernel class `kind` (PTEBD_KERNEL_*) since profiling was enabled;
 * waits for the handle's stream first.  Errors: EINVAL (bad handle, class or NULL out). */
int ptebd_get_kernel_stats(ptebd_mps_t h, int kind, ptebd_kernel_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* PTEBD_H */
