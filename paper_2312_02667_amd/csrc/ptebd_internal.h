// Internal declarations shared by the host runtime and the HIP kernels of libptebd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ptebd {

// Complex number of precision T, stored interleaved (re, im).
template <class T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

// Device descriptor of one bond update (one gate, or one tSU) of a layer.
//
// Device layout of Gamma[q] (shape chi_q x 2 x chi_{q+1}): two planes s = 0, 1, each a
// column-major chi_q x chi_{q+1} matrix (row a fastest); element (a, s, m) at
// s * chi_q * chi_{q+1} + m * chi_q + a, complex of the handle's precision.
//
// The two-site wavefunction theta is the (2 chi_q) x (2 chi_{q+2}) matrix with row index
// s' * chi_q + a and column index t' * chi_{q+2} + c.  The SVD works on the column-major
// work matrix W with R rows and C <= R columns: W = theta when 2 chi_{q+2} <= 2 chi_q,
// else W = theta^H (transposed = 1).  V is the C x C matrix of accumulated rotations.
struct GateDesc {
  int32_t cl, cm, cr;      // chi_q, chi_{q+1}, chi_{q+2}
  int32_t R, C;            // rows / columns of W
  int32_t transposed;      // 1: W = theta^H
  int32_t has_gate;        // 0: identity gate (tSU), the gate mix is skipped
  int32_t chi_max;         // truncation bound; <= 0: keep every sigma above the cutoff
  int32_t stabilize;       // 1: nu = (1 - eps)^(-1/2); 0: nu = 1
  int32_t eps_mode;        // 0: discarded sigma^2; 1: that / sum sigma^2; 2: 1 - kept sigma^2
  void* gq;                // Gamma[q] slot
  void* gq1;               // Gamma[q+1] slot
  const double* lam_l;     // Lambda[q]   (cl)
  double* lam_m;           // Lambda[q+1] (written: k values)
  const double* lam_r;     // Lambda[q+2] (cr)
  void* w;                 // R x C work matrix (complex T)
  void* v;                 // C x C rotation matrix (complex T), or nullptr: not accumulated
  const double* gate;      // 16 complex128, U[(s' t'), (s t)] row-major
  void* gram;              // preconditioned FP32 path: C x C complex FP64 (G, then R, then
                           // the right vectors as complex FP32), else nullptr
  void* left;              // preconditioned FP32 path: R x C complex FP32 (U S), else nullptr
};

// Per-gate side data of the preconditioned SVD (ptebd_precond.hip).
struct PrecondOut {
  int32_t* ps;       // column order of W by descending norm, n_gates * cmax
  double* gmax;      // largest column norm^2 of W, per gate
  int32_t cmax;
};

// Per-gate outputs of a layer's SVD + truncation, device arrays of length n_gates
// (sig / perm: n_gates * cmax).
struct LayerOut {
  double* sig;       // singular values, descending
  int32_t* perm;     // column of W holding the j-th largest
  int32_t* k;        // kept dimension
  int32_t* r;        // rank above the cutoff
  double* eps;       // discarded weight
  double* nu;        // stabilization factor
  int32_t* sweeps;   // Jacobi sweeps
  int32_t* conv;     // converged flag
  uint32_t* offbits; // max relative off-diagonal of the sweep (float bits)
  int32_t* counters; // [0..1] unconverged counts (double-buffered by sweep parity),
                     // [2] error flags: bit0 annihilated, bit1 non-finite
  uint32_t* work;    // executed Jacobi rows per (gate, pair slot): work[2 (g nslot + x)] sums
                     // the rows over which Gram matrices were formed, work[2 (g nslot + x) + 1]
                     // the rows rotated (W's, plus V's when accumulated).  One workgroup owns a
                     // slot in a launch, so these counts never contend (a handful of shared
                     // counters for every workgroup of a launch serialize in one L2 channel
                     // and cost a large share of the Gram phase).
  int32_t nslot;     // pair slots per gate: half the even block count of cmax
  int32_t* rstart;   // per gate and 16-column block: the first row of W that can be nonzero
                     // (n x nbmax).  A pair skips the 16-row chunks below the smaller of its
                     // blocks' starts (exact zeros in both); a rotated pair gives both blocks
                     // that start.
  int32_t nbmax;     // 16-column blocks of cmax
  int32_t triangular;  // 1: the Jacobi starts from a lower-triangular W (block b starts at
                       // row block_cols * b), 0: every block starts at row 0
  int32_t block_cols;  // columns per Jacobi block: 16 (jacobi_round_kernel) or 32
                       // (jacobi64_round_kernel, FP32 only); rstart is indexed by block
  int32_t cmax;
};

// Arguments of one site of perfect sampling (ptebd_sample.hip).
struct SampleSite {
  const void* gamma;         // Gamma[q] slot (complex T), planes cl x cm
  const double* lam_r;       // Lambda[q+1] (cm)
  int32_t cl, cm;            // chi_q, chi_{q+1}
  int32_t first;             // 1 at site 0 (prefix vector (1))
  int32_t n_samples;
  int32_t ldw;               // row stride of the W buffers (>= 2 * max chi)
  const void* w_in;          // previous site's rows (complex T), n_samples x ldw
  void* w_out;               // this site's rows
  const int32_t* sel_in;     // previous plane per sample
  const double* scale_in;    // previous 1 / sqrt(p_sel) per sample
  int32_t* sel_out;
  double* scale_out;
  const double* u;           // uniforms of this site, sample i at u[i * ustride]
  int32_t ustride;
  uint8_t* bits;             // bit of this site, sample i at bits[i * bstride]
  int32_t bstride;
  int32_t* err;              // bit0: a vanishing conditional probability
  double* part;              // per sample and column tile: partial p_0, p_1 (n_samples x
                             // ntiles x 2)
  int32_t ntiles;            // column tiles of 32 over the two planes: ceil(2 cm / 32)
};

// Kernel launchers (ptebd_kernels.hip).  All are asynchronous on `stream`.
template <class T>
void launch_theta(const GateDesc* d_desc, int n_gates, int max_tiles, hipStream_t stream);
// One round of a sweep; prev_slot >= 0: every workgroup returns at once when
// out.counters[prev_slot] (the previous sweep's count of unconverged gates) is zero.
template <class T>
void launch_jacobi_round(const GateDesc* d_desc, int n_gates, int round, int nbp,
                         const LayerOut& out, double tol_scale, int inner_sweeps,
                         double inner_repeat, int sort_pairs, int prev_slot,
                         hipStream_t stream);
// The same round with 32-column blocks (FP32 only; ptebd_jacobi64.hip); nbp counts 32-column
// blocks.
void launch_jacobi_round64(const GateDesc* d_desc, int n_gates, int round, int nbp,
                           const LayerOut& out, double tol_scale, int inner_sweeps,
                           double inner_repeat, int sort_pairs, int prev_slot,
                           hipStream_t stream);
void launch_sweep_check(const GateDesc* d_desc, int n_gates, int sweep, double tol_factor,
                        double unit_roundoff, const LayerOut& out, hipStream_t stream);
template <class T>
void launch_jacobi_init(const GateDesc* d_desc, int n_gates, int max_c, const LayerOut& out,
                        hipStream_t stream);
template <class T>
void launch_finalize(const GateDesc* d_desc, int n_gates, double cutoff, const LayerOut& out,
                     hipStream_t stream);
// Gamma[q], Gamma[q+1] and Lambda[q+1] of every gate: Lambda[q+1] = nu sigma[:k] for the
// gates with d_apply[g] != 0 (d_apply may be nullptr: none), sigma[:k] for the others.
template <class T>
void launch_writeback(const GateDesc* d_desc, int n_gates, const int32_t* d_apply,
                      const LayerOut& out, hipStream_t stream);

// Preconditioned SVD of the FP32 path (ptebd_precond.hip).  d_desc: the theta descriptors
// (w = theta, gram, left set); d_jdesc: the Jacobi descriptors (w = X, v = nullptr, R = C,
// gram as in d_desc).
void launch_colsort(const GateDesc* d_desc, int n_gates, const PrecondOut& po,
                    hipStream_t stream);
void launch_gram64(const GateDesc* d_desc, int n_gates, int max_c, const PrecondOut& po,
                   hipStream_t stream);
void launch_cholesky(const GateDesc* d_desc, int n_gates, int max_c, const PrecondOut& po,
                     hipStream_t stream);
void launch_xinit(const GateDesc* d_jdesc, int n_gates, int max_c, hipStream_t stream);
void launch_recover(const GateDesc* d_desc, const GateDesc* d_jdesc, int n_gates, int max_r,
                    int max_c, const PrecondOut& po, const LayerOut& out, hipStream_t stream);

// Sampling and normalization kernels (ptebd_sample.hip).
template <class T>
void launch_sample_site(const SampleSite& a, hipStream_t stream);
template <class T>
void launch_scale_state(void* gamma_base, size_t slot_elems, double* lam_base, int lam_stride,
                        const int32_t* d_dims, int n_sites, int max_elems, double nrm,
                        hipStream_t stream);

// Query kernels (ptebd_queries.hip), all FP64.
// Column-major complex GEMM C = alpha * op(A) * op(B) + beta * C, op: 'N', 'T' or 'C'.
void launch_zgemm(char opa, char opb, int m, int n, int k, double alpha_re,
                  const cplx<double>* a, int lda, const cplx<double>* b, int ldb,
                  double beta_re, cplx<double>* c, int ldc, hipStream_t stream);
// A_s = diag(lam) * Gamma_s for both planes, converted to FP64: out planes (cl x cm) each.
template <class T>
void launch_site_a(const void* gamma, const double* lam_left, const double* lam_right,
                   int cl, int cm, double scale_left, double scale_right, cplx<double>* out,
                   hipStream_t stream);
// out[0] = sum_ij |x_ij - delta_ij|^2 of an n x n matrix (canonical distance).
void launch_frob_minus_identity(const cplx<double>* x, int n, double* out, hipStream_t stream);
// out[0] += weight * Re sum_i conj(a_i) b_i (used by <Z>).
void launch_dot_conj(const cplx<double>* a, const cplx<double>* b, int count, double weight,
                     double* out_re, hipStream_t stream);
// x[0] = value (a 1 x 1 environment).
void launch_set_identity_scalar(cplx<double>* x, double value, hipStream_t stream);
// |0...0>: Gamma[q] = e_0 at the listed Gamma slots (byte offsets), Lambda = (1) at the
// listed Lambda slots (double offsets).
template <class T>
void launch_init_product(void* gamma_base, const size_t* d_gamma_offsets, int n_sites,
                         double* lam_base, const size_t* d_lam_offsets, int n_bonds,
                         hipStream_t stream);

// Host helpers of the runtime (ptebd_api.hip), shared with the allocation-free entry point.
// Sets the thread-local last error and returns code.
int report_error(int code, const char* msg);
// Bytes of the per-gate output block of a batch of n gates of at most cmax columns, and the
// block laid out at base (256-byte aligned pieces).
size_t layer_out_bytes(int n, int cmax);
LayerOut layer_out_at(void* base, int n, int cmax);
// The Jacobi sweeps of the batched SVD on descriptors already on the device (init kernel,
// rounds, a convergence check and one 4-byte read-back into h_counter per sweep).
template <class T>
int jacobi_sweeps(hipStream_t stream, const GateDesc* d_desc, int n, int max_c,
                  const LayerOut& lo, int precision, int max_sweeps, double tol_factor,
                  int inner_sweeps, double inner_repeat, int sort_pairs, int32_t* h_counter,
                  int* n_unconverged);

}  // namespace ptebd
