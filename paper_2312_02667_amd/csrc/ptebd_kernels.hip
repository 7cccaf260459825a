// HIP kernels of one pTEBD layer on gfx950 (theta_kernel, the two-site wavefunction, is in
// ptebd_theta.hip):
//   jacobi_*         -- batched one-sided block Jacobi SVD (Hestenes), MFMA Gram and
//                       column updates, FP64 inner rotations
//   finalize_kernel  -- singular values, sort, truncation and discarded weight (Sec. III.B,
//                       Theorem 1), norm stabilization nu (Sec. III.C.2, Eq. (lren))
//   writeback_kernel -- Vidal regauge with Lambda^{-1} (Sec. II.C) and the new Lambda
//                       (times nu on compressed layers) into the state arena
#include <type_traits>

#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

// ---------------------------------------------------------------- Jacobi
// V = I (C x C), per-gate convergence state cleared.
template <class T>
__global__ void jacobi_init_kernel(const GateDesc* __restrict__ descs, LayerOut out) {
  const int g = blockIdx.y;
  const GateDesc* d = descs + g;
  const int C = d->C;
  const gptr<cplx<T>> v = as_global((cplx<T>*)d->v);
  const size_t total = v != nullptr ? (size_t)C * C : 0;  // no V: right vectors not kept
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t col = e / C, row = e % C;
    cplx<T> z = czero<T>();
    if (row == col) z.re = T(1);
    gstore<T>(v + e, z);
  }
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < 2 * out.nslot; i += blockDim.x)
      out.work[(size_t)g * 2 * out.nslot + i] = 0u;
    for (int b = threadIdx.x; b < out.nbmax; b += blockDim.x)
      out.rstart[(size_t)g * out.nbmax + b] = out.triangular ? out.block_cols * b : 0;
    if (threadIdx.x == 0) {
      out.conv[g] = 0;
      out.sweeps[g] = 0;
      out.offbits[g] = 0u;
      if (g == 0) {
        out.counters[0] = 0;
        out.counters[1] = 0;
        out.counters[2] = 0;
      }
    }
  }
}

// One round of the block Jacobi sweep: every workgroup takes one pair (I, J) of 16-column
// blocks of one gate's W, forms the 32x32 Gram matrix G = W_IJ^H W_IJ on MFMA, records the
// largest relative off-diagonal |G_ij| / sqrt(G_ii G_jj), runs cyclic Jacobi sweeps on G
// (rotation angles computed in FP64; G and the accumulated rotation Q held in the path's
// precision T) and applies Q to the 32 columns of W and, when the descriptor has one, of V
// on MFMA.  Pairs of one round are disjoint, so no two workgroups of a gate touch the same
// column.
//
// Both complex products (the Gram tiles and W_IJ Q) take three real MFMA products per
// complex one instead of four (Re = P1 -+ P2, Im = P3 - P1 +- P2 with P3 the product of the
// sums): a quarter fewer MFMAs, for an error bound of the same order (normwise, a few units
// of the roundoff of T times the norms of the two factors).
//
// LDS: G and Q (2 x 32 rows of 48 (FP32) or 33 (FP64) complex T), both rotated in place, and
// Re + Im of the permuted Q; the cross-wave reduction of the Gram tiles and the permuted copy
// of Q used by the column update alias G and Q.
//
// Occupancy: the kernel is bound by the latency of its phases, so it is built for at least
// five waves per SIMD in FP32 (at most 96 registers, no spills) and three in FP64 (at most
// 168).
template <class T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 5 : 3) void jacobi_round_kernel(const GateDesc* __restrict__ descs,
                                                           int round, int nbp, LayerOut out,
                                                           double tol_scale, int inner_sweeps,
                                                           double inner_repeat, int sort_pairs,
                                                           int prev_slot) {
  // the previous sweep left no gate of the batch unconverged (a sweep queued ahead of the
  // host's convergence check): nothing to do
  if (prev_slot >= 0 && out.counters[prev_slot] == 0) return;
  const int g = blockIdx.y;
  if (out.conv[g]) return;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const int nb = (C + 15) >> 4;
  // Each gate follows its own tournament of nbg players (its block count, made even): the
  // launch covers the batch's largest, and a gate sits out the rounds and pairs beyond its
  // own, so its sequence of rotations does not depend on what it is batched with.
  const int nbg = max(2, nb + (nb & 1));
  (void)nbp;
  if (round >= nbg - 1 || (int)blockIdx.x >= nbg / 2) return;
  const int I = rr_player(blockIdx.x, round, nbg);
  const int J = rr_player(nbg - 1 - blockIdx.x, round, nbg);
  const bool dummy_i = I >= nb, dummy_j = J >= nb;
  if (dummy_i && dummy_j) return;
  // A pair with the padding player is skipped, except when the matrix has a single block:
  // then that block is diagonalized on its own against an empty second half.
  if ((dummy_i || dummy_j) && nb > 1) return;
  const int cI = dummy_i ? 0 : I * 16, cJ = dummy_j ? 0 : J * 16;
  const int nI = dummy_i ? 0 : min(16, C - cI), nJ = dummy_j ? 0 : min(16, C - cJ);
  // Rows below both blocks' first possibly nonzero row are exact zeros in all 32 columns
  // (on the mixed path W starts lower triangular): every wave skips its 16-row chunks there,
  // keeping the chunk-to-wave assignment (and so every sum) as without the skip.
  int32_t* __restrict__ rsg = out.rstart + (size_t)g * out.nbmax;
  const int rs0 = min(dummy_i ? R : rsg[I], dummy_j ? R : rsg[J]);
  const int c0 = rs0 >> 4;  // first chunk that can hold a nonzero row
  const gptr<cplx<T>> __restrict__ W = as_global((cplx<T>*)d->w);
  const gptr<cplx<T>> __restrict__ V = as_global((cplx<T>*)d->v);

  // FP32 rows padded to 48 entries (384 B): the two 16-lane row groups of each half-wave of
  // an 8-byte LDS access then fall on disjoint banks (a 33-entry row puts them 8 B apart).
  // FP64 entries are 16 B, whose accesses are conflict-free at 33.
  constexpr int kLd = sizeof(T) == 4 ? 48 : 33;
  __shared__ cplx<T> G[32][kLd];
  __shared__ cplx<T> Q[32][kLd];
  __shared__ __align__(16) T P[16][4];  // one round's rotations: c, Re s, Im s, (unused)
  __shared__ T Qs[32][kLd];  // Re + Im of the permuted Q
  __shared__ double red[4];
  __shared__ unsigned int rmax_bits;  // largest |g|^2 / (a b) rotated in this inner sweep
  __shared__ int pos[32];
  // reduction scratch: wave w < 2 owns region w (3 tiles of 16 x 16), aliasing G / Q
  cplx<T>* part0 = &G[0][0];
  cplx<T>* part1 = &Q[0][0];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar loop bounds
  const int wstart = 16 * (c0 + (((wave - c0) % 4) + 4) % 4);  // this wave's first chunk
  const int col = lane & 15, grp = lane >> 4;
  typedef typename Mfma<T>::v4 V4;

  // ---- Gram matrix: rows split over the four waves in chunks of 16, next chunk prefetched.
  // Every load is unconditional (out-of-range rows read row 0, a column beyond nI / nJ
  // reads column cI or cJ) and masked where it is used, so no load sits under a divergent
  // branch and the next chunk's loads stay in flight during this chunk's MFMAs.
  // Three real products per complex tile entry: for sum conj(x) y with x = p + iq,
  // y = u + iv: P1 = sum p u, P2 = sum q v, P3 = sum (p - q)(u + v);
  // Re = P1 + P2, Im = P3 - P1 + P2.  Tiles: 0 = I^H I, 1 = I^H J, 2 = J^H J.
  V4 acc[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);
  const bool okI = col < nI, okJ = col < nJ;
  const uint32_t baseI = (uint32_t)(cI + (okI ? col : 0)) * (uint32_t)R;
  const uint32_t baseJ = (uint32_t)(cJ + (okJ ? col : 0)) * (uint32_t)R;
  // Rows rbase .. rbase + 3 of the lane's I and J columns.  For even R (every theta: its
  // row count is twice a bond dimension) they are two 16-byte-aligned pairs, an
  // out-of-range pair reading rows 0 and 1; for odd R (a general batched SVD) one load per
  // row, an out-of-range row reading row 0.  Rows at or beyond R are masked where used.
  // The two loops are separate instantiations, chosen once per workgroup.
  auto gram_rows = [&](auto even_tag) {
    constexpr bool kEven = decltype(even_tag)::value;
    cplx<T> xi[4], xj[4], ni[4], nj[4];
    auto load_chunk = [&](int r0, cplx<T>(&a)[4], cplx<T>(&b)[4]) {
      const int rbase = r0 + grp * 4;
      if constexpr (kEven) {
        const uint32_t o0 = rbase < R ? rbase : 0, o1 = rbase + 2 < R ? rbase + 2 : 0;
        gload_pair<T>(W, baseI + o0, a[0], a[1]);
        gload_pair<T>(W, baseI + o1, a[2], a[3]);
        gload_pair<T>(W, baseJ + o0, b[0], b[1]);
        gload_pair<T>(W, baseJ + o1, b[2], b[3]);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t o = rbase + t < R ? rbase + t : 0;
          a[t] = gload<T>(gat<T>(W, baseI + o));
          b[t] = gload<T>(gat<T>(W, baseJ + o));
        }
      }
    };
    auto gram_chunk = [&](int r0, const cplx<T>(&a)[4], const cplx<T>(&b)[4]) {
      const int rbase = r0 + grp * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool vr = rbase + t < R;
        const cplx<T> x = cmask<T>(a[t], okI && vr), y = cmask<T>(b[t], okJ && vr);
        const T xd = x.re - x.im, xs = x.re + x.im, yd = y.re - y.im, ys = y.re + y.im;
        acc[0][0] = Mfma<T>::op(x.re, x.re, acc[0][0]);
        acc[0][1] = Mfma<T>::op(x.im, x.im, acc[0][1]);
        acc[0][2] = Mfma<T>::op(xd, xs, acc[0][2]);
        acc[1][0] = Mfma<T>::op(x.re, y.re, acc[1][0]);
        acc[1][1] = Mfma<T>::op(x.im, y.im, acc[1][1]);
        acc[1][2] = Mfma<T>::op(xd, ys, acc[1][2]);
        acc[2][0] = Mfma<T>::op(y.re, y.re, acc[2][0]);
        acc[2][1] = Mfma<T>::op(y.im, y.im, acc[2][1]);
        acc[2][2] = Mfma<T>::op(yd, ys, acc[2][2]);
      }
    };
    // The prefetch is unconditional (a wave's last chunk re-reads itself, from cache): a
    // load under a branch would make the compiler wait for it before this chunk's products.
    int r0 = wstart;
    if (r0 < R) load_chunk(r0, xi, xj);
    for (; r0 < R; r0 += 64) {
      load_chunk(r0 + 64 < R ? r0 + 64 : r0, ni, nj);
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
      gram_chunk(r0, xi, xj);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        xi[t] = ni[t];
        xj[t] = nj[t];
      }
    }
  };
  if (R & 1)
    gram_rows(std::false_type{});
  else
    gram_rows(std::true_type{});
  for (int tl = 0; tl < 3; ++tl)
    for (int v = 0; v < 4; ++v) {
      const T p1 = acc[tl][0][v], p2 = acc[tl][1][v];
      acc[tl][0][v] = p1 + p2;
      acc[tl][1][v] = acc[tl][2][v] - p1 + p2;
    }
  if (wave < 2) {
    cplx<T>* p = wave == 0 ? part0 : part1;
    for (int tl = 0; tl < 3; ++tl)
      for (int v = 0; v < 4; ++v) {
        cplx<T> z;
        z.re = acc[tl][0][v];
        z.im = acc[tl][1][v];
        p[(tl * 16 + Mfma<T>::row(lane, v)) * 16 + col] = z;
      }
  }
  __syncthreads();
  if (wave >= 2) {
    cplx<T>* p = wave == 2 ? part0 : part1;
    for (int tl = 0; tl < 3; ++tl)
      for (int v = 0; v < 4; ++v) {
        cplx<T>& z = p[(tl * 16 + Mfma<T>::row(lane, v)) * 16 + col];
        z.re += acc[tl][0][v];
        z.im += acc[tl][1][v];
      }
  }
  __syncthreads();
  cplx<T> gv[4];
  for (int k = 0; k < 4; ++k) {
    const int e = tid + 256 * k;
    const int i = e >> 5, j = e & 31;
    int tl, ii, jj;
    bool conj = false;
    if (i < 16 && j < 16) {
      tl = 0; ii = i; jj = j;
    } else if (i < 16) {
      tl = 1; ii = i; jj = j - 16;
    } else if (j >= 16) {
      tl = 2; ii = i - 16; jj = j - 16;
    } else {
      tl = 1; ii = j; jj = i - 16; conj = true;
    }
    const cplx<T> a = part0[(tl * 16 + ii) * 16 + jj], b = part1[(tl * 16 + ii) * 16 + jj];
    gv[k].re = a.re + b.re;
    gv[k].im = i == j ? T(0) : (conj ? -(a.im + b.im) : (a.im + b.im));  // real diagonal
  }
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    const int e = tid + 256 * k;
    G[e >> 5][e & 31] = gv[k];
  }
  __syncthreads();

  // ---- convergence measure of this pair.  Pairs with a numerically zero column (norm
  // below 16 u times its partner's, u the unit roundoff of T) do not count: their cosine is
  // rounding noise left by an earlier cancellation, and rotating the residue against its
  // partner sweep after sweep only shrinks it towards underflow.  tiny = (16 u)^2.  The
  // inner rotations below do not use this test, so a pair the measure counts is always
  // rotated.
  constexpr double tiny = sizeof(T) == 4 ? 9.094947017729282e-13 : 3.1554436208840472e-30;
  // FP32: the largest squared cosine |G_ij|^2 / (G_ii G_jj), one square root at the end
  // (the entries are FP32 values, so their squares and products are normal FP64 numbers).
  // FP64 entries may be small enough for their squares to underflow: scaled hypot there.
  constexpr bool kSq = sizeof(T) == 4;
  double mx = 0.0;
  for (int e = tid; e < 1024; e += 256) {
    const int i = e >> 5, j = e & 31;
    if (i < j) {
      const double di = (double)G[i][i].re, dj = (double)G[j][j].re;
      if (fmin(di, dj) > tiny * fmax(di, dj)) {
        const double gr = (double)G[i][j].re, gi = (double)G[i][j].im;
        if constexpr (kSq)
          mx = fmax(mx, (gr * gr + gi * gi) / (di * dj));
        else
          mx = fmax(mx, hypot(gr, gi) / sqrt(di * dj));
      }
    }
  }
  mx = wave_max(mx);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  if constexpr (kSq) mx = sqrt(mx);
  // Orthogonality threshold tol_factor u sqrt(R), but never below 8 u: the cosine of a
  // short column pair cannot be computed more accurately than a few units of u.
  constexpr double kUnit = sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  const double thr = fmax(tol_scale * sqrt((double)R), 8.0 * kUnit);
  const bool rotate = mx > thr;
  if (tid == 0) {
    atomicMax(&out.offbits[g], __float_as_uint((float)mx));
    uint32_t* wk = out.work + ((size_t)g * out.nslot + blockIdx.x) * 2;  // this pair's slot
    const uint32_t rows = (uint32_t)(R - 16 * c0 > 0 ? R - 16 * c0 : 0);
    atomicAdd(wk, rows);
    if (rotate) {
      atomicAdd(wk + 1, rows + (V != nullptr ? (uint32_t)C : 0u));
      // both blocks' columns are now combinations of the two: nonzero from rs0 on
      if (!dummy_i) rsg[I] = rs0;
      if (!dummy_j) rsg[J] = rs0;
    }
  }
  if (!rotate) return;  // uniform: every thread read the same red[]

  // ---- cyclic Jacobi on the 32x32 Hermitian G; Q accumulates the rotations.  The
  // threshold sits well below the outer tolerance so that a pair the outer test calls
  // unconverged is always rotated.
  const double inner_tol = 0.125 * thr;
  for (int e = tid; e < 1024; e += 256) {
    const int i = e >> 5, j = e & 31;
    cplx<T> z;
    z.re = (i == j) ? T(1) : T(0);
    z.im = T(0);
    Q[i][j] = z;
  }
  // G and Q are stored in tournament-slot order: in every round slot k is paired with slot
  // 31 - k, and thread (ia, ib) owns rows (ia, 31 - ia) and columns (ib, 31 - ib).  The
  // circle method moves every player except player 0 down one slot per round, so each
  // thread writes its rotated 2x2 block straight to the next round's slots; 16 consecutive
  // lanes then always touch 16 consecutive complex entries, which keeps the interleaved LDS
  // accesses free of bank conflicts.  After the 31 rounds of a sweep the slots are back in
  // natural order.  The update is in place: every thread holds its block in registers
  // across the barrier that publishes the round's rotations, so no thread overwrites an
  // entry another has still to read, and G and Q need one copy each (half the LDS of a
  // double-buffered scheme, twice the workgroups per CU).  Thread (k, k) holds exactly the
  // 2x2 block of pair k (G_pp, G_pq, G_qq), computes that pair's rotation in FP64 from its
  // registers and hands it to every thread through LDS; the 16 such threads are spread over
  // the four waves.
  const int ia = tid >> 4, ib = tid & 15;
  const int ra = ia, rb2 = 31 - ia, ca0 = ib, cb2 = 31 - ib;
  auto next_slot = [](int s) { return s >= 2 ? s - 1 : (s == 1 ? 31 : 0); };
  const int nra = next_slot(ra), nrb = next_slot(rb2), nca = next_slot(ca0), ncb = next_slot(cb2);
  const bool diag_owner = ia == ib;
  // Another inner sweep follows only while the last one still rotated a pair whose cosine
  // exceeded inner_repeat: cyclic Jacobi converges quadratically, so after a sweep whose
  // largest rotated cosine was c the remaining ones are of order c^2.
  // One round's rotation as one 16-byte LDS access (two for FP64) each way.
  auto put_rot = [&](int k, double c, double sr, double si) {
    if constexpr (sizeof(T) == 4) {
      vf4 w;
      w.x = (float)c;
      w.y = (float)sr;
      w.z = (float)si;
      w.w = 0.f;
      *reinterpret_cast<vf4*>(&P[k][0]) = w;
    } else {
      vd2 w0, w1;
      w0.x = c;
      w0.y = sr;
      w1.x = si;
      w1.y = 0.0;
      *reinterpret_cast<vd2*>(&P[k][0]) = w0;
      *reinterpret_cast<vd2*>(&P[k][2]) = w1;
    }
  };
  auto get_rot = [&](int k, T& c, T& sr, T& si) {
    if constexpr (sizeof(T) == 4) {
      const vf4 r = *reinterpret_cast<const vf4*>(&P[k][0]);
      c = r.x;
      sr = r.y;
      si = r.z;
    } else {
      const vd2 r0 = *reinterpret_cast<const vd2*>(&P[k][0]);
      const vd2 r1 = *reinterpret_cast<const vd2*>(&P[k][2]);
      c = r0.x;
      sr = r0.y;
      si = r1.x;
    }
  };
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    __syncthreads();
    if (tid == 0) rmax_bits = 0u;
    __syncthreads();
    // the largest squared cosine this thread's pair rotated in the sweep, published once
    float my_rmax = 0.f;
    for (int rd = 0; rd < 31; ++rd) {
      const cplx<T> b00 = G[ra][ca0], b01 = G[ra][cb2], b10 = G[rb2][ca0], b11 = G[rb2][cb2];
      const cplx<T> q00 = Q[ra][ca0], q01 = Q[ra][cb2], q10 = Q[rb2][ca0], q11 = Q[rb2][cb2];
      if (diag_owner) {
        double c, sr, si;
        const double gpp = (double)b00.re, gqq = (double)b11.re;
        const double gr = (double)b01.re, gi = (double)b01.im;
        if (jacobi_rotation<sizeof(T) == 4 ? 1 : 2>(gpp, gqq, gr, gi, inner_tol, c, sr, si)) {
          // squared cosine |g|^2 / (a b) of the rotated pair (a threshold test only: the
          // hardware reciprocal estimate is accurate enough)
          const double ab = gpp * gqq;
          const float cos2 =
              ab > 0.0 ? (float)((gr * gr + gi * gi) * __builtin_amdgcn_rcp(ab)) : 3.0e38f;
          my_rmax = fmaxf(my_rmax, cos2);
        }
        put_rot(ia, c, sr, si);
      }
      __syncthreads();
      T ca, sar, sai, cb, sbr, sbi;
      get_rot(ia, ca, sar, sai);
      get_rot(ib, cb, sbr, sbi);
      // X = B J_b: X[:,0] = c_b B[:,0] - conj(s_b) B[:,1];  X[:,1] = s_b B[:,0] + c_b B[:,1]
      cplx<T> x00, x01, x10, x11;
      x00.re = cb * b00.re - (sbr * b01.re + sbi * b01.im);
      x00.im = cb * b00.im - (sbr * b01.im - sbi * b01.re);
      x10.re = cb * b10.re - (sbr * b11.re + sbi * b11.im);
      x10.im = cb * b10.im - (sbr * b11.im - sbi * b11.re);
      x01.re = (sbr * b00.re - sbi * b00.im) + cb * b01.re;
      x01.im = (sbr * b00.im + sbi * b00.re) + cb * b01.im;
      x11.re = (sbr * b10.re - sbi * b10.im) + cb * b11.re;
      x11.im = (sbr * b10.im + sbi * b10.re) + cb * b11.im;
      // B' = J_a^H X: row0 = c_a X[0,:] - s_a X[1,:];  row1 = conj(s_a) X[0,:] + c_a X[1,:]
      cplx<T> n00, n01, n10, n11;
      n00.re = ca * x00.re - (sar * x10.re - sai * x10.im);
      n00.im = ca * x00.im - (sar * x10.im + sai * x10.re);
      n01.re = ca * x01.re - (sar * x11.re - sai * x11.im);
      n01.im = ca * x01.im - (sar * x11.im + sai * x11.re);
      n10.re = (sar * x00.re + sai * x00.im) + ca * x10.re;
      n10.im = (sar * x00.im - sai * x00.re) + ca * x10.im;
      n11.re = (sar * x01.re + sai * x01.im) + ca * x11.re;
      n11.im = (sar * x01.im - sai * x01.re) + ca * x11.im;
      // Q' = Q J_b (rows ra, rb2 of Q are a plain partition; its columns follow the slots)
      cplx<T> m00, m01, m10, m11;
      m00.re = cb * q00.re - (sbr * q01.re + sbi * q01.im);
      m00.im = cb * q00.im - (sbr * q01.im - sbi * q01.re);
      m10.re = cb * q10.re - (sbr * q11.re + sbi * q11.im);
      m10.im = cb * q10.im - (sbr * q11.im - sbi * q11.re);
      m01.re = (sbr * q00.re - sbi * q00.im) + cb * q01.re;
      m01.im = (sbr * q00.im + sbi * q00.re) + cb * q01.im;
      m11.re = (sbr * q10.re - sbi * q10.im) + cb * q11.re;
      m11.im = (sbr * q10.im + sbi * q10.re) + cb * q11.im;
      G[nra][nca] = n00;
      G[nra][ncb] = n01;
      G[nrb][nca] = n10;
      G[nrb][ncb] = n11;
      Q[ra][nca] = m00;
      Q[ra][ncb] = m01;
      Q[rb2][nca] = m10;
      Q[rb2][ncb] = m11;
      __syncthreads();
    }
    if (diag_owner && my_rmax > 0.f) atomicMax(&rmax_bits, __float_as_uint(my_rmax));
    __syncthreads();
    const float rmax2 = __uint_as_float(rmax_bits);
    if (!(rmax2 > (float)(inner_repeat * inner_repeat)) || rmax_bits == 0u) break;
  }
  __syncthreads();
  // Optional ordering of the pair's 32 new columns by norm: the 16 largest go to the
  // lower-numbered block (full blocks only), so that sweeps drift the columns towards
  // descending order.
  if (tid < 32) {
    int p = tid;
    if (sort_pairs && nI == 16 && nJ == 16) {
      const T dj = G[tid][tid].re;
      int rank = 0;
      for (int i = 0; i < 32; ++i) {
        const T di = G[i][i].re;
        rank += (di > dj || (di == dj && i < tid)) ? 1 : 0;
      }
      p = (I < J) ? rank : (rank < 16 ? rank + 16 : rank - 16);
    }
    pos[tid] = p;
  }
  __syncthreads();
  // column-permuted copy of Q in G, which is no longer needed, and Re + Im of its entries
  // for the three-product complex multiply of the update
  cplx<T>(*Qp)[kLd] = G;
  for (int e = tid; e < 1024; e += 256) {
    const int i = e >> 5, j = e & 31;
    const cplx<T> z = Q[i][j];
    Qp[i][pos[j]] = z;
    Qs[i][pos[j]] = z.re + z.im;
  }
  __syncthreads();

  // ---- column update [W_I W_J] <- [W_I W_J] Q and [V_I V_J] <- [V_I V_J] Q on MFMA,
  // next 16-row chunk prefetched
  const int npass = V != nullptr ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const gptr<cplx<T>> __restrict__ M = pass == 0 ? W : V;
    const int rows = pass == 0 ? R : C;
    // element offsets of this lane's 8 k-slice columns; a column beyond nI / nJ reads
    // column cI (masked where used), an out-of-range row reads row 0
    uint32_t coff[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int kk = ks * 4 + grp;
      const bool ok = kk < 16 ? kk < nI : kk - 16 < nJ;
      coff[ks] = (uint32_t)(ok ? (kk < 16 ? cI + kk : cJ + kk - 16) : cI) * (uint32_t)rows;
    }
    cplx<T> av[8], an[8];
    auto load_rows = [&](int rbase, cplx<T>(&dst)[8]) {
      const int r = rbase + col;
      const uint32_t rr = r < rows ? r : 0;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) dst[ks] = gload<T>(gat<T>(M, coff[ks] + rr));
    };
    int rb = pass == 0 ? wstart : wave * 16;  // V (pass 1) is not triangular
    if (rb < rows) load_rows(rb, av);
    for (; rb < rows; rb += 64) {
      load_rows(rb + 64 < rows ? rb + 64 : rb, an);  // unconditional, as in the Gram loop
      __builtin_amdgcn_sched_barrier(0);
      const bool rok = rb + col < rows;
      // Three real products per complex one: with a = x + iy, b = u + iv,
      // P1 = x u, P2 = y v, P3 = (x + y)(u + v); Re ab = P1 - P2, Im ab = P3 - P1 - P2.
      // The two 16-column output tiles one after the other (three accumulators live).
      for (int jt = 0; jt < 2; ++jt) {
        V4 o[3];
        for (int j = 0; j < 3; ++j)
          for (int v = 0; v < 4; ++v) o[j][v] = T(0);
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const int kk = ks * 4 + grp;
          const bool ok = rok && (kk < 16 ? kk < nI : kk - 16 < nJ);
          const cplx<T> a = cmask<T>(av[ks], ok);
          const cplx<T> b = Qp[kk][jt * 16 + col];
          const T bs = Qs[kk][jt * 16 + col];
          o[0] = Mfma<T>::op(a.re, b.re, o[0]);
          o[1] = Mfma<T>::op(a.im, b.im, o[1]);
          o[2] = Mfma<T>::op(a.re + a.im, bs, o[2]);
        }
        T ore[4], oim[4];
        for (int v = 0; v < 4; ++v) {
          ore[v] = o[0][v] - o[1][v];
          oim[v] = o[2][v] - o[0][v] - o[1][v];
        }
        const int jj = jt * 16 + col;
        const bool okc = jt == 0 ? jj < nI : jj - 16 < nJ;
        const int cidx = jt == 0 ? cI + jj : cJ + jj - 16;
        if (!okc) continue;
        const gptr<cplx<T>> __restrict__ dst = gat<T>(M, (uint32_t)cidx * (uint32_t)rows);
        if constexpr (sizeof(T) == 4) {
          // f32 layout: this lane's four values are rows rb + 4*grp + 0..3 of one column
          const int r4 = rb + 4 * grp;
          if (r4 + 3 < rows) {
            vf4 u, w;
            u.x = ore[0]; u.y = oim[0]; u.z = ore[1]; u.w = oim[1];
            w.x = ore[2]; w.y = oim[2]; w.z = ore[3]; w.w = oim[3];
            *reinterpret_cast<gptr<vf4>>(dst + r4) = u;
            *reinterpret_cast<gptr<vf4>>(dst + r4 + 2) = w;
            continue;
          }
        }
        for (int v = 0; v < 4; ++v) {
          const int rr = rb + Mfma<T>::row(lane, v);
          if (rr < rows) {
            cplx<T> z;
            z.re = ore[v];
            z.im = oim[v];
            gstore<T>(dst + rr, z);
          }
        }
      }
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) av[ks] = an[ks];
    }
  }
}

// After a sweep: a gate whose largest relative off-diagonal stayed at or below
// max(tol_factor sqrt(R), 8) u is converged.  counters[sweep & 1] counts the others.
__global__ void sweep_check_kernel(const GateDesc* __restrict__ descs, int n_gates, int sweep,
                                   double tol_factor, double unit_roundoff, LayerOut out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) out.counters[(sweep + 1) & 1] = 0;
  if (g >= n_gates) return;
  if (out.conv[g]) return;
  out.sweeps[g] += 1;
  const float off = __uint_as_float(out.offbits[g]);
  out.offbits[g] = 0u;
  const double tol = fmax(tol_factor * sqrt((double)descs[g].R), 8.0) * unit_roundoff;
  if ((double)off <= tol)
    out.conv[g] = 1;
  else
    atomicAdd(&out.counters[sweep & 1], 1);
}

// ---------------------------------------------------------------- finalize
// sigma_j = |W_j| (FP64), descending sort with the column permutation, r = #{sigma >
// cutoff sigma_1}, k = min(chi_max, r), eps = sum_{j >= k} sigma_j^2, nu = (1-eps)^(-1/2),
// and the batch's error word.  The state is not written here: whether nu multiplies
// Lambda[q+1] depends on the whole layer (Algorithm 1 compresses only when some bond
// exceeded chi), and a batch with an error must leave the state as it was, so the
// write-back sets Lambda[q+1] once every gate has been finalized and checked.
template <class T>
__global__ __launch_bounds__(256) void finalize_kernel(const GateDesc* __restrict__ descs,
                                                       double cutoff, LayerOut out) {
  const int g = blockIdx.x;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const gptr<const cplx<T>> __restrict__ W = as_global((const cplx<T>*)d->w);
  __shared__ double key[1024];
  __shared__ int idx[1024];
  __shared__ double red_d[4];
  __shared__ double red_w[4];
  __shared__ int red_i[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int P = 1;
  while (P < C) P <<= 1;
  for (int j = wave; j < C; j += 4) {
    double s = 0.0;
    for (int r = lane; r < R; r += 64) {
      const cplx<T> x = gload<T>(W + ((size_t)j * R + r));
      s += (double)x.re * (double)x.re + (double)x.im * (double)x.im;
    }
    s = wave_sum(s);
    if (lane == 0) {
      key[j] = s;
      idx[j] = j;
    }
  }
  for (int j = C + tid; j < P; j += 256) {
    key[j] = -1.0;
    idx[j] = j;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < (P >> 1); i += 256) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool descending = (lo & size) == 0;
        const double klo = key[lo], khi = key[hi];
        const bool sw = descending ? (klo < khi) : (klo > khi);
        if (sw) {
          key[lo] = khi;
          key[hi] = klo;
          const int t = idx[lo];
          idx[lo] = idx[hi];
          idx[hi] = t;
        }
      }
      __syncthreads();
    }
  }
  const double s1 = sqrt(fmax(key[0], 0.0));
  int cnt = 0;
  for (int j = tid; j < C; j += 256)
    if (sqrt(fmax(key[j], 0.0)) > cutoff * s1) ++cnt;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (lane == 0) red_i[wave] = cnt;
  __syncthreads();
  const int r = red_i[0] + red_i[1] + red_i[2] + red_i[3];
  const int chi_max = d->chi_max;
  int k = chi_max > 0 ? min(chi_max, r) : r;
  if (k < 1) k = 1;
  double part = 0.0, whole = 0.0;
  for (int j = tid; j < C; j += 256) {
    const double v = fmax(key[j], 0.0);
    whole += v;
    if (j >= k) part += v;
  }
  part = wave_sum(part);
  whole = wave_sum(whole);
  if (lane == 0) {
    red_d[wave] = part;
    red_w[wave] = whole;
  }
  __syncthreads();
  const double discarded = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
  const double total = (red_w[0] + red_w[1]) + (red_w[2] + red_w[3]);
  double eps = discarded;
  if (d->eps_mode == 1) eps = discarded / total;
  if (d->eps_mode == 2) eps = 1.0 - (total - discarded);
  const double nu = d->stabilize ? 1.0 / sqrt(1.0 - eps) : 1.0;
  for (int j = tid; j < C; j += 256) {
    out.sig[(size_t)g * out.cmax + j] = sqrt(fmax(key[j], 0.0));
    out.perm[(size_t)g * out.cmax + j] = idx[j];
  }
  if (tid == 0) {
    out.k[g] = k;
    out.r[g] = r;
    out.eps[g] = eps;
    out.nu[g] = nu;
    int err = 0;
    if (!(s1 > 0.0) || (d->stabilize && !(eps < 1.0))) err |= 1;
    if (!isfinite(s1) || !isfinite(eps) || !isfinite(nu)) err |= 2;
    if (err) atomicOr(&out.counters[2], err);
  }
}

// ---------------------------------------------------------------- write-back
// Gamma[q][a, s', j] = X[(s',a), j] / Lambda[q]_a and
// Gamma[q+1][j, t', c] = Ydag[j, (t',c)] / Lambda[q+2]_c for the k kept columns, where
// X = W/sigma, Ydag = V^H (W = theta) or X = V, Ydag = (W/sigma)^H (W = theta^H).
// blockIdx.z = 0 writes Gamma[q], 1 writes Gamma[q+1] (LDS-transposed 32x32 tiles).  Block
// (0, g, 0) also writes Lambda[q+1] = nu sigma[:k] where apply[g] != 0 (the state's layer
// was compressed: norm stabilization, Sec. III.C.2, Eq. (lren)), else sigma[:k].  This is
// the only kernel of a batch that writes the state: the host launches it once the batch's
// error word is clear, so a batch either commits every gate or leaves the state untouched.
template <class T>
__global__ __launch_bounds__(256) void writeback_kernel(const GateDesc* __restrict__ descs,
                                                        const int32_t* __restrict__ apply,
                                                        LayerOut out) {
  const int g = blockIdx.y;
  const GateDesc* d = descs + g;
  const int k = out.k[g];
  const int cl = d->cl, cr = d->cr, R = d->R, C = d->C, transposed = d->transposed;
  const double* __restrict__ sig = out.sig + (size_t)g * out.cmax;
  const int* __restrict__ perm = out.perm + (size_t)g * out.cmax;
  const gptr<const cplx<T>> __restrict__ W = as_global((const cplx<T>*)d->w);
  const gptr<const cplx<T>> __restrict__ V = as_global((const cplx<T>*)d->v);
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && blockIdx.z == 0 && d->lam_m != nullptr) {
    const double nu = (apply != nullptr && apply[g] != 0) ? out.nu[g] : 1.0;
    const gptr<double> lam_m = as_global(d->lam_m);
    for (int j = tid; j < k; j += 256) lam_m[j] = nu * sig[j];
  }
  if (blockIdx.z == 0) {
    const gptr<const cplx<T>> __restrict__ L = transposed ? V : W;
    const int ldl = transposed ? C : R;
    const bool divsig = !transposed;
    const gptr<const double> __restrict__ lam_l = as_global(d->lam_l);
    const gptr<cplx<T>> __restrict__ gout = as_global((cplx<T>*)d->gq);
    const size_t total = 2 * (size_t)cl * k;
    for (size_t e = (size_t)blockIdx.x * 256 + tid; e < total; e += (size_t)gridDim.x * 256) {
      const int a = (int)(e % cl);
      const size_t rest = e / cl;
      const int j = (int)(rest % k), sp = (int)(rest / k);
      const cplx<T> x = gload<T>(L + ((size_t)perm[j] * ldl + sp * cl + a));
      double sc = 1.0 / lam_l[a];
      if (divsig) sc /= sig[j];
      cplx<T> z;
      z.re = (T)((double)x.re * sc);
      z.im = (T)((double)x.im * sc);
      gstore<T>(gout + ((size_t)sp * cl * k + (size_t)j * cl + a), z);
    }
  } else {
    __shared__ cplx<T> tile[32][33];
    const gptr<const cplx<T>> __restrict__ Rs = transposed ? W : V;
    const int ldr = transposed ? R : C;
    const bool divsig = transposed;
    const gptr<const double> __restrict__ lam_r = as_global(d->lam_r);
    const gptr<cplx<T>> __restrict__ gout = as_global((cplx<T>*)d->gq1);
    const int tj = (k + 31) >> 5, tc = (cr + 31) >> 5;
    const int ntiles = 2 * tj * tc;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
      const int tp = t / (tj * tc), rem = t % (tj * tc);
      const int j0 = (rem / tc) * 32, c0 = (rem % tc) * 32;
      for (int i = 0; i < 4; ++i) {
        const int e = tid + 256 * i;
        const int jj = e >> 5, cc = e & 31;
        const int j = j0 + jj, c = c0 + cc;
        if (j < k && c < cr) {
          const cplx<T> x = gload<T>(Rs + ((size_t)perm[j] * ldr + tp * cr + c));
          double sc = 1.0 / lam_r[c];
          if (divsig) sc /= sig[j];
          cplx<T> z;
          z.re = (T)((double)x.re * sc);
          z.im = (T)(-(double)x.im * sc);
          tile[jj][cc] = z;
        }
      }
      __syncthreads();
      for (int i = 0; i < 4; ++i) {
        const int e = tid + 256 * i;
        const int jj = e & 31, cc = e >> 5;
        const int j = j0 + jj, c = c0 + cc;
        if (j < k && c < cr) gstore<T>(gout + ((size_t)tp * k * cr + (size_t)c * k + j), tile[jj][cc]);
      }
      __syncthreads();
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <class T>
void launch_jacobi_init(const GateDesc* d_desc, int n_gates, int max_c, const LayerOut& out,
                        hipStream_t stream) {
  if (n_gates <= 0) return;
  int blocks = (int)(((size_t)max_c * max_c + 255) / 256);
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(jacobi_init_kernel<T>, dim3(blocks, n_gates), dim3(256), 0, stream, d_desc,
                     out);
}

template <class T>
void launch_jacobi_round(const GateDesc* d_desc, int n_gates, int round, int nbp,
                         const LayerOut& out, double tol_scale, int inner_sweeps,
                         double inner_repeat, int sort_pairs, int prev_slot,
                         hipStream_t stream) {
  if (n_gates <= 0 || nbp < 2) return;
  hipLaunchKernelGGL(jacobi_round_kernel<T>, dim3(nbp / 2, n_gates), dim3(256), 0, stream,
                     d_desc, round, nbp, out, tol_scale, inner_sweeps, inner_repeat, sort_pairs,
                     prev_slot);
}

void launch_sweep_check(const GateDesc* d_desc, int n_gates, int sweep, double tol_factor,
                        double unit_roundoff, const LayerOut& out, hipStream_t stream) {
  const int blocks = (n_gates + 255) / 256;
  hipLaunchKernelGGL(sweep_check_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream,
                     d_desc, n_gates, sweep, tol_factor, unit_roundoff, out);
}

template <class T>
void launch_finalize(const GateDesc* d_desc, int n_gates, double cutoff, const LayerOut& out,
                     hipStream_t stream) {
  if (n_gates <= 0) return;
  hipLaunchKernelGGL(finalize_kernel<T>, dim3(n_gates), dim3(256), 0, stream, d_desc, cutoff,
                     out);
}

template <class T>
void launch_writeback(const GateDesc* d_desc, int n_gates, const int32_t* d_apply,
                      const LayerOut& out, hipStream_t stream) {
  if (n_gates <= 0) return;
  hipLaunchKernelGGL(writeback_kernel<T>, dim3(64, n_gates, 2), dim3(256), 0, stream, d_desc,
                     d_apply, out);
}

template void launch_jacobi_init<float>(const GateDesc*, int, int, const LayerOut&, hipStream_t);
template void launch_jacobi_init<double>(const GateDesc*, int, int, const LayerOut&, hipStream_t);
template void launch_jacobi_round<float>(const GateDesc*, int, int, int, const LayerOut&, double,
                                         int, double, int, int, hipStream_t);
template void launch_jacobi_round<double>(const GateDesc*, int, int, int, const LayerOut&, double,
                                          int, double, int, int, hipStream_t);
template void launch_finalize<float>(const GateDesc*, int, double, const LayerOut&, hipStream_t);
template void launch_finalize<double>(const GateDesc*, int, double, const LayerOut&, hipStream_t);
template void launch_writeback<float>(const GateDesc*, int, const int32_t*, const LayerOut&,
                                      hipStream_t);
template void launch_writeback<double>(const GateDesc*, int, const int32_t*, const LayerOut&,
                                       hipStream_t);

}  // namespace ptebd
