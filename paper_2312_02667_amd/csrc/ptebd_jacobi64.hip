// One round of the batched one-sided block Jacobi SVD with 32-column blocks (FP32 path).
//
// The same method as jacobi_round_kernel (ptebd_kernels.hip) with twice the block width:
// every workgroup (eight waves) takes one pair (I, J) of 32-column blocks of one gate's work
// matrix, forms the 64 x 64 Gram matrix G = [W_I W_J]^H [W_I W_J] on MFMA, records the
// largest relative off-diagonal, runs cyclic Jacobi sweeps on G (rotation angles in FP64; G
// and the accumulated rotation Q in FP32) and applies Q to the 64 columns of W and, when the
// descriptor has one, of the right-vector matrix V on MFMA.  A sweep
// over 16 blocks (C = 512) is 15 rounds of 8 pairs instead of 31 rounds of 16; every column
// pair is read once per round either way, so a sweep moves half the bytes of the 16-column
// kernel for the same MFMA work, and wider blocks take fewer sweeps to converge.
//
// Gram phase: the ten 16 x 16 upper tiles (a, b), a <= b, of the 4 x 4 tile grid of G are
// split over four tile groups {(0,0),(0,1),(1,1)}, {(2,2),(2,3),(3,3)}, {(0,2),(1,2)} and
// {(0,3),(1,3)} (16-column sub-blocks 0, 1 of W_I and 2, 3 of W_J); waves w and w + 4 form
// group w & 3 over the even and the odd 16-row chunks, and their partial tiles are summed in
// LDS.  Complex products take three real MFMA products (as in the 16-column kernel).
//
// Inner Jacobi: G and Q (64 x 65 complex FP32 each) in tournament-slot order, rotated in
// place.  Thread (ia, ib), ia < 32, ib < 16, owns rows (ia, 63 - ia) and the column pairs
// (ib, 63 - ib) and (ib + 16, 47 - ib); the owner of slot pair k's diagonal 2 x 2 block computes
// that pair's rotation in FP64.  63 rounds per inner sweep, two barriers per round.
//
// Column update: the eight waves split the 16-row chunks; per chunk a lane holds 16
// k-slices of the 64 input columns and the four 16-column output tiles are formed in turn.
//
// LDS: G and Q, about 67 KB: two workgroups (16 waves) per CU.
#include <type_traits>

#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

constexpr int kBs = 32;      // columns per block
constexpr int kN = 2 * kBs;  // columns per pair

__global__ __launch_bounds__(512, 4) void jacobi64_round_kernel(const GateDesc* __restrict__ descs,
                                                                int round, LayerOut out,
                                                                double tol_scale, int inner_sweeps,
                                                                double inner_repeat,
                                                                int sort_pairs, int prev_slot) {
  typedef float T;
  if (prev_slot >= 0 && out.counters[prev_slot] == 0) return;  // batch already converged
  const int g = blockIdx.y;
  if (out.conv[g]) return;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const int nb = (C + kBs - 1) / kBs;
  // each gate follows its own tournament of nbg players, as in the 16-column kernel
  const int nbg = max(2, nb + (nb & 1));
  if (round >= nbg - 1 || (int)blockIdx.x >= nbg / 2) return;
  const int I = rr_player(blockIdx.x, round, nbg);
  const int J = rr_player(nbg - 1 - blockIdx.x, round, nbg);
  const bool dummy_i = I >= nb, dummy_j = J >= nb;
  if (dummy_i && dummy_j) return;
  if ((dummy_i || dummy_j) && nb > 1) return;
  const int cI = dummy_i ? 0 : I * kBs, cJ = dummy_j ? 0 : J * kBs;
  const int nI = dummy_i ? 0 : min(kBs, C - cI), nJ = dummy_j ? 0 : min(kBs, C - cJ);
  int32_t* __restrict__ rsg = out.rstart + (size_t)g * out.nbmax;
  const int rs0 = min(dummy_i ? R : rsg[I], dummy_j ? R : rsg[J]);
  const int c0 = rs0 >> 4;
  const gptr<cplx<T>> __restrict__ W = as_global((cplx<T>*)d->w);

  __shared__ cplx<T> G[kN][kN + 1];
  __shared__ cplx<T> Q[kN][kN + 1];
  __shared__ __align__(16) T P[kBs][4];  // one round's rotations: c, Re s, Im s, (unused)
  __shared__ double red[8];
  __shared__ unsigned int rmax_bits;
  __shared__ int pos[kN];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, grp = lane >> 4;
  typedef Mfma<T>::v4 V4;

  // Local column lc (0..63) of the pair: W_I's column cI + lc for lc < 32, W_J's column
  // cJ + lc - 32 above; a column beyond nI / nJ reads the block's first column and is masked.
  auto col_ok = [&](int lc) { return lc < kBs ? lc < nI : lc - kBs < nJ; };
  auto col_off = [&](int lc) -> uint32_t {
    const int c = lc < kBs ? (lc < nI ? cI + lc : cI) : (lc - kBs < nJ ? cJ + lc - kBs : cJ);
    return (uint32_t)c * (uint32_t)R;
  };

  // ---- Gram matrix.  Tile group tg = wave & 3, row parity rh = wave >> 2; each group's tile
  // list and the 16-column sub-blocks it reads are compile-time constants.
  const int tg = wave & 3, rh = wave >> 2;
  auto gram_group = [&](auto tg_tag) {
    constexpr int TG = decltype(tg_tag)::value;
    // sub-blocks read (NSB of them) and tiles (NT of them) as (slot of a, slot of b)
    constexpr int NSB = TG < 2 ? 2 : 3;
    constexpr int NT = TG < 2 ? 3 : 2;
    constexpr int SB0 = TG == 1 ? 2 : 0, SB1 = TG == 1 ? 3 : 1, SB2 = TG == 3 ? 3 : 2;
    constexpr int TA[3] = {0, TG < 2 ? 0 : 1, 1};  // slots in the sub-block list
    constexpr int TB[3] = {TG < 2 ? 0 : 2, TG < 2 ? 1 : 2, 1};
    const int sbv[3] = {SB0, SB1, SB2};
    bool okc[NSB];
    uint32_t base[NSB];
#pragma unroll
    for (int q = 0; q < NSB; ++q) {
      const int lc = sbv[q] * 16 + col;
      okc[q] = col_ok(lc);
      base[q] = col_off(lc);
    }
    V4 acc[NT][3];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);
    // rows rbase .. rbase + 3 of the lane's columns (pairs of 16-byte loads for even R, one
    // load per row for odd R); out-of-range rows read row 0 and are masked where used
    const bool even = (R & 1) == 0;
    cplx<T> x[NSB][4], nx[NSB][4];
    auto load_chunk = [&](int r0, cplx<T>(&a)[NSB][4]) {
      const int rbase = r0 + grp * 4;
#pragma unroll
      for (int q = 0; q < NSB; ++q) {
        if (even) {
          const uint32_t o0 = rbase < R ? rbase : 0, o1 = rbase + 2 < R ? rbase + 2 : 0;
          gload_pair<T>(W, base[q] + o0, a[q][0], a[q][1]);
          gload_pair<T>(W, base[q] + o1, a[q][2], a[q][3]);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const uint32_t o = rbase + t < R ? rbase + t : 0;
            a[q][t] = gload<T>(gat<T>(W, base[q] + o));
          }
        }
      }
    };
    // this wave's chunks: c0 + rh, c0 + rh + 2, ... (16 rows each)
    int r0 = 16 * (c0 + rh);
    if (r0 < R) load_chunk(r0, x);
    for (; r0 < R; r0 += 32) {
      load_chunk(r0 + 32 < R ? r0 + 32 : r0, nx);
      __builtin_amdgcn_sched_barrier(0);
      const int rbase = r0 + grp * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool vr = rbase + t < R;
        cplx<T> y[NSB];
        T yd[NSB], ys[NSB];
#pragma unroll
        for (int q = 0; q < NSB; ++q) {
          y[q] = cmask<T>(x[q][t], okc[q] && vr);
          yd[q] = y[q].re - y[q].im;
          ys[q] = y[q].re + y[q].im;
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          acc[k][0] = Mfma<T>::op(y[TA[k]].re, y[TB[k]].re, acc[k][0]);
          acc[k][1] = Mfma<T>::op(y[TA[k]].im, y[TB[k]].im, acc[k][1]);
          acc[k][2] = Mfma<T>::op(yd[TA[k]], ys[TB[k]], acc[k][2]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < NSB; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) x[q][t] = nx[q][t];
    }
    // partial tiles: Re = P1 + P2, Im = P3 - P1 + P2, into the Q area (tile (a, b) of the
    // upper triangle at rows 16 a.., columns 16 b..); the even-row waves write, then the
    // odd-row waves add
#pragma unroll
    for (int k = 0; k < NT; ++k)
      for (int v = 0; v < 4; ++v) {
        const T p1 = acc[k][0][v], p2 = acc[k][1][v];
        acc[k][0][v] = p1 + p2;
        acc[k][1][v] = acc[k][2][v] - p1 + p2;
      }
    for (int half = 0; half < 2; ++half) {
      if (rh == half) {
#pragma unroll
        for (int k = 0; k < NT; ++k)
          for (int v = 0; v < 4; ++v) {
            cplx<T>& z = Q[sbv[TA[k]] * 16 + Mfma<T>::row(lane, v)][sbv[TB[k]] * 16 + col];
            if (half == 0) {
              z.re = acc[k][0][v];
              z.im = acc[k][1][v];
            } else {
              z.re += acc[k][0][v];
              z.im += acc[k][1][v];
            }
          }
      }
      __syncthreads();
    }
  };
  switch (tg) {
    case 0: gram_group(std::integral_constant<int, 0>{}); break;
    case 1: gram_group(std::integral_constant<int, 1>{}); break;
    case 2: gram_group(std::integral_constant<int, 2>{}); break;
    default: gram_group(std::integral_constant<int, 3>{}); break;
  }
  // full Hermitian G from the upper tiles (real diagonal)
  for (int e = tid; e < kN * kN; e += 512) {
    const int i = e >> 6, j = e & 63;
    const bool upper = (i >> 4) <= (j >> 4);
    cplx<T> z = upper ? Q[i][j] : Q[j][i];
    if (!upper) z.im = -z.im;
    if (i == j) z.im = T(0);
    G[i][j] = z;
  }
  __syncthreads();

  // ---- convergence measure (largest squared cosine of non-tiny column pairs)
  constexpr double tiny = 9.094947017729282e-13;  // (16 u)^2, u = 2^-24
  double mx = 0.0;
  for (int e = tid; e < kN * kN; e += 512) {
    const int i = e >> 6, j = e & 63;
    if (i < j) {
      const double di = (double)G[i][i].re, dj = (double)G[j][j].re;
      if (fmin(di, dj) > tiny * fmax(di, dj)) {
        const double gr = (double)G[i][j].re, gi = (double)G[i][j].im;
        mx = fmax(mx, (gr * gr + gi * gi) / (di * dj));
      }
    }
  }
  mx = wave_max(mx);
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  mx = red[0];
  for (int w = 1; w < 8; ++w) mx = fmax(mx, red[w]);
  mx = sqrt(mx);
  constexpr double kUnit = 5.9604644775390625e-08;
  const double thr = fmax(tol_scale * sqrt((double)R), 8.0 * kUnit);
  const bool rotate = mx > thr;
  if (tid == 0) {
    atomicMax(&out.offbits[g], __float_as_uint((float)mx));
    uint32_t* wk = out.work + ((size_t)g * out.nslot + blockIdx.x) * 2;
    const uint32_t rows = (uint32_t)(R - 16 * c0 > 0 ? R - 16 * c0 : 0);
    atomicAdd(wk, rows);
    if (rotate) {
      atomicAdd(wk + 1, rows + (d->v != nullptr ? (uint32_t)C : 0u));
      if (!dummy_i) rsg[I] = rs0;
      if (!dummy_j) rsg[J] = rs0;
    }
  }
  if (!rotate) return;  // uniform

  // ---- cyclic Jacobi on the 64 x 64 Hermitian G, Q accumulating the rotations
  const double inner_tol = 0.125 * thr;
  for (int e = tid; e < kN * kN; e += 512) {
    const int i = e >> 6, j = e & 63;
    cplx<T> z;
    z.re = (i == j) ? T(1) : T(0);
    z.im = T(0);
    Q[i][j] = z;
  }
  const int ia = tid >> 4, ib = tid & 15;
  const int ra = ia, rb = kN - 1 - ia;
  const int cA0 = ib, cA1 = kN - 1 - ib;            // column pair ib
  const int cB0 = ib + 16, cB1 = kN - 1 - 16 - ib;  // column pair ib + 16
  auto next_slot = [](int s) { return s >= 2 ? s - 1 : (s == 1 ? kN - 1 : 0); };
  const int nra = next_slot(ra), nrb = next_slot(rb);
  const int ncA0 = next_slot(cA0), ncA1 = next_slot(cA1), ncB0 = next_slot(cB0),
            ncB1 = next_slot(cB1);
  // the diagonal 2 x 2 block of slot pair ia lies in column pair A when ia == ib, B when
  // ia == ib + 16
  const bool ownA = ia == ib, ownB = ia == ib + 16;
  auto put_rot = [&](int k, double c, double sr, double si) {
    vf4 w;
    w.x = (float)c;
    w.y = (float)sr;
    w.z = (float)si;
    w.w = 0.f;
    *reinterpret_cast<vf4*>(&P[k][0]) = w;
  };
  auto get_rot = [&](int k, T& c, T& sr, T& si) {
    const vf4 r = *reinterpret_cast<const vf4*>(&P[k][0]);
    c = r.x;
    sr = r.y;
    si = r.z;
  };
  // B' = J_a^H B J_b for one 2 x 2 block (b00 b01; b10 b11), and Q' = Q J_b for its Q block
  auto rot_block = [](T ca, T sar, T sai, T cb, T sbr, T sbi, cplx<T>& b00, cplx<T>& b01,
                      cplx<T>& b10, cplx<T>& b11) {
    cplx<T> x00, x01, x10, x11;
    x00.re = cb * b00.re - (sbr * b01.re + sbi * b01.im);
    x00.im = cb * b00.im - (sbr * b01.im - sbi * b01.re);
    x10.re = cb * b10.re - (sbr * b11.re + sbi * b11.im);
    x10.im = cb * b10.im - (sbr * b11.im - sbi * b11.re);
    x01.re = (sbr * b00.re - sbi * b00.im) + cb * b01.re;
    x01.im = (sbr * b00.im + sbi * b00.re) + cb * b01.im;
    x11.re = (sbr * b10.re - sbi * b10.im) + cb * b11.re;
    x11.im = (sbr * b10.im + sbi * b10.re) + cb * b11.im;
    b00.re = ca * x00.re - (sar * x10.re - sai * x10.im);
    b00.im = ca * x00.im - (sar * x10.im + sai * x10.re);
    b01.re = ca * x01.re - (sar * x11.re - sai * x11.im);
    b01.im = ca * x01.im - (sar * x11.im + sai * x11.re);
    b10.re = (sar * x00.re + sai * x00.im) + ca * x10.re;
    b10.im = (sar * x00.im - sai * x00.re) + ca * x10.im;
    b11.re = (sar * x01.re + sai * x01.im) + ca * x11.re;
    b11.im = (sar * x01.im - sai * x01.re) + ca * x11.im;
  };
  auto rot_cols = [](T cb, T sbr, T sbi, cplx<T>& q00, cplx<T>& q01, cplx<T>& q10,
                     cplx<T>& q11) {
    cplx<T> m00, m01, m10, m11;
    m00.re = cb * q00.re - (sbr * q01.re + sbi * q01.im);
    m00.im = cb * q00.im - (sbr * q01.im - sbi * q01.re);
    m10.re = cb * q10.re - (sbr * q11.re + sbi * q11.im);
    m10.im = cb * q10.im - (sbr * q11.im - sbi * q11.re);
    m01.re = (sbr * q00.re - sbi * q00.im) + cb * q01.re;
    m01.im = (sbr * q00.im + sbi * q00.re) + cb * q01.im;
    m11.re = (sbr * q10.re - sbi * q10.im) + cb * q11.re;
    m11.im = (sbr * q10.im + sbi * q10.re) + cb * q11.im;
    q00 = m00;
    q01 = m01;
    q10 = m10;
    q11 = m11;
  };
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    __syncthreads();
    if (tid == 0) rmax_bits = 0u;
    __syncthreads();
    float my_rmax = 0.f;
    for (int rd = 0; rd < kN - 1; ++rd) {
      cplx<T> a00 = G[ra][cA0], a01 = G[ra][cA1], a10 = G[rb][cA0], a11 = G[rb][cA1];
      cplx<T> b00 = G[ra][cB0], b01 = G[ra][cB1], b10 = G[rb][cB0], b11 = G[rb][cB1];
      cplx<T> p00 = Q[ra][cA0], p01 = Q[ra][cA1], p10 = Q[rb][cA0], p11 = Q[rb][cA1];
      cplx<T> s00 = Q[ra][cB0], s01 = Q[ra][cB1], s10 = Q[rb][cB0], s11 = Q[rb][cB1];
      if (ownA || ownB) {
        double c, sr, si;
        const cplx<T> d00 = ownA ? a00 : b00, d01 = ownA ? a01 : b01, d11 = ownA ? a11 : b11;
        const double gpp = (double)d00.re, gqq = (double)d11.re;
        const double gr = (double)d01.re, gi = (double)d01.im;
        if (jacobi_rotation<1>(gpp, gqq, gr, gi, inner_tol, c, sr, si)) {
          const double ab = gpp * gqq;
          const float cos2 =
              ab > 0.0 ? (float)((gr * gr + gi * gi) * __builtin_amdgcn_rcp(ab)) : 3.0e38f;
          my_rmax = fmaxf(my_rmax, cos2);
        }
        put_rot(ia, c, sr, si);
      }
      __syncthreads();
      T ca, sar, sai, cb, sbr, sbi, cc, scr, sci;
      get_rot(ia, ca, sar, sai);
      get_rot(ib, cb, sbr, sbi);
      get_rot(ib + 16, cc, scr, sci);
      rot_block(ca, sar, sai, cb, sbr, sbi, a00, a01, a10, a11);
      rot_block(ca, sar, sai, cc, scr, sci, b00, b01, b10, b11);
      rot_cols(cb, sbr, sbi, p00, p01, p10, p11);
      rot_cols(cc, scr, sci, s00, s01, s10, s11);
      G[nra][ncA0] = a00;
      G[nra][ncA1] = a01;
      G[nrb][ncA0] = a10;
      G[nrb][ncA1] = a11;
      G[nra][ncB0] = b00;
      G[nra][ncB1] = b01;
      G[nrb][ncB0] = b10;
      G[nrb][ncB1] = b11;
      Q[ra][ncA0] = p00;
      Q[ra][ncA1] = p01;
      Q[rb][ncA0] = p10;
      Q[rb][ncA1] = p11;
      Q[ra][ncB0] = s00;
      Q[ra][ncB1] = s01;
      Q[rb][ncB0] = s10;
      Q[rb][ncB1] = s11;
      __syncthreads();
    }
    if ((ownA || ownB) && my_rmax > 0.f) atomicMax(&rmax_bits, __float_as_uint(my_rmax));
    __syncthreads();
    const float rmax2 = __uint_as_float(rmax_bits);
    if (!(rmax2 > (float)(inner_repeat * inner_repeat)) || rmax_bits == 0u) break;
  }
  __syncthreads();
  // order the pair's 64 new columns by norm: the 32 largest to the lower-numbered block
  if (tid < kN) {
    int p = tid;
    if (sort_pairs && nI == kBs && nJ == kBs) {
      const T dj = G[tid][tid].re;
      int rank = 0;
      for (int i = 0; i < kN; ++i) {
        const T di = G[i][i].re;
        rank += (di > dj || (di == dj && i < tid)) ? 1 : 0;
      }
      p = (I < J) ? rank : (rank < kBs ? rank + kBs : rank - kBs);
    }
    pos[tid] = p;
  }
  __syncthreads();
  // column-permuted Q into G's area, then Re + Im of its entries into Q's area
  cplx<T>(*Qp)[kN + 1] = G;
  for (int e = tid; e < kN * kN; e += 512) {
    const int i = e >> 6, j = e & 63;
    Qp[i][pos[j]] = Q[i][j];
  }
  __syncthreads();
  T(*Qs)[kN + 1] = reinterpret_cast<T(*)[kN + 1]>(&Q[0][0]);
  for (int e = tid; e < kN * kN; e += 512) {
    const int i = e >> 6, j = e & 63;
    const cplx<T> z = Qp[i][j];
    Qs[i][j] = z.re + z.im;
  }
  __syncthreads();

  // ---- column update [W_I W_J] <- [W_I W_J] Q and, when the descriptor has one,
  // [V_I V_J] <- [V_I V_J] Q on MFMA, next chunk prefetched.  The lane's k-slice ks reads
  // local column 4 ks + grp (offsets recomputed per load: cheaper than holding sixteen of
  // them in registers).
  const gptr<cplx<T>> __restrict__ V = as_global((cplx<T>*)d->v);
  const int npass = V != nullptr ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
  const gptr<cplx<T>> __restrict__ M = pass == 0 ? W : V;
  const int rows = pass == 0 ? R : C;
  auto off_in = [&](int lc) -> uint32_t {
    const int c = lc < kBs ? (lc < nI ? cI + lc : cI) : (lc - kBs < nJ ? cJ + lc - kBs : cJ);
    return (uint32_t)c * (uint32_t)rows;
  };
  cplx<T> av[16], an[16];
  auto load_rows = [&](int rbase, cplx<T>(&dst)[16]) {
    const int r = rbase + col;
    const uint32_t rr = r < rows ? r : 0;
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) dst[ks] = gload<T>(gat<T>(M, off_in(ks * 4 + grp) + rr));
  };
  // W skips its leading zero rows; V (pass 1) is not triangular
  int rbw = pass == 0 ? 16 * (c0 + (((wave - c0) % 8) + 8) % 8) : 16 * wave;
  if (rbw < rows) load_rows(rbw, av);
  for (; rbw < rows; rbw += 128) {
    load_rows(rbw + 128 < rows ? rbw + 128 : rbw, an);
    __builtin_amdgcn_sched_barrier(0);
    const bool rok = rbw + col < rows;
    for (int jt = 0; jt < 4; ++jt) {
      V4 o[3];
      for (int j = 0; j < 3; ++j)
        for (int v = 0; v < 4; ++v) o[j][v] = T(0);
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int kk = ks * 4 + grp;
        const cplx<T> a = cmask<T>(av[ks], rok && col_ok(kk));
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
      if (!col_ok(jj)) continue;
      const int cidx = jj < kBs ? cI + jj : cJ + jj - kBs;
      const gptr<cplx<T>> __restrict__ dst = gat<T>(M, (uint32_t)cidx * (uint32_t)rows);
      const int r4 = rbw + 4 * grp;
      if (r4 + 3 < rows) {
        vf4 u, w;
        u.x = ore[0]; u.y = oim[0]; u.z = ore[1]; u.w = oim[1];
        w.x = ore[2]; w.y = oim[2]; w.z = ore[3]; w.w = oim[3];
        *reinterpret_cast<gptr<vf4>>(dst + r4) = u;
        *reinterpret_cast<gptr<vf4>>(dst + r4 + 2) = w;
        continue;
      }
      for (int v = 0; v < 4; ++v) {
        const int rr = rbw + Mfma<T>::row(lane, v);
        if (rr < rows) {
          cplx<T> z;
          z.re = ore[v];
          z.im = oim[v];
          gstore<T>(dst + rr, z);
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) av[ks] = an[ks];
  }
  }
}

}  // namespace

void launch_jacobi_round64(const GateDesc* d_desc, int n_gates, int round, int nbp,
                           const LayerOut& out, double tol_scale, int inner_sweeps,
                           double inner_repeat, int sort_pairs, int prev_slot,
                           hipStream_t stream) {
  if (n_gates <= 0 || nbp < 2) return;
  hipLaunchKernelGGL(jacobi64_round_kernel, dim3(nbp / 2, n_gates), dim3(512), 0, stream, d_desc,
                     round, out, tol_scale, inner_sweeps, inner_repeat, sort_pairs, prev_slot);
}

}  // namespace ptebd
