// Preconditioning of the SVD on the mixed (FP32) path, one batch of gates per launch.
//
// For the work matrix W (R x C, R >= C; theta or theta^H):
//   colsort_kernel   -- column norms of W in FP64 and a permutation ps sorting them in
//                       descending order (A = W P, A[:, i] = W[:, ps[i]])
//   gram64_kernel    -- G = A^H A in FP64 on MFMA (upper 32x32 tiles)
//   potrf / trsm / herk_kernel -- blocked Cholesky G = R^H R (R upper), in place, FP64,
//                       with trailing updates deferred over groups of four panels;
//                       a pivot at or below 1e-13 G_00 marks a numerically dependent column
//                       (its row of R is set to zero)
//   xinit_kernel     -- X = R^H in FP32: the one-sided Jacobi then runs on X instead of W
//   recover_kernel   -- after the Jacobi (X Q = Y S, no V kept): the right vectors of W,
//                       Yhat[ps[i], j] = X[i, j] / ||X[:, j]||, and W Yhat = U S
// A = Q R with Q = A R^{-1} unitary, so R, and X = R^H, carry the singular values of W, and
// if X's columns after the rotations are Y S (Y orthonormal) then A = (A Y S^{-1}) S Y^H:
// right vectors P Y, left vectors W (P Y) / S.  Sorting the columns by norm first makes R
// graded, which halves the number of Jacobi sweeps on the saturated theta of a Haar layer.
// The Gram matrix squares the condition number: in FP64 it resolves every singular value
// above ~1e-7 sigma_1 of FP32 data to well below the FP32 rounding of theta, which is why the
// FP64 path does not use it.
#include <algorithm>

#include "ptebd_device.h"
#include "ptebd_internal.h"

namespace ptebd {
namespace {

typedef cplx<double> z64;
typedef cplx<float> z32;

// ---------------------------------------------------------------- column sort
// One workgroup per gate: column norms^2 of W (C <= 1024), bitonic sort, descending (ties
// by index).  Writes ps[0..C) and the largest norm^2 (the Cholesky pivot scale).
__global__ __launch_bounds__(256) void colsort_kernel(const GateDesc* __restrict__ descs,
                                                      PrecondOut po) {
  const int g = blockIdx.x;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const z32* __restrict__ W = (const z32*)d->w;
  __shared__ double key[1024];
  __shared__ int idx[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int P = 1;
  while (P < C) P <<= 1;
  for (int c = wave; c < C; c += 4) {
    double acc = 0.0;
    for (int r = lane; r < R; r += 64) {
      const z32 z = W[(size_t)c * R + r];
      acc += (double)z.re * z.re + (double)z.im * z.im;
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      key[c] = acc;
      idx[c] = c;
    }
  }
  for (int c = C + tid; c < P; c += 256) {
    key[c] = -1.0;
    idx[c] = c;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < (P >> 1); i += 256) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool descending = (lo & size) == 0;
        const double klo = key[lo], khi = key[hi];
        const int ilo = idx[lo], ihi = idx[hi];
        // descending by key, ascending index among equal keys
        const bool lo_first = klo > khi || (klo == khi && ilo < ihi);
        if (descending ? !lo_first : lo_first) {
          key[lo] = khi;
          key[hi] = klo;
          idx[lo] = ihi;
          idx[hi] = ilo;
        }
      }
      __syncthreads();
    }
  }
  int* ps = po.ps + (size_t)g * po.cmax;
  for (int c = tid; c < C; c += 256) ps[c] = idx[c];
  if (tid == 0) po.gmax[g] = key[0];
}

// ---------------------------------------------------------------- Gram matrix
// G[i, j] = sum_r conj(W[r, ps[i]]) W[r, ps[j]] in FP64 for the upper 32x32 tiles
// (ti <= tj); column-major C x C.  Four waves, each a 16x16 sub-tile; rows in steps of 16.
__device__ inline void tile_of(int t, int nt, int& ti, int& tj) {
  // upper-triangular tile t (row-major over ti, tj >= ti)
  ti = 0;
  int rowlen = nt;
  while (t >= rowlen) {
    t -= rowlen;
    ++ti;
    --rowlen;
  }
  tj = ti + t;
}

__global__ __launch_bounds__(256) void gram64_kernel(const GateDesc* __restrict__ descs,
                                                     int n_gates, int per_gate, PrecondOut po) {
  int g, tile;
  xcd_gate_tile(per_gate, g, tile);  // a gate's tiles on one XCD, its columns in one L2
  if (g >= n_gates) return;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const int nt = (C + 31) >> 5;
  if (tile >= nt * (nt + 1) / 2) return;
  int ti, tj;
  tile_of(tile, nt, ti, tj);
  const gptr<const z32> __restrict__ W = as_global((const z32*)d->w);
  const int* __restrict__ ps = po.ps + (size_t)g * po.cmax;
  z64* __restrict__ G = (z64*)d->gram;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int i0 = ti * 32 + (wave >> 1) * 16, j0 = tj * 32 + (wave & 1) * 16;
  const int ci = i0 + col, cj = j0 + col;
  const bool oki = ci < C, okj = cj < C;
  const uint32_t offi = (uint32_t)(oki ? ps[ci] : 0) * (uint32_t)R;
  const uint32_t offj = (uint32_t)(okj ? ps[cj] : 0) * (uint32_t)R;
  typedef Mfma<double>::v4 V4;
  // three real products per entry: for conj(x) y with x = p + iq, y = u + iv,
  // P1 = sum p u, P2 = sum q v, P3 = sum (p - q)(u + v); Re = P1 + P2, Im = P3 - P1 + P2.
  // The inputs are FP32 values, so p - q, u + v and every product are exact in FP64.
  V4 acc[3];
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < 4; ++v) acc[j][v] = 0.0;
  // 16 rows per step: the eight loads of a lane are unconditional (an out-of-range row
  // reads row 0) and issued together, masked where used; the next step's are in flight
  // during this step's products
  z32 xa[4], ya[4], xn[4], yn[4];
  auto load = [&](int r0, z32(&a)[4], z32(&b)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 4 * u + grp;
      const uint32_t rc = r < R ? r : 0;
      a[u] = gload<float>(gat<float>(W, offi + rc));
      b[u] = gload<float>(gat<float>(W, offj + rc));
    }
  };
  load(0, xa, ya);
  for (int r0 = 0; r0 < R; r0 += 16) {
    load(r0 + 16 < R ? r0 + 16 : r0, xn, yn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool rok = r0 + 4 * u + grp < R;
      const z32 a = cmask<float>(xa[u], oki && rok), b = cmask<float>(ya[u], okj && rok);
      const double p = a.re, q = a.im, uu = b.re, vv = b.im;
      acc[0] = Mfma<double>::op(p, uu, acc[0]);
      acc[1] = Mfma<double>::op(q, vv, acc[1]);
      acc[2] = Mfma<double>::op(p - q, uu + vv, acc[2]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xa[u] = xn[u];
      ya[u] = yn[u];
    }
  }
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + Mfma<double>::row(lane, v), j = j0 + col;
    if (i < C && j < C) {
      z64 z;
      z.re = acc[0][v] + acc[1][v];
      z.im = acc[2][v] - acc[0][v] + acc[1][v];
      G[(size_t)j * C + i] = z;
    }
  }
}

// ---------------------------------------------------------------- blocked Cholesky
// G = R^H R with R upper triangular, overwriting the upper triangle of G, 32 columns per
// block step kb: herk brings the block row kb up to date, potrf factors the diagonal
// block, trsm solves the block row R[kb, j] = R[kb, kb]^{-H} G[kb, j], and after every
// fourth panel herk updates the trailing upper tiles G[i, j] -= R[l, i]^H R[l, j] with the
// group's rows l.  A pivot d <= 1e-13 * G_00 (G_00 the largest column
// norm^2, the columns being sorted) is a numerically dependent column: its row of R is zero.
constexpr double kPivotTol = 1e-13;

__global__ __launch_bounds__(256) void potrf_kernel(const GateDesc* __restrict__ descs,
                                                    PrecondOut po, int kb) {
  const int g = blockIdx.x;
  const int C = descs[g].C;
  const int b0 = kb * 32;
  if (b0 >= C) return;
  const int nb = min(32, C - b0);
  z64* __restrict__ G = (z64*)descs[g].gram;
  const double thr = kPivotTol * po.gmax[g];
  __shared__ z64 A[32][33];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int e = tid; e < 1024; e += 256) {
    const int i = e & 31, j = e >> 5;
    z64 z;
    z.re = z.im = 0.0;
    if (i < nb && j < nb && i <= j) z = G[(size_t)(b0 + j) * C + b0 + i];
    A[i][j] = z;
  }
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    if (tid == 0) {
      const double dv = A[p][p].re;
      piv = dv > thr ? sqrt(dv) : 0.0;
    }
    __syncthreads();
    const double rp = piv;
    // row p of R: R[p][l] = A[p][l] / R[p][p] for l > p (zero row for a dropped pivot)
    if (tid < 32) {
      const int l = tid;
      if (l == p) {
        A[p][p].re = rp;
        A[p][p].im = 0.0;
      } else if (l > p && l < nb) {
        if (rp > 0.0) {
          A[p][l].re /= rp;
          A[p][l].im /= rp;
        } else {
          A[p][l].re = 0.0;
          A[p][l].im = 0.0;
        }
      }
    }
    __syncthreads();
    // trailing: A[l][m] -= conj(R[p][l]) R[p][m], p < l <= m
    for (int e = tid; e < 1024; e += 256) {
      const int l = e & 31, m = e >> 5;
      if (l > p && l <= m && m < nb) {
        const z64 a = A[p][l], b = A[p][m];
        A[l][m].re -= a.re * b.re + a.im * b.im;
        A[l][m].im -= a.re * b.im - a.im * b.re;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < 1024; e += 256) {
    const int i = e & 31, j = e >> 5;
    if (i < nb && j < nb && i <= j) G[(size_t)(b0 + j) * C + b0 + i] = A[i][j];
  }
}

// Block row: X = R_kk^{-H} G[kb, j] for the tiles j > kb (blockIdx.x + kb + 1), forward
// substitution with the lower-triangular R_kk^H.  Column j of the tile is solved by the 8
// lanes 8j .. 8j + 7 of one wave: lane s sums the terms l = s mod 8 of each row and keeps the
// solved rows l = s mod 8 in registers; shuffles complete the sum in all 8 lanes, which then
// scale by the reciprocal pivot (zero for a dropped pivot).
__global__ __launch_bounds__(256) void trsm_kernel(const GateDesc* __restrict__ descs,
                                                   int kb) {
  const int g = blockIdx.y;
  const int C = descs[g].C;
  const int b0 = kb * 32;
  const int c0 = (kb + 1 + blockIdx.x) * 32;
  if (c0 >= C) return;
  const int nb = min(32, C - b0), nc = min(32, C - c0);
  z64* __restrict__ G = (z64*)descs[g].gram;
  __shared__ z64 Rk[32][33];
  __shared__ z64 X[32][33];
  __shared__ double rinv[32];
  const int tid = threadIdx.x;
  for (int e = tid; e < 1024; e += 256) {
    const int i = e & 31, j = e >> 5;
    z64 z;
    z.re = z.im = 0.0;
    if (i < nb && j < nb && i <= j) z = G[(size_t)(b0 + j) * C + b0 + i];
    Rk[i][j] = z;
    z64 x;
    x.re = x.im = 0.0;
    if (i < nb && j < nc) x = G[(size_t)(c0 + j) * C + b0 + i];
    X[i][j] = x;
  }
  __syncthreads();
  if (tid < 32) {
    const double r = Rk[tid][tid].re;
    rinv[tid] = tid < nb && r > 0.0 ? 1.0 / r : 0.0;
  }
  __syncthreads();
  const int j = tid >> 3, s = tid & 7;
  double xr[4], xi[4];  // solved rows s, s + 8, s + 16, s + 24 of column j
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    xr[q] = 0.0;
    xi[q] = 0.0;
  }
  for (int i = 0; i < nb; ++i) {
    // sum_{l < i} conj(Rk[l][i]) X[l][j], this lane's share
    double pr = 0.0, pi = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int l = s + 8 * q;
      if (l < i) {
        const z64 r = Rk[l][i];
        pr += r.re * xr[q] + r.im * xi[q];
        pi += r.re * xi[q] - r.im * xr[q];
      }
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
      pr += __shfl_xor(pr, o);
      pi += __shfl_xor(pi, o);
    }
    const z64 b = X[i][j];
    const double ri = rinv[i];
    const double vr = (b.re - pr) * ri, vi = (b.im - pi) * ri;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (s + 8 * q == i) {
        xr[q] = vr;
        xi[q] = vi;
      }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int l = s + 8 * q;
    if (l < nb) {
      X[l][j].re = xr[q];
      X[l][j].im = xi[q];
    }
  }
  __syncthreads();
  for (int e = tid; e < 1024; e += 256) {
    const int i = e & 31, jj = e >> 5;
    if (i < nb && jj < nc) G[(size_t)(c0 + jj) * C + b0 + i] = X[i][jj];
  }
}

// Deferred updates of the blocked Cholesky: G[ti, tj] -= sum_l R[l, ti]^H R[l, tj] over the
// rows l in [32 l0, 32 l1) of R, which the earlier panels left in the upper triangle of G.
// mode 0: the block row ti = kb, tiles tj = kb + tile, before panel kb is factored
// (the rows of the panels since the last trailing update); mode 1: the upper tiles
// kb < ti <= tj once panel kb has closed a group (a rank 32 (l1 - l0) trailing update).
// Every operand entry has l < ti * 32 <= column, so it lies in the strict upper triangle,
// and no tile written here is read by the same launch.  Four waves, each a 16 x 16
// sub-tile on FP64 MFMA; K in steps of 16 rows with the next step's loads in flight,
// operands straight from global memory (column-major G: a column's rows are contiguous).
__global__ __launch_bounds__(256) void herk_kernel(const GateDesc* __restrict__ descs, int n_gates,
                                                   int per_gate, int kb, int l0, int l1, int mode) {
  int g, tile;
  xcd_gate_tile(per_gate, g, tile);  // a gate's tiles on one XCD, its R rows in one L2
  if (g >= n_gates) return;
  const int C = descs[g].C;
  const int nt = (C + 31) >> 5;
  int ti, tj;
  if (mode == 0) {
    ti = kb;
    tj = kb + tile;
    if (tj >= nt) return;
  } else {
    const int nrem = nt - kb - 1;
    if (nrem <= 0 || tile >= nrem * (nrem + 1) / 2) return;
    tile_of(tile, nrem, ti, tj);
    ti += kb + 1;
    tj += kb + 1;
  }
  const int k_lo = 32 * l0, k_hi = min(32 * l1, C);
  if (k_lo >= k_hi) return;
  z64* __restrict__ G = (z64*)descs[g].gram;
  const gptr<const z64> Gg = as_global((const z64*)G);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int i0 = ti * 32 + (wave >> 1) * 16, j0 = tj * 32 + (wave & 1) * 16;
  const int ci = i0 + col, cj = j0 + col;
  const bool oki = ci < C, okj = cj < C;
  // every matrix here has C <= 1024: 32-bit element offsets
  const uint32_t offi = (uint32_t)(oki ? ci : 0) * (uint32_t)C;
  const uint32_t offj = (uint32_t)(okj ? cj : 0) * (uint32_t)C;
  typedef Mfma<double>::v4 V4;
  V4 acc[2];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    acc[0][v] = 0.0;
    acc[1][v] = 0.0;
  }
  // rows k0 + 4u + grp of the lane's two columns; a row at or beyond k_hi reads row k_lo
  // (unconditional loads, masked where used)
  z64 xa[4], ya[4], xn[4], yn[4];
  auto load = [&](int k0, z64(&a)[4], z64(&b)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + grp;
      const uint32_t kc = (uint32_t)(k < k_hi ? k : k_lo);
      a[u] = gload<double>(gat<double>(Gg, offi + kc));
      b[u] = gload<double>(gat<double>(Gg, offj + kc));
    }
  };
  load(k_lo, xa, ya);
  for (int k0 = k_lo; k0 < k_hi; k0 += 16) {
    load(k0 + 16 < k_hi ? k0 + 16 : k0, xn, yn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool kok = k0 + 4 * u + grp < k_hi;
      gram_mfma<double>(acc, cmask<double>(xa[u], oki && kok), cmask<double>(ya[u], okj && kok));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xa[u] = xn[u];
      ya[u] = yn[u];
    }
  }
  const gptr<z64> Gw = as_global(G);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + Mfma<double>::row(lane, v);
    if (i < C && okj && i <= cj) {
      const gptr<z64> p = gat<double>(Gw, (uint32_t)cj * (uint32_t)C + (uint32_t)i);
      z64 z = gload<double>(p);
      z.re -= acc[0][v];
      z.im -= acc[1][v];
      gstore<double>(p, z);
    }
  }
}

// X = R^H in FP32 (C x C column-major, lower triangular) into the Jacobi work matrix,
// X[i, j] = conj(R[j, i]) = conj(G[j, i]) for i >= j.  One 32 x 32 tile of X per step,
// transposed through LDS: G's column i is read along its rows j and X's column j written
// along its rows i, both contiguous; tiles wholly above the diagonal are zeros.
__global__ __launch_bounds__(256) void xinit_kernel(const GateDesc* __restrict__ jdescs) {
  const int g = blockIdx.y;
  const int C = jdescs[g].C;
  const int nt = (C + 31) >> 5;
  const z64* __restrict__ G = (const z64*)jdescs[g].gram;
  z32* __restrict__ X = (z32*)jdescs[g].w;
  __shared__ z32 tile[32][33];  // tile[ii][jj] = X[32 a + ii, 32 b + jj]
  const int tid = threadIdx.x;
  for (int t = blockIdx.x; t < nt * nt; t += gridDim.x) {
    const int a = t % nt, b = t / nt;  // tile row (X rows i) and column (X columns j)
    if (a >= b) {
      for (int e = tid; e < 1024; e += 256) {
        const int jj = e & 31, ii = e >> 5;
        const int i = 32 * a + ii, j = 32 * b + jj;
        z32 z;
        z.re = z.im = 0.f;
        if (i < C && j < C && i >= j) {
          const z64 r = G[(size_t)i * C + j];  // R[j][i]
          z.re = (float)r.re;
          z.im = (float)(-r.im);
        }
        tile[ii][jj] = z;
      }
      __syncthreads();
      for (int e = tid; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        const int i = 32 * a + ii, j = 32 * b + jj;
        if (i < C && j < C) X[(size_t)j * C + i] = tile[ii][jj];
      }
      __syncthreads();
    } else {
      for (int e = tid; e < 1024; e += 256) {
        const int ii = e & 31, jj = e >> 5;
        const int i = 32 * a + ii, j = 32 * b + jj;
        z32 z;
        z.re = z.im = 0.f;
        if (i < C && j < C) X[(size_t)j * C + i] = z;
      }
    }
  }
}

// Right vectors of W: Yhat[ps[i], c] = X[i, c] / ||X[:, c]|| for the kept columns
// c = perm[j], j < k (stored in the G buffer, C x C FP32 column-major).
__global__ void yhat_kernel(const GateDesc* __restrict__ jdescs, PrecondOut po, LayerOut out) {
  const int g = blockIdx.y;
  const int C = jdescs[g].C;
  const int k = out.k[g];
  const z32* __restrict__ X = (const z32*)jdescs[g].w;
  z32* __restrict__ Y = (z32*)jdescs[g].gram;
  const int* __restrict__ ps = po.ps + (size_t)g * po.cmax;
  const int* __restrict__ perm = out.perm + (size_t)g * out.cmax;
  const double* __restrict__ sig = out.sig + (size_t)g * out.cmax;
  const size_t total = (size_t)C * k;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % C), j = (int)(e / C);
    const int c = perm[j];
    const double inv = sig[j] > 0.0 ? 1.0 / sig[j] : 0.0;
    const z32 x = X[(size_t)c * C + i];
    z32 z;
    z.re = (float)(x.re * inv);
    z.im = (float)(x.im * inv);
    Y[(size_t)c * C + ps[i]] = z;
  }
}

// U S = W Yhat for the kept columns (c = perm[j], j < k): 32 rows x 32 kept columns per
// workgroup, four waves of 16 x 16, K = C in steps of 16 on FP32 MFMA, the next step's loads
// in flight.  Three real products per complex one: with a = x + iy, b = u + iv,
// P1 = x u, P2 = y v, P3 = (x + y)(u + v); Re ab = P1 - P2, Im ab = P3 - P1 - P2.  Written
// into the column c of the U buffer (R x C), unnormalized (the write-back divides by sigma).
__global__ __launch_bounds__(256) void ugemm_kernel(const GateDesc* __restrict__ descs,
                                                    int n_gates, int per_gate, LayerOut out) {
  int g, tile;
  xcd_gate_tile(per_gate, g, tile);  // a gate's tiles on one XCD, its W and Y in one L2
  if (g >= n_gates) return;
  const GateDesc* d = descs + g;
  const int R = d->R, C = d->C;
  const int k = out.k[g];
  const int tr = (R + 31) >> 5, tk = (k + 31) >> 5;
  if (tile >= tr * tk) return;
  const int r0 = (tile % tr) * 32, j0 = (tile / tr) * 32;
  const z32* __restrict__ W = (const z32*)d->w;
  const z32* __restrict__ Y = (const z32*)d->gram;
  z32* __restrict__ U = (z32*)d->left;
  const int* __restrict__ perm = out.perm + (size_t)g * out.cmax;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int rr = r0 + (wave >> 1) * 16 + col;          // A operand row of this lane
  const int jb = j0 + (wave & 1) * 16;
  const int jl = jb + col;                              // B operand column of this lane
  const int cl = jl < k ? perm[jl] : -1;
  typedef Mfma<float>::v4 V4;
  V4 acc[3];
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < 4; ++v) acc[j][v] = 0.f;
  // 16 values of K per step, the eight loads of a lane issued together (out-of-range
  // indices read entry 0 and are masked where used)
  const gptr<const z32> Wg = as_global(W), Yg = as_global(Y);
  const uint32_t rc = rr < R ? rr : 0, yoff = (uint32_t)(cl >= 0 ? cl : 0) * (uint32_t)C;
  z32 aa[4], bb[4], an[4], bn[4];
  auto load = [&](int k0, z32(&a)[4], z32(&b)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + 4 * u + grp;
      const uint32_t kc = kk < C ? kk : 0;
      a[u] = gload<float>(gat<float>(Wg, kc * (uint32_t)R + rc));
      b[u] = gload<float>(gat<float>(Yg, yoff + kc));
    }
  };
  load(0, aa, bb);
  for (int k0 = 0; k0 < C; k0 += 16) {
    load(k0 + 16 < C ? k0 + 16 : k0, an, bn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool kok = k0 + 4 * u + grp < C;
      const z32 a = cmask<float>(aa[u], rr < R && kok), b = cmask<float>(bb[u], cl >= 0 && kok);
      acc[0] = Mfma<float>::op(a.re, b.re, acc[0]);
      acc[1] = Mfma<float>::op(a.im, b.im, acc[1]);
      acc[2] = Mfma<float>::op(a.re + a.im, b.re + b.im, acc[2]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      aa[u] = an[u];
      bb[u] = bn[u];
    }
  }
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + (wave >> 1) * 16 + Mfma<float>::row(lane, v);
    const int j = jb + col;
    if (r < R && j < k) {
      z32 z;
      z.re = acc[0][v] - acc[1][v];
      z.im = acc[2][v] - acc[0][v] - acc[1][v];
      U[(size_t)perm[j] * R + r] = z;
    }
  }
}

}  // namespace

void launch_colsort(const GateDesc* d_desc, int n_gates, const PrecondOut& po,
                    hipStream_t stream) {
  hipLaunchKernelGGL(colsort_kernel, dim3(n_gates), dim3(256), 0, stream, d_desc, po);
}

void launch_gram64(const GateDesc* d_desc, int n_gates, int max_c, const PrecondOut& po,
                   hipStream_t stream) {
  const int nt = (max_c + 31) / 32, per_gate = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(gram64_kernel, dim3(xcd_grid(per_gate, n_gates)), dim3(256), 0, stream,
                     d_desc, n_gates, per_gate, po);
}

// Panels of 32 columns; the trailing matrix is updated once per group of kGroup panels (a
// rank-128 update), and each panel's block row, just before it is factored, by the rows of
// the group's earlier panels.  Against a trailing update after every panel this reads and
// writes the trailing tiles a quarter as often, with K loops four times as long.
void launch_cholesky(const GateDesc* d_desc, int n_gates, int max_c, const PrecondOut& po,
                     hipStream_t stream) {
  constexpr int kGroup = 4;
  const int nt = (max_c + 31) / 32;
  for (int kb = 0; kb < nt; ++kb) {
    const int kb0 = kb - kb % kGroup;
    if (kb > kb0)
      hipLaunchKernelGGL(herk_kernel, dim3(xcd_grid(nt - kb, n_gates)), dim3(256), 0, stream,
                         d_desc, n_gates, nt - kb, kb, kb0, kb, 0);
    hipLaunchKernelGGL(potrf_kernel, dim3(n_gates), dim3(256), 0, stream, d_desc, po, kb);
    const int nrem = nt - kb - 1;
    if (nrem <= 0) break;
    hipLaunchKernelGGL(trsm_kernel, dim3(nrem, n_gates), dim3(256), 0, stream, d_desc, kb);
    if (kb % kGroup == kGroup - 1)
      hipLaunchKernelGGL(herk_kernel, dim3(xcd_grid(nrem * (nrem + 1) / 2, n_gates)), dim3(256),
                         0, stream, d_desc, n_gates, nrem * (nrem + 1) / 2, kb, kb0, kb + 1, 1);
  }
}

void launch_xinit(const GateDesc* d_jdesc, int n_gates, int max_c, hipStream_t stream) {
  const int nt = (max_c + 31) / 32;
  const int blocks = std::max(1, std::min(256, nt * nt));
  hipLaunchKernelGGL(xinit_kernel, dim3(blocks, n_gates), dim3(256), 0, stream, d_jdesc);
}

void launch_recover(const GateDesc* d_desc, const GateDesc* d_jdesc, int n_gates, int max_r,
                    int max_c, const PrecondOut& po, const LayerOut& out, hipStream_t stream) {
  const int blocks = std::max(1, std::min(256, (max_c * max_c + 255) / 256));
  hipLaunchKernelGGL(yhat_kernel, dim3(blocks, n_gates), dim3(256), 0, stream, d_jdesc, po, out);
  const int tiles = ((max_r + 31) / 32) * ((max_c + 31) / 32);
  hipLaunchKernelGGL(ugemm_kernel, dim3(xcd_grid(tiles, n_gates)), dim3(256), 0, stream, d_desc,
                     n_gates, tiles, out);
}

}  // namespace ptebd
