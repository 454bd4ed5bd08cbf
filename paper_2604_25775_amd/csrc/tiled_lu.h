// Register-tiled FP64 Gauss-Jordan inverse / LU determinant for one n x n
// matrix per 256-thread workgroup, n <= 16 R.
//
// Thread (tx = tid / 16, ty = tid % 16) holds rows ty + 16 a and columns
// tx + 16 b (cyclic distribution, so the work stays balanced as columns are
// eliminated).  The 16 threads owning a column sit in one wavefront, so the
// pivot search is a 16-lane reduction.  Partial pivoting without moving data:
// step p uses the unused row with the largest |entry| in column p.
//   INVERT:  in-place Gauss-Jordan; afterwards A^-1[p'][perm[q]] = X[perm[p']][q]
//   !INVERT: LU elimination of the unused rows only (determinant).
// det A = sign(perm) * prod(pivots).
#pragma once
#include "svmc_dev.h"

namespace svmc {

template <int R> struct GjShared {
  double colbuf[2][16 * R];      // pivot column, by step parity
  double rowbuf[2][16 * R];      // pivot row, by step parity
  double pvs[16 * R];            // pivot of each step
  int perm[16 * R];
  int perminv[16 * R];
  int piv[2];
  int inv;
  double red[4];
};

// Two barriers per step: the pivot column and row buffers alternate between
// steps, so a step's writes never meet the previous step's reads, and each
// thread keeps the used flags of its own rows in registers.  log|det| and
// the sign are formed from the stored pivots after the loop.
template <int R, bool INVERT>
SVMC_DEV void tiled_gj(double (&x)[R][R], int n, GjShared<R>& sh, double& logabs, double& sgn, bool& singular) {
  const int tid = threadIdx.x, tx = tid >> 4, ty = tid & 15;
  bool used[R];
#pragma unroll
  for (int a = 0; a < R; ++a) used[a] = ty + 16 * a >= n;
  logabs = 0.0;
  sgn = 1.0;
  singular = false;
  for (int p = 0; p < n; ++p) {
    const int bp = p >> 4, buf = p & 1;
    if (tx == (p & 15)) {
      double col[R];
#pragma unroll
      for (int a = 0; a < R; ++a) col[a] = 0.0;
#pragma unroll
      for (int b = 0; b < R; ++b)
        if (b == bp) {
#pragma unroll
          for (int a = 0; a < R; ++a) col[a] = x[a][b];
        }
      double best = -1.0;
      int bi = 1 << 20;
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const int k = ty + 16 * a;
        sh.colbuf[buf][k] = col[a];
        if (k < n && !used[a]) {
          const double v = fabs(col[a]);
          if (v > best) { best = v; bi = k; }
        }
      }
      for (int o = 8; o >= 1; o >>= 1) {
        const double b2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (b2 > best || (b2 == best && i2 < bi)) { best = b2; bi = i2; }
      }
      if (ty == 0) sh.piv[buf] = bi;
    }
    __syncthreads();
    const int pi = sh.piv[buf];
    const double pv = pi < n ? sh.colbuf[buf][pi] : 0.0;
    if (pv == 0.0) { singular = true; break; }              // the same in every thread
    if (ty == (pi & 15)) {
      const int ap = pi >> 4;
#pragma unroll
      for (int a = 0; a < R; ++a)
        if (a == ap) {
#pragma unroll
          for (int b = 0; b < R; ++b) sh.rowbuf[buf][tx + 16 * b] = x[a][b];
        }
    }
    if (tid == 0) { sh.perm[p] = pi; sh.pvs[p] = pv; }
    __syncthreads();
    const double inv = 1.0 / pv;
    // this thread's entries of the pivot row, read once per step
    double r[R];
#pragma unroll
    for (int b = 0; b < R; ++b) r[b] = sh.rowbuf[buf][tx + 16 * b];
    // column p sits in register column bp of the threads with tx = p mod 16
    const bool pcol = tx == (p & 15);
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int k = ty + 16 * a;
      const double f = sh.colbuf[buf][k] * inv;
      const bool isp = (k == pi);
      const bool live = !used[a] && !isp;
#pragma unroll
      for (int b = 0; b < R; ++b) {
        const int m = tx + 16 * b;
        if (INVERT) {
          // selects, not branches: the pivot row is scaled, every other row
          // eliminates column p, and column p takes the new inverse column
          const double upd = isp ? x[a][b] * inv : fma(-f, r[b], x[a][b]);
          const double newc = isp ? inv : -f;
          x[a][b] = (b == bp && pcol) ? newc : upd;
        } else if (live && m > p) {
          x[a][b] = fma(-f, r[b], x[a][b]);
        }
      }
      if (isp) used[a] = true;
    }
  }
  if (singular) return;
  __syncthreads();
  if (tid == 0) sh.inv = 0;
  for (int k = tid; k < n; k += 256) sh.perminv[sh.perm[k]] = k;
  // log|det| and the number of negative pivots, summed over the block
  double ls = 0.0;
  int neg = 0;
  for (int q = tid; q < n; q += 256) {
    ls += log(fabs(sh.pvs[q]));
    neg += sh.pvs[q] < 0.0 ? 1 : 0;
  }
  for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o, 64);
  if ((tid & 63) == 0) sh.red[tid >> 6] = ls;
  __syncthreads();
  // permutation inversions plus negative pivots: the sign's parity
  int cnt = neg;
  for (int q = tid; q < n; q += 256)
    for (int q2 = q + 1; q2 < n; ++q2) cnt += sh.perm[q2] < sh.perm[q];
  if (cnt) atomicAdd(&sh.inv, cnt);
  __syncthreads();
  logabs = sh.red[0] + sh.red[1] + sh.red[2] + sh.red[3];
  if (sh.inv & 1) sgn = -sgn;
}

// log|det| and sign of an n x n matrix in the layout of tiled_gj (thread
// (tx, ty) holds rows ty + 16 a, columns tx + 16 b; rows/columns >= n hold
// the identity), by LU elimination with partial pivoting (the same pivot
// choice as tiled_gj: largest |entry| of the unused rows, ties to the lower
// row).  The trailing update is applied to every element of every row
// without branches: rows already used (and the pivot row) take a zero
// multiplier, and columns already eliminated are changed but never read
// again, so the pivots - and the determinant - are those of the plain
// elimination.  Two barriers per step.
template <int R>
SVMC_DEV void tiled_lu_det(double (&x)[R][R], int n, GjShared<R>& sh, double& logabs, double& sgn, bool& singular) {
  const int tid = threadIdx.x, tx = tid >> 4, ty = tid & 15;
  bool used[R];
#pragma unroll
  for (int a = 0; a < R; ++a) used[a] = ty + 16 * a >= n;
  logabs = 0.0;
  sgn = 1.0;
  singular = false;
  for (int p = 0; p < n; ++p) {
    const int bp = p >> 4, buf = p & 1;
    if (tx == (p & 15)) {
      double col[R];
#pragma unroll
      for (int a = 0; a < R; ++a) col[a] = 0.0;
#pragma unroll
      for (int b = 0; b < R; ++b)
        if (b == bp) {
#pragma unroll
          for (int a = 0; a < R; ++a) col[a] = x[a][b];
        }
      double best = -1.0;
      int bi = 1 << 20;
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const int k = ty + 16 * a;
        sh.colbuf[buf][k] = col[a];
        const double v = used[a] ? -1.0 : fabs(col[a]);
        const bool take = v > best;
        best = take ? v : best;
        bi = take ? k : bi;
      }
      for (int o = 8; o >= 1; o >>= 1) {
        const double b2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        const bool take = b2 > best || (b2 == best && i2 < bi);
        best = take ? b2 : best;
        bi = take ? i2 : bi;
      }
      if (ty == 0) sh.piv[buf] = bi;
    }
    __syncthreads();
    const int pi = sh.piv[buf];
    const double pv = pi < n ? sh.colbuf[buf][pi] : 0.0;
    if (pv == 0.0) { singular = true; break; }              // the same in every thread
    if (ty == (pi & 15)) {
      const int ap = pi >> 4;
#pragma unroll
      for (int a = 0; a < R; ++a)
        if (a == ap) {
#pragma unroll
          for (int b = 0; b < R; ++b) sh.rowbuf[buf][tx + 16 * b] = x[a][b];
        }
    }
    if (tid == 0) { sh.perm[p] = pi; sh.pvs[p] = pv; }
    __syncthreads();
    const double inv = 1.0 / pv;
    double f[R], r[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int k = ty + 16 * a;
      const bool isp = k == pi;
      f[a] = (used[a] || isp) ? 0.0 : sh.colbuf[buf][k] * inv;
      used[a] = used[a] || isp;
    }
#pragma unroll
    for (int b = 0; b < R; ++b) r[b] = sh.rowbuf[buf][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) x[a][b] = fma(-f[a], r[b], x[a][b]);
  }
  if (singular) return;
  __syncthreads();
  if (tid == 0) sh.inv = 0;
  // log|det| and the number of negative pivots, summed over the block
  double ls = 0.0;
  int neg = 0;
  for (int q = tid; q < n; q += 256) {
    ls += log(fabs(sh.pvs[q]));
    neg += sh.pvs[q] < 0.0 ? 1 : 0;
  }
  for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o, 64);
  if ((tid & 63) == 0) sh.red[tid >> 6] = ls;
  __syncthreads();
  // permutation inversions plus negative pivots: the sign's parity
  int cnt = neg;
  for (int q = tid; q < n; q += 256)
    for (int q2 = q + 1; q2 < n; ++q2) cnt += sh.perm[q2] < sh.perm[q];
  if (cnt) atomicAdd(&sh.inv, cnt);
  __syncthreads();
  logabs = sh.red[0] + sh.red[1] + sh.red[2] + sh.red[3];
  if (sh.inv & 1) sgn = -sgn;
}

}  // namespace svmc
