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
  double colbuf[16 * R];
  double rowbuf[16 * R];
  int used[16 * R];
  int perm[16 * R];
  int perminv[16 * R];
  int piv;
  int inv;
};

template <int R, bool INVERT>
SVMC_DEV void tiled_gj(double (&x)[R][R], int n, GjShared<R>& sh, double& logabs, double& sgn, bool& singular) {
  const int tid = threadIdx.x, tx = tid >> 4, ty = tid & 15;
  for (int k = tid; k < 16 * R; k += 256) sh.used[k] = k >= n;
  __syncthreads();
  logabs = 0.0;
  sgn = 1.0;
  singular = false;
  for (int p = 0; p < n; ++p) {
    const int bp = p >> 4;
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
        sh.colbuf[k] = col[a];
        if (k < n && !sh.used[k]) {
          const double v = fabs(col[a]);
          if (v > best) { best = v; bi = k; }
        }
      }
      for (int o = 8; o >= 1; o >>= 1) {
        const double b2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (b2 > best || (b2 == best && i2 < bi)) { best = b2; bi = i2; }
      }
      if (ty == 0) sh.piv = bi;
    }
    __syncthreads();
    const int pi = sh.piv;
    const double pv = pi < n ? sh.colbuf[pi] : 0.0;
    if (pv == 0.0) { singular = true; break; }
    if (ty == (pi & 15)) {
      const int ap = pi >> 4;
#pragma unroll
      for (int a = 0; a < R; ++a)
        if (a == ap) {
#pragma unroll
          for (int b = 0; b < R; ++b) sh.rowbuf[tx + 16 * b] = x[a][b];
        }
    }
    __syncthreads();
    const double inv = 1.0 / pv;
    logabs += log(fabs(pv));
    if (pv < 0) sgn = -sgn;
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int k = ty + 16 * a;
      const double f = sh.colbuf[k] * inv;
      const bool isp = (k == pi);
      const bool live = !sh.used[k] && !isp;
#pragma unroll
      for (int b = 0; b < R; ++b) {
        const int m = tx + 16 * b;
        if (INVERT) {
          if (isp) x[a][b] = (m == p) ? inv : x[a][b] * inv;
          else x[a][b] = (m == p) ? -f : fma(-f, sh.rowbuf[m], x[a][b]);
        } else if (live && m > p) {
          x[a][b] = fma(-f, sh.rowbuf[m], x[a][b]);
        }
      }
    }
    __syncthreads();
    if (tid == 0) { sh.used[pi] = 1; sh.perm[p] = pi; }
    __syncthreads();
  }
  if (singular) return;
  if (tid == 0) sh.inv = 0;
  for (int k = tid; k < n; k += 256) sh.perminv[sh.perm[k]] = k;
  __syncthreads();
  int cnt = 0;
  for (int p = tid; p < n; p += 256)
    for (int q = p + 1; q < n; ++q) cnt += sh.perm[q] < sh.perm[p];
  if (cnt) atomicAdd(&sh.inv, cnt);
  __syncthreads();
  if (sh.inv & 1) sgn = -sgn;
}

}  // namespace svmc
