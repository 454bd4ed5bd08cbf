// Full-recompute local energies: the O(N^4)-per-sweep comparison scheme
// (Sec. III.A, global architectures: every connected configuration is
// re-evaluated from scratch).  Same inputs and precision policy as the
// low-rank path: conv stack on MFMA in the conv precision (the cold-setup
// forward kernels), orbital rows and determinants in FP64.
//
// Batched in stages over "configurations": for every walker its own
// configuration and every configuration one hop away, listed walker by
// walker in canonical hop order and processed in chunks:
//   1. k_full_configs writes each configuration's occupation bytes (and the
//      walker, hop index and Jordan-Wigner sign of its hop or spin exchange);
//   2. the forward of the cold setup (embedding, every conv layer over all
//      sites) runs on the chunk as if it were a batch of walkers;
//   3. k_full_det builds both Slater blocks of each configuration (rows of
//      the occupied sites in ascending order: base + H_L W + b, FP64) and
//      factorises them with the register-tiled LU, giving log|det| and sign
//      in canonical order; above 128 electrons per spin the cold-setup rows
//      and global-memory Gauss-Jordan kernels do the same;
//   4. k_full_post turns them into ratios psi(n')/psi(n) with the moving
//      electron keeping its row (the JW sign times the canonical ratio);
// and k_full_reduce sums the local energy per walker in canonical hop order.
#include "hop.h"
#include "svmc_launch.h"
#include "tiled_lu.h"

#include <algorithm>
#include <vector>

namespace svmc {

// Finds connection number h of the walker (canonical order, conn_mask
// items); one wavefront.  Returns its item e and direction d.
SVMC_DEV bool find_conn(const LatDev& lt, const int8_t* occ_s, int h, int& e_o, int& d_o, int lane) {
  const int items = conn_items(lt);
  int seen = 0;
  for (int base = 0; base < items; base += 64) {
    const int e = base + lane;
    const unsigned valid = e < items ? conn_mask(lt, occ_s, e) : 0u;
    const int cnt = __popc(valid);
    const int incl = wave_incl_scan(cnt, lane);
    const int tot = __shfl(incl, 63, 64);
    if (h < seen + tot) {
      const int excl = seen + incl - cnt;
      const bool mine = h >= excl && h < excl + cnt;
      const unsigned long long b = __ballot(mine);
      const int src = __ffsll((long long)b) - 1;
      int dsel = -1;
      if (mine) {
        unsigned m = valid;
        for (int r = h - excl; r > 0; --r) m &= m - 1;
        dsel = __ffs(m) - 1;
      }
      e_o = __shfl(e, src, 64);
      d_o = __shfl(dsel, src, 64);
      return true;
    }
    seen += tot;
  }
  return false;
}

// E_loc = diagonal term - sum_h amp_h ratio_h, connections in canonical order.
static __global__ void k_full_reduce(LatDev lt, Bufs bf, const double* ratio_tmp, int stride, ElocOut out) {
  const long long wl = blockIdx.x;
  const long long w = lt.w0 + wl;
  const int N = lt.N;
  __shared__ int8_t occ_s[4096];
  const int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  for (int s = threadIdx.x; s < N; s += blockDim.x) occ_s[s] = occ_g[s];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const bool bad = (bf.flags[w] & (1 | 8)) != 0;
  double e = 0.0;
  int hh = 0;
  const int items = conn_items(lt);
  for (int it = 0; it < items; ++it) {
    unsigned m = conn_mask(lt, occ_s, it);
    while (m) {
      const int d = __ffs(m) - 1;
      m &= m - 1;
      const int code = conn_code(lt, it, d);
      const double r = (bad || hh >= stride) ? NAN : ratio_tmp[wl * stride + hh];
      e += -conn_amp(lt, conn_decode(lt, code)) * r;
      if (out.ratio && hh < out.stride) {
        out.ratio[w * out.stride + hh] = r;
        out.code[w * out.stride + hh] = code;
      }
      ++hh;
    }
  }
  out.eloc[w] = bad ? NAN : diag_energy(lt, occ_s) + e;
  if (out.nhops) out.nhops[w] = min(hh, out.stride);
}

// Connections per walker (lattice-local), one wavefront per walker.
static __global__ __launch_bounds__(64) void k_full_count(LatDev lt, Bufs bf, int32_t* cnt) {
  const long long wl = blockIdx.x;
  const int N = lt.N, lane = threadIdx.x;
  const int8_t* occ = bf.occ + lt.occ_off + wl * N;
  int c = 0;
  for (int e = lane; e < conn_items(lt); e += 64) c += __popc(conn_mask(lt, occ, e));
  c = wave_sum_i(c);
  if (lane == 0) cnt[wl] = c;
}

// Configuration g = c0 + blockIdx.x of the listing: walker wl with
// off[wl] <= g < off[wl + 1]; slot g - off[wl] = 0 is the walker's own
// configuration, slot 1 + h its connection h (canonical order).  One
// wavefront.
static __global__ __launch_bounds__(64) void k_full_configs(LatDev lt, Bufs bf, const long long* __restrict__ off,
                                                            long long c0, int8_t* __restrict__ occ_h,
                                                            int32_t* __restrict__ cfg_w, int32_t* __restrict__ cfg_h,
                                                            double* __restrict__ cfg_jw) {
  __shared__ int8_t occ_s[4096];
  const long long g = c0 + blockIdx.x;
  const int N = lt.N, lane = threadIdx.x;
  long long lo = 0, hi = lt.nw;             // largest wl with off[wl] <= g
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (off[mid] <= g) lo = mid; else hi = mid;
  }
  const long long wl = lo;
  const int h = (int)(g - off[wl]) - 1;
  const int8_t* occ = bf.occ + lt.occ_off + wl * N;
  for (int s = lane; s < N; s += 64) occ_s[s] = occ[s];
  __syncthreads();
  double jw = 1.0;
  if (h >= 0) {
    int e = 0, d = 0;
    find_conn(lt, occ_s, h, e, d, lane);
    const Conn cn = conn_decode(lt, conn_code(lt, e, d));
    const int i = cn.i, j = conn_target(lt, i, d);
    // electrons strictly between i and j in site order, of the moving spin
    // (a hop) or of both spins (an exchange: the product of both signs)
    const int a = min(i, j), b = max(i, j), mask = cn.ex ? 3 : 1 << cn.sp;
    int between = 0;
    for (int s = a + 1 + lane; s < b; s += 64) between += __popc(occ_s[s] & mask);
    between = wave_sum_i(between);
    jw = (between & 1) ? -1.0 : 1.0;
    __syncthreads();
    if (lane == 0) {
      if (cn.ex) {
        const int8_t oi = occ_s[i];
        occ_s[i] = occ_s[j];
        occ_s[j] = oi;
      } else {
        occ_s[i] -= (int8_t)(1 << cn.sp);
        occ_s[j] += (int8_t)(1 << cn.sp);
      }
    }
    __syncthreads();
  }
  int8_t* o = occ_h + (long long)blockIdx.x * N;
  for (int s = lane; s < N; s += 64) o[s] = occ_s[s];
  if (lane == 0) {
    cfg_w[blockIdx.x] = (int32_t)wl;
    cfg_h[blockIdx.x] = h;
    cfg_jw[blockIdx.x] = jw;
  }
}

// Both Slater blocks of one configuration, spin tau = blockIdx.y, in
// canonical order (occupied sites ascending): rows base[s] + b + H_L[s] W
// (FP64, sum over channels in order), then log|det| and sign by the
// register-tiled LU with partial pivoting (tiled_lu_det).  H_L of the occupied sites
// ([n][C + 1] in the feature type) and W ([C][n] doubles) are staged in LDS.
template <class Tf, int R>
__global__ __launch_bounds__(256) void k_full_det(LatDev lt, int C, const int8_t* __restrict__ occ_h,
                                                  const Tf* __restrict__ featL, long long feat_stride,
                                                  double* __restrict__ ld_h, double* __restrict__ sg_h) {
  __shared__ GjShared<R> sh;
  __shared__ int wcnt[4];
  extern __shared__ __attribute__((aligned(16))) double fdl[];
  const long long c = blockIdx.x;
  const int tau = blockIdx.y;
  const int N = lt.N, n = lt.n[tau], nm = lt.nmax, HS = C + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* ldo = ld_h + 2 * c + tau;
  double* sgo = sg_h + 2 * c + tau;
  if (n == 0) {
    if (tid == 0) { *ldo = 0.0; *sgo = 1.0; }
    return;
  }
  double* Ws = fdl;                       // [C][n]
  Tf* Hs = (Tf*)(fdl + C * n);            // [n][C + 1]
  int* sites = (int*)(Hs + (long long)n * HS);
  const int8_t* occ = occ_h + c * N;
  // occupied sites of tau in ascending order (block-wide compaction)
  int base_cnt = 0;
  for (int s0 = 0; s0 < N; s0 += 256) {
    const int s = s0 + tid;
    const bool on = s < N && ((occ[s] >> tau) & 1);
    const unsigned long long m = __ballot(on);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
      pre += k < wv ? wcnt[k] : 0;
      tot += wcnt[k];
    }
    const int idx = base_cnt + pre + __popcll(m & ((1ULL << lane) - 1ULL));
    if (on && idx < n) sites[idx] = s;
    base_cnt += tot;
    __syncthreads();
  }
  const bool bad = base_cnt != n;         // wrong electron count: psi = 0
  const double* Wg = lt.W + (long long)tau * C * nm;
  for (int e = tid; e < C * n; e += 256) {
    const int cc = e / n, m = e - cc * n;
    Ws[e] = Wg[(long long)cc * nm + m];
  }
  const Tf* F = featL + c * feat_stride;
  for (int e = tid; e < n * C; e += 256) {
    const int k = e / C, cc = e - k * C;
    Hs[k * HS + cc] = bad ? Tf(0) : F[(long long)sites[k] * C + cc];
  }
  __syncthreads();
  const int tx = tid >> 4, ty = tid & 15;
  const double* base = lt.base + (long long)tau * N * nm;
  const double* bb = lt.b + tau * nm;
  double x[R][R];
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int k = ty + 16 * a, m = tx + 16 * b;
      x[a][b] = (k < n && m < n) ? base[(long long)(bad ? 0 : sites[k]) * nm + m] + bb[m] : (k == m ? 1.0 : 0.0);
    }
  for (int cc = 0; cc < C; ++cc) {
    double h[R], w[R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int k = ty + 16 * a;
      h[a] = k < n ? (double)Hs[k * HS + cc] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int m = tx + 16 * b;
      w[b] = m < n ? Ws[cc * n + m] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) x[a][b] = fma(h[a], w[b], x[a][b]);
  }
  double la, sg;
  bool sing;
  tiled_lu_det<R>(x, n, sh, la, sg, sing);
  if (tid == 0) {
    *ldo = (sing || bad) ? -INFINITY : la;
    *sgo = (sing || bad) ? 0.0 : sg;
  }
}

// pass 0: each walker's own configuration -> its log|psi| and sign;
// pass 1: every hop configuration -> ratio with the moving electron keeping
// its row, JW sign times psi(n')/psi(n) in canonical order.
static __global__ void k_full_post(int pass, int nc, const int32_t* __restrict__ cfg_w,
                                   const int32_t* __restrict__ cfg_h, const double* __restrict__ cfg_jw,
                                   const double* __restrict__ ld_h, const double* __restrict__ sg_h,
                                   double* __restrict__ ref, double* __restrict__ ratio, int stride) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  const long long wl = cfg_w[k];
  const int h = cfg_h[k];
  const double l = ld_h[2 * k] + ld_h[2 * k + 1], s = sg_h[2 * k] * sg_h[2 * k + 1];
  if (pass == 0) {
    if (h < 0) {
      ref[2 * wl] = l;
      ref[2 * wl + 1] = s;
    }
  } else if (h >= 0 && h < stride) {
    const double s0 = ref[2 * wl + 1], l0 = ref[2 * wl];
    ratio[wl * stride + h] = s == 0.0 ? 0.0 : cfg_jw[k] * s * s0 * exp(l - l0);
  }
}

// bytes per configuration of a chunk; L = feature planes per configuration
size_t full_config_bytes(const LatDev& lt, int L, int C, int tfb) {
  size_t b = (size_t)lt.N + (size_t)(L + 1) * lt.N * C * tfb + 4 * sizeof(double) + 16;
  if (lt.nmax > 128)
    b += 2ULL * lt.N * lt.nmax * 8 + 2ULL * lt.nmax * lt.nmax * 8 + 4ULL * lt.N + 4ULL * lt.nmax + 8;
  return b;
}

hipError_t launch_eloc_full(int prec, const ModelDev& md, const LatDev& lt, const Bufs& bf, const ElocOut& out,
                            double* ratio_tmp, int stride, const FullScratch& fs, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  if (lt.N > 4096 || lt.nmax > 512) return hipErrorInvalidValue;
  hipError_t e;
  const int L = feat_planes(md), C = md.C, N = lt.N;   // L: feature planes, the last feeds the rows
  const int tfb = prec == PREC_F64 ? 8 : 4;
  // hop counts -> configuration offsets (host prefix sum)
  hipLaunchKernelGGL(k_full_count, dim3((unsigned)lt.nw), dim3(64), 0, st, lt, bf, fs.cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<int32_t> cnt((size_t)lt.nw);
  if ((e = hipMemcpyAsync(cnt.data(), fs.cnt, cnt.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  std::vector<long long> off((size_t)lt.nw + 1, 0);
  for (long long w = 0; w < lt.nw; ++w) off[w + 1] = off[w] + 1 + cnt[w];
  if ((e = hipMemcpyAsync(fs.off, off.data(), off.size() * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
  const long long total = off[lt.nw];
  const long long chunk = fs.chunk;
  // view of a chunk of configurations as a batch of walkers
  LatDev v = lt;
  v.w0 = 0;
  v.occ_off = v.lab_off = v.pos_off = v.feat_off = v.inv_off = v.m_off = v.g_off = v.pt_off = 0;
  Bufs b = bf;
  b.occ = fs.occ;
  b.feat = fs.feat;
  b.lab = fs.lab;
  b.pos = fs.pos;
  b.M = fs.M;
  b.inv = fs.inv;
  b.ld = fs.ld;
  b.sg = fs.sg;
  b.flags = fs.flags;
  b.nacc = fs.nacc;
  b.G = nullptr;
  b.PT = nullptr;
  double* ratio = ratio_tmp;
  for (long long c0 = 0; c0 < total; c0 += chunk) {
    const int nc = (int)std::min(chunk, total - c0);
    v.nw = nc;
    hipLaunchKernelGGL(k_full_configs, dim3((unsigned)nc), dim3(64), 0, st, lt, bf, fs.off, c0, fs.occ, fs.cfg_w,
                       fs.cfg_h, fs.cfg_jw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_forward(prec, v, b, md, fs.h0, st)) != hipSuccess) return e;
    if (lt.nmax <= 128) {
      const int R = (lt.nmax + 15) / 16;
      const long long fstr = (long long)L * N * C;
      const size_t smem = (size_t)C * lt.nmax * 8 + (size_t)lt.nmax * (C + 1) * tfb + (size_t)lt.nmax * 4 + 16;
      const dim3 grid((unsigned)nc, 2);
      auto go = [&](auto kern, const auto* fl) {
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(kern, grid, dim3(256), smem, st, lt, C, fs.occ, fl + (long long)(L - 1) * N * C, fstr,
                             fs.ld, fs.sg);
          e = hipGetLastError();
        }
      };
#define SVMC_FD(R_)                                                                                 \
  case R_:                                                                                          \
    if (tfb == 8) go(k_full_det<double, R_>, (const double*)fs.feat);                               \
    else go(k_full_det<float, R_>, (const float*)fs.feat);                                          \
    break;
      switch (R) {
        SVMC_FD(1) SVMC_FD(2) SVMC_FD(3) SVMC_FD(4) SVMC_FD(5) SVMC_FD(6) SVMC_FD(7) SVMC_FD(8)
        default: return hipErrorInvalidValue;
      }
#undef SVMC_FD
      if (e != hipSuccess) return e;
    } else {
      // the cold-setup kernels on the chunk: labels (ascending order),
      // rows of every site, global-memory Gauss-Jordan -> log|det|, sign
      if ((e = launch_labels(v, b, st)) != hipSuccess) return e;
      if ((e = launch_rows(prec, v, b, L, C, st)) != hipSuccess) return e;
      if ((e = launch_gj(v, b, st)) != hipSuccess) return e;
    }
    const unsigned nb = (unsigned)((nc + 255) / 256);
    hipLaunchKernelGGL(k_full_post, dim3(nb), dim3(256), 0, st, 0, nc, fs.cfg_w, fs.cfg_h, fs.cfg_jw, fs.ld, fs.sg,
                       fs.ref, ratio, stride);
    hipLaunchKernelGGL(k_full_post, dim3(nb), dim3(256), 0, st, 1, nc, fs.cfg_w, fs.cfg_h, fs.cfg_jw, fs.ld, fs.sg,
                       fs.ref, ratio, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_full_reduce, dim3((unsigned)lt.nw), dim3(256), 0, st, lt, bf, ratio_tmp, stride, out);
  return hipGetLastError();
}

}  // namespace svmc
