// Full-recompute local energies: the O(N^4)-per-sweep comparison scheme
// (Sec. III.A, global architectures: every connected configuration is
// re-evaluated from scratch).  Same inputs and precision policy as the
// low-rank path: conv stack on MFMA in the conv precision (same conv tile),
// orbital rows and determinants in FP64.
//
// One workgroup per (walker, hop): the whole lattice's features of the new
// configuration live in LDS, rows of both Slater blocks are built in
// registers and factorised by the tiled LU; the ratio of determinants (moving
// electron keeps its row) goes to ratio_tmp, and a second kernel sums the
// local energy per walker in canonical hop order.
#include "hop.h"
#include "svmc_launch.h"
#include "tiled_lu.h"

namespace svmc {

// Finds hop number h of the walker (canonical order); wave 0 only.
SVMC_DEV bool find_hop(const LatDev& lt, const int8_t* occ_s, int h, int& sp_o, int& i_o, int& d_o, int lane) {
  const int N = lt.N, nd = lt.nd;
  int seen = 0;
  for (int base = 0; base < 2 * N; base += 64) {
    const int e = base + lane;
    int cnt = 0;
    unsigned valid = 0;
    if (e < 2 * N) {
      const int sp = e / N, i = e % N;
      if ((occ_s[i] >> sp) & 1) {
        const int xi = i % lt.Lx, yi = i / lt.Lx;
        for (int d = 0; d < nd; ++d) {
          int x = xi + dir_dx(d), y = yi + dir_dy(d);
          if (lt.pbc_x) x = imod(x, lt.Lx); else if (x < 0 || x >= lt.Lx) continue;
          if (lt.pbc_y) y = imod(y, lt.Ly); else if (y < 0 || y >= lt.Ly) continue;
          if ((occ_s[x + lt.Lx * y] >> sp) & 1) continue;
          valid |= 1u << d;
          ++cnt;
        }
      }
    }
    const int incl = wave_incl_scan(cnt, lane);
    const int tot = __shfl(incl, 63, 64);
    if (h < seen + tot) {
      const int excl = seen + incl - cnt;
      const bool mine = h >= excl && h < excl + cnt;
      const unsigned long long b = __ballot(mine);
      const int src = __ffsll((long long)b) - 1;
      int dsel = -1;
      if (mine) {
        int r = h - excl;
        for (int d = 0; d < 8; ++d)
          if ((valid >> d) & 1) {
            if (r == 0) { dsel = d; break; }
            --r;
          }
      }
      const int e_src = __shfl(e, src, 64);
      d_o = __shfl(dsel, src, 64);
      sp_o = e_src / N;
      i_o = e_src % N;
      return true;
    }
    seen += tot;
  }
  return false;
}

// E_loc = U * doubles - sum_h t_h ratio_h, hops in canonical order.
static __global__ void k_full_reduce(LatDev lt, Bufs bf, const double* ratio_tmp, int stride, ElocOut out) {
  const long long wl = blockIdx.x;
  const long long w = lt.w0 + wl;
  const int N = lt.N, nd = lt.nd;
  __shared__ int8_t occ_s[4096];
  const int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  for (int s = threadIdx.x; s < N; s += blockDim.x) occ_s[s] = occ_g[s];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const bool bad = (bf.flags[w] & (1 | 8)) != 0;
  double e = 0.0;
  int ndbl = 0;
  for (int s = 0; s < N; ++s) ndbl += occ_s[s] == 3;
  int hh = 0;
  for (int sp = 0; sp < 2; ++sp)
    for (int i = 0; i < N; ++i) {
      if (!((occ_s[i] >> sp) & 1)) continue;
      const int xi = i % lt.Lx, yi = i / lt.Lx;
      for (int d = 0; d < nd; ++d) {
        int x = xi + dir_dx(d), y = yi + dir_dy(d);
        if (lt.pbc_x) x = imod(x, lt.Lx); else if (x < 0 || x >= lt.Lx) continue;
        if (lt.pbc_y) y = imod(y, lt.Ly); else if (y < 0 || y >= lt.Ly) continue;
        if ((occ_s[x + lt.Lx * y] >> sp) & 1) continue;
        const double r = (bad || hh >= stride) ? NAN : ratio_tmp[wl * stride + hh];
        e += -(d < 4 ? lt.t : lt.tp) * r;
        if (out.ratio && hh < out.stride) {
          out.ratio[w * out.stride + hh] = r;
          out.code[w * out.stride + hh] = (i << 4) | (sp << 3) | d;
        }
        ++hh;
      }
    }
  out.eloc[w] = bad ? NAN : lt.U * ndbl + e;
  if (out.nhops) out.nhops[w] = min(hh, out.stride);
}

#ifdef SVMC_INST_P
template <int P, int C, int R, int TPW>
__global__ __launch_bounds__(256) void k_full_ratio(ModelDev md, LatDev lt, Bufs bf, double* ratio_tmp,
                                                    int stride) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ GjShared<R> sh;
  __shared__ int s_hop[4];
  const long long wl = blockIdx.y;
  const long long w = lt.w0 + wl;
  const int h = blockIdx.x;
  const int N = lt.N, nm = lt.nmax, Lx = lt.Lx;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (bf.flags[w] & (1 | 8)) return;
  constexpr int SP = SiteStride<Tf, C>::value;            // padded site stride
  Tf* grid = (Tf*)smem;                                    // [N][SP]
  int8_t* occ_s = (int8_t*)(smem + (size_t)N * SP * sizeof(Tf));
  double* wlds = (double*)(smem + (size_t)N * SP * sizeof(Tf) + ((N + 15) & ~15));   // [C][nmax]
  const int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  for (int s = tid; s < N; s += 256) occ_s[s] = occ_g[s];
  __syncthreads();
  if (wv == 0) {
    int sp = 0, i = 0, d = 0;
    const bool ok = find_hop(lt, occ_s, h, sp, i, d, lane);
    if (lane == 0) { s_hop[0] = ok; s_hop[1] = sp; s_hop[2] = i; s_hop[3] = d; }
  }
  __syncthreads();
  if (!s_hop[0]) return;
  const int sp = s_hop[1], i = s_hop[2], d = s_hop[3];
  const HopGeom g = hop_geom(lt, md.L, sp, i, d);
  const int bit = 1 << sp;
  __syncthreads();
  if (tid == 0) { occ_s[i] -= bit; occ_s[g.j] += bit; }
  __syncthreads();
  // H'_0
  const Tf* E = (const Tf*)md.embed;
  for (int e = tid; e < N * C; e += 256)
    grid[(e / C) * SP + (e % C)] = E[lt.emb_off + (long long)(e / C) * lt.emb_ss + occ_s[e / C] * C + (e % C)];
  __syncthreads();
  const int T = (N + 15) >> 4;
  for (int l = 0; l < md.L; ++l) {
    const Tb* Bl = (const Tb*)md.Bpack + (long long)l * CC::Q * CC::NT * 64;
    Acc acc[TPW][CC::NT];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wv + 4 * q;
      if (t < T) {
        const int m = 16 * t + (lane & 15);
        const int x = m % Lx, y = m / Lx;
        int nb[9];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
          int xx = x + (tp % 3) - 1, yy = y + (tp / 3) - 1;
          bool ok = m < N;
          if (lt.pbc_x) xx = imod(xx, Lx); else ok = ok && xx >= 0 && xx < Lx;
          if (lt.pbc_y) yy = imod(yy, lt.Ly); else ok = ok && yy >= 0 && yy < lt.Ly;
          nb[tp] = ok ? (xx + Lx * yy) * SP : -1;
        }
        conv_tile<P, C>(grid, nb, Bl, lane, acc[q]);
      }
    }
    const Tf* bias = (const Tf*)md.bias + l * C;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wv + 4 * q;
      if (t < T) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + OutMap<P>::site(lane, v);
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            if (r < N && n < C) acc[q][nt][v] = layer_out<P, Tf>(md.act, grid[r * SP + n], acc[q][nt][v] + bias[n]);
          }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wv + 4 * q;
      if (t < T) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + OutMap<P>::site(lane, v);
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            if (r < N && n < C) grid[r * SP + n] = acc[q][nt][v];
          }
      }
    }
    __syncthreads();
  }
  // determinants of both new Slater blocks, rows in label order with the
  // moving electron keeping its label
  const int16_t* posg = bf.pos + lt.pos_off + wl * 2LL * nm;
  const int16_t* labg = bf.lab + lt.lab_off + wl * 2LL * N;
  const int kmove = labg[sp * N + i];
  const int tx = tid >> 4, ty = tid & 15;
  double dlog = 0.0, dsign = 1.0;
  bool zero = false;
  for (int tau = 0; tau < 2; ++tau) {
    const int n = lt.n[tau];
    if (n == 0) continue;
    const double* base = lt.base + (long long)tau * N * nm;
    const double* Wg = lt.W + (long long)tau * C * nm;
    const double* b = lt.b + tau * nm;
    // this spin's projection W [C][n] into LDS (after the feature grid)
    double* W = wlds;
    for (int e = tid; e < C * n; e += 256) {
      const int c = e / n, m = e - c * n;
      W[c * n + m] = Wg[(long long)c * nm + m];
    }
    __syncthreads();
    double x[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a) {
      const int k = ty + 16 * a;
      int site = 0;
      if (k < n) site = (tau == sp && k == kmove) ? g.j : posg[tau * nm + k];
      const Tf* hl = grid + site * SP;
#pragma unroll
      for (int bb = 0; bb < R; ++bb) {
        const int m = tx + 16 * bb;
        double v;
        if (k < n && m < n) {
          v = base[(long long)site * nm + m] + b[m];
          for (int c = 0; c < C; ++c) v = fma((double)hl[c], W[c * n + m], v);
        } else {
          v = (k == m) ? 1.0 : 0.0;
        }
        x[a][bb] = v;
      }
    }
    double la, sg;
    bool sing;
    tiled_gj<R, false>(x, n, sh, la, sg, sing);
    if (sing) { zero = true; break; }
    dlog += la - bf.ld[2 * w + tau];
    dsign *= sg * bf.sg[2 * w + tau];
    __syncthreads();
  }
  if (tid == 0) ratio_tmp[wl * stride + h] = zero ? 0.0 : dsign * exp(dlog);
}

template <int P, int C, int R>
static hipError_t full_impl(const ModelDev& md, const LatDev& lt, const Bufs& bf, const ElocOut& out,
                            double* ratio_tmp, int stride, hipStream_t st) {
  typedef typename PrecT<P>::Tf Tf;
  const size_t smem = (size_t)lt.N * SiteStride<Tf, C>::value * sizeof(Tf) + ((lt.N + 15) & ~15) +
                      (size_t)C * lt.nmax * sizeof(double);
  auto kern = k_full_ratio<P, C, R, 4>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  // walkers in chunks so that grid.y stays below 65536
  for (long long w0 = 0; w0 < lt.nw; w0 += 32768) {
    LatDev part = lt;
    part.w0 = lt.w0 + w0;
    part.nw = std::min<long long>(32768, lt.nw - w0);
    part.occ_off = lt.occ_off + w0 * lt.N;
    part.lab_off = lt.lab_off + w0 * 2LL * lt.N;
    part.pos_off = lt.pos_off + w0 * 2LL * lt.nmax;
    hipLaunchKernelGGL(kern, dim3((unsigned)lt.maxhops, (unsigned)part.nw), dim3(256), smem, st, md, part, bf,
                       ratio_tmp + w0 * stride, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_full_reduce, dim3((unsigned)lt.nw), dim3(256), 0, st, lt, bf, ratio_tmp, stride, out);
  return hipGetLastError();
}

hipError_t SVMC_CAT3(eloc_full_, SVMC_INST_P, SVMC_INST_C)(const ModelDev& md, const LatDev& lt, const Bufs& bf,
                                                           const ElocOut& out, double* ratio_tmp, int stride,
                                                           hipStream_t st) {
  if (lt.nmax <= 16) return full_impl<SVMC_INST_P, SVMC_INST_C, 1>(md, lt, bf, out, ratio_tmp, stride, st);
  if (lt.nmax <= 32) return full_impl<SVMC_INST_P, SVMC_INST_C, 2>(md, lt, bf, out, ratio_tmp, stride, st);
  if (lt.nmax <= 64) return full_impl<SVMC_INST_P, SVMC_INST_C, 4>(md, lt, bf, out, ratio_tmp, stride, st);
  return full_impl<SVMC_INST_P, SVMC_INST_C, 8>(md, lt, bf, out, ratio_tmp, stride, st);
}
#else
hipError_t launch_eloc_full(int prec, const ModelDev& md, const LatDev& lt, const Bufs& bf, const ElocOut& out,
                            double* ratio_tmp, int stride_tmp, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  if (lt.N > 256 || lt.nmax > 128 || lt.N > 4096) return hipErrorInvalidValue;
#define SVMC_FU(P_, C_) \
  if (prec == P_ && md.C == C_) return eloc_full_##P_##_##C_(md, lt, bf, out, ratio_tmp, stride_tmp, st);
  SVMC_FOR_EACH_PREC_C(SVMC_FU)
#undef SVMC_FU
  return hipErrorInvalidValue;
}

#endif

}  // namespace svmc
