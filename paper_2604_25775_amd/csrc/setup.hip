// Walker set-up and FP64 refresh kernels:
//   labels      occupation -> electron labels (ascending sites) and site->label
//   embed       H_0 = E_s[n_s]                   (Sec. II.B, embedding layer; one
//                                                table for all sites or one per site)
//   forward     H_l = H_{l-1} + act(conv(H_{l-1}))  one launch per layer
//               (Sec. II.B, residual conv equation)
//   rows        M_s[x] = base_s[x] + H_L[x] W_s + b_s for every site
//               (Sec. II.B, orbital projection)
//   gj          Phi_s = M_s[pos], FP64 Gauss-Jordan inverse with partial
//               pivoting, log|det|, sign
//   gp          G_s = M_s Phi_s^-1 and P_s^T = (W_s Phi_s^-1)^T, the two
//               factors every low-rank ratio reads (Sec. II.C, SMW equations)
//   logpsi      canonical sign and log|psi| per walker
#include "svmc_dev.h"
#include "svmc_launch.h"
#include "tiled_lu.h"
#include "hop.h"

namespace svmc {

#ifdef SVMC_INST_P
template <class Tf>
__global__ void k_embed(LatDev lt, Bufs bf, ModelDev md, Tf* __restrict__ h0) {
  const int C = md.C;
  const long long total = lt.nw * (long long)lt.N * C;
  const Tf* E = (const Tf*)md.embed;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long site = e / C;
    const int c = (int)(e % C);
    const int o = bf.occ[lt.occ_off + site] & 3;
    const int s = (int)(site % lt.N);
    h0[e] = E[lt.emb_off + (long long)s * lt.emb_ss + o * C + c];
  }
}

// One conv layer over every site of every walker of a lattice.  Block = 4
// waves; each wave takes FWD_TPW consecutive 16-site tiles of one walker
// (the tiles of a lattice are dealt to the waves of a row of blocks), so the
// layer's weight fragments are loaded once per wave and reused.  src =
// H_{l-1} ([nw][N][C]), dst = H_l.
constexpr int FWD_TPW = 4;
template <int P, int C>
__global__ __launch_bounds__(256) void k_forward_layer(LatDev lt, ModelDev md, int layer,
                                                       const typename PrecT<P>::Tf* __restrict__ src,
                                                       long long src_stride,
                                                       typename PrecT<P>::Tf* __restrict__ dst,
                                                       long long dst_stride) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  const int lane = threadIdx.x & 63;
  const int tile0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * FWD_TPW;
  const long long wl = blockIdx.y;
  const int N = lt.N;
  if (tile0 * 16 >= N) return;
  const Tf* S = src + wl * src_stride;
  Tf* D = dst + wl * dst_stride;
  const Tb* Bl = (const Tb*)md.Bpack + (long long)layer * CC::Q * CC::NT * 64;
  const Tf* bias = (const Tf*)md.bias + layer * C;
  // the layer's weight fragments in registers when they fit (16-bit modes),
  // else read per tile
  constexpr bool RB = CC::Q * CC::NT * (int)sizeof(Tb) <= 80 * 4;
  Tb breg[RB ? CC::Q : 1][CC::NT];
  if constexpr (RB) {
#pragma unroll
    for (int q = 0; q < CC::Q; ++q)
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) breg[q][nt] = Bl[(q * CC::NT + nt) * 64 + lane];
  }
  for (int tt = 0; tt < FWD_TPW; ++tt) {
    const int tile = tile0 + tt;
    if (tile * 16 >= N) break;
    const int m = tile * 16 + (lane & 15);
    int nb[9];
    {
      const int x = m % lt.Lx, y = m / lt.Lx;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        int xx = x + (t % 3) - 1, yy = y + (t / 3) - 1;
        bool ok = m < N;
        if (lt.pbc_x) xx = imod(xx, lt.Lx); else ok = ok && xx >= 0 && xx < lt.Lx;
        if (lt.pbc_y) yy = imod(yy, lt.Ly); else ok = ok && yy >= 0 && yy < lt.Ly;
        nb[t] = ok ? (xx + lt.Lx * yy) * C : -1;
      }
    }
    Acc acc[CC::NT];
    if constexpr (RB) conv_tile_regb<P, C>(S, nb, breg, lane, acc);
    else conv_tile<P, C>(S, nb, Bl, lane, acc);
#pragma unroll
    for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = tile * 16 + OutMap<P>::site(lane, v);
        const int n = nt * 16 + OutMap<P>::chan(lane, v);
        if (r < N && n < C) {
          const Tf z = acc[nt][v] + bias[n];
          D[(long long)r * C + n] = layer_out<P, Tf>(md.act, S[(long long)r * C + n], z);
        }
      }
  }
}

// Every layer of the forward for one walker per workgroup, the lattice in
// LDS.  The LDS grid is the lattice with a one-site halo, (Lx + 2) x (Ly + 2)
// records of the incremental grid's layout (FP16-pair planes in F16X2):
// halo records repeat the opposite edge on periodic axes and hold zeros on
// open ones, so each conv tap of a site is a fixed record offset
// (conv_tile_win).  Per layer the waves convolve their tiles, form
// H_l = H_{l-1} + act(z + b) (layer_out, the same arithmetic as
// k_forward_layer), hold it in registers over a barrier, then write it over
// the layer input (with its halo copies) and to the feature cache.
constexpr int FUSED_MAXT = 6;             // tiles per wave: N <= 4 * 16 * 6 sites
template <int P, int C>
__global__ __launch_bounds__(256) void k_forward_fused(LatDev lt, Bufs bf, ModelDev md) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  constexpr int SP = SiteStride<Tf, C>::value;
  constexpr bool PL = GridPlanes<P>::value;
  constexpr int V = 16 / (int)sizeof(Tf), CV = C / V;
  constexpr int RV = SP * (int)sizeof(Tf) / 16;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  Tf* grid = (Tf*)smem;
  const long long wl = blockIdx.x;
  const int N = lt.N, Lx = lt.Lx, Ly = lt.Ly, GX = Lx + 2, GG = GX * (Ly + 2), L = md.L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int8_t* occ = bf.occ + lt.occ_off + wl * N;
  Tf* featw = (Tf*)bf.feat + lt.feat_off + wl * (long long)feat_planes(md) * N * C;
  // records of site s: itself and its halo copies (periodic axes)
  auto records = [&](int s, int (&r)[4]) -> int {
    const int x = s % Lx, y = s / Lx;
    const int X = x + 1, Y = y + 1;
    const int X2 = lt.pbc_x ? (x == 0 ? Lx + 1 : (x == Lx - 1 ? 0 : -1)) : -1;
    const int Y2 = lt.pbc_y ? (y == 0 ? Ly + 1 : (y == Ly - 1 ? 0 : -1)) : -1;
    int k = 0;
    r[k++] = Y * GX + X;
    if (X2 >= 0) r[k++] = Y * GX + X2;
    if (Y2 >= 0) r[k++] = Y2 * GX + X;
    if (X2 >= 0 && Y2 >= 0) r[k++] = Y2 * GX + X2;
    return k;
  };
  for (int e = tid; e < GG * RV; e += 256) reinterpret_cast<float4*>(grid)[e] = float4{0.0f, 0.0f, 0.0f, 0.0f};
  __syncthreads();
  // layer-0 input: the embedding of each site's occupation
  const Tf* E = (const Tf*)md.embed;
  for (int e = tid; e < N * CV; e += 256) {
    const int s = e / CV, cv = e - s * CV;
    const int o = occ[s] & 3;
    const float4 v = *reinterpret_cast<const float4*>(E + lt.emb_off + (long long)s * lt.emb_ss + o * C + cv * V);
    int r[4];
    const int k = records(s, r);
    for (int u = 0; u < k; ++u) {
      if constexpr (PL) grid_put4<P, C>(grid, r[u], cv * V, v);
      else *reinterpret_cast<float4*>(grid + r[u] * SP + cv * V) = v;
    }
  }
  __syncthreads();
  const int T = (N + 15) >> 4;
  const Tf* bias = (const Tf*)md.bias;
  for (int l = 1; l <= L; ++l) {
    const Tb* Bl = (const Tb*)md.Bpack + (long long)(l - 1) * CC::Q * CC::NT * 64;
    constexpr int QB = RegB<P, C>::value ? CC::Q : 1;
    Tb breg[QB][CC::NT];
    if constexpr (RegB<P, C>::value) {
#pragma unroll
      for (int q = 0; q < CC::Q; ++q)
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt) breg[q][nt] = Bl[(q * CC::NT + nt) * 64 + lane];
    }
    Acc acc[FUSED_MAXT][CC::NT];
    int cenr[FUSED_MAXT];
#pragma unroll
    for (int ti = 0; ti < FUSED_MAXT; ++ti) {
      const int t = wave + 4 * ti;
      if (t >= T) break;
      const int m = 16 * t + (lane & 15);
      const int mm = m < N ? m : N - 1;             // padding rows compute from a real site
      const int cen = (mm / Lx + 1) * GX + (mm % Lx + 1);
      cenr[ti] = cen;
      conv_tile_win<P, C>(grid, GX, cen, breg, Bl, lane, acc[ti]);
    }
#pragma unroll
    for (int ti = 0; ti < FUSED_MAXT; ++ti) {
      const int t = wave + 4 * ti;
      if (t >= T) break;
      const Tf* rec = grid + cenr[ti] * SP;
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = 16 * nt + OutMap<P>::chan(lane, v);
          if (n >= C) continue;
          Tf xres;
          if constexpr (PL) {
            float x4[4];
            planes_get4<C>(reinterpret_cast<const char*>(rec), 16 * nt + OutMap<P>::chan(lane, 0), x4);
            xres = x4[v];
          } else {
            xres = rec[n];
          }
          const Tf z = acc[ti][nt][v] + bias[(l - 1) * C + n];
          acc[ti][nt][v] = layer_out<P, Tf>(md.act, xres, z);
        }
    }
    __syncthreads();
#pragma unroll
    for (int ti = 0; ti < FUSED_MAXT; ++ti) {
      const int t = wave + 4 * ti;
      if (t >= T) break;
      const int m = 16 * t + (lane & 15);
      if (m >= N) continue;
      int r[4];
      const int k = records(m, r);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) {
        if constexpr (PL) {
          const int n0 = 16 * nt + OutMap<P>::chan(lane, 0);
          if (n0 >= C) continue;
          const float4 v4 = {acc[ti][nt][0], acc[ti][nt][1], acc[ti][nt][2], acc[ti][nt][3]};
          for (int u = 0; u < k; ++u) grid_put4<P, C>(grid, r[u], n0, v4);
          *reinterpret_cast<float4*>(featw + ((long long)(l - 1) * N + m) * C + n0) = v4;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            if (n >= C) continue;
            for (int u = 0; u < k; ++u) grid[r[u] * SP + n] = acc[ti][nt][v];
            featw[((long long)(l - 1) * N + m) * C + n] = acc[ti][nt][v];
          }
        }
      }
    }
    __syncthreads();
  }
}

// One site-wise layer m (Sec. II.B, site-wise MLP equation) over every site
// of every walker of a lattice: dst = act(src W_m + b_m) per site, no
// residual, rounded like every cached feature.  One wavefront per 16-site
// tile, four per block; blockIdx.y = walker.  src / dst: planes of the
// feature cache (walker stride `stride`).
template <int P, int C>
__global__ __launch_bounds__(256) void k_mlp_layer(LatDev lt, ModelDev md, int m,
                                                   const typename PrecT<P>::Tf* __restrict__ src,
                                                   typename PrecT<P>::Tf* __restrict__ dst, long long stride) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef MlpCfg<P, C> MC;
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int N = lt.N;
  if (tile * 16 >= N) return;
  const long long wl = blockIdx.y;
  const Tf* S = src + wl * stride;
  Tf* D = dst + wl * stride;
  const Tb* Bm = (const Tb*)md.Bmlp + (long long)m * MC::Q * MC::NT * 64;
  const Tf* bias = (const Tf*)md.bias + (long long)(md.L + m) * C;
  const int s = tile * 16 + (lane & 15);
  typename PrecT<P>::Acc acc[MC::NT];
  mlp_tile<P, C>(s < N ? S + (long long)s * C : nullptr, Bm, lane, acc);
  if (s >= N) return;
#pragma unroll
  for (int nt = 0; nt < MC::NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = 16 * nt + OutMap<P>::chan(lane, v);
      if (n < C) D[(long long)s * C + n] = mlp_out<P, Tf>(md.act, Tf(acc[nt][v] + bias[n]));
    }
}

template <int P, int C>
static hipError_t mlp_layers(const LatDev& lt, const Bufs& bf, const ModelDev& md, hipStream_t st) {
  typedef typename PrecT<P>::Tf Tf;
  const long long NC = (long long)lt.N * C, fs = (long long)feat_planes(md) * NC;
  Tf* feat = (Tf*)bf.feat + lt.feat_off;
  const dim3 grid((unsigned)((lt.N + 63) / 64), (unsigned)lt.nw);
  for (int m = 0; m < md.M; ++m)
    hipLaunchKernelGGL((k_mlp_layer<P, C>), grid, dim3(256), 0, st, lt, md, m,
                       feat + (long long)(md.L - 1 + m) * NC, feat + (long long)(md.L + m) * NC, fs);
  return hipGetLastError();
}

template <int P, int C>
size_t fused_smem(const LatDev& lt) {
  typedef typename PrecT<P>::Tf Tf;
  return (size_t)(lt.Lx + 2) * (lt.Ly + 2) * SiteStride<Tf, C>::value * sizeof(Tf);
}

template <int P, int C>
static hipError_t forward_impl(const LatDev& lt, const Bufs& bf, const ModelDev& md, void* h0tmp,
                               hipStream_t st) {
  typedef typename PrecT<P>::Tf Tf;
  if (lt.nw == 0) return hipSuccess;
  const size_t fsm = fused_smem<P, C>(lt);
  if (fsm <= 64 * 1024 && (lt.N + 15) / 16 <= 4 * FUSED_MAXT) {
    auto kern = k_forward_fused<P, C>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fsm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)lt.nw), dim3(256), fsm, st, lt, bf, md);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return mlp_layers<P, C>(lt, bf, md, st);
  }
  const long long NC = (long long)lt.N * C;
  Tf* h0 = (Tf*)h0tmp;
  hipLaunchKernelGGL(k_embed<Tf>, dim3(4096), dim3(256), 0, st, lt, bf, md, h0);
  Tf* feat = (Tf*)bf.feat + lt.feat_off;
  const long long fs = (long long)feat_planes(md) * NC;
  const dim3 grid((unsigned)((lt.N + 64 * FWD_TPW - 1) / (64 * FWD_TPW)), (unsigned)lt.nw);
  for (int l = 0; l < md.L; ++l) {
    const Tf* src = l == 0 ? h0 : feat + (long long)(l - 1) * NC;
    const long long ss = l == 0 ? NC : fs;
    hipLaunchKernelGGL((k_forward_layer<P, C>), grid, dim3(256), 0, st, lt, md, l, src, ss,
                       feat + (long long)l * NC, fs);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_layers<P, C>(lt, bf, md, st);
}

hipError_t SVMC_CAT3(forward_, SVMC_INST_P, SVMC_INST_C)(const LatDev& lt, const Bufs& bf, const ModelDev& md,
                                                         void* h0tmp, hipStream_t st) {
  return forward_impl<SVMC_INST_P, SVMC_INST_C>(lt, bf, md, h0tmp, st);
}
#else
__global__ void k_labels(LatDev lt, Bufs bf) {
  const long long wl = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (wl >= lt.nw) return;
  const int N = lt.N, nm = lt.nmax;
  const int8_t* occ = bf.occ + lt.occ_off + wl * N;
  int16_t* lab = bf.lab + lt.lab_off + wl * 2 * N;
  int16_t* pos = bf.pos + lt.pos_off + wl * 2 * nm;
  int cnt[2] = {0, 0};
  for (int s = 0; s < N; ++s) {
    const int o = occ[s];
    for (int sp = 0; sp < 2; ++sp) {
      if ((o >> sp) & 1) {
        if (cnt[sp] < nm) pos[sp * nm + cnt[sp]] = (int16_t)s;
        lab[sp * N + s] = (int16_t)cnt[sp];
        ++cnt[sp];
      } else {
        lab[sp * N + s] = -1;
      }
    }
  }
  for (int sp = 0; sp < 2; ++sp)
    for (int k = cnt[sp]; k < nm; ++k) pos[sp * nm + k] = -1;
  bool bad = cnt[0] != lt.n[0] || cnt[1] != lt.n[1];
  for (int s = 0; s < N; ++s) bad |= (occ[s] < 0 || occ[s] > 3 || (lt.tj && occ[s] == 3));
  const long long w = lt.w0 + wl;
  bf.flags[w] = bad ? 8 : 0;
  bf.nacc[w] = 0;
}

// M_s[x][m] = base_s[x][m] + sum_c H_L[x][c] W_s[c][m] + b_s[m] (zero for
// m >= n_s) on the FP64 matrix cores: one workgroup of four wavefronts per
// (walker, spin), wavefront w taking the 16-row tiles w, w + 4, ...; the W_s
// fragments of RC_CT column tiles stay in registers while the wavefront runs
// over its row tiles.  16 x 16 x 4 tiles: A[i][k] = H_L[16 ti + i][4 q + k]
// from lane i + 16 k, B[k][j] = W_s[4 q + k][16 tj + j] from lane j + 16 k,
// result row 4 v + l / 16, column l % 16 in slot v of lane l.
constexpr int RC_CT = 4;
template <class Tf, int KS>
SVMC_DEV void rows_one(const LatDev& lt, const Bufs& bf, int L, int C, long long wl, int sp) {
  const int N = lt.N, nm = lt.nmax, n = lt.n[sp];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lj = lane & 15, lk = lane >> 4;
  double* M = bf.M + lt.m_off + wl * 2LL * N * nm + (long long)sp * N * nm;
  const Tf* H = (const Tf*)bf.feat + lt.feat_off + wl * (long long)L * N * C + (long long)(L - 1) * N * C;
  const double* W = lt.W + (long long)sp * C * nm;
  const double* base = lt.base + (long long)sp * N * nm;
  const double* bb = lt.b + sp * nm;
  const int ntr = (N + 15) / 16, ntc = (nm + 15) / 16;
  for (int tc0 = 0; tc0 < ntc; tc0 += RC_CT) {
    // with C a multiple of 16, product q covers k = 16 (q / 4) + 4 lk + q % 4
    // in lane group lk (the same sum in another order), so a lane's four A
    // values of a block are consecutive in H and load as one vector
    constexpr bool BLK = KS % 4 == 0;
    auto kidx = [&](int q) { return BLK ? 16 * (q >> 2) + 4 * lk + (q & 3) : 4 * q + lk; };
    double bw[RC_CT][KS];
#pragma unroll
    for (int ct = 0; ct < RC_CT; ++ct)
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        const int col = 16 * (tc0 + ct) + lj, k = kidx(q);
        bw[ct][q] = (col < n && k < C) ? W[(long long)k * nm + col] : 0.0;
      }
    for (int ti = wave; ti < ntr; ti += 4) {
      double av[KS];
      const int row = 16 * ti + lj;
      if constexpr (BLK) {
#pragma unroll
        for (int q4 = 0; q4 < KS / 4; ++q4) {
          Tf x[4] = {Tf(0), Tf(0), Tf(0), Tf(0)};
          if (row < N) {
            const Tf* hp = H + (long long)row * C + 16 * q4 + 4 * lk;
            if constexpr (sizeof(Tf) == 4) {
              const float4 v = *reinterpret_cast<const float4*>(hp);
              x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
            } else {
              const double2 v0 = *reinterpret_cast<const double2*>(hp);
              const double2 v1 = *reinterpret_cast<const double2*>(hp + 2);
              x[0] = v0.x; x[1] = v0.y; x[2] = v1.x; x[3] = v1.y;
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) av[4 * q4 + e] = (double)x[e];
        }
      } else {
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          const int k = kidx(q);
          av[q] = (row < N && k < C) ? (double)H[(long long)row * C + k] : 0.0;
        }
      }
#pragma unroll
      for (int ct = 0; ct < RC_CT; ++ct) {
        const int col = 16 * (tc0 + ct) + lj;
        if (16 * (tc0 + ct) >= nm) break;
        v4d acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * ti + lk + 4 * v;
          acc[v] = (r < N && col < n) ? base[(long long)r * nm + col] + bb[col] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) mfma(acc, av[q], bw[ct][q]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * ti + lk + 4 * v;
          if (r < N && col < nm) M[(long long)r * nm + col] = acc[v];
        }
      }
    }
  }
}
template <class Tf, int KS>
__global__ __launch_bounds__(256) void k_rows(LatDev lt, Bufs bf, int L, int C, WalkerSel sel) {
  const int sp = blockIdx.y;
  for (long long z = blockIdx.x;; z += gridDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);    // uniform in the block
    if (r == 0) break;
    if (r == 1) rows_one<Tf, KS>(lt, bf, L, C, wl, sp);
  }
}

// Phi_s = M_s[pos] (rows in label order) -> Phi_s^-1, log|det|, sign, with
// the register-tiled Gauss-Jordan elimination of tiled_lu.h (n <= 16 R).
template <int R>
SVMC_DEV void gj_one(const LatDev& lt, const Bufs& bf, long long wl, int sp, GjShared<R>& sh) {
  const long long w = lt.w0 + wl;
  const int n = lt.n[sp], nm = lt.nmax;
  const int tid = threadIdx.x, tx = tid >> 4, ty = tid & 15;
  double* ldo = bf.ld + 2 * w + sp;
  double* sgo = bf.sg + 2 * w + sp;
  if (n == 0) {
    if (tid == 0) { *ldo = 0.0; *sgo = 1.0; }
    return;
  }
  if (bf.flags[w] & 8) {
    if (tid == 0) { *ldo = -INFINITY; *sgo = 0.0; }
    return;
  }
  const double* M = bf.M + lt.m_off + wl * 2LL * lt.N * nm + (long long)sp * lt.N * nm;
  const int16_t* pos = bf.pos + lt.pos_off + wl * 2LL * nm + sp * nm;
  double x[R][R];
#pragma unroll
  for (int a = 0; a < R; ++a) {
    const int k = ty + 16 * a;
    const int site = k < n ? pos[k] : 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int m = tx + 16 * b;
      x[a][b] = (k < n && m < n) ? M[(long long)site * nm + m] : (k == m ? 1.0 : 0.0);
    }
  }
  double logabs, sgn;
  bool singular;
  tiled_gj<R, true>(x, n, sh, logabs, sgn, singular);
  if (singular) {
    if (tid == 0) { *ldo = -INFINITY; *sgo = 0.0; atomicOr(bf.flags + w, 1); }
    return;
  }
  if (tid == 0) {
    *ldo = logabs;
    *sgo = sgn;
    if (!isfinite(logabs)) atomicOr(bf.flags + w, 2);
  }
  double* Y = bf.inv + lt.inv_off + wl * 2LL * nm * nm + (long long)sp * nm * nm;
#pragma unroll
  for (int a = 0; a < R; ++a) {
    const int k = ty + 16 * a;
    if (k >= n) continue;
    const int row = sh.perminv[k];
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int m = tx + 16 * b;
      if (m < n) Y[(long long)row * nm + sh.perm[m]] = x[a][b];
    }
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_gj(LatDev lt, Bufs bf, WalkerSel sel) {
  __shared__ GjShared<R> sh;
  const int sp = blockIdx.y;
  for (long long z = blockIdx.x;; z += gridDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);    // uniform in the block
    if (r == 0) break;
    if (r == 1) gj_one<R>(lt, bf, wl, sp, sh);
    __syncthreads();
  }
}

// Gauss-Jordan inverse of one Slater block for N_sigma > 128 (up to 512):
// Phi (rows in label order) is gathered into the walker's inverse slot and
// inverted in place with partial pivoting; rows are swapped physically and
// the swaps undone as column swaps at the end.  One workgroup of 256 threads
// per (walker, spin); the pivot row and the pivot column are staged in LDS,
// each step then updates the whole block (rows in order, columns across
// threads).  log|det| and its sign come from the pivots and the swaps.
struct GjBigShared {
  double prow[512], fcol[512], rv[256];
  int ri[256];
  int16_t sw[512];
};
SVMC_DEV void gj_big_one(const LatDev& lt, const Bufs& bf, long long wl, int sp, GjBigShared& sb) {
  const long long w = lt.w0 + wl;
  const int n = lt.n[sp], nm = lt.nmax, tid = threadIdx.x;
  double* prow = sb.prow;
  double* fcol = sb.fcol;
  double* rv = sb.rv;
  int* ri = sb.ri;
  int16_t* sw = sb.sw;
  double* ldo = bf.ld + 2 * w + sp;
  double* sgo = bf.sg + 2 * w + sp;
  if (n == 0) {
    if (tid == 0) { *ldo = 0.0; *sgo = 1.0; }
    return;
  }
  if (bf.flags[w] & 8) {
    if (tid == 0) { *ldo = -INFINITY; *sgo = 0.0; }
    return;
  }
  const double* M = bf.M + lt.m_off + wl * 2LL * lt.N * nm + (long long)sp * lt.N * nm;
  const int16_t* pos = bf.pos + lt.pos_off + wl * 2LL * nm + sp * nm;
  double* Y = bf.inv + lt.inv_off + wl * 2LL * nm * nm + (long long)sp * nm * nm;
  for (int k = 0; k < n; ++k) {
    const double* src = M + (long long)pos[k] * nm;
    for (int c = tid; c < n; c += 256) Y[(long long)k * nm + c] = src[c];
  }
  __syncthreads();
  double logabs = 0.0, sgn = 1.0;
  bool singular = false;
  for (int p = 0; p < n; ++p) {
    // pivot: largest |Y[r][p]| over r >= p, ties to the lower row
    double best = -1.0;
    int bi = n;
    for (int r = p + tid; r < n; r += 256) {
      const double v = fabs(Y[(long long)r * nm + p]);
      if (v > best) { best = v; bi = r; }
    }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) {
        const double a = rv[tid], b = rv[tid + o];
        if (b > a || (b == a && ri[tid + o] < ri[tid])) { rv[tid] = b; ri[tid] = ri[tid + o]; }
      }
      __syncthreads();
    }
    const int piv = ri[0];
    const double pmax = rv[0];
    __syncthreads();
    if (!(pmax > 0.0)) { singular = true; break; }
    if (piv != p)
      for (int c = tid; c < n; c += 256) {
        const double a = Y[(long long)p * nm + c];
        Y[(long long)p * nm + c] = Y[(long long)piv * nm + c];
        Y[(long long)piv * nm + c] = a;
      }
    if (tid == 0) sw[p] = (int16_t)piv;
    __syncthreads();
    const double pv = Y[(long long)p * nm + p];
    logabs += log(fabs(pv));
    if (pv < 0.0) sgn = -sgn;
    if (piv != p) sgn = -sgn;
    const double ipv = 1.0 / pv;
    for (int c = tid; c < n; c += 256) {
      prow[c] = c == p ? ipv : Y[(long long)p * nm + c] * ipv;
      fcol[c] = Y[(long long)c * nm + p];
    }
    __syncthreads();
    for (int r = 0; r < n; ++r) {
      double* yr = Y + (long long)r * nm;
      const double f = fcol[r];
      for (int c = tid; c < n; c += 256) {
        if (r == p) yr[c] = prow[c];
        else yr[c] = c == p ? -f * prow[p] : fma(-f, prow[c], yr[c]);
      }
    }
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) { *ldo = -INFINITY; *sgo = 0.0; atomicOr(bf.flags + w, 1); }
    return;
  }
  // the row swaps of Phi become column swaps of its inverse, undone in reverse
  for (int p = n - 1; p >= 0; --p) {
    const int q = sw[p];
    if (q != p)
      for (int r = tid; r < n; r += 256) {
        const double a = Y[(long long)r * nm + p];
        Y[(long long)r * nm + p] = Y[(long long)r * nm + q];
        Y[(long long)r * nm + q] = a;
      }
    __syncthreads();
  }
  if (tid == 0) {
    *ldo = logabs;
    *sgo = sgn;
    if (!isfinite(logabs)) atomicOr(bf.flags + w, 2);
  }
}

__global__ __launch_bounds__(256) void k_gj_big(LatDev lt, Bufs bf, WalkerSel sel) {
  __shared__ GjBigShared sb;
  const int sp = blockIdx.y;
  for (long long z = blockIdx.x;; z += gridDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);    // uniform in the block
    if (r == 0) break;
    if (r == 1) gj_big_one(lt, bf, wl, sp, sb);
    __syncthreads();
  }
}

// G_s = M_s Y_s and P_s = W_s Y_s (Y_s = Phi_s^-1) without the row buffer:
// M_s = B_s + 1 b_s + H_L W_s, so G_s = (B_s + 1 b_s) Y_s + H_L P_s, a product
// with inner dimension n_s + C whose left factor is the lattice's base
// orbitals plus bias (shared by all walkers: L2-resident) and the walker's
// final features.  On the FP64 matrix cores: one workgroup of four
// wavefronts per (walker, spin); wavefront w takes the 32-column blocks
// w, w + 4, ...: it first forms its block of P (C x 32, inner dimension n_s)
// into LDS and into P^T, then every 32 x 32 block of G in that column range
// (two row tiles by two column tiles, four 16 x 16 x 4 accumulators), four
// k-steps at a time.  Columns m >= n_s are not written.
template <class Tf>
SVMC_DEV void gp_one(const LatDev& lt, const Bufs& bf, int C, int planes, long long wl, int sp,
                     double (*Ps)[32]) {
  const int N = lt.N, nm = lt.nmax;
  const int n = lt.n[sp];
  if (n == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lj = lane & 15, lk = lane >> 4;
  const Tf* H = (const Tf*)bf.feat + lt.feat_off + wl * (long long)planes * N * C + (long long)(planes - 1) * N * C;
  const double* W = lt.W + (long long)sp * C * nm;
  const double* base = lt.base + (long long)sp * N * nm;
  const double* bb = lt.b + sp * nm;
  const double* Y = bf.inv + lt.inv_off + wl * 2LL * nm * nm + (long long)sp * nm * nm;
  double* G = bf.G + lt.g_off + wl * 2LL * N * nm + (long long)sp * N * nm;
  double* PT = bf.PT + lt.pt_off + wl * 2LL * nm * C + (long long)sp * nm * C;
  const int nbc = (n + 31) / 32;
  const bool vec = (nm & 1) == 0;          // rows of B_s and W_s start 16-byte aligned
  for (int cb = wave; cb < nbc; cb += 4) {
    const int c0 = 32 * cb;
    bool bok[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) bok[u] = c0 + 16 * u + lj < n;
    // B operand over the orbital index: k = k0 + 4 lk + e in product e of a
    // block of 16 (any order of k gives the same sum when A and B agree)
    auto load_y = [&](int k0, double (&b)[4][2]) {
      const int ka = k0 + 4 * lk;
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int t = 0; t < 2; ++t) b[e][t] = (ka + e < n && bok[t]) ? Y[(long long)(ka + e) * nm + c0 + 16 * t + lj] : 0.0;
    };
    auto load_row = [&](const double* row, bool ok, int k0, double (&a)[4]) {
      const int ka = k0 + 4 * lk;
      if (vec && ok && ka + 3 < n) {
        const double2 x0 = *reinterpret_cast<const double2*>(row + ka);
        const double2 x1 = *reinterpret_cast<const double2*>(row + ka + 2);
        a[0] = x0.x; a[1] = x0.y; a[2] = x1.x; a[3] = x1.y;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = (ok && ka + e < n) ? row[ka + e] : 0.0;
      }
    };
    // ---- P block: rows c < C of W_s Y_s, columns c0 .. c0 + 31
    {
      v4d acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[u][t] = v4d{0.0, 0.0, 0.0, 0.0};
      bool aok[2];
      const double* arow[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        aok[u] = 16 * u + lj < C;
        arow[u] = W + (long long)(aok[u] ? 16 * u + lj : 0) * nm;
      }
      for (int k0 = 0; k0 < n; k0 += 16) {
        double a[2][4], b[4][2];
#pragma unroll
        for (int u = 0; u < 2; ++u) load_row(arow[u], aok[u], k0, a[u]);
        load_y(k0, b);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t) mfma(acc[u][t], a[u][e], b[e][t]);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int m = c0 + 16 * t + lj;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int c = 16 * u + lk + 4 * v;
            if (c < C) {
              Ps[c][16 * t + lj] = m < n ? acc[u][t][v] : 0.0;
              if (m < n) PT[(long long)m * C + c] = acc[u][t][v];
            }
          }
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // ---- G blocks in this column range: (B_s + 1 b_s) Y_s + H_L P_s, 32
    // rows at a time (two row tiles share each B fragment; four would spill
    // at this register budget)
    constexpr int RT = 2;
    for (int r0 = 0; r0 < N; r0 += 16 * RT) {
      bool aok[RT];
      const double* arow[RT];
#pragma unroll
      for (int u = 0; u < RT; ++u) {
        const int r = r0 + 16 * u + lj;
        aok[u] = r < N;
        arow[u] = base + (long long)(aok[u] ? r : 0) * nm;
      }
      v4d acc[RT][2];
#pragma unroll
      for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[u][t] = v4d{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < n; k0 += 16) {
        double a[RT][4], b[4][2], bk[4];
        const int ka = k0 + 4 * lk;
#pragma unroll
        for (int e = 0; e < 4; ++e) bk[e] = ka + e < n ? bb[ka + e] : 0.0;
#pragma unroll
        for (int u = 0; u < RT; ++u) {
          load_row(arow[u], aok[u], k0, a[u]);
#pragma unroll
          for (int e = 0; e < 4; ++e) a[u][e] = aok[u] ? a[u][e] + bk[e] : 0.0;
        }
        load_y(k0, b);
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int u = 0; u < RT; ++u)
#pragma unroll
            for (int t = 0; t < 2; ++t) mfma(acc[u][t], a[u][e], b[e][t]);
      }
      // the features' part: inner index c over the channels, four at a time
      for (int q = 0; 4 * q < C; ++q) {
        const int c = 4 * q + lk;
        double a[RT], b[2];
#pragma unroll
        for (int u = 0; u < RT; ++u) {
          const int r = r0 + 16 * u + lj;
          a[u] = (r < N && c < C) ? (double)H[(long long)r * C + c] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) b[t] = c < C ? Ps[c][16 * t + lj] : 0.0;
#pragma unroll
        for (int u = 0; u < RT; ++u)
#pragma unroll
          for (int t = 0; t < 2; ++t) mfma(acc[u][t], a[u], b[t]);
      }
#pragma unroll
      for (int u = 0; u < RT; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int m = c0 + 16 * t + lj;
          if (m >= n) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = r0 + 16 * u + lk + 4 * v;
            if (r < N) G[(long long)r * nm + m] = acc[u][t][v];
          }
        }
    }
    // this wavefront's P block is read by no one else; the next column
    // block overwrites it only after every read above
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}
template <class Tf>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gp(LatDev lt, Bufs bf, int C, int planes,
                                                                                 WalkerSel sel) {
  __shared__ double ps[4][32][32];               // each wavefront's block of P
  const int sp = blockIdx.y;
  for (long long z = blockIdx.x;; z += gridDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);    // uniform in the block
    if (r == 0) break;
    if (r == 1) gp_one<Tf>(lt, bf, C, planes, wl, sp, ps[threadIdx.x >> 6]);
  }
}

// sign with canonical (site-ascending) row order = label-order sign times the
// parity of the label -> site map; log|psi| = sum over spins.
__global__ void k_logpsi(LatDev lt, Bufs bf, double* sign, double* logabs) {
  const long long wl = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (wl >= lt.nw) return;
  const long long w = lt.w0 + wl;
  const int nm = lt.nmax;
  double s = bf.sg[2 * w] * bf.sg[2 * w + 1];
  const double la = bf.ld[2 * w] + bf.ld[2 * w + 1];
  for (int sp = 0; sp < 2; ++sp) {
    const int16_t* pos = bf.pos + lt.pos_off + wl * 2LL * nm + sp * nm;
    int inv = 0;
    for (int p = 0; p < lt.n[sp]; ++p)
      for (int q = p + 1; q < lt.n[sp]; ++q) inv += pos[q] < pos[p];
    if (inv & 1) s = -s;
  }
  if (sign) sign[w] = s;
  if (logabs) logabs[w] = la;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_labels(const LatDev& lt, const Bufs& bf, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  const unsigned nb = (unsigned)((lt.nw + 255) / 256);
  hipLaunchKernelGGL(k_labels, dim3(nb), dim3(256), 0, st, lt, bf);
  return hipGetLastError();
}

hipError_t launch_forward(int prec, const LatDev& lt, const Bufs& bf, const ModelDev& md, void* h0tmp,
                          hipStream_t st) {
#define SVMC_FWD(P_, C_) if (prec == P_ && md.C == C_) return forward_##P_##_##C_(lt, bf, md, h0tmp, st);
  SVMC_FOR_EACH_PREC_C(SVMC_FWD)
#undef SVMC_FWD
  return hipErrorInvalidValue;
}


// Walker slots of a launch: every walker of the lattice (one slot each), or
// `list_slots` slots that loop over the list.
static long long walker_slots(const LatDev& lt, const WalkerSel& sel, int list_slots) {
  return sel.list ? std::min<long long>(lt.nw, list_slots) : lt.nw;
}

hipError_t launch_rows(int prec, const LatDev& lt, const Bufs& bf, int L, int C, hipStream_t st, WalkerSel sel) {
  if (lt.nw == 0) return hipSuccess;
  const dim3 grid((unsigned)walker_slots(lt, sel, 256), 2);
  auto go = [&](auto kf) { hipLaunchKernelGGL(kf, grid, dim3(256), 0, st, lt, bf, L, C, sel); };
  const bool f64 = prec == PREC_F64;
  switch (C) {
    case 8: f64 ? go(k_rows<double, 2>) : go(k_rows<float, 2>); break;
    case 16: f64 ? go(k_rows<double, 4>) : go(k_rows<float, 4>); break;
    case 24: f64 ? go(k_rows<double, 6>) : go(k_rows<float, 6>); break;
    case 32: f64 ? go(k_rows<double, 8>) : go(k_rows<float, 8>); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gj(const LatDev& lt, const Bufs& bf, hipStream_t st, WalkerSel sel) {
  if (lt.nw == 0) return hipSuccess;
  const dim3 grid((unsigned)walker_slots(lt, sel, 256), 2);
  if (lt.nmax <= 16) hipLaunchKernelGGL((k_gj<1>), grid, dim3(256), 0, st, lt, bf, sel);
  else if (lt.nmax <= 32) hipLaunchKernelGGL((k_gj<2>), grid, dim3(256), 0, st, lt, bf, sel);
  else if (lt.nmax <= 64) hipLaunchKernelGGL((k_gj<4>), grid, dim3(256), 0, st, lt, bf, sel);
  else if (lt.nmax <= 128) hipLaunchKernelGGL((k_gj<8>), grid, dim3(256), 0, st, lt, bf, sel);
  else if (lt.nmax <= 512) hipLaunchKernelGGL(k_gj_big, grid, dim3(256), 0, st, lt, bf, sel);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gp(int prec, const LatDev& lt, const Bufs& bf, int planes, int C, hipStream_t st, WalkerSel sel) {
  if (lt.nw == 0) return hipSuccess;
  if (C > 32) return hipErrorInvalidValue;
  const dim3 grid((unsigned)walker_slots(lt, sel, 256), 2);
  if (prec == PREC_F64) hipLaunchKernelGGL(k_gp<double>, grid, dim3(256), 0, st, lt, bf, C, planes, sel);
  else hipLaunchKernelGGL(k_gp<float>, grid, dim3(256), 0, st, lt, bf, C, planes, sel);
  return hipGetLastError();
}

hipError_t launch_logpsi(const LatDev& lt, const Bufs& bf, double* sign, double* logabs, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_logpsi, dim3((unsigned)((lt.nw + 127) / 128)), dim3(128), 0, st, lt, bf, sign, logabs);
  return hipGetLastError();
}

#endif

}  // namespace svmc
