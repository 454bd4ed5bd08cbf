// Amplitude ratio of one hop by local update (Sec. II.C):
//  1. cached features are reused outside the hop's receptive field; inside it
//     the conv stack is re-evaluated on a box that grows by one site per
//     layer (affected-sites equation: Chebyshev neighbourhood of the two
//     changed sites), so layer l touches at most (2l+2) x (2l+2) sites;
//  2. the changed orbital rows form a low-rank update of the Slater matrix;
//     the ratio is det(A) with A built from the cached inverse through
//     G = M Phi^-1 and P = W Phi^-1 (Sherman-Morrison-Woodbury / matrix
//     determinant lemma), one small FP64 LU per spin.
//
// Two wavefronts evaluate one hop together: the conv tiles, ring fills and
// difference rows are split between them, then wavefront s computes the
// determinant of spin s.  LDS scratch per hop: see HopScratch.
#pragma once
#include "svmc_dev.h"

namespace svmc {

SVMC_DEV int dir_dx(int d) { return (d == 0 || d == 4 || d == 5) ? 1 : ((d == 1 || d == 6 || d == 7) ? -1 : 0); }
SVMC_DEV int dir_dy(int d) { return (d == 2 || d == 4 || d == 6) ? 1 : ((d == 3 || d == 5 || d == 7) ? -1 : 0); }

// One lattice axis as seen from a hop.  Coordinates u are "unwrapped"
// (may leave [0, La) on periodic axes).  Window mode: grid index u - go.
// Torus mode (periodic axis shorter than the largest box): grid index u mod La.
struct Axis {
  int La, per, torus, go;
};
SVMC_DEV int gidx(const Axis& a, int u) { return a.torus ? imod(u, a.La) : u - a.go; }
SVMC_DEV bool inlat(const Axis& a, int u) { return a.per || (u >= 0 && u < a.La); }
SVMC_DEV int latc(const Axis& a, int u) { return a.per ? imod(u, a.La) : u; }
// Sites within distance l of {x_i, x_i + dx} along the axis, clipped at open
// edges and capped at the axis length on periodic ones: [lo, lo + w).
SVMC_DEV void box1(const Axis& a, int xi, int dx, int l, int& lo, int& w) {
  int L0 = xi + min(0, dx) - l, H0 = xi + max(0, dx) + l;
  if (!a.per) { L0 = max(L0, 0); H0 = min(H0, a.La - 1); }
  w = H0 - L0 + 1;
  if (a.per && w > a.La) w = a.La;
  lo = L0;
}
SVMC_DEV bool inbox(const Axis& a, int lo, int w, int u) {
  return a.torus ? imod(u - lo, a.La) < w : (u >= lo && u < lo + w);
}


struct HopGeom {
  int i, j, sigma, d;
  Axis ax, ay;
  int xi, yi, dx, dy;
};

SVMC_DEV HopGeom hop_geom(const LatDev& lt, int L, int sigma, int i, int d) {
  HopGeom h;
  h.i = i; h.sigma = sigma; h.d = d;
  h.dx = dir_dx(d); h.dy = dir_dy(d);
  h.xi = i % lt.Lx; h.yi = i / lt.Lx;
  const int xj = lt.pbc_x ? imod(h.xi + h.dx, lt.Lx) : h.xi + h.dx;
  const int yj = lt.pbc_y ? imod(h.yi + h.dy, lt.Ly) : h.yi + h.dy;
  h.j = xj + lt.Lx * yj;
  h.ax = Axis{lt.Lx, lt.pbc_x, lt.torus_x, h.xi + min(0, h.dx) - L - 1};
  h.ay = Axis{lt.Ly, lt.pbc_y, lt.torus_y, h.yi + min(0, h.dy) - L - 1};
  return h;
}

// Site stride of the LDS feature arrays: C channels plus 16 bytes, so that
// the 16 rows of an MFMA fragment (16 different sites) fall into different
// LDS banks.
template <class Tf, int C> struct SiteStride {
  static constexpr int value = C + 16 / (int)sizeof(Tf);
};
constexpr int KSP = 50;   // row stride (doubles) of the transposed P^T staging

// LDS scratch of one hop, in bytes:
//   grid   [Gy][Gx][SP] Tf  features of one layer on the update box; after the
//                           last layer, D = H'_L - H_L densely as [m][SP]
//   stage0 max(OUT box x C Tf, P^T staging)  layer outputs before they
//                           replace the grid; later spin 0's staged P^T rows,
//                           G values and LU pivot row
//   stage1 P^T staging of spin 1
//   klists [2][Gx Gy] int   changed-row lists per spin
//   misc   64 bytes         per-spin results
constexpr int KSTAGE = 48;
struct HopScratch {
  int stage0, stage1, klists, misc, bytes;
};
__host__ __device__ inline int align16i(int x) { return (x + 15) & ~15; }
__host__ __device__ inline HopScratch hop_scratch(int Gx, int Gy, int L, int C, int tfb) {
  HopScratch h;
  const int SP = C + 16 / tfb;
  const int grid = align16i(Gx * Gy * SP * tfb);
  const int ox = Gx < 2 * L + 2 ? Gx : 2 * L + 2, oy = Gy < 2 * L + 2 ? Gy : 2 * L + 2;
  const int outb = ox * oy * SP * tfb;
  const int pkc = (C * KSP > KSTAGE * C ? C * KSP : KSTAGE * C);
  const int pkb = (pkc + KSTAGE + 64) * 8;
  h.stage0 = grid;
  h.stage1 = h.stage0 + align16i(outb > pkb ? outb : pkb);
  h.klists = h.stage1 + align16i(pkb);
  h.misc = h.klists + align16i(2 * Gx * Gy * 4);
  h.bytes = h.misc + 64;
  return h;
}

// B fragments of a layer kept in registers when they fit (<= 80 VGPRs).
template <int P, int C> struct RegB {
  static constexpr bool value =
      ConvCfg<P, C>::Q * ConvCfg<P, C>::NT * (int)sizeof(typename PrecT<P>::Tb) <= 80 * 4;
};

// One 16-site tile of a layer on the LDS grid.  px / py: packed grid
// coordinates of the lane's row (byte k = offset k - 1, 0xFF = zero padding).
// B fragments come from registers (breg) or global memory (Bl).  Per output
// element the accumulation order equals conv_tile's.
template <int P, int C>
SVMC_DEV void conv_tile_grid(const typename PrecT<P>::Tf* __restrict__ grid, int Gx, unsigned px, unsigned py,
                             const typename PrecT<P>::Tb (&breg)[RegB<P, C>::value ? ConvCfg<P, C>::Q : 1]
                                                               [ConvCfg<P, C>::NT],
                             const typename PrecT<P>::Tb* __restrict__ Bl, int lane,
                             typename PrecT<P>::Acc (&acc)[ConvCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef ConvCfg<P, C> CC;
  const int g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[nt][v] = 0;
#pragma unroll
  for (int q = 0; q < CC::Q; ++q) {
    Tb b[CC::NT];
#pragma unroll
    for (int nt = 0; nt < CC::NT; ++nt) {
      if constexpr (RegB<P, C>::value) b[nt] = breg[q][nt];
      else b[nt] = Bl[(q * CC::NT + nt) * 64 + lane];
    }
    int tap, c0;
    bool kok;
    if constexpr (P == PREC_BF16 || P == PREC_BF16X3) {
      const int k0 = 32 * q + 8 * g;
      kok = k0 < CC::K;
      tap = kok ? k0 / C : 0;
      c0 = k0 % C;
    } else {
      kok = true;
      tap = (4 * q) / C;
      c0 = (4 * q) % C + g;
    }
    const unsigned gx = (px >> (8 * (tap % 3))) & 0xFFu, gy = (py >> (8 * (tap / 3))) & 0xFFu;
    const bool ok = kok && gx != 0xFFu && gy != 0xFFu;
    const int off = ((int)gy * Gx + (int)gx) * SiteStride<Tf, C>::value + c0;
    if constexpr (P == PREC_BF16 || P == PREC_BF16X3) {
      float x[8];
      if (ok) {
        const float4* p4 = reinterpret_cast<const float4*>(grid + off);
        const float4 x0 = p4[0], x1 = p4[1];
        x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
        x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      }
      v8bf a;
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (__bf16)x[e];
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], a, b[nt]);
      if constexpr (P == PREC_BF16X3) {
        v8bf a2, a3;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float r1 = x[e] - (float)a[e];
          a2[e] = (__bf16)r1;
          a3[e] = (__bf16)(r1 - (float)a2[e]);
        }
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt) {
          mfma(acc[nt], a2, b[nt]);
          mfma(acc[nt], a3, b[nt]);
        }
      }
    } else {
      const Tf a = ok ? grid[off] : Tf(0);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], a, b[nt]);
    }
  }
}

// Incremental conv stack for one hop, computed by the NW wavefronts of the
// workgroup (wave = this thread's wavefront).  On return (after a barrier)
// the grid's first count*C entries hold D = H'_L - H_L on the layer-L box
// (index m = ox + owx * oy).  If `commit` is non-null every new layer value is
// also stored into the cache (accepted move); commit may equal featw (the
// box of a layer never overlaps the ring read from the cache for the next).
template <int P, int C, int NW>
SVMC_DEV void hop_features(const ModelDev& md, const LatDev& lt, const HopGeom& h, const int8_t* occ_s,
                           const typename PrecT<P>::Tf* featw,
                           typename PrecT<P>::Tf* commit, char* scratch, const HopScratch& hs,
                           int& olx, int& owx, int& oly, int& owy) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NT_ = 64 * NW;
  constexpr int SP = SiteStride<Tf, C>::value;
  const int L = md.L, N = lt.N, Lx = lt.Lx, Gx = lt.Gx;
  const Axis ax = h.ax, ay = h.ay;
  Tf* grid = (Tf*)scratch;
  Tf* obuf = (Tf*)(scratch + hs.stage0);
  const int bit = 1 << h.sigma;
  // layer-1 input: embedding of the new configuration on the layer-1 input
  // box (layer-1 output box grown by one site)
  {
    int lx, wx, ly, wy;
    box1(ax, h.xi, h.dx, 2, lx, wx);
    box1(ay, h.yi, h.dy, 2, ly, wy);
    const Tf* E = (const Tf*)md.embed;
    const int tot = wx * wy * C;
    for (int e = tid; e < tot; e += NT_) {
      const int c = e % C, q = e / C;
      const int ux = lx + q % wx, uy = ly + q / wx;
      const int s = latc(ax, ux) + Lx * latc(ay, uy);
      int o = occ_s[s];
      if (s == h.i) o -= bit;
      if (s == h.j) o += bit;
      grid[(gidx(ay, uy) * Gx + gidx(ax, ux)) * SP + c] = E[o * C + c];
    }
  }
  __syncthreads();
  constexpr int QB = RegB<P, C>::value ? CC::Q : 1;
  constexpr int V = 16 / sizeof(Tf);          // elements per 16-byte vector
  constexpr int CV = C / V;
  for (int l = 1; l <= L; ++l) {
    box1(ax, h.xi, h.dx, l, olx, owx);
    box1(ay, h.yi, h.dy, l, oly, owy);
    const int cnt = uniform_i(owx * owy);
    const int T = (cnt + 15) >> 4;
    const Tb* Bl = (const Tb*)md.Bpack + (long long)(l - 1) * CC::Q * CC::NT * 64;
    Tb breg[QB][CC::NT];
    if constexpr (RegB<P, C>::value) {
      if (wave < T) {
#pragma unroll
        for (int q = 0; q < CC::Q; ++q)
#pragma unroll
          for (int nt = 0; nt < CC::NT; ++nt) breg[q][nt] = Bl[(q * CC::NT + nt) * 64 + lane];
      }
    }
    const Tf* bias = (const Tf*)md.bias + (l - 1) * C;
    for (int t = wave; t < T; t += NW) {
      const int m = 16 * t + (lane & 15);
      unsigned px = 0xFFFFFFu, py = 0xFFFFFFu;
      if (m < cnt) {
        const int ux = olx + m % owx, uy = oly + m / owx;
        px = 0;
        py = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int nx = ux + k - 1, ny = uy + k - 1;
          px |= (inlat(ax, nx) ? (unsigned)gidx(ax, nx) : 0xFFu) << (8 * k);
          py |= (inlat(ay, ny) ? (unsigned)gidx(ay, ny) : 0xFFu) << (8 * k);
        }
      }
      Acc acc[CC::NT];
      conv_tile_grid<P, C>(grid, Gx, px, py, breg, Bl, lane, acc);
      // epilogue: H'_l = H'_{l-1} + act(conv + b); residual read from the grid
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * t + OutMap<P>::row(lane, v);
          const int n = 16 * nt + OutMap<P>::col(lane, v);
          if (r < cnt && n < C) {
            const int ux = olx + r % owx, uy = oly + r / owx;
            const Tf z = acc[nt][v] + bias[n];
            obuf[r * SP + n] = grid[(gidx(ay, uy) * Gx + gidx(ax, ux)) * SP + n] + act_fn<Tf>(md.act, z);
          }
        }
    }
    __syncthreads();
    if (l < L) {
      // H'_l replaces H'_{l-1} on the box ...
      for (int e = tid; e < cnt * CV; e += NT_) {
        const int r = e / CV, cv = e % CV;
        const int ux = olx + r % owx, uy = oly + r / owx;
        const float4 val = *reinterpret_cast<const float4*>(obuf + r * SP + cv * V);
        *reinterpret_cast<float4*>(grid + (gidx(ay, uy) * Gx + gidx(ax, ux)) * SP + cv * V) = val;
        if (commit) {
          const int s = latc(ax, ux) + Lx * latc(ay, uy);
          *reinterpret_cast<float4*>(commit + ((long long)(l - 1) * N + s) * C + cv * V) = val;
        }
      }
      // ... and the ring of the next input box (output box at distance l+1
      // grown by one) gets the cached H_l
      int ilx, iwx, ily, iwy;
      box1(ax, h.xi, h.dx, l + 2, ilx, iwx);
      box1(ay, h.yi, h.dy, l + 2, ily, iwy);
      const Tf* Hl = featw + (long long)(l - 1) * N * C;
      const int tot = iwx * iwy * CV;
      constexpr int U = 4;          // loads in flight per thread
      for (int e0 = 0; e0 < tot; e0 += NT_ * U) {
        float4 val[U];
        int dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + NT_ * u + tid;
          const int q = e / CV, cv = e % CV;
          const int ux = ilx + q % iwx, uy = ily + q / iwx;
          const bool ok = e < tot && !(inbox(ax, olx, owx, ux) && inbox(ay, oly, owy, uy));
          const int s = ok ? latc(ax, ux) + Lx * latc(ay, uy) : 0;
          dst[u] = ok ? (gidx(ay, uy) * Gx + gidx(ax, ux)) * SP + cv * V : -1;
          val[u] = ok ? *reinterpret_cast<const float4*>(Hl + (long long)s * C + cv * V) : float4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (dst[u] >= 0) *reinterpret_cast<float4*>(grid + dst[u]) = val[u];
      }
    } else {
      // D = H'_L - H_L, densely [m][C] at the start of the grid
      const Tf* HL = featw + (long long)(L - 1) * N * C;
      const int tot = cnt * CV;
      constexpr int U = 4;
      for (int e0 = 0; e0 < tot; e0 += NT_ * U) {
        float4 old[U];
        int ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + NT_ * u + tid;
          ok[u] = e < tot;
          const int r = e / CV, cv = e % CV;
          const int ux = olx + r % owx, uy = oly + r / owx;
          const int s = ok[u] ? latc(ax, ux) + Lx * latc(ay, uy) : 0;
          old[u] = ok[u] ? *reinterpret_cast<const float4*>(HL + (long long)s * C + cv * V) : float4{0, 0, 0, 0};
          if (ok[u] && commit)
            *reinterpret_cast<float4*>(commit + ((long long)(L - 1) * N + s) * C + cv * V) =
                *reinterpret_cast<const float4*>(obuf + r * SP + cv * V);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!ok[u]) continue;
          const int e = e0 + NT_ * u + tid;
          const int r = e / CV, cv = e % CV;
          Tf* d = grid + r * SP + cv * V;
          const Tf* nv = obuf + r * SP + cv * V;
          const Tf* ov = reinterpret_cast<const Tf*>(&old[u]);
#pragma unroll
          for (int k = 0; k < V; ++k) d[k] = nv[k] - ov[k];
        }
      }
    }
    __syncthreads();
  }
}

// Changed-row list of spin tau (one wavefront): every electron of spin tau
// in the new configuration on the layer-L box, entry (m << 16) | label, m
// indexing the box.  The moving electron keeps its label at its new site.
// Returns the list length; *hpos gets the mover's position (tau = sigma).
SVMC_DEV int hop_klist(const LatDev& lt, const HopGeom& h, const int8_t* occ_s, const int16_t* lab_s, int tau,
                       int olx, int owx, int oly, int owy, int* kl, int& hpos, int lane) {
  const int N = lt.N, Lx = lt.Lx;
  const int cnt = owx * owy;
  const int bit = 1 << h.sigma;
  int nk = 0;
  hpos = -1;
  for (int base = 0; base < cnt; base += 64) {
    const int m = base + lane;
    int s = 0, o = 0;
    if (m < cnt) {
      const int ux = olx + m % owx, uy = oly + m / owx;
      s = latc(h.ax, ux) + Lx * latc(h.ay, uy);
      o = occ_s[s];
      if (s == h.i) o -= bit;
      if (s == h.j) o += bit;
    }
    const bool pred = m < cnt && ((o >> tau) & 1);
    const unsigned long long mask = __ballot(pred);
    const int idx = nk + __popcll(mask & ((1ULL << lane) - 1ULL));
    const bool mover = pred && tau == h.sigma && s == h.j;
    if (pred) {
      const int k = mover ? lab_s[h.sigma * N + h.i] : lab_s[tau * N + s];
      kl[idx] = (m << 16) | k;
    }
    const unsigned long long mm = __ballot(mover);
    if (mm) hpos = nk + __popcll(mask & ((1ULL << (__ffsll((long long)mm) - 1)) - 1ULL));
    nk += __popcll(mask);
  }
  return nk;
}

// One-wave LU determinant of an r x r FP64 matrix, r <= RM <= 64.
// Lane a (< r) holds row a in a[0..RM).  Columns rotate: at every step the
// current pivot column is a[0] and the remaining columns shift left, so all
// register indices stay static in a runtime step loop.  Partial pivoting
// without moving rows: the unused row with the largest |a[0]| pivots (the
// search compares |a| rounded to FP32, ties to the lower lane; pivots below
// FP32's smallest denormal count as zero).  The pivot row reaches the other
// lanes through v_readlane (scalar registers), eight columns at a time, and
// only the columns still in play are updated.
// det = sign(permutation) * prod(pivots).
template <int RM>
SVMC_DEV double lu_det_rot(double (&a)[RM], int r_in, int lane) {
  const int r = uniform_i(r_in);
  bool used = lane >= r;
  int step = 64;
  double det = 1.0;
  for (int p = 0; p < r; ++p) {
    const double cp = a[0];
    const unsigned key0 = used ? 0u : ((__float_as_uint((float)fabs(cp)) & ~63u) | (unsigned)(63 - lane));
    const unsigned key = wave_max_u32(key0);
    if ((key & ~63u) == 0u) return 0.0;
    const int piv = 63 - (int)(key & 63u);
    const double pv = readlane_d(cp, piv);
    det *= pv;
    if (lane == piv) { used = true; step = p; }
    const double l = used ? 0.0 : cp * (1.0 / pv);
    const int live = r - 1 - p;               // columns right of the pivot
#pragma unroll
    for (int c0 = 1; c0 < RM; c0 += 8) {
      if (c0 <= live) {
#pragma unroll
        for (int c = c0; c < c0 + 8 && c < RM; ++c) a[c - 1] = fma(-l, readlane_d(a[c], piv), a[c]);
      }
    }
  }
  int inv = 0;
  for (int b = 0; b < r; ++b) {
    const int sb = __builtin_amdgcn_readlane(step, b);
    if (lane < r && b > lane && sb < step) ++inv;
  }
  inv = wave_sum_i(inv);
  return (inv & 1) ? -det : det;
}

// det of the Woodbury/determinant-lemma matrix of spin tau for one hop
// (one wavefront).
//   row form (|K| <= C):  A[a][b] = delta_ab + D(m_a) . P[:, k_b]
//                         + [a = mover] (G[j][k_b] - delta_ab)
//   column form (|K| > C): det(I + V U) with U = [D_K, e_h], V = [P_K; g - e_h]
// Both equal det(Phi'[K] Phi^-1[:, K]).  All in FP64.  The P^T rows (and G
// values) of the K labels are first copied into LDS with coalesced loads
// (row form: transposed [c][b]; column form [b][c] when |K| <= KSTAGE).
template <class Tf, int C>
SVMC_DEV double hop_det(const int* kl, int K_in, bool hopspin, int hpos_in, const Tf* Dbuf,
                        const double* __restrict__ PTt, const double* __restrict__ Gj, double* stage, int lane) {
  const int K = uniform_i(K_in), hpos = uniform_i(hpos_in);
  if (K == 0) return 1.0;
  constexpr int RM = C + 1;
  const bool rowform = K <= C;
  const bool staged = K <= KSTAGE;
  constexpr int SP = SiteStride<Tf, C>::value;
  constexpr int PKN = (C * KSP > KSTAGE * C ? C * KSP : KSTAGE * C);
  double* pk = stage;                 // row form [C][KSP], column form [K][C]
  double* gk = stage + PKN;           // [KSTAGE]
  if (staged) {
    constexpr int U = 4;
    const int tot = K * C;
    for (int e0 = 0; e0 < tot; e0 += 64 * U) {
      double v[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + 64 * u + lane;
        const bool ok = e < tot;
        const int b = e / C, c = e % C;
        const int kb = ok ? (kl[b] & 0xffff) : 0;
        dst[u] = ok ? (rowform ? c * KSP + b : e) : -1;
        v[u] = ok ? PTt[kb * C + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (dst[u] >= 0) pk[dst[u]] = v[u];
    }
    if (hopspin && lane < K) gk[lane] = Gj[kl[lane] & 0xffff];
    __builtin_amdgcn_wave_barrier();
  }
  double a[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) a[c] = 0.0;
  int rdim;
  if (rowform) {
    const int ma = lane < K ? (kl[lane] >> 16) : 0;
    for (int c = 0; c < C; ++c) {
      const double dc = lane < K ? (double)Dbuf[ma * SP + c] : 0.0;
      const double* pr = pk + c * KSP;
#pragma unroll
      for (int b = 0; b < RM; ++b) a[b] = fma(dc, pr[b], a[b]);
    }
    const bool hrow = hopspin && lane == hpos;
#pragma unroll
    for (int b = 0; b < RM; ++b) {
      double x = (b < K) ? a[b] : 0.0;
      if (lane == b) x += 1.0;
      if (hrow && b < K) x += gk[b] - (b == hpos ? 1.0 : 0.0);
      a[b] = x;
    }
    rdim = K;
  } else {
    for (int q = 0; q < K; ++q) {
      const int e = kl[q];
      const int mq = e >> 16, kq = e & 0xffff;
      double p = 0.0;
      if (lane < C) p = staged ? pk[q * C + lane] : PTt[kq * C + lane];
      else if (hopspin && lane == C) p = (staged ? gk[q] : Gj[kq]) - (q == hpos ? 1.0 : 0.0);
      const Tf* Dq = Dbuf + mq * SP;
#pragma unroll
      for (int c = 0; c < C; ++c) a[c] = fma(p, (double)Dq[c], a[c]);
    }
    const int kh = hopspin ? (kl[hpos] & 0xffff) : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (lane == c) a[c] += 1.0;
      if (lane > C || (!hopspin && lane == C)) a[c] = 0.0;
    }
    if (hopspin) a[C] = lane < C ? PTt[kh * C + lane] : (lane == C ? Gj[kh] : 0.0);
    else a[C] = lane == C ? 1.0 : 0.0;
    rdim = C + (hopspin ? 1 : 0);
  }
  return lu_det_rot<RM>(a, rdim, lane);
}

}  // namespace svmc
