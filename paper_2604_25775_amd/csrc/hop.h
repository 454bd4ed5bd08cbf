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
// One wavefront evaluates one hop.  Per-wave LDS scratch: a grid holding one
// layer's features on the box ([Gy][Gx][C], Tf) and two label lists.
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

// Per-wave scratch bytes for a lattice.
inline size_t hop_scratch_bytes(int Gx, int Gy, int C, int tf_bytes) {
  size_t g = (size_t)Gx * Gy * C * tf_bytes;
  g = (g + 15) & ~(size_t)15;
  return g + (size_t)2 * Gx * Gy * sizeof(int);
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

// Incremental conv stack for one hop.  On return the accumulators hold H'_L
// on the layer-L box (count sites, index m = ox + owx * oy), and the grid's
// first count*C entries hold D = H'_L - H_L there.  If `commit` is non-null
// every new layer value is also stored into the cache (accepted move).
template <int P, int C, int MAXT>
SVMC_DEV void hop_features(const ModelDev& md, const LatDev& lt, const HopGeom& h, const int8_t* occ_s,
                           const typename PrecT<P>::Tf* __restrict__ featw,
                           typename PrecT<P>::Tf* commit, char* scratch, int lane,
                           int& olx, int& owx, int& oly, int& owy) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  const int L = md.L, N = lt.N, Lx = lt.Lx, Gx = lt.Gx;
  const Axis ax = h.ax, ay = h.ay;
  Tf* grid = (Tf*)scratch;
  const int bit = 1 << h.sigma;
  auto occp = [&](int s) {
    int o = occ_s[s];
    if (s == h.i) o -= bit;
    if (s == h.j) o += bit;
    return o;
  };
  // layer-1 input: embedding of the new configuration on the layer-1 input
  // box (layer-1 output box grown by one site)
  {
    int lx, wx, ly, wy;
    box1(ax, h.xi, h.dx, 2, lx, wx);
    box1(ay, h.yi, h.dy, 2, ly, wy);
    const Tf* E = (const Tf*)md.embed;
    const int tot = wx * wy * C;
    for (int e = lane; e < tot; e += 64) {
      const int c = e % C, q = e / C;
      const int ux = lx + q % wx, uy = ly + q / wx;
      const int s = latc(ax, ux) + Lx * latc(ay, uy);
      grid[(gidx(ay, uy) * Gx + gidx(ax, ux)) * C + c] = E[occp(s) * C + c];
    }
  }
  Acc acc[MAXT][CC::NT];
  for (int l = 1; l <= L; ++l) {
    box1(ax, h.xi, h.dx, l, olx, owx);
    box1(ay, h.yi, h.dy, l, oly, owy);
    const int cnt = owx * owy;
    const int T = (cnt + 15) >> 4;
    const Tb* Bl = (const Tb*)md.Bpack + (long long)(l - 1) * CC::Q * CC::NT * 64;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < T) {
        const int m = 16 * t + (lane & 15);
        const int ux = olx + m % owx, uy = oly + m / owx;
        int nb[9];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
          const int nx = ux + (tp % 3) - 1, ny = uy + (tp / 3) - 1;
          const bool ok = m < cnt && inlat(ax, nx) && inlat(ay, ny);
          nb[tp] = ok ? (gidx(ay, ny) * Gx + gidx(ax, nx)) * C : -1;
        }
        conv_tile<P, C>(grid, nb, Bl, lane, acc[t]);
      }
    }
    // epilogue: H'_l = H'_{l-1} + act(conv + b) (residual read from the grid)
    const Tf* bias = (const Tf*)md.bias + (l - 1) * C;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < T) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + OutMap<P>::row(lane, v);
            const int n = 16 * nt + OutMap<P>::col(lane, v);
            if (r < cnt && n < C) {
              const int ux = olx + r % owx, uy = oly + r / owx;
              const Tf z = acc[t][nt][v] + bias[n];
              acc[t][nt][v] = grid[(gidx(ay, uy) * Gx + gidx(ax, ux)) * C + n] + act_fn<Tf>(md.act, z);
            }
          }
      }
    }
    if (l < L) {
      // store H'_l on the box, then fill the ring of the next input box
      // with cached H_l
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t < T) {
#pragma unroll
          for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = 16 * t + OutMap<P>::row(lane, v);
              const int n = 16 * nt + OutMap<P>::col(lane, v);
              if (r < cnt && n < C) {
                const int ux = olx + r % owx, uy = oly + r / owx;
                grid[(gidx(ay, uy) * Gx + gidx(ax, ux)) * C + n] = acc[t][nt][v];
                if (commit) {
                  const int s = latc(ax, ux) + Lx * latc(ay, uy);
                  commit[((long long)(l - 1) * N + s) * C + n] = acc[t][nt][v];
                }
              }
            }
        }
      }
      // input box of layer l+1 = its output box (distance l+1) grown by one
      int ilx, iwx, ily, iwy;
      box1(ax, h.xi, h.dx, l + 2, ilx, iwx);
      box1(ay, h.yi, h.dy, l + 2, ily, iwy);
      const Tf* Hl = featw + (long long)(l - 1) * N * C;
      constexpr int V = 16 / sizeof(Tf);          // elements per 16-byte vector
      constexpr int CV = C / V;
      const int tot = iwx * iwy * CV;
      for (int e = lane; e < tot; e += 64) {
        const int q = e / CV, cv = e % CV;
        const int ux = ilx + q % iwx, uy = ily + q / iwx;
        if (inbox(ax, olx, owx, ux) && inbox(ay, oly, owy, uy)) continue;
        const int s = latc(ax, ux) + Lx * latc(ay, uy);
        const float4 val = *reinterpret_cast<const float4*>(Hl + (long long)s * C + cv * V);
        *reinterpret_cast<float4*>(grid + (gidx(ay, uy) * Gx + gidx(ax, ux)) * C + cv * V) = val;
      }
    }
  }
  // D = H'_L - H_L on the layer-L box, stored densely as [m][C]
  {
    const int cnt = owx * owy;
    const int T = (cnt + 15) >> 4;
    const Tf* HL = featw + (long long)(L - 1) * N * C;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < T) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + OutMap<P>::row(lane, v);
            const int n = 16 * nt + OutMap<P>::col(lane, v);
            if (r < cnt && n < C) {
              const int ux = olx + r % owx, uy = oly + r / owx;
              const int s = latc(ax, ux) + Lx * latc(ay, uy);
              const Tf old = HL[(long long)s * C + n];
              if (commit) commit[((long long)(L - 1) * N + s) * C + n] = acc[t][nt][v];
              acc[t][nt][v] = acc[t][nt][v] - old;
            }
          }
      }
    }
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < T) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * t + OutMap<P>::row(lane, v);
            const int n = 16 * nt + OutMap<P>::col(lane, v);
            if (r < cnt && n < C) grid[r * C + n] = acc[t][nt][v];
          }
      }
    }
  }
}

// Lists, per spin, the electrons whose orbital row changes: every electron of
// the new configuration on the layer-L box, entry (m << 16) | label, where m
// indexes the box.  The moving electron keeps its label at its new site.
// Returns the list position of the moving electron in its spin's list.
SVMC_DEV int hop_klists(const LatDev& lt, const HopGeom& h, const int8_t* occ_s, const int16_t* lab_s,
                        int olx, int owx, int oly, int owy, int* kl, int KM, int (&nk)[2], int lane) {
  const int N = lt.N, Lx = lt.Lx;
  const int cnt = owx * owy;
  const int bit = 1 << h.sigma;
  nk[0] = nk[1] = 0;
  int hpos = -1;
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
#pragma unroll
    for (int tau = 0; tau < 2; ++tau) {
      const bool pred = m < cnt && ((o >> tau) & 1);
      const unsigned long long mask = __ballot(pred);
      const int idx = nk[tau] + __popcll(mask & ((1ULL << lane) - 1ULL));
      const bool mover = pred && tau == h.sigma && s == h.j;
      if (pred) {
        const int k = mover ? lab_s[h.sigma * N + h.i] : lab_s[tau * N + s];
        kl[tau * KM + idx] = (m << 16) | k;
      }
      const unsigned long long mm = __ballot(mover);
      if (mm) hpos = nk[tau] + __popcll(mask & ((1ULL << (__ffsll((long long)mm) - 1)) - 1ULL));
      nk[tau] += __popcll(mask);
    }
  }
  return hpos;
}

// det of the Woodbury/determinant-lemma matrix of spin tau for one hop.
//   row form (|K| <= C):  A[a][b] = delta_ab + D(m_a) . P[:, k_b]
//                         + [a = mover] (G[j][k_b] - delta_ab)
//   column form (|K| > C): det(I + V U) with U = [D_K, e_h], V = [P_K; g - e_h]
// Both equal det(Phi'[K] Phi^-1[:, K]).  All in FP64.
template <class Tf, int C>
SVMC_DEV double hop_det(const int* kl, int K, bool hopspin, int hpos, const Tf* Dbuf,
                        const double* __restrict__ PTt, const double* __restrict__ Gj, int lane) {
  if (K == 0) return 1.0;
  constexpr int RM = C + 1;
  double a[RM];
  int rdim;
  if (K <= C) {
    const int e = lane < K ? kl[lane] : 0;
    const int ma = e >> 16;
    double Da[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Da[c] = lane < K ? (double)Dbuf[ma * C + c] : 0.0;
#pragma unroll
    for (int b = 0; b < RM; ++b) {
      if (b < K) {
        const int kb = uniform_i(kl[b]) & 0xffff;
        const double* pt = PTt + kb * C;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) s = fma(Da[c], pt[c], s);
        s += (lane == b) ? 1.0 : 0.0;
        if (hopspin && lane == hpos) s += Gj[kb] - (b == hpos ? 1.0 : 0.0);
        a[b] = s;
      } else {
        a[b] = (lane == b) ? 1.0 : 0.0;
      }
    }
    rdim = K;
  } else {
#pragma unroll
    for (int c = 0; c < RM; ++c) a[c] = 0.0;
    for (int q = 0; q < K; ++q) {
      const int e = uniform_i(kl[q]);
      const int mq = e >> 16, kq = e & 0xffff;
      double p = 0.0;
      if (lane < C) p = PTt[kq * C + lane];
      else if (hopspin && lane == C) p = Gj[kq] - (q == hpos ? 1.0 : 0.0);
      const Tf* Dq = Dbuf + mq * C;
#pragma unroll
      for (int c = 0; c < C; ++c) a[c] = fma(p, (double)Dq[c], a[c]);
    }
    const int kh = hopspin ? (uniform_i(kl[hpos]) & 0xffff) : 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (lane == c) a[c] += 1.0;
      if (lane > C || (!hopspin && lane == C)) a[c] = 0.0;
    }
    if (hopspin) a[C] = lane < C ? PTt[kh * C + lane] : (lane == C ? Gj[kh] : 0.0);
    else a[C] = lane == C ? 1.0 : 0.0;
    rdim = C + (hopspin ? 1 : 0);
  }
  return lu_det_rows<RM>(a, rdim, lane);
}

}  // namespace svmc
