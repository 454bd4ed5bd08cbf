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

// ---------------------------------------------------------------------------
// Connected configurations of the Hamiltonians of Sec. III, in canonical
// order.  Items e in [0, 2N): the electron of spin e / N on site e % N,
// hopping in directions 0 .. nd-1 (+x, -x, +y, -y, then the diagonals when
// t' != 0) to a site without an electron of that spin (t-J: to an empty
// site, the Gutzwiller projection); items e in [2N, 3N), t-J only: the spin
// exchange of the lone up electron on site e - 2N with a lone down electron
// on a nearest-neighbour site (directions 0..3).  Codes: (i << 4) | (spin
// << 3) | d for a hop, ((N + i) << 4) | d for an exchange (N <= 2048 then).
// ---------------------------------------------------------------------------
SVMC_DEV int conn_items(const LatDev& lt) { return lt.tj ? 3 * lt.N : 2 * lt.N; }

// site at direction d from i, or -1 off an open edge
SVMC_DEV int conn_target(const LatDev& lt, int i, int d) {
  int x = i % lt.Lx + dir_dx(d), y = i / lt.Lx + dir_dy(d);
  if (lt.pbc_x) x = imod(x, lt.Lx); else if (x < 0 || x >= lt.Lx) return -1;
  if (lt.pbc_y) y = imod(y, lt.Ly); else if (y < 0 || y >= lt.Ly) return -1;
  return x + lt.Lx * y;
}

// valid directions of item e as a bit mask
SVMC_DEV unsigned conn_mask(const LatDev& lt, const int8_t* occ, int e) {
  const int N = lt.N;
  unsigned m = 0;
  if (e < 2 * N) {
    const int sp = e >= N ? 1 : 0, i = e - sp * N;
    if (!((occ[i] >> sp) & 1)) return 0;
    for (int d = 0; d < lt.nd; ++d) {
      const int j = conn_target(lt, i, d);
      if (j < 0) continue;
      const int o = occ[j];
      if (lt.tj ? o != 0 : ((o >> sp) & 1)) continue;
      m |= 1u << d;
    }
  } else {
    const int i = e - 2 * N;
    if (occ[i] != 1) return 0;
    for (int d = 0; d < 4; ++d) {
      const int j = conn_target(lt, i, d);
      if (j >= 0 && occ[j] == 2) m |= 1u << d;
    }
  }
  return m;
}

SVMC_DEV int conn_code(const LatDev& lt, int e, int d) {
  const int N = lt.N;
  if (e >= 2 * N) return ((e - N) << 4) | d;
  const int sp = e >= N ? 1 : 0;
  return ((e - sp * N) << 4) | (sp << 3) | d;
}

// Decoded code: ex = spin exchange (sp = 0: the up electron leaves i).
struct Conn {
  int i, sp, d, ex;
};
SVMC_DEV Conn conn_decode(const LatDev& lt, int code) {
  Conn c;
  const int a = code >> 4;
  c.ex = a >= lt.N ? 1 : 0;
  c.i = c.ex ? a - lt.N : a;
  c.sp = c.ex ? 0 : (code >> 3) & 1;
  c.d = code & 7;
  return c;
}

// Hopping amplitude of a connection: the local-energy term is -amp * R with
// R the in-place ratio (for a spin exchange both spins move in place and
// the matrix element of (J/2)(S+S- + S-S+) is -(J/2) times the product of
// the two spins' signs, so amp = J/2).
SVMC_DEV double conn_amp(const LatDev& lt, const Conn& c) { return c.ex ? 0.5 * lt.J : (c.d < 4 ? lt.t : lt.tp); }

// Diagonal part of the local energy: U per doubly occupied site (Hubbard);
// t-J: J S^z_i S^z_j over nearest-neighbour bonds (each once, via the +x and
// +y neighbours) plus the staggered pinning field hpin (-1)^y S^z on the
// column x = 0.  One thread.
SVMC_DEV double diag_energy(const LatDev& lt, const int8_t* occ) {
  const int N = lt.N;
  if (!lt.tj) {
    int ndbl = 0;
    for (int s = 0; s < N; ++s) ndbl += occ[s] == 3;
    return lt.U * ndbl;
  }
  auto sz = [&](int s) { return 0.5 * (double)((occ[s] & 1) - ((occ[s] >> 1) & 1)); };
  double zz = 0.0, pin = 0.0;
  for (int s = 0; s < N; ++s) {
    const double z = sz(s);
    if (z == 0.0) continue;
    const int a = conn_target(lt, s, 0), b = conn_target(lt, s, 2);
    if (a >= 0) zz += z * sz(a);
    if (b >= 0) zz += z * sz(b);
  }
  for (int y = 0; y < lt.Ly; ++y) pin += (y & 1 ? -1.0 : 1.0) * sz(lt.Lx * y);
  return lt.J * zz + lt.hpin * pin;
}

// q / w for 0 <= q < 1087 and 1 <= w <= 64 as (q * m) >> 16 with
// m = 65536 / w + 1 (checked exhaustively over that range).  Box widths are
// at most 2L + 4 and box sizes at most (2L + 4)^2 sites.
__constant__ const int kMagic16[65] = {
    0,     65537, 32769, 21846, 16385, 13108, 10923, 9363, 8193, 7282, 6554, 5958, 5462, 5042, 4682, 4370, 4097,
    3856,  3641,  3450,  3277,  3121,  2979,  2850,  2731, 2622, 2521, 2428, 2341, 2260, 2185, 2115, 2049,
    1986,  1928,  1873,  1821,  1772,  1725,  1681,  1639, 1599, 1561, 1525, 1490, 1457, 1425, 1395, 1366,
    1338,  1311,  1286,  1261,  1237,  1214,  1192,  1171, 1150, 1130, 1111, 1093, 1075, 1058, 1041, 1025};
SVMC_DEV int fdiv16(int q, int m) { return (q * m) >> 16; }

// One lattice axis as seen from a hop.  Coordinates u are "unwrapped"
// (may leave [0, La) on periodic axes, by at most L + 2).  Window mode: grid
// index u - go.  Torus mode (periodic axis shorter than the largest box,
// La < 2L + 4): grid index u mod La.
struct Axis {
  int La, per, torus, go, m;    // m = kMagic16[La] (torus mode)
};
// u mod La: torus axes (La <= 2L + 3, u >= -8 La) by the magic division,
// window-mode periodic axes (u in [-La, 2 La)) by one conditional step.
SVMC_DEV int wrapt(const Axis& a, int u) {
  const int v = u + 8 * a.La;
  return v - a.La * fdiv16(v, a.m);
}
SVMC_DEV int wrapw(const Axis& a, int u) { return u < 0 ? u + a.La : (u >= a.La ? u - a.La : u); }
SVMC_DEV int gidx(const Axis& a, int u) { return a.torus ? wrapt(a, u) : u - a.go; }
SVMC_DEV bool inlat(const Axis& a, int u) { return a.per || (u >= 0 && u < a.La); }
SVMC_DEV int latc(const Axis& a, int u) { return a.per ? (a.torus ? wrapt(a, u) : wrapw(a, u)) : u; }
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
  return a.torus ? wrapt(a, u - lo) < w : (u >= lo && u < lo + w);
}
// Box site q (x fastest) -> unwrapped coordinates; m = kMagic16[w].
SVMC_DEV void box_site(int q, int lx, int w, int m, int ly, int& ux, int& uy) {
  const int qy = fdiv16(q, m);
  ux = lx + q - qy * w;
  uy = ly + qy;
}


// One connected configuration seen as a local move: sites i and j change.
// A hop of spin sigma: occupation codes change by di = -(1 << sigma) at i
// and -di at j.  A spin exchange (sigma = 0): the up electron goes i -> j
// and the down electron j -> i, di = +1 at i and -1 at j; di > 0 marks it.
struct HopGeom {
  int i, j, sigma, d, di;
  Axis ax, ay;
  int xi, yi, dx, dy;
};

SVMC_DEV HopGeom hop_geom(const LatDev& lt, int L, int sigma, int i, int d, int ex = 0) {
  HopGeom h;
  h.i = i; h.sigma = sigma; h.d = d;
  h.di = ex ? 1 : -(1 << sigma);
  h.dx = dir_dx(d); h.dy = dir_dy(d);
  h.xi = i % lt.Lx; h.yi = i / lt.Lx;
  const int xj = lt.pbc_x ? imod(h.xi + h.dx, lt.Lx) : h.xi + h.dx;
  const int yj = lt.pbc_y ? imod(h.yi + h.dy, lt.Ly) : h.yi + h.dy;
  h.j = xj + lt.Lx * yj;
  h.ax = Axis{lt.Lx, lt.pbc_x, lt.torus_x, h.xi + min(0, h.dx) - L - 1, kMagic16[lt.torus_x ? lt.Lx : 1]};
  h.ay = Axis{lt.Ly, lt.pbc_y, lt.torus_y, h.yi + min(0, h.dy) - L - 1, kMagic16[lt.torus_y ? lt.Ly : 1]};
  return h;
}

// Site stride of the LDS feature arrays: C channels plus 16 bytes, so that
// the 16 rows of an MFMA fragment (16 different sites) fall into different
// LDS banks.
template <class Tf, int C> struct SiteStride {
  static constexpr int value = C + 16 / (int)sizeof(Tf);
};

// Storage of the dense difference D = H'_L - H_L that the determinant
// assembly reads: the feature type (the difference is formed in FP64 and
// rounded once), row stride C + 4 elements.  FP32 storage keeps the hop's
// LDS at the size of its feature grid.
template <int P> struct DType {
  typedef typename PrecT<P>::Tf type;
};
template <int C> struct DStride {
  static constexpr int value = C + 4;
};

// LDS scratch of one hop, in bytes:
//   grid   [Gy][Gx][SP] Tf  features of one layer on the update box, then one
//                           all-zero record (the conv's zero padding); after the
//                           last layer, D = H'_L - H_L densely as Tf [m][C + 4];
//                           once both determinant matrices are built, their
//                           row-major copies [2][C + 1][C + 2] f64
//   klists [2][Gx Gy] int   changed-row lists per spin
//   misc   64 bytes         per-spin results
//   bias   [L][C] f32       conv biases (FP32 feature modes), filled once per
//                           workgroup by hop_scratch_init
//   emb    [4][C] Tf        the shared embedding table (first 4 C entries of
//                           the embedding), filled once per workgroup
struct HopScratch {
  int klists, misc, bias, emb, bytes;
};
__host__ __device__ inline int align16i(int x) { return (x + 15) & ~15; }
// rows_only: the caller stages only row-form matrices (16 x 17 per wavefront)
__host__ __device__ inline HopScratch hop_scratch(int Gx, int Gy, int L, int C, int tfb, bool rows_only = false) {
  HopScratch h;
  const int SP = C + 16 / tfb;
  const int ox = Gx < 2 * L + 2 ? Gx : 2 * L + 2, oy = Gy < 2 * L + 2 ? Gy : 2 * L + 2;
  const int gb = (Gx * Gy + 1) * SP * tfb, db = ox * oy * (C + 4) * tfb;
  // two determinant stagings: column form (C + 1) x (C + 2) or row form
  // 16 x 17 doubles per wavefront, whichever is larger
  const int sc = rows_only ? 0 : (C + 1) * (C + 2), sr = 16 * 17;
  const int sb = 2 * (sc > sr ? sc : sr) * 8;
  const int rb = gb > db ? gb : db;
  h.klists = align16i(rb > sb ? rb : sb);
  h.misc = h.klists + align16i(2 * Gx * Gy * 4);
  h.bias = h.misc + 64;
  h.emb = h.bias + align16i(L * C * 4);
  h.bytes = h.emb + align16i(4 * C * tfb);
  return h;
}

// Per-workgroup set-up of the hop scratch: the conv biases (FP32 feature
// modes) and the shared embedding table into LDS (with per-site tables the
// copy is not used).  All threads of the block call it; a barrier must follow
// before the first hop.
template <int P>
SVMC_DEV void hop_scratch_init(const ModelDev& md, char* scratch, const HopScratch& hs) {
  typedef typename PrecT<P>::Tf Tf;
  if constexpr (sizeof(Tf) == 4) {
    const float* b = (const float*)md.bias;
    float* d = (float*)(scratch + hs.bias);
    for (int e = threadIdx.x; e < md.L * md.C; e += blockDim.x) d[e] = b[e];
  }
  const Tf* E = (const Tf*)md.embed;
  Tf* de = (Tf*)(scratch + hs.emb);
  for (int e = threadIdx.x; e < 4 * md.C; e += blockDim.x) de[e] = E[e];
}

// B fragments of a layer kept in registers when they fit (<= 80 VGPRs).
template <int P, int C> struct RegB {
  static constexpr bool value =
      ConvCfg<P, C>::Q * ConvCfg<P, C>::NT * (int)sizeof(typename PrecT<P>::Tb) <= 80 * 4;
};

// LDS feature grid of the hop: per site a record of SiteStride<Tf, C> Tf.
// In PREC_F16X2 the record holds the features already split into their FP16
// pair: hi[C] then lo[C] (FP16), then 16 bytes of padding (same size as the
// FP32 record), so the conv reads MFMA operands directly.
template <int P> struct GridPlanes {
  static constexpr bool value = P == PREC_F16X2;
};

// Four consecutive channels n0 .. n0 + 3 of grid site record `rec`.
template <int C> SVMC_DEV void planes_put4(char* rec, int n0, float a, float b, float c, float d) {
  unsigned h0, l0, h1, l1;
  pair_split2(a, b, h0, l0);
  pair_split2(c, d, h1, l1);
  *reinterpret_cast<uint2*>(rec + 2 * n0) = uint2{h0, h1};
  *reinterpret_cast<uint2*>(rec + 2 * C + 2 * n0) = uint2{l0, l1};
}
template <int C> SVMC_DEV void planes_get4(const char* rec, int n0, float (&x)[4]) {
  const uint2 h = *reinterpret_cast<const uint2*>(rec + 2 * n0);
  const uint2 l = *reinterpret_cast<const uint2*>(rec + 2 * C + 2 * n0);
  const v2h h0 = __builtin_bit_cast(v2h, h.x), h1 = __builtin_bit_cast(v2h, h.y);
  const v2h l0 = __builtin_bit_cast(v2h, l.x), l1 = __builtin_bit_cast(v2h, l.y);
  x[0] = (float)h0[0] + (float)l0[0];
  x[1] = (float)h0[1] + (float)l0[1];
  x[2] = (float)h1[0] + (float)l1[0];
  x[3] = (float)h1[1] + (float)l1[1];
}

// One 16-site tile of a layer on the LDS grid.  px / py: packed grid
// coordinates of the lane's site (byte k = offset k - 1, 0xFF = zero padding).
// B fragments come from registers (breg) or global memory (Bl).  Per output
// element the accumulation order equals conv_tile's (chunk by chunk; in the
// split modes all output tiles of one term before the next term).
template <int P, int C>
SVMC_DEV void conv_tile_grid(const typename PrecT<P>::Tf* __restrict__ grid, int Gx, int zsite, unsigned px, unsigned py,
                             const typename PrecT<P>::Tb (&breg)[RegB<P, C>::value ? ConvCfg<P, C>::Q : 1]
                                                               [ConvCfg<P, C>::NT],
                             const typename PrecT<P>::Tb* __restrict__ Bl, int lane,
                             typename PrecT<P>::Acc (&acc)[ConvCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef ConvCfg<P, C> CC;
  constexpr int SP = SiteStride<Tf, C>::value;
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
    if constexpr (Mma16<P>::value) {
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
    // zero padding reads the all-zero record: the loads need no branch
    const bool ok = kok && gx != 0xFFu && gy != 0xFFu;
    const int site = ok ? (int)gy * Gx + (int)gx : zsite;
    if constexpr (GridPlanes<P>::value) {
      const char* rec = reinterpret_cast<const char*>(grid) + site * SP * (int)sizeof(Tf) + 2 * c0;
      const v8h hi = *reinterpret_cast<const v8h*>(rec);
      const v8h lo = *reinterpret_cast<const v8h*>(rec + 2 * C);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], hi);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], lo);
    } else if constexpr (Mma16<P>::value) {
      const int off = site * SP + c0;
      float x[8];
      const float4* p4 = reinterpret_cast<const float4*>(grid + off);
      const float4 x0 = p4[0], x1 = p4[1];
      x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
      x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
      mma_chunk16<P, CC::NT>(acc, x, b);
    } else {
      const int off = site * SP + c0;
      const Tf a = grid[off];
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], a);
    }
  }
}

// The same tile when both axes are in window mode (no torus wrap): the grid
// is a window of unwrapped coordinates whose off-lattice records hold zeros,
// so tap t of the lane's site is the record cen + (t/3 - 1) Gx + (t%3 - 1),
// one add per K chunk (a uniform tap offset when a chunk holds one tap).  cen
// must be a record whose 3 x 3 neighbourhood lies in the window (padding rows
// pass any box site; their results are not used).  Same products in the same
// order as conv_tile_grid.
template <int P, int C>
SVMC_DEV void conv_tile_win(const typename PrecT<P>::Tf* __restrict__ grid, int Gx, int cen,
                            const typename PrecT<P>::Tb (&breg)[RegB<P, C>::value ? ConvCfg<P, C>::Q : 1]
                                                              [ConvCfg<P, C>::NT],
                            const typename PrecT<P>::Tb* __restrict__ Bl, int lane,
                            typename PrecT<P>::Acc (&acc)[ConvCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef ConvCfg<P, C> CC;
  constexpr int SP = SiteStride<Tf, C>::value;
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
    if constexpr (Mma16<P>::value) {
      const int k0 = 32 * q + 8 * g;
      kok = k0 < CC::K;
      tap = kok ? k0 / C : 4;
      c0 = kok ? k0 % C : 0;
    } else {
      kok = true;
      tap = (4 * q) / C;
      c0 = (4 * q) % C + g;
    }
    const int site = cen + (tap / 3 - 1) * Gx + (tap % 3 - 1);
    if constexpr (GridPlanes<P>::value) {
      const char* rec = reinterpret_cast<const char*>(grid) + site * SP * (int)sizeof(Tf) + 2 * c0;
      v8h hi = *reinterpret_cast<const v8h*>(rec);
      v8h lo = *reinterpret_cast<const v8h*>(rec + 2 * C);
      if (!kok) { hi = v8h{}; lo = v8h{}; }
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], hi);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], lo);
    } else if constexpr (Mma16<P>::value) {
      const int off = site * SP + c0;
      float x[8];
      const float4* p4 = reinterpret_cast<const float4*>(grid + off);
      const float4 x0 = p4[0], x1 = p4[1];
      x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
      x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
      if (!kok)
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      mma_chunk16<P, CC::NT>(acc, x, b);
    } else {
      const Tf a = grid[site * SP + c0];
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], b[nt], a);
    }
  }
}

// Writes four consecutive channels n0 .. n0 + 3 of FP32 features to grid
// record `site` (16-byte vector loads and stores on both layouts).
template <int P, int C>
SVMC_DEV void grid_put4(typename PrecT<P>::Tf* grid, int site, int n0, const float4& v) {
  constexpr int SP = SiteStride<typename PrecT<P>::Tf, C>::value;
  if constexpr (GridPlanes<P>::value)
    planes_put4<C>(reinterpret_cast<char*>(grid) + site * SP * 4, n0, v.x, v.y, v.z, v.w);
  else
    *reinterpret_cast<float4*>(grid + site * SP + n0) = v;
}

// Per-hop coordinate table of one wavefront, one entry per lane: for the 16
// unwrapped coordinates u = base + k of each axis (base = the hop's lower
// changed coordinate minus L + 2, enough for the layer-(L+1) box and its
// neighbours when L <= 4, also on axes shorter than 2L + 4), lane k holds for x and lane 16 + k for y the grid
// indices of u - 1, u, u + 1 in bytes 0, 1, 2 (0xFF off an open edge); lanes
// 32 + k and 48 + k hold the lattice coordinates of u.  Looked up with one
// lane permute instead of the wrap and clip arithmetic per site; lookups run
// with all lanes of the wavefront active.
struct AxisTab {
  int v;          // this lane's entry
  int bx, by;     // base coordinates (uniform)
};
SVMC_DEV AxisTab axis_tab(const HopGeom& h, int L, int lane) {
  AxisTab t;
  t.bx = h.xi + min(0, h.dx) - (L + 2);
  t.by = h.yi + min(0, h.dy) - (L + 2);
  const bool isy = (lane >> 4) & 1;
  const Axis a = isy ? h.ay : h.ax;
  const int u = (isy ? t.by : t.bx) + (lane & 15);
  int v;
  if (lane < 32) {
    v = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int uu = u + k - 1;
      // (bytes of coordinates outside the grid hold junk that no box site reads)
      v |= ((inlat(a, uu) ? gidx(a, uu) : 0xFF) & 0xFF) << (8 * k);
    }
  } else {
    v = inlat(a, u) ? latc(a, u) : 0;
  }
  t.v = v;
  return t;
}
SVMC_DEV int tab_get(const AxisTab& t, int idx) { return __builtin_amdgcn_ds_bpermute(4 * idx, t.v); }
// neighbour grid indices of unwrapped (ux, uy): bytes as in the table
SVMC_DEV unsigned tab_gx(const AxisTab& t, int ux) { return (unsigned)tab_get(t, ux - t.bx) & 0xFFFFFFu; }
SVMC_DEV unsigned tab_gy(const AxisTab& t, int uy) { return (unsigned)tab_get(t, 16 + uy - t.by) & 0xFFFFFFu; }
SVMC_DEV int tab_site(const AxisTab& t, int ux, int uy, int Lx) {
  return tab_get(t, 32 + ux - t.bx) + Lx * tab_get(t, 48 + uy - t.by);
}

// Site-wise layer tile on the LDS grid: the 16 sites' own records (record
// `site` of this lane; the all-zero record for padding rows).  In PREC_F16X2
// the record's FP16 planes are the MFMA operands directly; the products and
// their order are those of mlp_tile on the same values.
template <int P, int C>
SVMC_DEV void mlp_tile_grid(const typename PrecT<P>::Tf* __restrict__ grid, int site,
                            const typename PrecT<P>::Tb* __restrict__ Bm, int lane,
                            typename PrecT<P>::Acc (&acc)[MlpCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef MlpCfg<P, C> MC;
  constexpr int SP = SiteStride<Tf, C>::value;
  if constexpr (GridPlanes<P>::value) {
    const int g = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < MC::NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[nt][v] = 0;
#pragma unroll
    for (int q = 0; q < MC::Q; ++q) {
      typename PrecT<P>::Tb b[MC::NT];
#pragma unroll
      for (int nt = 0; nt < MC::NT; ++nt) b[nt] = Bm[(q * MC::NT + nt) * 64 + lane];
      const int k0 = 32 * q + 8 * g;
      v8h hi = {}, lo = {};
      if (k0 < C) {
        const char* rec = reinterpret_cast<const char*>(grid) + site * SP * (int)sizeof(Tf) + 2 * k0;
        hi = *reinterpret_cast<const v8h*>(rec);
        lo = *reinterpret_cast<const v8h*>(rec + 2 * C);
      }
#pragma unroll
      for (int nt = 0; nt < MC::NT; ++nt) mfma(acc[nt], b[nt], hi);
#pragma unroll
      for (int nt = 0; nt < MC::NT; ++nt) mfma(acc[nt], b[nt], lo);
    }
  } else {
    mlp_tile<P, C>(grid + site * SP, Bm, lane, acc);
  }
}

// Incremental conv stack for one hop, computed by the NW wavefronts of the
// workgroup (wave = this thread's wavefront); `tab` = axis_tab of the hop.  On return (after a barrier)
// the scratch starts with D = H'_L - H_L on the layer-L box as Tf
// [m][C + 4] (index m = ox + owx * oy).  If `commit` is non-null every new layer value is
// also stored into the cache (accepted move); commit may equal featw (the
// box of a layer never overlaps the ring read from the cache for the next).
// Each layer: the wave's tiles are convolved, the next layer's B fragments
// are requested, the new values are formed (still in registers), a barrier,
// then they replace the layer input on the grid and the ring of the next
// input box is filled from the cache.
// MAXTILES: 16-site tiles of the largest layer box the caller allows (7 for
// up to four conv layers: at most 10 x 10 sites; 1 for one conv layer: at
// most 4 x 4), which sizes the registers holding a layer's results.  MLP:
// the network may have site-wise layers (md.M > 0); without them the
// site-wise stage is not compiled in.
template <int P, int C, int NW, int MAXTILES = 7, bool MLP = false>
SVMC_DEV void hop_features(const ModelDev& md, const LatDev& lt, const HopGeom& h, const int8_t* occ_s,
                           const typename PrecT<P>::Tf* featw,
                           typename PrecT<P>::Tf* commit, char* scratch, const HopScratch& hs,
                           const AxisTab& tab, int& olx, int& owx, int& oly, int& owy) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename PrecT<P>::Tb Tb;
  typedef typename PrecT<P>::Acc Acc;
  typedef ConvCfg<P, C> CC;
  // thread index through an opaque copy: the lane-dependent index arithmetic
  // below is recomputed per hop instead of being hoisted out of the callers'
  // hop loops into registers (where it would be spilled)
  int tid;
  asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NT_ = 64 * NW;
  constexpr int SP = SiteStride<Tf, C>::value;
  constexpr bool PL = GridPlanes<P>::value;
  const int L = md.L, N = lt.N, Lx = lt.Lx, Gx = lt.Gx;
  const Axis ax = h.ax, ay = h.ay;
  // window mode on both axes: grid index = unwrapped coordinate - origin, and
  // every tap of a box site is a fixed record offset (off-lattice records of
  // the window hold zeros); otherwise taps go through the coordinate table
  const bool win = !(lt.torus_x | lt.torus_y);
  Tf* grid = (Tf*)scratch;
  constexpr int V = 16 / sizeof(Tf);          // elements per 16-byte vector
  constexpr int CV = C / V;
  constexpr int QB = RegB<P, C>::value ? CC::Q : 1;
  // B fragments of layer 1 (when held in registers), requested before the
  // embedding fill
  Tb breg[QB][CC::NT];
  auto load_b = [&](int l) {
    if constexpr (RegB<P, C>::value) {
      const Tb* Bl = (const Tb*)md.Bpack + (long long)(l - 1) * CC::Q * CC::NT * 64;
#pragma unroll
      for (int q = 0; q < CC::Q; ++q)
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt) breg[q][nt] = Bl[(q * CC::NT + nt) * 64 + lane];
    }
  };
  load_b(1);
  const int zsite = Gx * lt.Gy;             // the all-zero record after the grid
  constexpr int RV = SP * (int)sizeof(Tf) / 16;   // 16-byte vectors per grid record
  if (tid < RV) reinterpret_cast<float4*>(grid + zsite * SP)[tid] = float4{0.0f, 0.0f, 0.0f, 0.0f};
  if (win) {
    // zeros on the window's off-lattice records (open axes); the grid area
    // held the previous hop's determinant staging
    const int mg = kMagic16[Gx], GG = Gx * lt.Gy;
    for (int r = tid; r < GG; r += NT_) {
      const int gy = fdiv16(r, mg), gx = r - gy * Gx;
      if (inlat(ax, ax.go + gx) && inlat(ay, ay.go + gy)) continue;
      float4* d = reinterpret_cast<float4*>(grid + r * SP);
#pragma unroll
      for (int k = 0; k < RV; ++k) d[k] = float4{0.0f, 0.0f, 0.0f, 0.0f};
    }
  }
  // layer-1 input: embedding of the new configuration on the layer-1 input
  // box (layer-1 output box grown by one site)
  {
    int lx, wx, ly, wy;
    box1(ax, h.xi, h.dx, 2, lx, wx);
    box1(ay, h.yi, h.dy, 2, ly, wy);
    const Tf* E = (const Tf*)md.embed;
    const int mw = kMagic16[wx];
    const int tot = wx * wy * CV;
    for (int e0 = 0; e0 < tot; e0 += NT_) {
      // table lookups with every lane active (a permute reads nothing useful
      // from a disabled lane)
      const int e = e0 + tid;
      const int q = e / CV, cv = e - q * CV;
      int ux, uy;
      box_site(q, lx, wx, mw, ly, ux, uy);
      const int s = tab_site(tab, ux, uy, Lx);
      const int site = (int)((tab_gy(tab, uy) >> 8) & 0xFFu) * Gx + (int)((tab_gx(tab, ux) >> 8) & 0xFFu);
      if (e >= tot) continue;
      int o = occ_s[s];
      if (s == h.i) o += h.di;
      if (s == h.j) o -= h.di;
      // one shared table: its LDS copy; per-site tables from memory
      const float4 ev = lt.emb_ss == 0
                            ? *reinterpret_cast<const float4*>((const Tf*)(scratch + hs.emb) + o * C + cv * V)
                            : *reinterpret_cast<const float4*>(E + lt.emb_off + (long long)s * lt.emb_ss + o * C + cv * V);
      if constexpr (PL)
        grid_put4<P, C>(grid, site, cv * V, ev);
      else
        *reinterpret_cast<float4*>(grid + site * SP + cv * V) = ev;
    }
  }
  __syncthreads();
  for (int l = 1; l <= L; ++l) {
    // the thread index once more through an opaque copy per layer: the
    // per-tile lane addresses below are then recomputed in each layer rather
    // than hoisted out of the layer loop and spilled
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    const int lane = tid & 63;
    box1(ax, h.xi, h.dx, l, olx, owx);
    box1(ay, h.yi, h.dy, l, oly, owy);
    const int cnt = uniform_i(owx * owy);
    const int mow = kMagic16[owx];
    const int T = (cnt + 15) >> 4;
    const Tb* Bl = (const Tb*)md.Bpack + (long long)(l - 1) * CC::Q * CC::NT * 64;
    const Tf* bias = (const Tf*)md.bias + (l - 1) * C;
    constexpr bool FULLC = C % 16 == 0;        // every channel of every output tile exists
    const float* bias_s = (const float*)(scratch + hs.bias) + (l - 1) * C;   // the same biases in LDS
    // Each wave keeps its tiles' results in registers until every wave has
    // finished reading the grid of this layer (at most 7 tiles: the layer-L
    // box of L <= 4 has at most 10 x 10 sites).  The lane's site is the same
    // in all four slots v (OutMap).
    constexpr int MAXT = (MAXTILES + NW - 1) / NW;
    Acc acc[MAXT][CC::NT];
    int gsite[MAXT];               // grid record of the lane's site, -1 for padding rows
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int t = wave + NW * ti;
      gsite[ti] = -1;
      if (t >= T) break;
      const int m = 16 * t + (lane & 15);
      if (win) {
        // padding rows compute from the box's last site
        const int mm = m < cnt ? m : cnt - 1;
        int ux, uy;
        box_site(mm, olx, owx, mow, oly, ux, uy);
        const int cen = (uy - ay.go) * Gx + (ux - ax.go);
        if (m < cnt) gsite[ti] = cen;
        conv_tile_win<P, C>(grid, Gx, cen, breg, Bl, lane, acc[ti]);
      } else {
        unsigned px = 0xFFFFFFu, py = 0xFFFFFFu;
        int ux, uy;
        box_site(m, olx, owx, mow, oly, ux, uy);
        const unsigned tx = tab_gx(tab, ux), ty = tab_gy(tab, uy);
        if (m < cnt) {
          px = tx;
          py = ty;
          gsite[ti] = (int)((ty >> 8) & 0xFFu) * Gx + (int)((tx >> 8) & 0xFFu);
        }
        conv_tile_grid<P, C>(grid, Gx, zsite, px, py, breg, Bl, lane, acc[ti]);
      }
    }
    // the next layer's B fragments are in flight during the rest of this one
    if (l < L) load_b(l + 1);
    // H'_l = H'_{l-1} + act(conv + b); the residual is this site's own grid
    // value (padding rows compute from another record and are not stored)
    if constexpr (PL) {
      auto epilogue = [&](auto actc) {
        constexpr int A = decltype(actc)::value;
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti) {
          const int t = wave + NW * ti;
          if (t >= T) break;
          const char* rec = reinterpret_cast<const char*>(grid + (gsite[ti] >= 0 ? gsite[ti] : zsite) * SP);
#pragma unroll
          for (int nt = 0; nt < CC::NT; ++nt) {
            const int n0 = 16 * nt + OutMap<P>::chan(lane, 0);
            if (!FULLC && n0 >= C) continue;
            float x[4];
            planes_get4<C>(rec, n0, x);
            const float4 b4 = *reinterpret_cast<const float4*>(bias_s + n0);
            const float bv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[ti][nt][v] = layer_out_c<P, A>(x[v], acc[ti][nt][v] + bv[v]);
          }
        }
      };
      if (md.act == ACT_TANH) epilogue(ActC<ACT_TANH>());
      else epilogue(ActC<ACT_SILU>());
    } else {
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int t = wave + NW * ti;
      if (t >= T) break;
      const bool on = gsite[ti] >= 0;
      const int gofs = (on ? gsite[ti] : zsite) * SP;
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) {
        {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            Tf val = Tf(0);
            if (on && n < C) val = layer_out<P, Tf>(md.act, grid[gofs + n], Tf(acc[ti][nt][v] + bias[n]));
            acc[ti][nt][v] = val;
          }
        }
      }
    }
    }
    __syncthreads();
    // the cached features the new ones replace: the last plane (conv layer L,
    // or the last site-wise layer)
    const int M = MLP ? md.M : 0, FL = L + M - 1;
    const Tf* HL = featw + (long long)FL * N * C;
    typedef typename DType<P>::type DT;
    // this tile's new values replace the old ones on the grid (and go to
    // cache plane cp on accept)
    auto put_tile = [&](int ti, int s, int cp) {
      const int site = gsite[ti];
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) {
        if constexpr (PL) {
          const int n0 = 16 * nt + OutMap<P>::chan(lane, 0);
          if (n0 >= C) continue;
          const float4 v4 = {acc[ti][nt][0], acc[ti][nt][1], acc[ti][nt][2], acc[ti][nt][3]};
          grid_put4<P, C>(grid, site, n0, v4);
          if (commit) *reinterpret_cast<float4*>(commit + ((long long)cp * N + s) * C + n0) = v4;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            if (n >= C) continue;
            grid[site * SP + n] = acc[ti][nt][v];
            if (commit) commit[((long long)cp * N + s) * C + n] = acc[ti][nt][v];
          }
        }
      }
    };
    // D = H'_F - H_F (F the last plane), densely [m][C + 4] at the start of
    // the scratch
    auto put_D = [&](int ti, int r, int s) {
      DT* D = reinterpret_cast<DT*>(grid);
      if constexpr (PL) {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt) {
          const int n0 = 16 * nt + OutMap<P>::chan(lane, 0);
          if (!FULLC && n0 >= C) continue;
          const long long gi = (long long)s * C + n0;
          const float4 old = *reinterpret_cast<const float4*>(HL + gi);
          const float4 nw = {acc[ti][nt][0], acc[ti][nt][1], acc[ti][nt][2], acc[ti][nt][3]};
          const float4 d = {(float)((double)nw.x - (double)old.x), (float)((double)nw.y - (double)old.y),
                            (float)((double)nw.z - (double)old.z), (float)((double)nw.w - (double)old.w)};
          *reinterpret_cast<float4*>(D + r * DStride<C>::value + n0) = d;
          if (commit) *reinterpret_cast<float4*>(commit + (long long)FL * N * C + gi) = nw;
        }
      } else {
#pragma unroll
        for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int n = 16 * nt + OutMap<P>::chan(lane, v);
            if (n >= C) continue;
            const long long gi = (long long)s * C + n;
            const Tf old = HL[gi];
            D[r * DStride<C>::value + n] = (DT)((double)acc[ti][nt][v] - (double)old);
            if (commit) commit[(long long)FL * N * C + gi] = acc[ti][nt][v];
          }
      }
    };
    const bool dnow = l == L && M == 0;
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int t = wave + NW * ti;
      if (t >= T) break;
      const int r = 16 * t + (lane & 15);
      int ux, uy;
      box_site(r, olx, owx, mow, oly, ux, uy);
      const int s = tab_site(tab, ux, uy, Lx);     // every lane active
      if (gsite[ti] < 0) continue;
      if (!dnow) put_tile(ti, s, l - 1);
      else put_D(ti, r, s);
    }
    if (MLP && l == L && M > 0) {
      // the site-wise layers (Sec. II.B, site-wise MLP equation) on the
      // layer-L box: each wavefront runs its own tiles, a site reading only
      // its own record, so the wavefronts do not wait for each other
      for (int m = 0; m < M; ++m) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const Tb* Bm = (const Tb*)md.Bmlp + (long long)m * MlpCfg<P, C>::Q * CC::NT * 64;
        const Tf* mb = (const Tf*)md.bias + (long long)(L + m) * C;
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti) {
          const int t = wave + NW * ti;
          if (t >= T) break;
          mlp_tile_grid<P, C>(grid, gsite[ti] >= 0 ? gsite[ti] : zsite, Bm, lane, acc[ti]);
#pragma unroll
          for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int n = 16 * nt + OutMap<P>::chan(lane, v);
              acc[ti][nt][v] = n < C ? mlp_out<P, Tf>(md.act, Tf(acc[ti][nt][v] + mb[n])) : Tf(0);
            }
        }
        if (m + 1 == M) break;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int ti = 0; ti < MAXT; ++ti) {
          const int t = wave + NW * ti;
          if (t >= T) break;
          const int r = 16 * t + (lane & 15);
          int ux, uy;
          box_site(r, olx, owx, mow, oly, ux, uy);
          const int s = tab_site(tab, ux, uy, Lx);
          if (gsite[ti] >= 0) put_tile(ti, s, L + m);
        }
      }
      __syncthreads();    // every wavefront is done with the grid: D may overwrite it
#pragma unroll
      for (int ti = 0; ti < MAXT; ++ti) {
        const int t = wave + NW * ti;
        if (t >= T) break;
        const int r = 16 * t + (lane & 15);
        int ux, uy;
        box_site(r, olx, owx, mow, oly, ux, uy);
        const int s = tab_site(tab, ux, uy, Lx);
        if (gsite[ti] >= 0) put_D(ti, r, s);
      }
    }
    if (l < L) {
      // the ring of the next input box (output box at distance l+1 grown by
      // one) gets the cached H_l; ring sites lie outside this layer's box, so
      // they are never written above.  Two threads per site, each moving half
      // of its channels, so the site's coordinates are worked out once per
      // half record.
      int ilx, iwx, ily, iwy;
      box1(ax, h.xi, h.dx, l + 2, ilx, iwx);
      box1(ay, h.yi, h.dy, l + 2, ily, iwy);
      const Tf* Hl = featw + (long long)(l - 1) * N * C;
      const int miw = kMagic16[iwx];
      constexpr int HV = CV / 2;           // 16-byte vectors per half record
      static_assert(CV % 2 == 0, "half records of whole vectors");
      const int tot = iwx * iwy * 2;
      for (int e0 = 0; e0 < tot; e0 += NT_) {
        const int e = e0 + tid;
        const int q = e >> 1, half = e & 1;
        int ux, uy;
        box_site(q, ilx, iwx, miw, ily, ux, uy);
        const int s = tab_site(tab, ux, uy, Lx);
        const int site = (int)((tab_gy(tab, uy) >> 8) & 0xFFu) * Gx + (int)((tab_gx(tab, ux) >> 8) & 0xFFu);
        const bool ok = e < tot && !(inbox(ax, olx, owx, ux) && inbox(ay, oly, owy, uy));
        if (!ok) continue;
        const Tf* src = Hl + (long long)s * C + half * HV * V;
        float4 val[HV];
#pragma unroll
        for (int u = 0; u < HV; ++u) val[u] = reinterpret_cast<const float4*>(src)[u];
#pragma unroll
        for (int u = 0; u < HV; ++u) {
          const int n0 = (half * HV + u) * V;
          if constexpr (PL) grid_put4<P, C>(grid, site, n0, val[u]);
          else *reinterpret_cast<float4*>(grid + site * SP + n0) = val[u];
        }
      }
    }
    __syncthreads();
  }
}

// Changed-row list of spin tau (one wavefront): every electron of spin tau
// in the new configuration on the layer-L box, entry (m << 16) | label, m
// indexing the box.  A moving electron keeps its label at its new site.
// Returns the list length; *hpos gets the mover's position (-1 if spin tau
// does not move: tau != sigma of a hop).
SVMC_DEV int hop_klist(const LatDev& lt, const HopGeom& h, const AxisTab& tab, const int8_t* occ_s,
                       const int16_t* lab_s, int tau, int olx, int owx, int oly, int owy, int* kl, int& hpos,
                       int lane) {
  const int N = lt.N, Lx = lt.Lx;
  const int cnt = owx * owy;
  const int mow = kMagic16[owx];
  // the moving electron of spin tau: from msrc to mdst (mdst = -1: none)
  const int mdst = tau == h.sigma ? h.j : (h.di > 0 ? h.i : -1);
  const int msrc = tau == h.sigma ? h.i : h.j;
  int nk = 0;
  hpos = -1;
  for (int base = 0; base < cnt; base += 64) {
    const int m = base + lane;
    int ux, uy;
    box_site(m, olx, owx, mow, oly, ux, uy);
    const int sl = tab_site(tab, ux, uy, Lx);      // every lane active
    int s = 0, o = 0;
    if (m < cnt) {
      s = sl;
      o = occ_s[s];
      if (s == h.i) o += h.di;
      if (s == h.j) o -= h.di;
    }
    const bool pred = m < cnt && ((o >> tau) & 1);
    const unsigned long long mask = __ballot(pred);
    const int idx = nk + __popcll(mask & ((1ULL << lane) - 1ULL));
    const bool mover = pred && s == mdst;
    if (pred) {
      const int k = mover ? lab_s[tau * N + msrc] : lab_s[tau * N + s];
      kl[idx] = (m << 16) | k;
    }
    const unsigned long long mm = __ballot(mover);
    if (mm) hpos = nk + __popcll(mask & ((1ULL << (__ffsll((long long)mm) - 1)) - 1ULL));
    nk += __popcll(mask);
  }
  return nk;
}

// Number of electrons of spin tau in the new configuration on the layer-L
// box (the length hop_klist would return), one wavefront, every lane active.
SVMC_DEV int hop_kcount(const LatDev& lt, const HopGeom& h, const AxisTab& tab, const int8_t* occ_s, int tau,
                        int olx, int owx, int oly, int owy, int lane) {
  const int Lx = lt.Lx, cnt = owx * owy, mow = kMagic16[owx];
  int nk = 0;
  for (int base = 0; base < cnt; base += 64) {
    const int m = base + lane;
    int ux, uy;
    box_site(m, olx, owx, mow, oly, ux, uy);
    const int s = tab_site(tab, ux, uy, Lx);
    int o = 0;
    if (m < cnt) {
      o = occ_s[s];
      if (s == h.i) o += h.di;
      if (s == h.j) o -= h.di;
    }
    nk += __popcll(__ballot(m < cnt && ((o >> tau) & 1)));
  }
  return nk;
}

// FP64 reciprocal: hardware estimate refined by two Newton steps (error
// below one ulp of the IEEE quotient, enough for an elimination multiplier).
SVMC_DEV double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// One-wave LU determinant of an RM x RM FP64 matrix held one row per lane
// (lanes < RM; lanes >= RM take no part), all RM elimination steps unrolled
// so that column counts are static and the code has no branches on them.
// Partial pivoting without moving rows: at step p the unused row with the
// largest |a[p]| pivots (the search compares |a| rounded to FP32, ties to
// the lower lane; a pivot column below FP32's smallest denormal makes the
// matrix count as singular and the result 0).  The pivot row reaches the
// other lanes by lane reads (its own multiplier is zero, so it does not
// change during the step).  Each step first updates the next pivot column
// and starts its search, then the remaining columns, so the search overlaps
// the update.  det = sign(permutation) * prod(pivots).
SVMC_DEV unsigned piv_key(double v, bool used, int lane) {
  return used ? 0u : ((__float_as_uint((float)fabs(v)) & ~63u) | (unsigned)(63 - lane));
}
template <int RM>
SVMC_DEV double lu_det_unrolled(double (&a)[RM], int lane) {
  bool used = lane >= RM;
  int step = 64;
  double det = 1.0;
  bool sing = false;
  unsigned kmax = wave_max_u32(piv_key(a[0], used, lane));
#pragma unroll
  for (int p = 0; p < RM; ++p) {
    sing = sing || (kmax & ~63u) == 0u;
    const int piv = 63 - (int)(kmax & 63u);
    const double pv = readlane_d(a[p], piv);
    det *= pv;
    if (lane == piv) {
      used = true;
      step = p;
    }
    if (p + 1 < RM) {
      const double l = used ? 0.0 : a[p] * rcp_d(sing ? 1.0 : pv);
      a[p + 1] = fma(-l, readlane_d(a[p + 1], piv), a[p + 1]);
      kmax = wave_max_u32(piv_key(a[p + 1], used, lane));
#pragma unroll
      for (int c = p + 2; c < RM; ++c) a[c] = fma(-l, readlane_d(a[c], piv), a[c]);
    }
  }
  int inv = 0;
#pragma unroll 1
  for (int b = 0; b < RM; ++b) {
    const int sb = __builtin_amdgcn_readlane(step, b);
    if (lane < RM && b > lane && sb < step) ++inv;
  }
  const unsigned long long odd = __ballot(inv & 1);
  if (sing) return 0.0;
  return (__popcll(odd) & 1) ? -det : det;
}

// The Woodbury / determinant-lemma matrix of spin tau for one hop (one
// wavefront), in the column form
//   A = I + V U,  U = [D_K, e_h] (changed rows K carry D(m_a); the mover's
//   row also e_h),  V = [P_K; g_K - e_h]  (P = W Phi^-1, g = G[j] = M[j] Phi^-1)
// of size C + [tau = moving spin]; det A = det(Phi'[K] Phi^-1[:, K]).
// The product V U over the changed rows is a (C + 1) x r x C contraction and
// runs on the FP64 matrix cores (16 x 16 x 4 tiles: row tiles over the C rows
// of P plus row C = g, column tiles over the C channels of D, four changed
// rows per step).  Lane l supplies changed row 4 s + l / 16 of step s.
template <int C> struct DetTiles {
  static constexpr int I = (C + 16) / 16;     // row tiles (rows 0 .. C)
  static constexpr int J = (C + 15) / 16;     // column tiles (columns 0 .. C-1)
  static constexpr int RS = C + 2;            // staged row stride (doubles)
};

template <int C, class DT>
SVMC_DEV void hop_det_build(const int* kl, int K_in, bool hopspin, int hpos_in, const DT* Dbuf,
                            const double* __restrict__ PTt, const double* __restrict__ Gj, int lane,
                            v4d (&acc)[DetTiles<C>::I][DetTiles<C>::J]) {
  typedef DetTiles<C> T;
  constexpr int SD = DStride<C>::value;
  constexpr int U = 4;                         // steps whose loads are in flight together
  // with C a multiple of 16, row C sits alone in the last row tile: it is
  // summed on the vector units (changed row q of lane group q mod 4) instead
  // of taking a row tile of products for one row
  constexpr bool ROWC_V = C % 16 == 0;
  const int K = uniform_i(K_in), hpos = uniform_i(hpos_in);
  const int r16 = lane & 15, qo = lane >> 4;
  double rc[T::J];
#pragma unroll
  for (int tj = 0; tj < T::J; ++tj) rc[tj] = 0.0;
#pragma unroll
  for (int ti = 0; ti < T::I; ++ti)
#pragma unroll
    for (int tj = 0; tj < T::J; ++tj) acc[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int q0 = 0; q0 < K; q0 += 4 * U) {
    double x[U][T::I], y[U][T::J];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + 4 * u + qo;
      const bool ok = q < K;
      const int e = ok ? kl[q] : 0;
      const int kq = e & 0xffff, mo = (e >> 16) * SD;
#pragma unroll
      for (int ti = 0; ti < T::I; ++ti) {
        const int c = ROWC_V && ti == T::I - 1 ? C : 16 * ti + r16;
        double v = 0.0;
        if (ok) {
          if (c < C) v = PTt[kq * C + c];
          else if (c == C && hopspin) v = Gj[kq] - (q == hpos ? 1.0 : 0.0);
        }
        x[u][ti] = v;
      }
#pragma unroll
      for (int tj = 0; tj < T::J; ++tj) {
        const int c = 16 * tj + r16;
        y[u][tj] = (ok && c < C) ? (double)Dbuf[mo + c] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (q0 + 4 * u >= K) break;
#pragma unroll
      for (int ti = 0; ti < T::I; ++ti) {
        if (16 * ti >= C && !hopspin) continue;          // row C only for the moving spin
        if (ROWC_V && ti == T::I - 1) {
#pragma unroll
          for (int tj = 0; tj < T::J; ++tj) rc[tj] = fma(x[u][ti], y[u][tj], rc[tj]);
          continue;
        }
#pragma unroll
        for (int tj = 0; tj < T::J; ++tj) mfma(acc[ti][tj], x[u][ti], y[u][tj]);
      }
    }
  }
  if constexpr (ROWC_V) {
    // the four lane groups' partial sums of row C to lanes 0 .. 15, where the
    // row tile's result would hold it (row 16 (I - 1) + 0 in slot 0)
#pragma unroll
    for (int tj = 0; tj < T::J; ++tj) {
      double v = rc[tj];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      acc[T::I - 1][tj][0] = qo == 0 ? v : 0.0;
    }
  }
}

// Adds the identity and column C (moving spin: P^T[k_h], G[j][k_h]) and
// stages the matrix row-major in `stage` ((C + 1) x (C + 2) doubles of this
// wavefront; the caller makes sure nothing else uses it): C x C for the spin
// that does not move, (C + 1) x (C + 1) for the moving one; with no changed
// rows (K = 0) the identity.  The 16 x 16 f64 MFMA result holds
// A[16 ti + l / 16 + 4 v][16 tj + l % 16] in slot v of lane l.
template <int C>
SVMC_DEV void hop_det_stage(const v4d (&acc)[DetTiles<C>::I][DetTiles<C>::J], const int* kl, int K_in,
                            bool hopspin, int hpos_in, const double* __restrict__ PTt,
                            const double* __restrict__ Gj, double* stage, int lane) {
  typedef DetTiles<C> T;
  constexpr int RS = T::RS;
  const int K = uniform_i(K_in), hpos = uniform_i(hpos_in);
  const int R = C + (hopspin ? 1 : 0);
  const int r16 = lane & 15, qo = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < T::I; ++ti)
#pragma unroll
    for (int tj = 0; tj < T::J; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * ti + qo + 4 * v, c = 16 * tj + r16;
        if (r < R && c < C) stage[r * RS + c] = (K > 0 ? acc[ti][tj][v] : 0.0) + (r == c ? 1.0 : 0.0);
      }
  if (hopspin) {
    const int kh = K > 0 ? kl[hpos] & 0xffff : 0;
    const double pv = PTt[kh * C + (lane < C ? lane : 0)], gv = Gj[kh];    // unconditional loads
    if (lane < C) stage[lane * RS + C] = K > 0 ? pv : 0.0;
    else if (lane == C) stage[C * RS + C] = K > 0 ? gv : 1.0;
  }
  // lanes read rows other lanes wrote: order the accesses for the compiler
  // (the hardware keeps a wavefront's LDS operations in order)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One elimination step on the staged (C + 1) x (C + 1) matrix of the moving
// spin (one wavefront, one row per lane): pivot on column 0 over all rows,
// then the C x C Schur complement (the other rows in their order, columns
// 1 .. C) replaces the matrix at the top left of the stage.  Returns the
// factor it takes off the determinant, (-1)^piv * pivot (the pivot row moved
// to the top), or 0 for a zero column.
template <int C>
SVMC_DEV double hop_det_reduce(double* stage, int lane) {
  constexpr int RM = C + 1, RS = DetTiles<C>::RS;
  double a[RM];
  const double2* rp = reinterpret_cast<const double2*>(stage + (lane < RM ? lane : 0) * RS);
#pragma unroll
  for (int c2 = 0; c2 < RS / 2; ++c2) {
    const double2 v = rp[c2];
    if (2 * c2 < RM) a[2 * c2] = lane < RM ? v.x : 0.0;
    if (2 * c2 + 1 < RM) a[2 * c2 + 1] = lane < RM ? v.y : 0.0;
  }
  const bool out = lane >= RM;
  const unsigned kmax = wave_max_u32(piv_key(a[0], out, lane));
  const bool sing = (kmax & ~63u) == 0u;
  const int piv = 63 - (int)(kmax & 63u);
  const double pv = readlane_d(a[0], piv);
  const double l = (out || lane == piv) ? 0.0 : a[0] * rcp_d(sing ? 1.0 : pv);
#pragma unroll
  for (int c = 1; c < RM; ++c) a[c] = fma(-l, readlane_d(a[c], piv), a[c]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!out && lane != piv) {
    double2* wp = reinterpret_cast<double2*>(stage + (lane - (lane > piv ? 1 : 0)) * RS);
#pragma unroll
    for (int c2 = 0; c2 < C / 2; ++c2) wp[c2] = double2{a[2 * c2 + 1], a[2 * c2 + 2]};
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (sing) return 0.0;
  return (piv & 1) ? -pv : pv;
}

// Value of lane src of a 64-bit register (src given as byte address 4 src;
// every lane must be active).
SVMC_DEV double bperm_d(int addr, double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(v & 0xffffffffLL));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(v >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Two C x C LU determinants in one wavefront: lanes 0 .. 31 hold the rows of
// the first matrix, lanes 32 .. 63 those of the second (row = lane mod 32,
// rows >= C take no part).  The same steps as the one-matrix LU above, with
// each half searching its own pivot (row maxima by DPP, the two rows of a
// half joined by a row broadcast, read back from lanes 31 and 63) and taking
// its pivot row by lane permutes.  The sign of each half's pivot order is
// kept step by step: moving the pivot ahead of the unused rows before it
// costs one transposition per such row.  Lane 0 returns the first
// determinant, lane 32 the second.
template <int C>
SVMC_DEV double lu_det_pair(double (&a)[C], int lane) {
  static_assert(C <= 32 && C % 2 == 0, "one matrix per half wavefront, rows read in pairs");
  const bool hi_half = lane >= 32;
  bool used = (lane & 31) >= C;
  double det = 1.0;
  unsigned par_lo = 0, par_hi = 0;
  bool sing_lo = false, sing_hi = false;
  auto half_max = [&](unsigned v, unsigned& k_lo, unsigned& k_hi) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    k_lo = (unsigned)__builtin_amdgcn_readlane((int)v, 31);
    k_hi = (unsigned)__builtin_amdgcn_readlane((int)v, 63);
  };
  unsigned k_lo, k_hi;
  half_max(piv_key(a[0], used, lane), k_lo, k_hi);
#pragma unroll
  for (int p = 0; p < C; ++p) {
    sing_lo = sing_lo || (k_lo & ~63u) == 0u;
    sing_hi = sing_hi || (k_hi & ~63u) == 0u;
    const int piv_lo = 63 - (int)(k_lo & 63u), piv_hi = 63 - (int)(k_hi & 63u);
    const int piv = hi_half ? piv_hi : piv_lo;
    const int addr = piv << 2;
    // rows of this half still unused and before the pivot
    const unsigned long long before = __ballot(!used && lane < piv);
    par_lo ^= (unsigned)__popcll(before & 0xffffffffULL);
    par_hi ^= (unsigned)__popcll(before >> 32);
    const double pv = bperm_d(addr, a[p]);
    det *= pv;
    if (lane == piv) used = true;
    if (p + 1 < C) {
      const bool sing = hi_half ? sing_hi : sing_lo;
      const double l = used ? 0.0 : a[p] * rcp_d(sing ? 1.0 : pv);
      a[p + 1] = fma(-l, bperm_d(addr, a[p + 1]), a[p + 1]);
      half_max(piv_key(a[p + 1], used, lane), k_lo, k_hi);
#pragma unroll
      for (int c = p + 2; c < C; ++c) a[c] = fma(-l, bperm_d(addr, a[c]), a[c]);
    }
  }
  const bool sing = hi_half ? sing_hi : sing_lo;
  const bool odd = ((hi_half ? par_hi : par_lo) & 1u) != 0u;
  if (sing) return 0.0;
  return odd ? -det : det;
}

// Value of the other lane of this lane's pair (lanes 2 r and 2 r + 1), by a
// DPP quad permutation (every lane active).
SVMC_DEV double swap_pair_d(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One C x C LU determinant per wavefront, two lanes per row: lane 2 r + h
// holds the columns of parity h of row r (a[j] = A[r][2 j + h]; rows >= C
// take no part).  Partial pivoting as in the LUs above (FP32-rounded |a|
// keys, ties to the lower lane, a column below FP32's smallest normal counts
// as zero), with the pivot searched over the lanes that hold column p.  The
// pivot value is one lane read; a row's multiplier comes from its other lane
// by a pair swap; each lane fetches the pivot row's entries of its own
// parity by lane permutes.  At step p the registers from (p + 1) / 2 on are
// updated in every lane: the one or two columns at or left of p this touches
// are never read again.  The permutation sign is kept step by step as in
// lu_det_pair.  Every lane returns the determinant.
template <int C>
SVMC_DEV double lu_det_split(double (&a)[C / 2], int lane) {
  static_assert(C % 2 == 0 && C <= 32, "two lanes per row, at most 32 rows");
  constexpr int J = C / 2;
  const int row = lane >> 1, par = lane & 1;
  bool used = row >= C;
  double det = 1.0;
  unsigned parity = 0;
  bool sing = false;
  auto key = [&](double v, int p) -> unsigned {
    return (used || par != (p & 1)) ? 0u : ((__float_as_uint((float)fabs(v)) & ~63u) | (unsigned)(63 - lane));
  };
  unsigned kmax = wave_max_u32(key(a[0], 0));
#pragma unroll
  for (int p = 0; p < C; ++p) {
    sing = sing || (kmax & ~63u) == 0u;
    const int pl = 63 - (int)(kmax & 63u);      // pivot lane: row pl / 2, parity p & 1
    const int prow = pl >> 1;
    const double pv = readlane_d(a[p >> 1], pl);
    det *= pv;
    parity ^= (unsigned)__popcll(__ballot(!used && par == 0 && row < prow)) & 1u;
    if (row == prow) used = true;
    if (p + 1 < C) {
      const double own = a[p >> 1];
      const double other = swap_pair_d(own);
      const double ap = par == (p & 1) ? own : other;
      const double l = used ? 0.0 : ap * rcp_d(sing ? 1.0 : pv);
      const int src = (2 * prow + par) << 2;
      const int jn = (p + 1) >> 1;
      a[jn] = fma(-l, bperm_d(src, a[jn]), a[jn]);
      kmax = wave_max_u32(key(a[jn], p + 1));
#pragma unroll
      for (int j = jn + 1; j < J; ++j) a[j] = fma(-l, bperm_d(src, a[j]), a[j]);
    }
  }
  if (sing) return 0.0;
  return (parity & 1u) ? -det : det;
}

// The determinant-lemma matrix of spin tau in the row form (one wavefront),
// for K <= 16 changed rows:
//   A[a][b] = E[a][b] + sum_c D(m_a)[c] P[c][k_b],   a, b < K,
// with E the identity except for the moving electron's row (a = hpos), which
// is G[j][k_b] (its orbital row at the new site against the cached inverse);
// det A = det(Phi'[K] Phi^-1[:, K]), the ratio the column form of size
// C + [tau moves] gives (Sylvester's determinant identity).  The product is
// one 16 x 16 tile on the FP64 matrix cores, C / 4 k-steps (A[i][k] from
// lane i + 16 k, B[k][j] from lane j + 16 k); slot v of lane l then holds row
// l / 16 + 4 v, column l % 16.
template <int C, class DT>
SVMC_DEV v4d hop_det_row_build(const int* kl, int K_in, const DT* Dbuf, const double* __restrict__ PTt, int lane) {
  static_assert(C % 4 == 0, "k-steps of four channels");
  constexpr int SD = DStride<C>::value;
  const int K = uniform_i(K_in);
  const int li = lane & 15, lk = lane >> 4;
  const bool ok = li < K;
  const int e = kl[ok ? li : 0];
  const int mrow = ok ? (e >> 16) * SD : 0, kcol = ok ? e & 0xffff : 0;
  // all operands requested at once (unconditional loads from valid
  // addresses, masked afterwards), then the C / 4 k-steps; k-step q takes
  // channel (C / 4) lk + q in lane group lk, so a lane's operands are
  // contiguous runs of its D row and P^T row (wide loads)
  double av[C / 4], bv[C / 4];
#pragma unroll
  for (int q = 0; q < C / 4; ++q) {
    av[q] = (double)Dbuf[mrow + (C / 4) * lk + q];
    bv[q] = PTt[kcol * C + (C / 4) * lk + q];
  }
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < C / 4; ++q) mfma(acc, ok ? av[q] : 0.0, ok ? bv[q] : 0.0);
  return acc;
}
// Adds E and stages the matrix row-major [KS][KS + 1] (KS = 8 or 16 >= K);
// rows and columns >= K hold the identity.
template <int KS>
SVMC_DEV void hop_det_row_stage(const v4d& acc, const int* kl, int K_in, bool hopspin, int hpos_in,
                                const double* __restrict__ Gj, double* stage, int lane) {
  const int K = uniform_i(K_in), hpos = uniform_i(hpos_in);
  const int li = lane & 15, lk = lane >> 4;
  const int kcol = li < K ? kl[li < K ? li : 0] & 0xffff : 0;
  const double gk = Gj[kcol];       // unconditional (valid address), used on the mover's row
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = lk + 4 * v, c = li;
    if (r >= KS || c >= KS) continue;
    double val;
    if (r < K && c < K) val = acc[v] + ((hopspin && r == hpos) ? gk : (r == c ? 1.0 : 0.0));
    else val = r == c ? 1.0 : 0.0;
    stage[r * (KS + 1) + c] = val;
  }
}

// Stages the matrix (hop_det_stage) and returns its determinant by the
// one-wave LU.
template <int C>
SVMC_DEV double hop_det_finish(const v4d (&acc)[DetTiles<C>::I][DetTiles<C>::J], const int* kl, int K_in,
                               bool hopspin, int hpos_in, const double* __restrict__ PTt,
                               const double* __restrict__ Gj, double* stage, int lane) {
  typedef DetTiles<C> T;
  constexpr int RM = C + 1, RS = T::RS;
  const int K = uniform_i(K_in);
  if (K == 0) return 1.0;
  const int R = C + (hopspin ? 1 : 0);
  hop_det_stage<C>(acc, kl, K_in, hopspin, hpos_in, PTt, Gj, stage, lane);
  // rows in lanes < RM; the spin that does not move gets an identity row and
  // column C (same determinant), so both matrices take the same RM steps
  double a[RM];
  const double2* rp = reinterpret_cast<const double2*>(stage + (lane < R ? lane : 0) * RS);
#pragma unroll
  for (int c2 = 0; c2 < RS / 2; ++c2) {
    const double2 v = rp[c2];
    if (2 * c2 < RM) a[2 * c2] = (lane < R && 2 * c2 < R) ? v.x : 0.0;
    if (2 * c2 + 1 < RM) a[2 * c2 + 1] = (lane < R && 2 * c2 + 1 < R) ? v.y : 0.0;
  }
  if (!hopspin && lane == C) a[C] = 1.0;
  __builtin_amdgcn_wave_barrier();
  return lu_det_unrolled<RM>(a, lane);
}

}  // namespace svmc
