// Metropolis sampling of |psi|^2 with single-electron nearest-neighbour moves
// (Sec. II.A: configurations drawn by Markov chain Monte Carlo), with the
// local update of Sec. II.C for both the ratio and the accepted move:
//   ratio   incremental conv on the update box + determinant-lemma matrix per
//           spin (the same routines as the local-energy kernel);
//   accept  the new features are written into the cache, and the inverse
//           information kept per walker, G = M Phi^-1 (all sites) and
//           P = W Phi^-1, is brought up to date with the Sherman-Morrison-
//           Woodbury formula (Sec. II.C).  Per spin the change of the Slater
//           matrix has rank <= C + 1:  Phi' - Phi = U V with
//             U = [rows K carry D(m_a) (C columns), e_k for the mover],
//             V = [W; M[j] - M[i]],
//           so with A = I + V Phi^-1 U ((C+1) x (C+1), det A = ratio) and
//           Z = A^-1 V Phi^-1 (V Phi^-1 = [P; G[j] - e_k], column w_k):
//             G' = G_old' - (G_old' U) Z,   P' = P - (P U) Z,
//           where G_old' = M' Phi^-1 = G + D P on the box sites.  Evaluated
//           as G'[s][k] = G[s][k] + e_s . w_k with one coefficient vector per
//           site, e_s = [[s in box] D(s) - A^-T (G_old' U)[s]; -(G_old' U)[s]
//           . A^-1[:, C]], and P' = P - (PU A^-1) w_k.  log|psi| and the sign
//           take the ratio per spin.
//
// Proposal q of walker w uses one Philox4x64-10 block (key (seed, 0), counter
// (w, step0 + q, 0, 0)), written from the published definition (Salmon et
// al., SC'11).  A walker stops after `refresh_every` accepted moves; the host
// rebuilds its inverse in FP64 and restarts it at the next proposal, so the
// chain is the same as without the pause.
#include "hop.h"
#include "svmc_launch.h"

namespace svmc {

constexpr int SW_NW = 4;        // wavefronts per workgroup
constexpr int SCH = 32;         // sites per chunk of the G update
// nacc value of a walker whose update matrix was singular: its G and P were
// not updated, so the refresh rebuilds it without a drift check
constexpr int SW_REBUILD = 0x7fffffff;

struct SweepLds {
  int occ, lab, pos, misc, pu, rowc, ainv, qm, perm, corder, pkbm, gk, mk, gkc, ec, mbs, scratch, bytes, kmax;
};
__host__ __device__ inline int al16(int x) { return (x + 15) & ~15; }
// LDS of one walker: configuration, labels, positions, per-hop results, the
// update matrices of one spin (PU [C][C+1], row C of A, A^-1 and Q = PU A^-1,
// pivot order, label order [2 nmax], the changed rows' P^T [kmax][C] which
// later holds B = U A^-1 [kmax][C+1], their G[j] entries and box offsets, a
// chunk's G[s, K] [SCH][kmax] and E rows [SCH][C+1]) and the hop scratch.
// kmax = changed rows per spin at most = sites of the layer-L box.
__host__ __device__ inline SweepLds sweep_layout(int N, int nmax, int Gx, int Gy, int L, int C, int tfb) {
  const int ra = C + 1;
  SweepLds o;
  o.kmax = (Gx < 2 * L + 2 ? Gx : 2 * L + 2) * (Gy < 2 * L + 2 ? Gy : 2 * L + 2);
  o.occ = 0;
  o.lab = al16(N);
  o.pos = o.lab + al16(4 * N);
  o.misc = o.pos + al16(4 * nmax);
  o.pu = o.misc + 128;
  o.rowc = o.pu + al16(8 * C * ra);
  o.ainv = o.rowc + al16(8 * ra);
  o.qm = o.ainv + al16(8 * ra * ra);
  o.perm = o.qm + al16(8 * C * ra);
  o.corder = o.perm + al16(4 * ra);
  o.pkbm = o.corder + al16(2 * 2 * nmax);
  o.gk = o.pkbm + al16(8 * o.kmax * ra);
  o.mk = o.gk + al16(8 * o.kmax);
  o.gkc = o.mk + al16(4 * o.kmax);
  o.ec = o.gkc + al16(8 * SCH * o.kmax);
  o.mbs = o.ec + al16(8 * SCH * ra);
  o.scratch = o.mbs + al16(4 * SCH);
  o.bytes = o.scratch + hop_scratch(Gx, Gy, L, C, tfb).bytes;
  return o;
}

// Dense index of site s in the layer-L update box (origin (olx, oly), size
// owx x owy, periodic axes wrapped), or -1 outside.
SVMC_DEV int box_index(const LatDev& lt, int s, int olx, int owx, int oly, int owy) {
  const int xs = s % lt.Lx, ys = s / lt.Lx;
  const int dx = lt.pbc_x ? imod(xs - olx, lt.Lx) : xs - olx;
  const int dy = lt.pbc_y ? imod(ys - oly, lt.Ly) : ys - oly;
  return (dx >= 0 && dx < owx && dy >= 0 && dy < owy) ? dx + owx * dy : -1;
}

SVMC_DEV void philox4x64_10(unsigned long long (&c)[4], unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const unsigned long long lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// Gauss-Jordan inverse of an r x r FP64 matrix in one wavefront (r <= RM),
// rows in lanes with rotating columns: at step p the current column is a[0];
// the pivot row is scaled, the other rows eliminate it, every row shifts left
// and the new column of the inverse enters at a[RM - 1].  Partial pivoting
// by row choice only (largest |a[0]| among unused rows, compared in FP32).
// Afterwards lane perm[p] holds row p of the inverse, column perm[q] in slot
// RM - r + q.  Returns false when a pivot column is zero.
template <int RM>
SVMC_DEV bool gj_inverse_rot(double (&a)[RM], int r_in, int lane, int* perm, int& mystep) {
  const int r = uniform_i(r_in);
  bool used = lane >= r;
  mystep = -1;
  for (int p = 0; p < r; ++p) {
    const double cp = a[0];
    const unsigned key0 = used ? 0u : ((__float_as_uint((float)fabs(cp)) & ~63u) | (unsigned)(63 - lane));
    const unsigned key = wave_max_u32(key0);
    if ((key & ~63u) == 0u) return false;
    const int piv = 63 - (int)(key & 63u);
    const double pv = readlane_d(cp, piv);
    const double ipv = 1.0 / pv;
    const bool me = lane == piv;
    if (me) { used = true; mystep = p; }
    if (lane == 0) perm[p] = piv;
    const double f = me ? 0.0 : cp;
#pragma unroll
    for (int c = 1; c < RM; ++c) {
      const double pr = readlane_d(a[c], piv) * ipv;       // scaled pivot row
      a[c - 1] = me ? pr : fma(-f, pr, a[c]);
    }
    a[RM - 1] = me ? ipv : -f * ipv;
  }
  return true;
}

#ifdef SVMC_INST_P
template <int P, int C>
__global__ __launch_bounds__(64 * SW_NW) void k_sweep(ModelDev md, const LatDev* __restrict__ lats, int nlats,
                                                      Bufs bf, SweepArgs sa) {
  typedef typename PrecT<P>::Tf Tf;
  constexpr int NW = SW_NW, NTH = 64 * NW;
  constexpr int SP = SiteStride<Tf, C>::value;
  constexpr int RA = C + 1;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const long long w = blockIdx.x;
  int li = 0;
  while (li + 1 < nlats && w >= lats[li + 1].w0) ++li;
  const LatDev lt = lats[li];
  const long long wl = w - lt.w0;
  const int N = lt.N, nm = lt.nmax;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long long qend = (long long)sa.n_sweeps * N;
  long long q = sa.prog[w];
  if (q >= qend) return;
  const unsigned long long step0 = sa.step0_dev ? *sa.step0_dev : sa.step0;
  if (bf.flags[w] & (1 | 2 | 8)) {
    if (tid == 0) sa.prog[w] = qend;
    return;
  }
  const SweepLds lay = sweep_layout(N, nm, lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf));
  int8_t* occ_s = (int8_t*)(smem + lay.occ);
  int16_t* lab_s = (int16_t*)(smem + lay.lab);
  int16_t* pos_s = (int16_t*)(smem + lay.pos);
  double* misc = (double*)(smem + lay.misc);
  double* pu = (double*)(smem + lay.pu);
  double* rowc = (double*)(smem + lay.rowc);
  double* ainv = (double*)(smem + lay.ainv);
  double* qm = (double*)(smem + lay.qm);
  int* perm = (int*)(smem + lay.perm);
  int16_t* corder = (int16_t*)(smem + lay.corder);
  double* pk = (double*)(smem + lay.pkbm);
  double* bm = pk;                  // B = U A^-1 replaces P^T_K once PU is formed
  double* gk = (double*)(smem + lay.gk);
  int* mk = (int*)(smem + lay.mk);
  double* gkc = (double*)(smem + lay.gkc);
  double* ec = (double*)(smem + lay.ec);
  int* mbs = (int*)(smem + lay.mbs);
  const int kmax = lay.kmax;
  char* scratch = smem + lay.scratch;
  const HopScratch hsc = hop_scratch(lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf));
  const int KM = lt.Gx * lt.Gy;
  int* klb = (int*)(scratch + hsc.klists);
  const typename DType<P>::type* Dbuf = (const typename DType<P>::type*)scratch;
  constexpr int SD = DStride<C>::value;

  int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  int16_t* lab_g = bf.lab + lt.lab_off + wl * 2LL * N;
  int16_t* pos_g = bf.pos + lt.pos_off + wl * 2LL * nm;
  for (int s = tid; s < N; s += NTH) occ_s[s] = occ_g[s];
  for (int s = tid; s < 2 * N; s += NTH) lab_s[s] = lab_g[s];
  for (int s = tid; s < 2 * nm; s += NTH) pos_s[s] = pos_g[s];
  Tf* featw = (Tf*)bf.feat + lt.feat_off + wl * (long long)md.L * N * C;
  double* Gw = bf.G + lt.g_off + wl * 2LL * N * nm;
  double* PTw = bf.PT + lt.pt_off + wl * 2LL * nm * C;
  // electron counts as scalars: indexing the local descriptor copy with a
  // runtime spin would move it to scratch memory
  const int n_up = lt.n[0], n_dn = lt.n[1];
  const int ne = n_up + n_dn;
  int nacc = bf.nacc[w];
  long long accepted = 0;
  bool stop_refresh = false;
  hop_scratch_init<P>(md, scratch, hsc);
  __syncthreads();

  for (; q < qend && ne > 0; ++q) {
    // ---- draw (identical in every thread)
    unsigned long long ctr[4] = {(unsigned long long)w, step0 + (unsigned long long)q, 0ULL, 0ULL};
    philox4x64_10(ctr, sa.seed, 0ULL);
    const int e = (int)__umul64hi(ctr[0], (unsigned long long)ne);
    const int d = (int)(ctr[1] >> 62);
    const double u = (double)(ctr[2] >> 11) * 0x1.0p-53;
    const int sp = e < n_up ? 0 : 1;
    const int k = sp == 0 ? e : e - n_up;
    const int i = uniform_i(pos_s[sp * nm + k]);
    const int bit = 1 << sp;
    {
      int x = i % lt.Lx + dir_dx(d), y = i / lt.Lx + dir_dy(d);
      bool ok = true;
      if (lt.pbc_x) x = imod(x, lt.Lx); else ok = ok && x >= 0 && x < lt.Lx;
      if (lt.pbc_y) y = imod(y, lt.Ly); else ok = ok && y >= 0 && y < lt.Ly;
      if (!ok || ((occ_s[x + lt.Lx * y] >> sp) & 1)) continue;   // uniform
    }
    const HopGeom g = hop_geom(lt, md.L, sp, i, d);
    int olx, owx, oly, owy;
    const AxisTab tab = axis_tab(g, md.L, lane);
    hop_features<P, C, NW>(md, lt, g, occ_s, featw, (Tf*)nullptr, scratch, hsc, tab, olx, owx, oly, owy);
    int K = 0, hpos = -1;
    const int wd = wv < 2 ? wv : 0;           // spin of this wavefront's determinant
    const double* PTt = PTw + (long long)wd * nm * C;
    const double* Gj = Gw + ((long long)wd * N + g.j) * nm;
    v4d dacc[DetTiles<C>::I][DetTiles<C>::J];
    if (wv < 2) {
      K = hop_klist(lt, g, tab, occ_s, lab_s, wv, olx, owx, oly, owy, klb + wv * KM, hpos, lane);
      hop_det_build<C>(klb + wv * KM, K, wv == sp, hpos, Dbuf, PTt, Gj, lane, dacc);
    }
    __syncthreads();      // both matrices built: their staging may overwrite D
    if (wv < 2) {
      double* stage = (double*)scratch + wv * (C + 1) * DetTiles<C>::RS;
      const double Rt = hop_det_finish<C>(dacc, klb + wv * KM, K, wv == sp, hpos, PTt, Gj, stage, lane);
      if (lane == 0) {
        misc[wv] = Rt;
        misc[2 + wv] = (double)K;
        misc[4 + wv] = (double)hpos;
      }
    }
    __syncthreads();
    const double R0 = misc[0], R1 = misc[1];
    const double R = R0 * R1;
    if (!(u < R * R)) continue;                                       // uniform

    // ---- accepted: commit the new features (and recompute D on the box)
    hop_features<P, C, NW>(md, lt, g, occ_s, featw, featw, scratch, hsc, tab, olx, owx, oly, owy);
    bool fallback = false;
    for (int tau = 0; tau < 2; ++tau) {
      const int n = tau == 0 ? n_up : n_dn;
      if (n == 0) continue;
      const int r = (int)misc[2 + tau];
      const bool hs = tau == sp;
      const int R = C + (hs ? 1 : 0);
      const int* kl = klb + tau * KM;
      double* Gt = Gw + (long long)tau * N * nm;
      double* PTt = PTw + (long long)tau * nm * C;
      const double* Gj = Gt + (long long)g.j * nm;
      // (0) stage the changed labels' P^T rows, G[j] entries and box rows:
      //     pk[a][c] = P^T[k_a][c], gk[a] = G[j][k_a] - [k_a = k], mk[a] = m_a
      for (int a = tid; a < r; a += NTH) {
        const int e = kl[a];
        mk[a] = (e >> 16) * SD;
        gk[a] = hs ? Gj[e & 0xffff] - ((e & 0xffff) == k ? 1.0 : 0.0) : 0.0;
      }
      {
        const int tot = r * C;
        for (int e0 = 0; e0 < tot; e0 += NTH * 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e2 = e0 + NTH * u + tid;
            v[u] = e2 < tot ? PTt[(long long)(kl[e2 / C] & 0xffff) * C + (e2 % C)] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e2 = e0 + NTH * u + tid;
            if (e2 < tot) pk[e2] = v[u];
          }
        }
      }
      __syncthreads();
      // (1) PU = P U: PU[c'][c] = sum_a P^T[k_a][c'] D(m_a)[c] (c < C), PU[c'][C] = P^T[k][c'];
      //     row C of A - I (hop spin): sum_a (G[j][k_a] - [k_a = k]) D(m_a)[c], G[j][k] - 1
      for (int e2 = tid; e2 < C * RA; e2 += NTH) {
        const int cp = e2 / RA, c = e2 - cp * RA;
        double v = 0.0;
        if (c < C) {
#pragma unroll 8
          for (int a = 0; a < r; ++a) v = fma(pk[a * C + cp], (double)Dbuf[mk[a] + c], v);
        } else if (hs) {
          v = PTt[(long long)k * C + cp];
        }
        pu[e2] = v;
      }
      for (int c = tid; c < RA; c += NTH) {
        double v = 0.0;
        if (hs) {
          if (c < C) {
#pragma unroll 8
            for (int a = 0; a < r; ++a) v = fma(gk[a], (double)Dbuf[mk[a] + c], v);
          } else {
            v = Gj[k] - 1.0;
          }
        }
        rowc[c] = v;
      }
      for (int e2 = tid; e2 < RA * RA; e2 += NTH) ainv[e2] = 0.0;
      __syncthreads();
      // (2) A = I + V Phi^-1 U, inverted by wavefront 0
      if (wv == 0) {
        double arow[RA];
#pragma unroll
        for (int c = 0; c < RA; ++c) {
          double v = 0.0;
          if (lane < R && c < R) v = (lane < C ? pu[lane * RA + c] : rowc[c]) + (lane == c ? 1.0 : 0.0);
          arow[c] = v;
        }
        int mystep;
        const bool ok = gj_inverse_rot<RA>(arow, R, lane, perm, mystep);
        // every lane reads the pivot order lane 0 wrote: order the accesses
        // for the compiler (a wavefront's LDS operations stay in order)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ok && lane < R) {
#pragma unroll
          for (int qq = 0; qq < RA; ++qq) {
            if (qq < R) {
              const int slot = RA - R + qq;
              double v = 0.0;
#pragma unroll
              for (int s2 = 0; s2 < RA; ++s2) v = (s2 == slot) ? arow[s2] : v;
              ainv[mystep * RA + perm[qq]] = v;   // A^-1[p][perm[q]]
            }
          }
        }
        if (lane == 0) misc[6] = ok ? 1.0 : 0.0;
      }
      __syncthreads();
      if (misc[6] == 0.0) { fallback = true; continue; }                 // uniform
      // Q = PU A^-1 (C x RA) and B = U A^-1 (r x RA), U[a] = [D(m_a), [k_a = k]]:
      //   G' = G + E W,  E[s] = [s in box] (D_ext(s) - D(s) Q) - G[s, K] B,
      //   P^T' = P^T - (Q W)^T,  W[:, k'] = [P^T[k']; G[j][k'] - [k' = k]]
      for (int e2 = tid; e2 < C * RA; e2 += NTH) {
        const int cp = e2 / RA, c = e2 - cp * RA;
        double v = 0.0;
        for (int c1 = 0; c1 < R; ++c1) v = fma(pu[cp * RA + c1], ainv[c1 * RA + c], v);
        qm[e2] = v;
      }
      for (int e2 = tid; e2 < r * RA; e2 += NTH) {
        const int a = e2 / RA, c2 = e2 - a * RA;
        const typename DType<P>::type* Da = Dbuf + mk[a];
        double v = (hs && (kl[a] & 0xffff) == k) ? ainv[C * RA + c2] : 0.0;
#pragma unroll 8
        for (int c = 0; c < C; ++c) v = fma((double)Da[c], ainv[c * RA + c2], v);
        bm[e2] = v;
      }
      // Columns (labels) go in passes of NTH / 2, each column on two threads
      // (even and odd sites of a chunk).  With more than one pass the labels
      // of K come last and all fall in the last pass: E of a chunk reads the
      // old G[s, K] of its sites.
      constexpr int NCOL = NTH / 2;
      const int npass = (n + NCOL - 1) / NCOL;
      if (npass > 1) {
        for (int kk = tid; kk < n; kk += NTH) corder[kk] = 0;
        __syncthreads();
        for (int a = tid; a < r; a += NTH) corder[kl[a] & 0xffff] = 1;
        __syncthreads();
        if (tid == 0) {
          int lo = 0, hi = n;
          for (int kk = 0; kk < n; ++kk) {
            if (corder[kk] == 0) corder[n + lo++] = (int16_t)kk;
            else corder[n + --hi] = (int16_t)kk;
          }
        }
      }
      __syncthreads();
      const int half = tid / NCOL, tcol = tid - half * NCOL;
      for (int b = 0; b < npass; ++b) {
        // passes are cut from the end of the order, so the last one holds the
        // final NCOL labels and with them all of K (r <= (2L+2)^2 <= NCOL)
        const int slot = n - (npass - b) * NCOL + tcol;
        const bool col = slot >= 0;
        const int kc = !col ? 0 : (npass > 1 ? (int)corder[n + slot] : slot);
        double wcol[RA];
#pragma unroll
        for (int c = 0; c < C; ++c) wcol[c] = col ? PTt[(long long)kc * C + c] : 0.0;
        wcol[C] = (col && hs) ? Gj[kc] - (kc == k ? 1.0 : 0.0) : 0.0;
        __syncthreads();            // every read of G[j] and P done before they change
        for (int s0 = 0; s0 < N; s0 += SCH) {
          const int ns = min(SCH, N - s0);
          // this thread's G entries of the chunk, requested first so that the
          // loads overlap the gather and E rows below (no other thread writes
          // them before this thread's update)
          constexpr int SPT = SCH / 2;
          double gv[SPT];
#pragma unroll
          for (int i2 = 0; i2 < SPT; ++i2) {
            const int sl = half + 2 * i2;
            gv[i2] = (col && sl < ns) ? Gt[(long long)(s0 + sl) * nm + kc] : 0.0;
          }
          {
            // G[s, K] of the chunk's sites: all of this thread's loads first
            // (at most SCH * kmax / NTH <= 13 of them for L <= 4)
            constexpr int GI = (SCH * 100 + NTH - 1) / NTH;
            double gg[GI];
            int gd[GI];
#pragma unroll
            for (int u2 = 0; u2 < GI; ++u2) {
              const int e2 = tid + u2 * NTH;
              const bool ok = e2 < ns * r;
              const int sl = ok ? e2 / r : 0, a = ok ? e2 - sl * r : 0;
              gd[u2] = ok ? sl * kmax + a : -1;
              gg[u2] = ok ? Gt[(long long)(s0 + sl) * nm + (kl[a] & 0xffff)] : 0.0;
            }
#pragma unroll
            for (int u2 = 0; u2 < GI; ++u2)
              if (gd[u2] >= 0) gkc[gd[u2]] = gg[u2];
          }
          if (tid < ns) mbs[tid] = box_index(lt, s0 + tid, olx, owx, oly, owy);
          __syncthreads();
          for (int e2 = tid; e2 < ns * RA; e2 += NTH) {
            const int sl = e2 / RA, c2 = e2 - sl * RA;
            const int mb = mbs[sl];
            double v = 0.0;
            if (mb >= 0) {
              const typename DType<P>::type* Dm = Dbuf + mb * SD;
              v = c2 < C ? (double)Dm[c2] : 0.0;
#pragma unroll 8
              for (int c = 0; c < C; ++c) v = fma(-(double)Dm[c], qm[c * RA + c2], v);
            }
            const double* gr = gkc + sl * kmax;
#pragma unroll 8
            for (int a = 0; a < r; ++a) v = fma(-gr[a], bm[a * RA + c2], v);
            ec[sl * RA + c2] = v;
          }
          __syncthreads();
          if (col) {
#pragma unroll
            for (int i2 = 0; i2 < SPT; ++i2) {
              const int sl = half + 2 * i2;
              if (sl >= ns) break;
              const double* es = ec + sl * RA;
              double v = gv[i2];
#pragma unroll
              for (int c = 0; c < RA; ++c) v = fma(es[c], wcol[c], v);
              Gt[(long long)(s0 + sl) * nm + kc] = v;
            }
          }
          __syncthreads();
        }
        if (col && half == 0) {
#pragma unroll
          for (int cp = 0; cp < C; ++cp) {
            const double* qr = qm + cp * RA;
            double v = wcol[cp];
#pragma unroll
            for (int c = 0; c < RA; ++c) v = fma(-qr[c], wcol[c], v);
            PTt[(long long)kc * C + cp] = v;
          }
        }
        __syncthreads();
      }
    }
    // ---- configuration, labels, log|psi|
    if (tid == 0) {
      const int j = g.j;
      occ_s[i] -= bit;
      occ_s[j] += bit;
      lab_s[sp * N + j] = (int16_t)k;
      lab_s[sp * N + i] = -1;
      pos_s[sp * nm + k] = (int16_t)j;
      bf.ld[2 * w] += log(fabs(R0));
      bf.ld[2 * w + 1] += log(fabs(R1));
      if (R0 < 0) bf.sg[2 * w] = -bf.sg[2 * w];
      if (R1 < 0) bf.sg[2 * w + 1] = -bf.sg[2 * w + 1];
    }
    __syncthreads();
    ++accepted;
    ++nacc;
    if (nacc >= sa.refresh_every || fallback) {
      if (fallback) nacc = SW_REBUILD;
      stop_refresh = true;
      ++q;
      break;
    }
  }
  // write back
  for (int s = tid; s < N; s += NTH) occ_g[s] = occ_s[s];
  for (int s = tid; s < 2 * N; s += NTH) lab_g[s] = lab_s[s];
  for (int s = tid; s < 2 * nm; s += NTH) pos_g[s] = pos_s[s];
  if (tid == 0) {
    sa.prog[w] = (ne > 0) ? q : qend;
    bf.nacc[w] = nacc;
    if (sa.n_accept) sa.n_accept[w] += accepted;
    if (stop_refresh && sa.paused) atomicAdd(sa.paused, 1);
  }
}

template <int P, int C>
static hipError_t sweep_impl(const ModelDev& md, const LatDev* lats_dev, int nlats, long long W, const Bufs& bf,
                             const SweepArgs& sa, size_t smem, hipStream_t st) {
  auto kern = k_sweep<P, C>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)W), dim3(64 * SW_NW), smem, st, md, lats_dev, nlats, bf, sa);
  return hipGetLastError();
}

hipError_t SVMC_CAT3(sweep_, SVMC_INST_P, SVMC_INST_C)(const ModelDev& md, const LatDev* lats_dev, int nlats,
                                                       long long W, const Bufs& bf, const SweepArgs& sa,
                                                       size_t smem, hipStream_t st) {
  return sweep_impl<SVMC_INST_P, SVMC_INST_C>(md, lats_dev, nlats, W, bf, sa, smem, st);
}
#else
// Drift of the maintained G before a refresh: max |G[pos_k][k'] - delta|
// over occupied rows (these rows of M Phi^-1 are unit rows in exact
// arithmetic); sets the DRIFT flag above 1e-8.  Only walkers due for a
// refresh (nacc >= refresh_every) when only_due != 0.
__global__ void k_drift(LatDev lt, Bufs bf, int only_due, int refresh_every) {
  const long long wl = blockIdx.x;
  const long long w = lt.w0 + wl;
  if (only_due && bf.nacc[w] < refresh_every) return;
  if (bf.nacc[w] == SW_REBUILD) return;
  const int N = lt.N, nm = lt.nmax;
  double mx = 0.0;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = lt.n[sp];
    const double* G = bf.G + lt.g_off + wl * 2LL * N * nm + (long long)sp * N * nm;
    const int16_t* pos = bf.pos + lt.pos_off + wl * 2LL * nm + sp * nm;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int k = e / n, k2 = e % n;
      const double v = G[(long long)pos[k] * nm + k2] - (k == k2 ? 1.0 : 0.0);
      mx = fmax(mx, fabs(v));
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(red[0] <= 1e-8)) atomicOr(bf.flags + w, 4);
}

__global__ void k_clear_nacc(LatDev lt, Bufs bf, int refresh_every) {
  const long long wl = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (wl >= lt.nw) return;
  const long long w = lt.w0 + wl;
  if (bf.nacc[w] >= refresh_every) bf.nacc[w] = 0;
}

__global__ void k_fill_i64(int64_t* p, long long n, int64_t v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i64(int64_t* p, long long n, int64_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

size_t sweep_smem(const LatDev* lats, int nlats, int prec, int L, int C) {
  const int tfb = prec == PREC_F64 ? 8 : 4;
  size_t mx = 0;
  for (int l = 0; l < nlats; ++l)
    mx = std::max(mx, (size_t)sweep_layout(lats[l].N, lats[l].nmax, lats[l].Gx, lats[l].Gy, L, C, tfb).bytes);
  return mx;
}

hipError_t launch_drift(const LatDev& lt, const Bufs& bf, int only_due, int refresh_every, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_drift, dim3((unsigned)lt.nw), dim3(256), 0, st, lt, bf, only_due, refresh_every);
  return hipGetLastError();
}

hipError_t launch_clear_nacc(const LatDev& lt, const Bufs& bf, int refresh_every, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_nacc, dim3((unsigned)((lt.nw + 255) / 256)), dim3(256), 0, st, lt, bf,
                     refresh_every);
  return hipGetLastError();
}

hipError_t launch_sweep(int prec, const ModelDev& md, const LatDev* lats_dev, const LatDev* lats_host, int nlats,
                        long long W, const Bufs& bf, const SweepArgs& sa, hipStream_t st) {
  const size_t smem = sweep_smem(lats_host, nlats, prec, md.L, md.C);
  if (smem > 160 * 1024) return hipErrorInvalidValue;
#define SVMC_SW(P_, C_) \
  if (prec == P_ && md.C == C_) return sweep_##P_##_##C_(md, lats_dev, nlats, W, bf, sa, smem, st);
  SVMC_FOR_EACH_PREC_C(SVMC_SW)
#undef SVMC_SW
  return hipErrorInvalidValue;
}
#endif

}  // namespace svmc
