// Metropolis sampling of |psi|^2 with single-electron nearest-neighbour moves
// (Sec. II.A: configurations drawn by Markov chain Monte Carlo), with the
// local update of Sec. II.C for both the ratio and the accepted move.  In
// the t-J model (Sec. III) a move onto an occupied site is rejected without
// evaluation: the Gutzwiller projection gives it amplitude zero.
//
// The sweep is step-synchronous across walkers: proposal q of every walker
// is one launch of k_step_propose (one workgroup per walker), followed by
// one launch of k_step_update over the walkers that accepted; every few
// steps the FP64 refresh of the walkers that reached `refresh_every`
// accepted moves, driven by a device-side list.
//   propose  incremental conv on the update box + determinant-lemma matrix A
//            per spin (the routines of the local-energy kernel); on accept
//            the new features are committed to the cache, A^-1 (Gauss-Jordan
//            on the staged A), the changed-row lists, the old row G[j] and
//            D = H'_L - H_L on the box are staged for the update, and the
//            configuration, labels and log|psi| are updated;
//   update   the inverse information kept per walker, G = M Phi^-1 (all
//            sites) and P = W Phi^-1, follows the Sherman-Morrison-Woodbury
//            formula (Sec. II.C).  Per spin Phi' - Phi = U V with
//              U = [rows K carry D(m_a) (C columns), e_k for the mover],
//              V = [W; M[j] - M[i]],  A = I + V Phi^-1 U = [PU; g-row] + I,
//            so Q = PU A^-1 = (I - A^-1)[0:C] and, with B = U A^-1 and
//            W[:, k'] = [P^T[k']; G[j][k'] - [k' = k]],
//              G'[s][k'] = G[s][k'] + E[s] . W[:, k'],
//              E[s] = [s in box] D(s) A^-1[0:C, :] - G[s, K] B,
//              P^T'[k'] = A^-1[0:C, :] W[:, k'].
//            One workgroup per (walker, spin): E and G in chunks of sites,
//            with E formed as [D(s) - G[s, K] D_K | -G[s, k_mover]] A^-1
//            (no B), then P.
//
// Proposal q of walker w uses one Philox4x64-10 block (key (seed, 0), counter
// (w, step0 + q, 0, 0)), written from the published definition (Salmon et
// al., SC'11), so the chain does not depend on when refreshes happen.
#include "hop.h"
#include "svmc_launch.h"

namespace svmc {

// nacc value of a walker whose update matrix was singular: its G and P were
// not updated, so the refresh rebuilds it without a drift check
constexpr int SW_REBUILD = 0x7fffffff;
constexpr int UPD_SC = 64;      // sites per chunk of the G update

__host__ __device__ inline int al16(int x) { return (x + 15) & ~15; }
// sites of the layer-L update box at most: (2L + 2) along the hop and
// (2L + 1) across it for nearest-neighbour hops only (nd = 4), (2L + 2)
// along both axes with diagonal hops (nd = 8); each axis capped by the grid
__host__ __device__ inline int box_kmax(int Gx, int Gy, int L, int nd) {
  const int ax = Gx < 2 * L + 2 ? Gx : 2 * L + 2, ay = Gy < 2 * L + 2 ? Gy : 2 * L + 2;
  const int bx = Gx < 2 * L + 1 ? Gx : 2 * L + 1, by = Gy < 2 * L + 1 ? Gy : 2 * L + 1;
  if (nd == 8) return ax * ay;
  return ax * by > bx * ay ? ax * by : bx * ay;
}

// Staging record of one walker's accepted move (global memory, byte offsets):
//   hdr   int [16]            flags and scalars (HD_*)
//   kl    int [2][kmax]       changed-row lists per spin, (m << 16) | label
//   D     DT  [kmax][C + 4]   D = H'_L - H_L on the layer-L box
//   ainv  f64 [2][C+1][C+1]   A^-1 per spin (zero row / column C for the
//                             spin that does not move)
//   gj    f64 [2][nmax]       G[j] per spin before the update
struct StepStage {
  int hdr, kl, D, ainv, gj, bytes;
};
__host__ __device__ inline StepStage step_stage(int nmax, int Gx, int Gy, int L, int nd, int C, int dtb) {
  const int km = box_kmax(Gx, Gy, L, nd), ra = C + 1;
  StepStage o;
  o.hdr = 0;
  o.kl = 64;
  o.D = o.kl + al16(2 * km * 4);
  o.ainv = o.D + al16(km * (C + 4) * dtb);
  o.gj = o.ainv + 2 * ra * ra * 8;
  o.bytes = o.gj + al16(2 * nmax * 8);
  return o;
}
enum { HD_ACC = 0, HD_SP, HD_K, HD_J, HD_OLX, HD_OWX, HD_OLY, HD_OWY, HD_R0, HD_R1, HD_HPOS };

// LDS of the proposal kernel: configuration, labels, pivot orders of the two
// inverse wavefronts, per-hop scratch.
struct ProposeLds {
  int occ, lab, perm, scratch, bytes;
};
__host__ __device__ inline ProposeLds propose_layout(int N, int Gx, int Gy, int L, int C, int tfb) {
  ProposeLds o;
  o.occ = 0;
  o.lab = al16(N);
  o.perm = o.lab + al16(4 * N);
  o.scratch = o.perm + 2 * 64 * 4;
  o.bytes = o.scratch + hop_scratch(Gx, Gy, L, C, tfb).bytes;
  return o;
}
// LDS of the update kernel: A^-1, the changed-row list, the D rows of the
// changed electrons, E rows of a chunk of sites.
__host__ __device__ inline int update_lds_bytes(int kmax, int C, int dtb) {
  const int ra = C + 1;
  return al16(ra * ra * 8) + al16(kmax * 4) + al16(kmax * C * dtb) + UPD_SC * (4 * ((ra + 3) / 4)) * 8;
}

// Dense index of site s in the layer-L update box (origin (olx, oly), size
// owx x owy, periodic axes wrapped), or -1 outside.
SVMC_DEV int box_index(const LatDev& lt, int s, int olx, int owx, int oly, int owy) {
  const int xs = s % lt.Lx, ys = s / lt.Lx;
  const int dx = lt.pbc_x ? imod(xs - olx, lt.Lx) : xs - olx;
  const int dy = lt.pbc_y ? imod(ys - oly, lt.Ly) : ys - oly;
  return (dx >= 0 && dx < owx && dy >= 0 && dy < owy) ? dx + owx * dy : -1;
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
// Proposal sa.q of every walker (one workgroup of two wavefronts per walker).
// MLP: the instance for networks with site-wise layers.
template <int P, int C, bool MLP>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_step_propose(ModelDev md, const LatDev* __restrict__ lats, int nlats,
                                                      Bufs bf, StepArgs sa) {
  typedef typename PrecT<P>::Tf Tf;
  typedef typename DType<P>::type DT;
  constexpr int NW = 2, NTH = 64 * NW, RA = C + 1;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const long long w = blockIdx.x;
  int li = 0;
  while (li + 1 < nlats && w >= lats[li + 1].w0) ++li;
  const LatDev lt = lats[li];
  const long long wl = w - lt.w0;
  const int N = lt.N, nm = lt.nmax;
  const int tid = threadIdx.x, lane = tid & 63, wv = uniform_i(tid >> 6);
  const StepStage sl = step_stage(nm, lt.Gx, lt.Gy, md.L, lt.nd, C, (int)sizeof(DT));
  char* st = sa.stage + w * sa.stage_stride;
  int* hdr = (int*)(st + sl.hdr);
  // electron counts as scalars: indexing the local descriptor copy with a
  // runtime spin would move it to scratch memory
  const int n_up = lt.n[0], n_dn = lt.n[1], ne = n_up + n_dn;
  const long long qend = (long long)sa.n_sweeps * N;
  const int mv = sa.sym_mode ? uniform_i(sa.sym_move[w]) : 0;
  if (sa.q >= qend || ne == 0 || (bf.flags[w] & (1 | 2 | 8)) || mv < 0) {
    if (tid == 0) {
      hdr[HD_ACC] = 0;
      if (sa.sym_mode == 1) sa.sym_ratio[w] = 0.0;
    }
    return;
  }
  int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  int16_t* lab_g = bf.lab + lt.lab_off + wl * 2LL * N;
  int16_t* pos_g = bf.pos + lt.pos_off + wl * 2LL * nm;
  // ---- draw (identical in every thread), or the move given
  int d, sp, k, i;
  double u = 0.0;
  if (sa.sym_mode == 0) {
    const unsigned long long step0 = sa.step0_dev ? *sa.step0_dev : sa.step0;
    unsigned long long ctr[4] = {(unsigned long long)w, step0 + (unsigned long long)sa.q, 0ULL, 0ULL};
    philox4x64_10(ctr, sa.seed, 0ULL);
    const int e = (int)__umul64hi(ctr[0], (unsigned long long)ne);
    d = (int)(ctr[1] >> 62);
    u = (double)(ctr[2] >> 11) * 0x1.0p-53;
    sp = e < n_up ? 0 : 1;
    k = sp == 0 ? e : e - n_up;
    i = uniform_i(pos_g[sp * nm + k]);
  } else {
    i = mv >> 4;
    sp = (mv >> 3) & 1;
    d = mv & 7;
    k = uniform_i(lab_g[sp * N + i]);
  }
  const int bit = 1 << sp;
  {
    int x = i % lt.Lx + dir_dx(d), y = i / lt.Lx + dir_dy(d);
    bool ok = k >= 0;
    if (lt.pbc_x) x = imod(x, lt.Lx); else ok = ok && x >= 0 && x < lt.Lx;
    if (lt.pbc_y) y = imod(y, lt.Ly); else ok = ok && y >= 0 && y < lt.Ly;
    const int tgt = ok ? uniform_i(occ_g[x + lt.Lx * y]) : 0;
    // (t-J: the Gutzwiller projection also rejects a site of the other spin)
    if (!ok || (lt.tj ? tgt != 0 : ((tgt >> sp) & 1))) {              // uniform
      if (tid == 0) {
        hdr[HD_ACC] = 0;
        if (sa.sym_mode == 1) sa.sym_ratio[w] = 0.0;
      }
      return;
    }
  }
  const ProposeLds lay = propose_layout(N, lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf));
  int8_t* occ_s = (int8_t*)(smem + lay.occ);
  int16_t* lab_s = (int16_t*)(smem + lay.lab);
  int* perm = (int*)(smem + lay.perm) + wv * 64;
  char* scratch = smem + lay.scratch;
  const HopScratch hsc = hop_scratch(lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf));
  hop_scratch_init<P>(md, scratch, hsc);
  for (int s = tid; s < N; s += NTH) occ_s[s] = occ_g[s];
  for (int s = tid; s < 2 * N; s += NTH) lab_s[s] = lab_g[s];
  __syncthreads();

  // ---- ratio
  Tf* featw = (Tf*)bf.feat + lt.feat_off + wl * (long long)feat_planes(md) * N * C;
  const double* Gw = bf.G + lt.g_off + wl * 2LL * N * nm;
  const double* PTw = bf.PT + lt.pt_off + wl * 2LL * nm * C;
  const HopGeom g = hop_geom(lt, md.L, sp, i, d);
  const AxisTab tab = axis_tab(g, md.L, lane);
  int olx, owx, oly, owy;
  hop_features<P, C, NW, 7, MLP>(md, lt, g, occ_s, featw, (Tf*)nullptr, scratch, hsc, tab, olx, owx, oly, owy);
  const int KM = lt.Gx * lt.Gy;
  int* kl = (int*)(scratch + hsc.klists) + wv * KM;
  double* misc = (double*)(scratch + hsc.misc);
  int hpos;
  const int K = hop_klist(lt, g, tab, occ_s, lab_s, wv, olx, owx, oly, owy, kl, hpos, lane);
  const double* PTt = PTw + (long long)wv * nm * C;
  const double* Gj = Gw + ((long long)wv * N + g.j) * nm;
  v4d dacc[DetTiles<C>::I][DetTiles<C>::J];
  hop_det_build<C>(kl, K, wv == sp, hpos, (const DT*)scratch, PTt, Gj, lane, dacc);
  __syncthreads();      // both matrices built: their staging may overwrite D
  double* stage = (double*)scratch + wv * (C + 1) * DetTiles<C>::RS;
  const double Rt = hop_det_finish<C>(dacc, kl, K, wv == sp, hpos, PTt, Gj, stage, lane);
  if (lane == 0) misc[wv] = Rt;
  __syncthreads();
  const double R0 = misc[0], R1 = misc[1];
  const double R = R0 * R1;
  if (sa.sym_mode == 1) {
    if (tid == 0) {
      sa.sym_ratio[w] = R;
      hdr[HD_ACC] = 0;
    }
    return;
  }
  if (sa.sym_mode == 2 ? sa.sym_acc[w] == 0 : !(u < R * R)) {         // uniform
    if (tid == 0) hdr[HD_ACC] = 0;
    return;
  }

  // ---- accepted.  Wavefront tau: A^-1 of spin tau from the staged A (still
  // in LDS: the LU worked on registers), its changed-row list and G[j].
  const int kmaxb = box_kmax(lt.Gx, lt.Gy, md.L, lt.nd);
  const int ntau = wv == 0 ? n_up : n_dn;
  bool ok = true;
  if (ntau > 0) {
    const bool hs = wv == sp;
    const int R_ = C + (hs ? 1 : 0);
    double* ai = (double*)(st + sl.ainv) + (long long)wv * RA * RA;
    if (K == 0) {
      // no changed row of this spin (never the moving one): A = I
      for (int e2 = lane; e2 < RA * RA; e2 += 64) ai[e2] = (e2 / RA == e2 % RA && e2 / RA < R_) ? 1.0 : 0.0;
    } else {
      double arow[RA];
      const double2* rp = reinterpret_cast<const double2*>(stage + (lane < R_ ? lane : 0) * DetTiles<C>::RS);
#pragma unroll
      for (int c2 = 0; c2 < DetTiles<C>::RS / 2; ++c2) {
        const double2 v = rp[c2];
        if (2 * c2 < RA) arow[2 * c2] = (lane < R_ && 2 * c2 < R_) ? v.x : 0.0;
        if (2 * c2 + 1 < RA) arow[2 * c2 + 1] = (lane < R_ && 2 * c2 + 1 < R_) ? v.y : 0.0;
      }
      int mystep;
      ok = gj_inverse_rot<RA>(arow, R_, lane, perm, mystep);
      // every lane reads the pivot order lane 0 wrote: order the accesses
      // for the compiler (a wavefront's LDS operations stay in order)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ok) {
        if (lane < R_) {
#pragma unroll
          for (int qq = 0; qq < RA; ++qq) {
            if (qq < R_) {
              const int slot = RA - R_ + qq;
              double v = 0.0;
#pragma unroll
              for (int s2 = 0; s2 < RA; ++s2) v = (s2 == slot) ? arow[s2] : v;
              ai[mystep * RA + perm[qq]] = v;   // A^-1[p][perm[q]]
            }
          }
        }
        if (R_ < RA) {   // zero row and column C
          if (lane < RA) ai[C * RA + lane] = 0.0;
          if (lane < C) ai[lane * RA + C] = 0.0;
        }
      }
    }
    int* klo = (int*)(st + sl.kl) + wv * kmaxb;
    for (int a = lane; a < K; a += 64) klo[a] = kl[a];
    double* gjo = (double*)(st + sl.gj) + (long long)wv * nm;
    for (int kc = lane; kc < ntau; kc += 64) gjo[kc] = Gj[kc];
  }
  if (lane == 0) {
    misc[2 + wv] = (double)K;
    misc[4 + wv] = (double)hpos;
    misc[6 + wv] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  const bool fallback = misc[6] == 0.0 || misc[7] == 0.0;

  // ---- commit: the box features recomputed with write-back (D fresh in LDS)
  hop_features<P, C, NW, 7, MLP>(md, lt, g, occ_s, featw, featw, scratch, hsc, tab, olx, owx, oly, owy);
  {
    const int nv = owx * owy * (C + 4) * (int)sizeof(DT) / 16;
    const float4* src = reinterpret_cast<const float4*>(scratch);
    float4* dst = reinterpret_cast<float4*>(st + sl.D);
    for (int e2 = tid; e2 < nv; e2 += NTH) dst[e2] = src[e2];
  }
  // ---- configuration, labels, log|psi|, counters, header
  if (tid == 0) {
    const int j = g.j;
    occ_g[i] -= bit;
    occ_g[j] += bit;
    lab_g[sp * N + j] = (int16_t)k;
    lab_g[sp * N + i] = -1;
    pos_g[sp * nm + k] = (int16_t)j;
    bf.ld[2 * w] += log(fabs(R0));
    bf.ld[2 * w + 1] += log(fabs(R1));
    if (R0 < 0) bf.sg[2 * w] = -bf.sg[2 * w];
    if (R1 < 0) bf.sg[2 * w + 1] = -bf.sg[2 * w + 1];
    // a walker whose G and P could not be updated is rebuilt after this step
    // (urgent list); one that reaches refresh_every accepted moves at the
    // next batch refresh (its G and P stay current meanwhile)
    const int na = fallback ? SW_REBUILD : bf.nacc[w] + 1;
    bf.nacc[w] = na;
    if (fallback) sa.urgent_list[atomicAdd(sa.urgent_count, 1)] = (int)w;
    else if (na == sa.refresh_every) sa.due_list[atomicAdd(sa.due_count, 1)] = (int)w;
    if (sa.n_accept) sa.n_accept[w] += 1;
    hdr[HD_SP] = sp;
    hdr[HD_K] = k;
    hdr[HD_J] = j;
    hdr[HD_OLX] = olx;
    hdr[HD_OWX] = owx;
    hdr[HD_OLY] = oly;
    hdr[HD_OWY] = owy;
    hdr[HD_R0] = (int)misc[2];
    hdr[HD_R1] = (int)misc[3];
    hdr[HD_HPOS] = (int)misc[4 + sp];
    hdr[HD_ACC] = fallback ? 0 : 1;
    if (!fallback) sa.acc_list[atomicAdd(sa.count, 1)] = (int)w;
  }
}

// G and P updates of the walkers that accepted at this step: one item per
// (walker, spin), items dealt to a persistent grid.  Block 0 clears the
// counter of the next step.
template <int P, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_step_update(int L, const LatDev* __restrict__ lats, int nlats, Bufs bf,
                                                     StepArgs sa) {
  typedef typename DType<P>::type DT;
  constexpr int NTH = 256, RA = C + 1, SC = UPD_SC, SD = DStride<C>::value;
  constexpr int KS = (RA + 3) / 4;                          // k-steps of the 16x16x4 f64 MFMA
  constexpr int ECS = 4 * KS;                               // E row stride (zero padded)
  static_assert(RA <= 48 && SC == 16 * (NTH / 64), "E product tiles: 3 column tiles, one row tile per wave");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) *sa.count_next = 0;
  const long long items = 2LL * uniform_i(*(volatile int*)sa.count);
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const long long w = sa.acc_list[it >> 1];
    const int tau = (int)(it & 1);
    int li = 0;
    while (li + 1 < nlats && w >= lats[li + 1].w0) ++li;
    const LatDev lt = lats[li];
    const long long wl = w - lt.w0;
    const int N = lt.N, nm = lt.nmax;
    const int n = tau == 0 ? lt.n[0] : lt.n[1];
    if (n == 0) continue;                                             // uniform
    const int kmaxb = box_kmax(lt.Gx, lt.Gy, L, lt.nd);
    const StepStage sl = step_stage(nm, lt.Gx, lt.Gy, L, lt.nd, C, (int)sizeof(DT));
    const char* st = sa.stage + w * sa.stage_stride;
    const int* hdr = (const int*)(st + sl.hdr);
    const int sp = hdr[HD_SP], kmv = hdr[HD_K], olx = hdr[HD_OLX], owx = hdr[HD_OWX], oly = hdr[HD_OLY],
              owy = hdr[HD_OWY];
    const int r = hdr[HD_R0 + tau], hpos = hdr[HD_HPOS];
    const bool hs = tau == sp;
    const int* klg = (const int*)(st + sl.kl) + tau * kmaxb;
    const DT* Dg = (const DT*)(st + sl.D);
    const double* aig = (const double*)(st + sl.ainv) + (long long)tau * RA * RA;
    const double* gjs = (const double*)(st + sl.gj) + (long long)tau * nm;
    double* Gt = bf.G + lt.g_off + wl * 2LL * N * nm + (long long)tau * N * nm;
    double* PTt = bf.PT + lt.pt_off + wl * 2LL * nm * C + (long long)tau * nm * C;
    double* ainv = (double*)smem;
    int* kls = (int*)(smem + al16(RA * RA * 8));
    DT* dk = (DT*)(smem + al16(RA * RA * 8) + al16(kmaxb * 4));          // D(m_a), row a
    double* ec = (double*)(smem + al16(RA * RA * 8) + al16(kmaxb * 4) + al16(kmaxb * C * (int)sizeof(DT)));
    for (int e2 = tid; e2 < RA * RA; e2 += NTH) ainv[e2] = aig[e2];
    for (int a = tid; a < r; a += NTH) kls[a] = klg[a];
    __syncthreads();
    for (int e2 = tid; e2 < r * C; e2 += NTH) {
      const int a = e2 / C, c = e2 - a * C;
      dk[e2] = Dg[(kls[a] >> 16) * SD + c];
    }
    __syncthreads();
    // G'[s][k'] = G[s][k'] + E[s] . W[:, k'] in chunks of SC sites, with
    //   E[s] = D(s) A^-1[0:C, :] - G[s, K] B,  B = U A^-1,
    // U[a] = [D(m_a), 1 if a is the mover's row of the moving spin].  Taken
    // as E[s] = [Et(s) | -g(s)] A^-1 with Et(s) = D(s) - sum_a G[s, k_a] D(m_a)
    // and g(s) = G[s, k_mover] (moving spin): two products on the FP64
    // matrix cores per chunk, wavefront t forming the rows of sites
    // 16 t .. 16 t + 15 (D(s) is zero off the box).
    const int wave = tid >> 6, lane = tid & 63, lj = lane & 15, lk = lane >> 4;
    constexpr int CT = (C + 15) / 16;               // column tiles of Et
    const int ke1 = (r + 3) / 4;                    // k-steps of the first product
    const int kmov = hs ? kls[hpos] & 0xffff : 0;
    for (int s0 = 0; s0 < N; s0 += SC) {
      const int ns = min(SC, N - s0);
      double* ew = ec + 16 * wave * ECS;            // this wavefront's 16 rows
      if (16 * wave < ns) {
        const int si = 16 * wave + lj;              // this lane's A row (site)
        const bool sok = si < ns;
        const double* Gs = Gt + (long long)(s0 + (sok ? si : 0)) * nm;
        // Et: accumulator starts at D(s) of the result rows (lk + 4 v)
        v4d acc1[CT];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int so = 16 * wave + lk + 4 * v;
          const int mb = so < ns ? box_index(lt, s0 + so, olx, owx, oly, owy) : -1;
#pragma unroll
          for (int tj = 0; tj < CT; ++tj) {
            const int col = 16 * tj + lj;
            acc1[tj][v] = (mb >= 0 && col < C) ? (double)Dg[mb * SD + col] : 0.0;
          }
        }
        for (int q0 = 0; q0 < ke1; q0 += 4) {
          double av[4], bv[4][CT];                  // four k-steps in flight
#pragma unroll
          for (int u2 = 0; u2 < 4; ++u2) {
            const int a = 4 * (q0 + u2) + lk;
            const bool ok = a < r;
            const int e = ok ? kls[a] : 0;
            av[u2] = (ok && sok) ? -Gs[e & 0xffff] : 0.0;
#pragma unroll
            for (int tj = 0; tj < CT; ++tj) {
              const int col = 16 * tj + lj;
              bv[u2][tj] = (ok && col < C) ? (double)dk[a * C + col] : 0.0;
            }
          }
#pragma unroll
          for (int u2 = 0; u2 < 4; ++u2) {
            if (q0 + u2 >= ke1) break;
#pragma unroll
            for (int tj = 0; tj < CT; ++tj) mfma(acc1[tj], av[u2], bv[u2][tj]);
          }
        }
        // [Et | -g | 0] to this wavefront's rows, then read back as A rows
#pragma unroll
        for (int tj = 0; tj < CT; ++tj) {
          const int col = 16 * tj + lj;
          if (col >= C) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) ew[(lk + 4 * v) * ECS + col] = acc1[tj][v];
        }
        if (lk == 0)
          for (int c = C; c < ECS; ++c) ew[lj * ECS + c] = (c == C && hs && sok) ? -Gs[kmov] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        v4d eacc[3];
#pragma unroll
        for (int tj = 0; tj < 3; ++tj) eacc[tj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          const int c2 = 4 * q + lk;
          const double a2 = ew[lj * ECS + c2];
#pragma unroll
          for (int tj = 0; tj < 3; ++tj) {
            const int col = 16 * tj + lj;
            const double b2 = (c2 < RA && col < RA) ? ainv[c2 * RA + col] : 0.0;
            mfma(eacc[tj], a2, b2);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // E rows to LDS (columns C + 1 .. ECS - 1 are zero)
#pragma unroll
        for (int tj = 0; tj < 3; ++tj) {
          const int col = 16 * tj + lj;
          if (col >= ECS) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) ew[(lk + 4 * v) * ECS + col] = eacc[tj][v];
        }
      }
      __syncthreads();
      // G[s0 + i][16 tj + j] += sum_c2 E[i][c2] W[c2][16 tj + j] on the FP64
      // matrix cores: A = E rows (LDS), B = W fragments, C = the G tile
      {
        const int ntj = (n + 15) / 16;
        for (int tj = wave; tj < ntj; tj += NTH / 64) {
          const int kc = 16 * tj + lj;
          const int kcc = kc < n ? kc : n - 1;
          // contraction index c2 = KS * lk + qq: a lane's W operands are a
          // contiguous run of its P^T row (wide loads; past the row's end
          // masked, slack after the array), its E operands a run of an E row
          const double* prow = PTt + (long long)kcc * C + KS * lk;
          double pv[KS];
#pragma unroll
          for (int qq = 0; qq < KS; ++qq) pv[qq] = prow[qq];
          const double gv = gjs[kcc] - (kc == kmv ? 1.0 : 0.0);
          double bw[KS];
#pragma unroll
          for (int qq = 0; qq < KS; ++qq) {
            const int c2 = KS * lk + qq;
            bw[qq] = kc >= n ? 0.0 : c2 < C ? pv[qq] : (c2 == C && hs) ? gv : 0.0;
          }
          for (int ti = 0; 16 * ti < ns; ++ti) {
            v4d acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int sr = 16 * ti + lk + 4 * v;
              acc[v] = (sr < ns && kc < n) ? Gt[(long long)(s0 + sr) * nm + kc] : 0.0;
            }
            const double* er = ec + (16 * ti + lj) * ECS + KS * lk;
#pragma unroll
            for (int qq = 0; qq < KS; ++qq) mfma(acc, er[qq], bw[qq]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int sr = 16 * ti + lk + 4 * v;
              if (sr < ns && kc < n) Gt[(long long)(s0 + sr) * nm + kc] = acc[v];
            }
          }
        }
      }
      __syncthreads();
    }
    // P^T'[k'][cp] = sum_c2 W[c2][k'] A^-1[cp][c2] (W from the old P^T and
    // G[j]) on the FP64 matrix cores, in place: a wavefront reads all of its
    // 16 rows of P^T before it writes them, and no other wavefront touches them
    for (int ti = wave; 16 * ti < n; ti += NTH / 64) {
      const int kr = 16 * ti + lj;
      const int krc = kr < n ? kr : n - 1;
      // contraction index c2 = KS * lk + q, as in the G update: contiguous runs
      const double* prow = PTt + (long long)krc * C + KS * lk;
      double pv[KS];
#pragma unroll
      for (int q = 0; q < KS; ++q) pv[q] = prow[q];
      const double gv = gjs[krc] - (kr == kmv ? 1.0 : 0.0);
      double av[KS];
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        const int c2 = KS * lk + q;
        av[q] = kr >= n ? 0.0 : c2 < C ? pv[q] : (c2 == C && hs) ? gv : 0.0;
      }
      v4d pacc[CT];
#pragma unroll
      for (int tj = 0; tj < CT; ++tj) {
        pacc[tj] = v4d{0.0, 0.0, 0.0, 0.0};
        const int col = 16 * tj + lj;
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          const int c2 = KS * lk + q;
          const double b2 = (c2 < RA && col < C) ? ainv[col * RA + c2] : 0.0;
          mfma(pacc[tj], av[q], b2);
        }
      }
#pragma unroll
      for (int tj = 0; tj < CT; ++tj) {
        const int col = 16 * tj + lj;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ko = 16 * ti + lk + 4 * v;
          if (ko < n && col < C) PTt[(long long)ko * C + col] = pacc[tj][v];
        }
      }
    }
    __syncthreads();
  }
}

template <int P, int C>
static hipError_t step_impl(const ModelDev& md, const LatDev* lats_dev, int nlats, long long W, const Bufs& bf,
                            const StepArgs& sa, size_t smem_p, size_t smem_u, int upd_blocks, hipStream_t st) {
  auto kp = md.M > 0 ? k_step_propose<P, C, true> : k_step_propose<P, C, false>;
  auto ku = k_step_update<P, C>;
  hipError_t e = hipFuncSetAttribute((const void*)kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_p);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)ku, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_u);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kp, dim3((unsigned)W), dim3(128), smem_p, st, md, lats_dev, nlats, bf, sa);
  // (the ratio-only pass of symmetric sampling changes nothing to update)
  if (sa.sym_mode != 1)
    hipLaunchKernelGGL(ku, dim3((unsigned)upd_blocks), dim3(256), smem_u, st, md.L, lats_dev, nlats, bf, sa);
  return hipGetLastError();
}

hipError_t SVMC_CAT3(sweep_step_, SVMC_INST_P, SVMC_INST_C)(const ModelDev& md, const LatDev* lats_dev, int nlats,
                                                            long long W, const Bufs& bf, const StepArgs& sa,
                                                            size_t smem_p, size_t smem_u, int upd_blocks,
                                                            hipStream_t st) {
  return step_impl<SVMC_INST_P, SVMC_INST_C>(md, lats_dev, nlats, W, bf, sa, smem_p, smem_u, upd_blocks, st);
}
#else
// Drift of the maintained G before a refresh: max |G[pos_k][k'] - delta|
// over occupied rows (these rows of M Phi^-1 are unit rows in exact
// arithmetic); sets the DRIFT flag above 1e-8.  Only walkers due for a
// refresh (nacc >= refresh_every) when only_due != 0.
SVMC_DEV void drift_one(const LatDev& lt, const Bufs& bf, long long wl, double* red) {
  const long long w = lt.w0 + wl;
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
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(red[0] <= 1e-8)) atomicOr(bf.flags + w, 4);
}
__global__ __launch_bounds__(256) void k_drift(LatDev lt, Bufs bf, WalkerSel sel) {
  __shared__ double red[256];
  for (long long z = blockIdx.x;; z += gridDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);    // uniform in the block
    if (r == 0) break;
    if (r == 1) drift_one(lt, bf, wl, red);
    __syncthreads();
  }
}

// accept counters of the selected walkers back to zero (after their rebuild)
__global__ void k_clear_nacc(LatDev lt, Bufs bf, WalkerSel sel) {
  for (long long z = blockIdx.x * (long long)blockDim.x + threadIdx.x;; z += (long long)gridDim.x * blockDim.x) {
    long long wl;
    const int r = pick_walker(sel, lt, z, wl);
    if (r == 0) break;
    if (r == 1) bf.nacc[lt.w0 + wl] = 0;
  }
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

// Workspace of one step: LDS of the proposal kernel, LDS of the update
// kernel, and the staging bytes per walker.
StepSizes step_sizes(const LatDev* lats, int nlats, int prec, int L, int C) {
  const int tfb = prec == PREC_F64 ? 8 : 4;
  StepSizes z{0, 0, 0};
  for (int l = 0; l < nlats; ++l) {
    const LatDev& lt = lats[l];
    z.smem_propose = std::max(z.smem_propose, (size_t)propose_layout(lt.N, lt.Gx, lt.Gy, L, C, tfb).bytes);
    z.smem_update = std::max(z.smem_update, (size_t)update_lds_bytes(box_kmax(lt.Gx, lt.Gy, L, lt.nd), C, tfb));
    z.stage_bytes = std::max(z.stage_bytes, (size_t)step_stage(lt.nmax, lt.Gx, lt.Gy, L, lt.nd, C, tfb).bytes);
  }
  return z;
}
__global__ void k_fill_i32(int32_t* p, long long n, int32_t v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_drift(const LatDev& lt, const Bufs& bf, WalkerSel sel, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  const long long slots = sel.list ? std::min<long long>(lt.nw, 256) : lt.nw;
  hipLaunchKernelGGL(k_drift, dim3((unsigned)slots), dim3(256), 0, st, lt, bf, sel);
  return hipGetLastError();
}

hipError_t launch_clear_nacc(const LatDev& lt, const Bufs& bf, WalkerSel sel, hipStream_t st) {
  if (lt.nw == 0) return hipSuccess;
  const long long slots = sel.list ? std::min<long long>(lt.nw, 256) : lt.nw;
  hipLaunchKernelGGL(k_clear_nacc, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st, lt, bf, sel);
  return hipGetLastError();
}

hipError_t launch_sweep_step(int prec, const ModelDev& md, const LatDev* lats_dev, const LatDev* lats_host,
                             int nlats, long long W, const Bufs& bf, const StepArgs& sa, hipStream_t st) {
  const StepSizes z = step_sizes(lats_host, nlats, prec, md.L, md.C);
  if (z.smem_propose > 160 * 1024 || z.smem_update > 160 * 1024) return hipErrorInvalidValue;
  // persistent update grid: as many workgroups as fit at once
  const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / std::max<size_t>(z.smem_update, 1))));
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
  }
  const int blocks = ncu * per_cu;
#define SVMC_SW(P_, C_)                                                                                     \
  if (prec == P_ && md.C == C_)                                                                           \
    return sweep_step_##P_##_##C_(md, lats_dev, nlats, W, bf, sa, z.smem_propose, z.smem_update, blocks, st);
  SVMC_FOR_EACH_PREC_C(SVMC_SW)
#undef SVMC_SW
  return hipErrorInvalidValue;
}
#endif

}  // namespace svmc
