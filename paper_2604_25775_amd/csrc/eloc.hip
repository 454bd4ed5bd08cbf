// Low-rank local energies (Sec. II.A definition of E_loc with the Hubbard
// Hamiltonian of Sec. III; ratios by the local update of Sec. II.C).
//
// A walker's connected configurations are enumerated in canonical order (spin
// up first, source site ascending, directions +x, -x, +y, -y, then the four
// diagonals when t' != 0) and split into `slices` contiguous ranges; one
// workgroup (two wavefronts) evaluates one range, hop after hop (conv split
// between the wavefronts, then one determinant per wavefront).  Lattices of
// a mixed batch share the launch.  Partial sums are added per walker in
// slice order by a second small kernel (deterministic).
#include "hop.h"
#include "svmc_launch.h"

namespace svmc {

struct ElocLds {
  int occ, lab, hops, red, scratch;   // byte offsets
  int wave_bytes;
};

inline __host__ __device__ int align16(int x) { return (x + 15) & ~15; }

constexpr int ELOC_NW = 2;     // wavefronts per workgroup

// the one-conv-layer instance serves (see k_eloc_lowrank's SMALL)
inline bool eloc_small(const ModelDev& md, const ElocOut& out) { return md.L == 1 && out.row_form_max >= 16; }

__host__ __device__ inline ElocLds eloc_layout(int N, int maxhops, int Gx, int Gy, int L, int C, int tfb,
                                               bool rows_only) {
  ElocLds o;
  o.occ = 0;
  o.lab = align16(N);
  o.hops = o.lab + align16(4 * N);
  o.red = o.hops + align16(2 * maxhops);
  o.scratch = o.red + 64;
  o.wave_bytes = hop_scratch(Gx, Gy, L, C, tfb, rows_only).bytes;
  return o;
}

// exclusive block scan of one int per thread (blockDim.x = 64 * waves)
SVMC_DEV int block_excl_scan(int v, int* tmp, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int incl = wave_incl_scan(v, lane);
  if (lane == 63) tmp[wv] = incl;
  __syncthreads();
  int off = 0;
  total = 0;
  for (int k = 0; k < nwv; ++k) {
    if (k < wv) off += tmp[k];
    total += tmp[k];
  }
  __syncthreads();
  return off + incl - v;
}

// Enumerate the walker's connected configurations into `hops` (16-bit codes
// of conn_code, canonical order); returns the count.  At most `cap` codes
// are stored (a walker with a wrong electron count may have more).  All
// threads of the block take part.
SVMC_DEV int enumerate_hops(const LatDev& lt, const int8_t* occ_s, uint16_t* hops, int* tmp, int cap) {
  const int items = conn_items(lt), tid = threadIdx.x;
  const int per = (items + blockDim.x - 1) / blockDim.x;
  const int e0 = tid * per;
  int cnt = 0;
  for (int e = e0; e < min(items, e0 + per); ++e) cnt += __popc(conn_mask(lt, occ_s, e));
  int total;
  int off = block_excl_scan(cnt, tmp, total);
  for (int e = e0; e < min(items, e0 + per); ++e) {
    unsigned m = conn_mask(lt, occ_s, e);
    while (m) {
      const int d = __ffs(m) - 1;
      m &= m - 1;
      if (off < cap) hops[off] = (uint16_t)conn_code(lt, e, d);
      ++off;
    }
  }
  __syncthreads();
  return total;
}

#ifdef SVMC_INST_P
// Block b -> (walker, slice).  Blocks are dealt to the 8 XCDs round-robin
// (XCD = b mod 8); the slices of one walker get consecutive positions on the
// same XCD so that walker's features, P^T and G stay in that XCD's L2.
SVMC_DEV void eloc_block(long long b, int S, long long& w, int& slice) {
  const long long xcd = b & 7, r = b >> 3;
  slice = (int)(r % S);
  w = (r / S) * 8 + xcd;
}

// SMALL: the instance for one conv layer, whose update boxes hold at most
// 4 x 4 sites, so at most 16 changed rows per spin: the row form always
// applies, the column form and the registers of larger boxes are left out,
// and more wavefronts fit per SIMD.  Its workgroups are one wavefront, which
// evaluates a hop alone (conv tiles, both spins' change lists and row-form
// matrices, both determinants): twice the hops in flight per CU, and no
// barrier waits on another wavefront.  MLP: the instance for networks with
// site-wise layers (the others do not carry that code).
template <int P, int C, bool SMALL, bool MLP>
__global__ __launch_bounds__(SMALL ? 64 : 64 * ELOC_NW) __attribute__((amdgpu_waves_per_eu(SMALL ? 4 : 3))) void
k_eloc_lowrank(ModelDev md, const LatDev* __restrict__ lats, int nlats, Bufs bf, ElocOut out, long long Wtot) {
  typedef typename PrecT<P>::Tf Tf;
  constexpr int NW = SMALL ? 1 : ELOC_NW, NTH = 64 * NW;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  long long w;
  int slice;
  eloc_block(blockIdx.x, out.slices, w, slice);
  if (w >= Wtot) return;
  int li = 0;
  while (li + 1 < nlats && w >= lats[li + 1].w0) ++li;
  const LatDev lt = lats[li];
  const long long wl = w - lt.w0;
  const int N = lt.N, nm = lt.nmax;
  const int tid = threadIdx.x, wv = uniform_i(tid >> 6);
  const ElocLds lay = eloc_layout(N, lt.maxhops, lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf), SMALL);
  int8_t* occ_s = (int8_t*)(smem + lay.occ);
  int16_t* lab_s = (int16_t*)(smem + lay.lab);
  uint16_t* hops = (uint16_t*)(smem + lay.hops);
  double* red = (double*)(smem + lay.red);
  char* scratch = smem + lay.scratch;
  const HopScratch hsc = hop_scratch(lt.Gx, lt.Gy, md.L, C, (int)sizeof(Tf), SMALL);
  hop_scratch_init<P>(md, scratch, hsc);

  const int8_t* occ_g = bf.occ + lt.occ_off + wl * N;
  const int16_t* lab_g = bf.lab + lt.lab_off + wl * 2LL * N;
  for (int s = tid; s < N; s += NTH) occ_s[s] = occ_g[s];
  for (int s = tid; s < 2 * N; s += NTH) lab_s[s] = lab_g[s];
  __syncthreads();
  const int H = uniform_i(min(enumerate_hops(lt, occ_s, hops, (int*)red, lt.maxhops), lt.maxhops));
  const bool bad = (bf.flags[w] & (1 | 8)) != 0;
  // this block's hops: a contiguous slice of the canonical order
  const int h0 = (int)(((long long)H * slice) / out.slices), h1 = (int)(((long long)H * (slice + 1)) / out.slices);

  const Tf* featw = (const Tf*)bf.feat + lt.feat_off + wl * (long long)feat_planes(md) * N * C;
  const double* Gw = bf.G + lt.g_off + wl * 2LL * N * nm;
  const double* PTw = bf.PT + lt.pt_off + wl * 2LL * nm * C;
  const int KM = lt.Gx * lt.Gy;
  int* kl = (int*)(scratch + hsc.klists) + wv * KM;
  double* misc = (double*)(scratch + hsc.misc);

  // the slice's running sum sits in LDS, read and written by thread 0 only:
  // as a register it is held by every lane through the hop loop (and spilled
  // around the conv, one scratch store per hop)
  double* part_s = red + 7;
  // the hopping amplitudes t, t' and J/2 (an exchange) in LDS, read by
  // thread 0 per hop: as values they stay live through the hop loop
  double* amp_s = red + 1;
  if (tid == 0) {
    *part_s = 0.0;
    amp_s[0] = lt.t;
    amp_s[1] = lt.tp;
    amp_s[2] = 0.5 * lt.J;
  }
  bool nonfinite = false;
  if (!bad) {
    for (int hh = h0; hh < h1; ++hh) {
      // lane index through an opaque copy (see hop_features)
      int lane;
      asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"((int)threadIdx.x & 63));
      const Conn cn = conn_decode(lt, uniform_i(hops[hh]));
      const int sp = cn.sp;
      // the hop's amplitude waits in LDS for the end of the hop
      if (tid == 0) misc[4] = amp_s[cn.ex ? 2 : (cn.d < 4 ? 0 : 1)];
      const HopGeom g = hop_geom(lt, md.L, sp, cn.i, cn.d, cn.ex);
      int olx, owx, oly, owy;
      const AxisTab tab = axis_tab(g, md.L, lane);
      hop_features<P, C, NW, SMALL ? 1 : 7, MLP>(md, lt, g, occ_s, featw, (Tf*)nullptr, scratch, hsc, tab, olx, owx,
                                                 oly, owy);
      if constexpr (SMALL) {
        // one wavefront: both spins' change lists and row-form matrices
        // (at most 16 rows each), then both determinants at once
        int Kt[2], hp[2];
        v4d racc[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) Kt[q] = hop_klist(lt, g, tab, occ_s, lab_s, q, olx, owx, oly, owy, kl + q * KM, hp[q], lane);
        const int KMx = uniform_i(max(Kt[0], Kt[1]));
#pragma unroll
        for (int q = 0; q < 2; ++q)
          racc[q] = hop_det_row_build<C>(kl + q * KM, Kt[q], (const typename DType<P>::type*)scratch,
                                         PTw + (long long)q * nm * C, lane);
        __syncthreads();    // both matrices built: their staging may overwrite D
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const bool mvq = q == sp || cn.ex;
          const double* Gq = Gw + ((long long)q * N + (q == sp ? g.j : g.i)) * nm;
          double* rstage = (double*)scratch + q * 16 * 17;
          if (KMx <= 8) hop_det_row_stage<8>(racc[q], kl + q * KM, Kt[q], mvq, hp[q], Gq, rstage, lane);
          else hop_det_row_stage<16>(racc[q], kl + q * KM, Kt[q], mvq, hp[q], Gq, rstage, lane);
        }
        __syncthreads();
        auto pair = [&](auto ks) {
          constexpr int KS = decltype(ks)::value;
          const double* sr = (const double*)scratch + (lane >> 5) * 16 * 17 +
                             ((lane & 31) < KS ? (lane & 31) : 0) * (KS + 1);
          double a[KS];
#pragma unroll
          for (int c2 = 0; c2 < KS; ++c2) a[c2] = (lane & 31) < KS ? sr[c2] : 0.0;
          __builtin_amdgcn_wave_barrier();
          return lu_det_pair<KS>(a, lane);
        };
        const double dt = KMx <= 8 ? pair(IntC<8>()) : pair(IntC<16>());
        if ((lane & 31) == 0) misc[lane >> 5] = dt;
        // (more than 16 rows cannot occur with one conv layer; if a caller
        // broke that, the ratio is flagged rather than wrong)
        if (lane == 0) {
          misc[2] = KMx > 16 ? NAN : 1.0;
          misc[3] = 1.0;
        }
        __syncthreads();
      } else {
        // wavefront wv: determinant of spin wv
        int hpos;
        const int K = hop_klist(lt, g, tab, occ_s, lab_s, wv, olx, owx, oly, owy, kl, hpos, lane);
        const double* PTt = PTw + (long long)wv * nm * C;
        // spin wv's moving electron (a hop: spin sp, i -> j; an exchange: both
        // spins, the down electron j -> i) and the G row of its new site
        const bool mv = wv == sp || cn.ex;
        const double* Gj = Gw + ((long long)wv * N + (wv == sp ? g.j : g.i)) * nm;
        // few changed rows in both spins: the row form (K x K, padded to 8 or
        // 16) instead of the column form of size C + 1
        const int Ko = hop_kcount(lt, g, tab, occ_s, 1 - wv, olx, owx, oly, owy, lane);
        const int KM = uniform_i(max(K, Ko));
        if (KM <= out.row_form_max) {
          const v4d racc = hop_det_row_build<C>(kl, K, (const typename DType<P>::type*)scratch, PTt, lane);
          __syncthreads();    // both matrices built: their staging may overwrite D
          double* rstage = (double*)scratch + wv * 16 * 17;
          if (KM <= 8) hop_det_row_stage<8>(racc, kl, K, mv, hpos, Gj, rstage, lane);
          else hop_det_row_stage<16>(racc, kl, K, mv, hpos, Gj, rstage, lane);
          __syncthreads();
          if (wv == 0) {
            // both K x K determinants in wavefront 0, one matrix per half
            auto pair = [&](auto ks) {
              constexpr int KS = decltype(ks)::value;
              const double* sr = (const double*)scratch + (lane >> 5) * 16 * 17 +
                                 ((lane & 31) < KS ? (lane & 31) : 0) * (KS + 1);
              double a[KS];
#pragma unroll
              for (int c2 = 0; c2 < KS; ++c2) a[c2] = (lane & 31) < KS ? sr[c2] : 0.0;
              __builtin_amdgcn_wave_barrier();
              return lu_det_pair<KS>(a, lane);
            };
            const double dt = KM <= 8 ? pair(IntC<8>()) : pair(IntC<16>());
            if ((lane & 31) == 0) misc[lane >> 5] = dt;
            if (lane == 0) misc[2] = misc[3] = 1.0;
          }
          __syncthreads();
        } else {
          v4d dacc[DetTiles<C>::I][DetTiles<C>::J];
          hop_det_build<C>(kl, K, mv, hpos, (const typename DType<P>::type*)scratch, PTt, Gj, lane, dacc);
          __syncthreads();      // both matrices built: their staging may overwrite D
          double* stage = (double*)scratch + wv * (C + 1) * DetTiles<C>::RS;
          hop_det_stage<C>(dacc, kl, K, mv, hpos, PTt, Gj, stage, lane);
          // a moving spin's matrix is brought to C x C by one elimination step
          if (mv) {
            const double f = hop_det_reduce<C>(stage, lane);
            if (lane == 0) misc[wv == sp ? 2 : 3] = f;
          } else if (lane == 0) {
            misc[3] = 1.0;
          }
          // each wavefront factors its own spin's C x C matrix (its own staging
          // area: no barrier with the other wavefront), two lanes per row
          {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int r = lane >> 1;
            const double* sr = stage + (r < C ? r : 0) * DetTiles<C>::RS + (lane & 1);
            double a[C / 2];
#pragma unroll
            for (int j = 0; j < C / 2; ++j) a[j] = r < C ? sr[2 * j] : 0.0;
            __builtin_amdgcn_wave_barrier();
            const double dt = lu_det_split<C>(a, lane);
            if (lane == 0) misc[wv] = dt;
          }
          __syncthreads();
        }
      }
      if (tid == 0) {
        // misc[2], misc[3]: the moving spins' reduction factors (1 where
        // none was taken)
        const double R = misc[0] * misc[1] * misc[2] * misc[3];
        *part_s += -misc[4] * R;
        nonfinite |= !isfinite(R);
        if (out.ratio) {
          out.ratio[w * out.stride + hh] = R;
          out.code[w * out.stride + hh] = hops[hh];
        }
      }
    }
  }
  if (tid == 0) {
    double part = *part_s;
    if (nonfinite) atomicOr(bf.flags + w, 2);
    if (slice == 0) {
      // the diagonal term and the per-walker outputs go with slice 0
      part += diag_energy(lt, occ_s);
      if (out.nhops) out.nhops[w] = H;
    }
    out.part[w * out.slices + slice] = bad ? NAN : part;
  }
  if (bad && out.ratio && slice == 0) {
    for (int hh = tid; hh < H; hh += NTH) {
      out.ratio[w * out.stride + hh] = NAN;
      out.code[w * out.stride + hh] = hops[hh];
    }
  }
}

template <int P, int C>
static hipError_t eloc_impl(const ModelDev& md, const LatDev* lats_dev, int nlats, long long W, const Bufs& bf,
                            const ElocOut& out, size_t smem, hipStream_t st) {
  // one conv layer with the row form allowed up to 16 rows: every hop takes
  // the row form, so the smaller instance serves
  const bool sm = eloc_small(md, out), ml = md.M > 0;
  auto kern = sm ? (ml ? k_eloc_lowrank<P, C, true, true> : k_eloc_lowrank<P, C, true, false>)
                 : (ml ? k_eloc_lowrank<P, C, false, true> : k_eloc_lowrank<P, C, false, false>);
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const long long nblk = ((W + 7) / 8) * 8 * out.slices;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(sm ? 64 : 64 * ELOC_NW), smem, st, md, lats_dev, nlats, bf, out,
                     W);
  return hipGetLastError();
}

hipError_t SVMC_CAT3(eloc_lowrank_, SVMC_INST_P, SVMC_INST_C)(const ModelDev& md, const LatDev* lats_dev,
                                                              int nlats, long long W, const Bufs& bf,
                                                              const ElocOut& out, size_t smem, hipStream_t st) {
  return eloc_impl<SVMC_INST_P, SVMC_INST_C>(md, lats_dev, nlats, W, bf, out, smem, st);
}
#else
// Partial sums of the allocation-free local-energy entry point: a fixed
// array per device, shared by every call on that device (each call writes
// every slot it reads, so nothing needs clearing; calls that overlap on one
// device race).  Host code uses only the address hipGetSymbolAddress gives
// for the device that was current at set-up, never the symbol itself.
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = (double*)p;
  return hipSuccess;
}

double* noalloc_scratch(int dev) { return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr; }

size_t eloc_lowrank_smem(const LatDev* lats, int nlats, int prec, int L, int C, bool rows_only) {
  const int tfb = prec == PREC_F64 ? 8 : 4;
  size_t mx = 0;
  for (int l = 0; l < nlats; ++l) {
    const ElocLds o = eloc_layout(lats[l].N, lats[l].maxhops, lats[l].Gx, lats[l].Gy, L, C, tfb, rows_only);
    mx = std::max(mx, (size_t)o.scratch + (size_t)o.wave_bytes);
  }
  return mx;
}

// E_loc[w] = sum over the walker's slices of the partial sums, in slice order.
__global__ void k_eloc_sum(const double* __restrict__ part, int S, long long W, double* eloc) {
  const long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (w >= W) return;
  double e = 0.0;
  for (int k = 0; k < S; ++k) e += part[w * S + k];
  eloc[w] = e;
}

hipError_t launch_eloc_lowrank(int prec, const ModelDev& md, const LatDev* lats_dev, const LatDev* lats_host,
                               int nlats, long long W, const Bufs& bf, const ElocOut& out, hipStream_t st) {
  const size_t smem = eloc_lowrank_smem(lats_host, nlats, prec, md.L, md.C, eloc_small(md, out));
  if (smem > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
#define SVMC_EL(P_, C_) \
  if (prec == P_ && md.C == C_) e = eloc_lowrank_##P_##_##C_(md, lats_dev, nlats, W, bf, out, smem, st);
  SVMC_FOR_EACH_PREC_C(SVMC_EL)
#undef SVMC_EL
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eloc_sum, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, st, out.part, out.slices, W,
                     out.eloc);
  return hipGetLastError();
}

#endif

}  // namespace svmc
