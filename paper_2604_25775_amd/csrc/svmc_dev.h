// Device-side definitions shared by the scalevmc kernels: descriptors,
// wavefront helpers, the MFMA conv tile and the one-wave LU determinant.
//
// Target: gfx950 (CDNA4), wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SVMC_DEV __device__ __forceinline__

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));

// PREC_BF16X3: conv multiplier inputs split exactly into three BF16 terms
// (x = hi + mid + lo), three MFMA passes with FP32 accumulation, so the conv
// sees FP32 activations and BF16 weights.
// PREC_F16X2: features carried as pairs of FP16 terms: every layer output
// (and the embedding) is rounded to hi + lo with hi = x rounded toward zero to
// FP16 and lo = (x - hi) rounded toward zero to FP16 (22 significant bits,
// |x - (hi + lo)| < 2^-21 |x| in FP16's normal range), so the conv inputs
// split exactly into two FP16 MFMA passes with FP32 accumulation; FP16
// weights.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2, PREC_BF16X3 = 3, PREC_F16X2 = 4 };
// conv on the 16-bit matrix-core instructions (K chunks of 32)
template <int P> struct Mma16 {
  static constexpr bool value = P == PREC_BF16 || P == PREC_BF16X3 || P == PREC_F16X2;
};
enum { ACT_TANH = 0, ACT_SILU = 1 };

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
// One lattice of a (possibly mixed) batch.  Walkers [w0, w0 + nw) belong to
// it; every per-walker array below is addressed as base + off + (w - w0) *
// stride, with the strides implied by N, nmax and the model.
struct LatDev {
  int Lx, Ly, pbc_x, pbc_y, N;
  int n[2];       // electrons per spin
  int nmax;       // max(n[0], n[1]), leading dimension of per-spin matrices
  int nd;         // hop directions: 4 (t' = 0) or 8
  int maxhops;    // (n0 + n1) * nd, plus 4 min(n0, n1) spin exchanges (t-J)
  int torus_x, torus_y;   // incremental boxes wrap (axis shorter than 2L+4)
  int Gx, Gy;             // incremental grid extent per axis
  double t, tp, U;
  int tj;              // 1: t-J model (Gutzwiller projection, exchange J, pinning field hpin)
  double J, hpin;
  long long w0, nw;
  long long occ_off;   // int8  [N]
  long long lab_off;   // int16 [2][N]     label of the electron at a site, -1
  long long pos_off;   // int16 [2][nmax]  site of each label
  long long feat_off;  // Tf    [L + M][N][C]  H_1..H_L, then the M site-wise layers' outputs
  long long inv_off;   // f64   [2][nmax][nmax]  Phi^-1[m][k]
  long long m_off;     // f64   [2][N][nmax]     orbital rows of all sites
  long long g_off;     // f64   [2][N][nmax]     G = M Phi^-1
  long long pt_off;    // f64   [2][nmax][C]     P^T = (W Phi^-1)^T
  const double* base;  // [2][N][nmax]
  const double* W;     // [2][C][nmax]
  const double* b;     // [2][nmax]
  long long poff;      // offset of this lattice's W_up in the flat parameter vector
  // embedding of site s with occupation o, channel c: embed[emb_off + s * emb_ss + o * C + c]
  // (emb_ss = 0 for one table shared by all sites, 4 C for per-site tables)
  long long emb_off;
  int emb_ss;
};

// Device buffers of one context (walker-indexed arrays, see LatDev offsets).
struct Bufs {
  int8_t* occ;
  int16_t* lab;
  int16_t* pos;
  void* feat;        // Tf
  double* inv;
  double* M;
  double* G;
  double* PT;
  double* ld;        // [W][2] log|det Phi_s| (label order)
  double* sg;        // [W][2] sign of det Phi_s (label order)
  int32_t* flags;    // [W]
  int32_t* nacc;     // [W] accepted moves since the last refresh
};

// Network constants.  Bpack holds the conv kernels pre-arranged as MFMA B
// fragments: [layer][chunk q][out-tile nt][lane] of PrecT<P>::Tb; Bmlp the
// site-wise layers' C x C weights in the same arrangement (one tap).
struct ModelDev {
  int L, C, act;
  int M;               // site-wise layers after the conv stack
  const void* Bpack;
  const void* Bmlp;
  const void* embed;   // Tf [4][C], or per lattice [N][4][C] (LatDev::emb_off)
  const void* bias;    // Tf [L + M][C]: conv biases, then the site-wise biases
};
// feature planes cached per walker: the conv layers, then the site-wise ones
__host__ __device__ inline int feat_planes(const ModelDev& md) { return md.L + md.M; }

template <int P> struct PrecT;
template <> struct PrecT<PREC_F64> {
  typedef double Tf; typedef double Tb; typedef v4d Acc; static constexpr int KC = 4;
};
template <> struct PrecT<PREC_F32> {
  typedef float Tf; typedef float Tb; typedef v4f Acc; static constexpr int KC = 4;
};
template <> struct PrecT<PREC_BF16> {
  typedef float Tf; typedef v8bf Tb; typedef v4f Acc; static constexpr int KC = 32;
};
template <> struct PrecT<PREC_BF16X3> {
  typedef float Tf; typedef v8bf Tb; typedef v4f Acc; static constexpr int KC = 32;
};
template <> struct PrecT<PREC_F16X2> {
  typedef float Tf; typedef v8h Tb; typedef v4f Acc; static constexpr int KC = 32;
};

template <int P, int C> struct ConvCfg {
  static constexpr int KC = PrecT<P>::KC;
  static constexpr int K = 9 * C;
  static constexpr int Q = (K + KC - 1) / KC;   // K chunks per layer
  static constexpr int NT = (C + 15) / 16;      // 16-wide output tiles
};
// the same for a site-wise layer (one tap: K = C)
template <int P, int C> struct MlpCfg {
  static constexpr int KC = PrecT<P>::KC;
  static constexpr int K = C;
  static constexpr int Q = (K + KC - 1) / KC;
  static constexpr int NT = (C + 15) / 16;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
SVMC_DEV int imod(int a, int m) { int r = a % m; return r < 0 ? r + m : r; }

SVMC_DEV double readlane_d(double x, int lane) {
  long long v = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), lane);
  int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

SVMC_DEV int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Philox4x64-10 counter-based generator (Salmon et al., SC'11): ten rounds
// on the counter c with key (k0, k1); the Metropolis proposals draw one block
// each.
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


// Maximum of an unsigned key over the wavefront with DPP lane exchanges
// (quad swaps, half-row and row mirrors, then row broadcasts 15 and 31);
// lane 63 ends with the maximum, which is returned to every lane.
SVMC_DEV unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

SVMC_DEV double wave_sum_d(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
SVMC_DEV int wave_sum_i(int v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// inclusive prefix sum over the wave
SVMC_DEV int wave_incl_scan(int v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

template <class T> SVMC_DEV T act_fn(int act, T x);
// FP32: from the hardware exp2 and reciprocal, tanh(x) = sign(x) (1 - t) / (1 + t)
// with t = exp(-2|x|) (absolute error a few 1e-8, the rounding level of the
// FP32 residual stream it is added to); SiLU(x) = x / (1 + exp(-x)).
// act_c<A> is the same function with the activation fixed at compile time.
template <int A> SVMC_DEV float act_c(float x);
template <> SVMC_DEV float act_c<ACT_TANH>(float x) {
  constexpr float kLog2e = 1.4426950408889634f;
  const float t = __builtin_amdgcn_exp2f(-2.0f * kLog2e * fabsf(x));
  const float r = (1.0f - t) * __builtin_amdgcn_rcpf(1.0f + t);
  return copysignf(r, x);
}
template <> SVMC_DEV float act_c<ACT_SILU>(float x) {
  constexpr float kLog2e = 1.4426950408889634f;
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-kLog2e * x));
}
template <> SVMC_DEV float act_fn<float>(int act, float x) {
  return act == ACT_TANH ? act_c<ACT_TANH>(x) : act_c<ACT_SILU>(x);
}
template <> SVMC_DEV double act_fn<double>(int act, double x) {
  return act == ACT_TANH ? tanh(x) : x / (1.0 + exp(-x));
}

// ---------------------------------------------------------------------------
// MFMA step per precision
// ---------------------------------------------------------------------------
SVMC_DEV void mfma(v4d& c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
SVMC_DEV void mfma(v4f& c, float a, float b) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
SVMC_DEV void mfma(v4f& c, v8h a, v8h b) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
SVMC_DEV void mfma(v4f& c, v8bf a, v8bf b) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// FP16 pair of an FP32 value (round toward zero twice; see PREC_F16X2): hi and
// lo of two values packed per dword.
SVMC_DEV void pair_split2(float a, float b, unsigned& hi, unsigned& lo) {
  const v2h h = __builtin_bit_cast(v2h, __builtin_amdgcn_cvt_pkrtz(a, b));
  const v2h l = __builtin_bit_cast(v2h, __builtin_amdgcn_cvt_pkrtz(a - (float)h[0], b - (float)h[1]));
  hi = __builtin_bit_cast(unsigned, h);
  lo = __builtin_bit_cast(unsigned, l);
}
// hi + lo of one value (exact in FP32)
SVMC_DEV float pair_round(float x) {
  const v2h h = __builtin_bit_cast(v2h, __builtin_amdgcn_cvt_pkrtz(x, 0.0f));
  const float hf = (float)h[0];
  const v2h l = __builtin_bit_cast(v2h, __builtin_amdgcn_cvt_pkrtz(x - hf, 0.0f));
  return hf + (float)l[0];
}

// New feature of one layer: H_l = H_{l-1} + act(z), rounded to an FP16 pair
// in PREC_F16X2.  Every conv kernel forms its outputs here.
template <int P, class T> SVMC_DEV T layer_out(int act, T x, T z) {
  const T y = x + act_fn<T>(act, z);
  if constexpr (P == PREC_F16X2) return pair_round(y);
  return y;
}
// the same with the activation fixed at compile time (FP32 features)
template <int P, int A> SVMC_DEV float layer_out_c(float x, float z) {
  const float y = x + act_c<A>(z);
  if constexpr (P == PREC_F16X2) return pair_round(y);
  return y;
}
// Output of a site-wise layer: act(z), no residual, rounded to an FP16 pair
// in PREC_F16X2 like every other cached feature.
template <int P, class T> SVMC_DEV T mlp_out(int act, T z) {
  const T y = act_fn<T>(act, z);
  if constexpr (P == PREC_F16X2) return pair_round(y);
  return y;
}
template <int A> struct ActC {
  static constexpr int value = A;
};
template <int V> struct IntC {
  static constexpr int value = V;
};

// One K chunk of a 16-bit mode: the B fragments b[nt] (weights, the MFMA A
// operand) times this lane's 8 activations x (FP32, the B operand),
// accumulated into acc[nt].  Every conv kernel goes through here or through
// the same sequence on pre-split activations, so the arithmetic per output
// element is the same in all of them.
template <int P, int NT>
SVMC_DEV void mma_chunk16(v4f (&acc)[NT], const float (&x)[8], const typename PrecT<P>::Tb (&b)[NT]) {
  if constexpr (P == PREC_F16X2) {
    // x is an FP16 pair (hi + lo): the round-toward-zero conversions recover
    // both terms exactly
    v8h hi, lo;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      unsigned h, l;
      pair_split2(x[e], x[e + 1], h, l);
      const v2h h2 = __builtin_bit_cast(v2h, h), l2 = __builtin_bit_cast(v2h, l);
      hi[e] = h2[0]; hi[e + 1] = h2[1];
      lo[e] = l2[0]; lo[e + 1] = l2[1];
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) mfma(acc[nt], b[nt], hi);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) mfma(acc[nt], b[nt], lo);
  } else {
    v8bf a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (__bf16)x[e];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) mfma(acc[nt], b[nt], a);
    if constexpr (P == PREC_BF16X3) {
      // remainders: x - hi is exact in FP32, and so is (x - hi) - mid
      v8bf a2, a3;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float r1 = x[e] - (float)a[e];
        a2[e] = (__bf16)r1;
        a3[e] = (__bf16)(r1 - (float)a2[e]);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        mfma(acc[nt], b[nt], a2);
        mfma(acc[nt], b[nt], a3);
      }
    }
  }
}

// Output element held in accumulator slot v of `lane` for the 16x16 MFMA
// tiles used here, with the weights as the A operand (rows = output channels)
// and the activations as the B operand (columns = sites); measured on gfx950:
//   f32 16x16x4, bf16 / f16 16x16x32: channel = 4*(lane/16) + v, site = lane%16
//   f64 16x16x4:                      channel = lane/16 + 4*v,  site = lane%16
// Inputs: A[i][k] from lane i + 16*(k/kpl) (kpl = k-values per lane),
// B[k][j] from lane j + 16*(k/kpl).
template <int P> struct OutMap {
  SVMC_DEV static int site(int lane, int v) { return lane & 15; }
  SVMC_DEV static int chan(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct OutMap<PREC_F64> {
  SVMC_DEV static int site(int lane, int v) { return lane & 15; }
  SVMC_DEV static int chan(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// ---------------------------------------------------------------------------
// conv tile: 16 output sites x C output channels of
//   acc[site][n] = sum_{tap t, c} X(site, t)[c] * K[t][c][n]
// Lane l supplies site (l % 16), a column of the B operand; the weights are
// the A operand, so acc[nt] holds acc[site][16 nt + channel] transposed (see
// OutMap).  nb[t] is the element offset
// (into `src`) of the C-channel feature vector of this lane's site's
// neighbour at tap t (t = 3*ky + kx, offset (kx-1, ky-1)), or -1 for zero
// padding.  The arithmetic per output element depends only on that element's
// own inputs, in a fixed order, so every caller (full forward or incremental
// box) produces identical values for identical inputs.
// ---------------------------------------------------------------------------
template <int P, int C>
SVMC_DEV void conv_tile(const typename PrecT<P>::Tf* __restrict__ src, const int (&nb)[9],
                        const typename PrecT<P>::Tb* __restrict__ Bl,   // layer's packed B
                        int lane, typename PrecT<P>::Acc (&acc)[ConvCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef ConvCfg<P, C> CC;
  const int g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[nt][v] = 0;
#pragma unroll
  for (int q = 0; q < CC::Q; ++q) {
    if constexpr (Mma16<P>::value) {
      const int k0 = 32 * q + 8 * g;
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      if (k0 < CC::K) {
        const int t = k0 / C, c0 = k0 % C;
        int off = nb[0];
#pragma unroll
        for (int tt = 1; tt < 9; ++tt) off = (t == tt) ? nb[tt] : off;
        if (off >= 0) {
          const float4* p4 = reinterpret_cast<const float4*>(src + off + c0);
          const float4 x0 = p4[0], x1 = p4[1];
          x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
          x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
        }
      }
      typename PrecT<P>::Tb b[CC::NT];
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) b[nt] = Bl[(q * CC::NT + nt) * 64 + lane];
      mma_chunk16<P, CC::NT>(acc, x, b);
    } else {
      // K chunk of 4: all four k of the chunk lie in one tap (C % 4 == 0)
      const int t = (4 * q) / C;
      const int c = (4 * q) % C + g;
      const int off = nb[t];
      Tf a = off >= 0 ? src[off + c] : Tf(0);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt)
        mfma(acc[nt], Bl[(q * CC::NT + nt) * 64 + lane], a);
    }
  }
}

// The same tile with the layer's weight fragments already in registers
// (breg[q][nt] = Bl[(q NT + nt) 64 + lane]); identical arithmetic.
template <int P, int C>
SVMC_DEV void conv_tile_regb(const typename PrecT<P>::Tf* __restrict__ src, const int (&nb)[9],
                             const typename PrecT<P>::Tb (&breg)[ConvCfg<P, C>::Q][ConvCfg<P, C>::NT], int lane,
                             typename PrecT<P>::Acc (&acc)[ConvCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef ConvCfg<P, C> CC;
  const int g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < CC::NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[nt][v] = 0;
#pragma unroll
  for (int q = 0; q < CC::Q; ++q) {
    if constexpr (Mma16<P>::value) {
      const int k0 = 32 * q + 8 * g;
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      if (k0 < CC::K) {
        const int t = k0 / C, c0 = k0 % C;
        int off = nb[0];
#pragma unroll
        for (int tt = 1; tt < 9; ++tt) off = (t == tt) ? nb[tt] : off;
        if (off >= 0) {
          const float4* p4 = reinterpret_cast<const float4*>(src + off + c0);
          const float4 x0 = p4[0], x1 = p4[1];
          x[0] = x0.x; x[1] = x0.y; x[2] = x0.z; x[3] = x0.w;
          x[4] = x1.x; x[5] = x1.y; x[6] = x1.z; x[7] = x1.w;
        }
      }
      mma_chunk16<P, CC::NT>(acc, x, breg[q]);
    } else {
      const int t = (4 * q) / C;
      const int c = (4 * q) % C + g;
      const int off = nb[t];
      Tf a = off >= 0 ? src[off + c] : Tf(0);
#pragma unroll
      for (int nt = 0; nt < CC::NT; ++nt) mfma(acc[nt], breg[q][nt], a);
    }
  }
}

// ---------------------------------------------------------------------------
// Site-wise layer tile (Sec. II.B, site-wise MLP equation): 16 sites x C
// outputs of acc[site][n] = sum_c x_site[c] W[c][n], weights as the A operand
// as in the conv tiles (OutMap gives the result layout).  x: this lane's
// site's C features in memory (FP32 / FP64 values; FP16 pairs in F16X2), or
// nullptr for a padding row.  Bm: the layer's packed B fragments
// [chunk q][out-tile nt][lane].  The chunk order is that of the conv tiles,
// so every kernel that evaluates a site-wise layer (forward over all sites,
// incremental update on a box) gives identical values for identical inputs.
// ---------------------------------------------------------------------------
template <int P, int C>
SVMC_DEV void mlp_tile(const typename PrecT<P>::Tf* x, const typename PrecT<P>::Tb* __restrict__ Bm, int lane,
                       typename PrecT<P>::Acc (&acc)[MlpCfg<P, C>::NT]) {
  typedef typename PrecT<P>::Tf Tf;
  typedef MlpCfg<P, C> MC;
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
    if constexpr (Mma16<P>::value) {
      const int k0 = 32 * q + 8 * g;
      float xv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xv[e] = 0.0f;
      if (x && k0 < C) {
        const float4* p4 = reinterpret_cast<const float4*>(x + k0);
        const float4 x0 = p4[0], x1 = p4[1];
        xv[0] = x0.x; xv[1] = x0.y; xv[2] = x0.z; xv[3] = x0.w;
        xv[4] = x1.x; xv[5] = x1.y; xv[6] = x1.z; xv[7] = x1.w;
      }
      mma_chunk16<P, MC::NT>(acc, xv, b);
    } else {
      const Tf a = x ? x[4 * q + g] : Tf(0);
#pragma unroll
      for (int nt = 0; nt < MC::NT; ++nt) mfma(acc[nt], b[nt], a);
    }
  }
}

// ---------------------------------------------------------------------------
// One-wave LU determinant of an r x r FP64 matrix, r <= RMAX <= 64.
// Lane a (< r) holds row a in a[0..RMAX); lanes >= r must hold identity rows.
// Partial pivoting without moving data: at step p the not-yet-used row with
// the largest |a[p]| is the pivot; det = sign(permutation) * prod(pivots).
// Returns 0 when a pivot column is exactly zero.
// ---------------------------------------------------------------------------
template <int RMAX>
SVMC_DEV double lu_det_rows(double (&a)[RMAX], int r, int lane) {
  bool used = lane >= r;
  int step = 64;
  double det = 1.0;
  bool zero = false;
#pragma unroll
  for (int p = 0; p < RMAX; ++p) {
    if (p < r && !zero) {
      double v = used ? -1.0 : fabs(a[p]);
      int li = lane;
      for (int o = 32; o >= 1; o >>= 1) {
        double v2 = __shfl_xor(v, o, 64);
        int l2 = __shfl_xor(li, o, 64);
        if (v2 > v || (v2 == v && l2 < li)) { v = v2; li = l2; }
      }
      const int piv = uniform_i(li);
      const double pv = readlane_d(a[p], piv);
      if (pv == 0.0) {
        zero = true;
      } else {
        det *= pv;
        if (lane == piv) { used = true; step = p; }
        const double inv = 1.0 / pv;
        const double l = used ? 0.0 : a[p] * inv;
#pragma unroll
        for (int c = p + 1; c < RMAX; ++c) {
          const double pr = readlane_d(a[c], piv);
          a[c] = fma(-l, pr, a[c]);
        }
      }
    }
  }
  if (zero) return 0.0;
  // parity of the pivot order: inversions among lanes < r
  int inv = 0;
  for (int b = 0; b < r; ++b) {
    int sb = __builtin_amdgcn_readlane(step, b);
    if (lane < r && b > lane && sb < step) ++inv;
  }
  inv = wave_sum_i(inv);
  return (inv & 1) ? -det : det;
}
