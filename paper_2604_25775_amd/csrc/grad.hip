// Gradient of log|psi| with respect to the network parameters (the amplitude
// of Sec. II.B; Sec. II.F optimises these parameters by gradients).
//
// Projection (per spin, Phi[k] = base[pos_k] + H_L[pos_k] W + b):
//   d log|det Phi| = tr(Phi^-1 dPhi), so
//     dW[c][m] = sum_k H_L[pos_k][c] Phi^-1[m][k],   db[m] = sum_k Phi^-1[m][k],
//     dH_L[pos_k] += (W Phi^-1)[:, k] = P[:, k]      (P is the low-rank precompute).
// Site-wise layers, m = M-1 .. 0, with H_{L+m+1} = act(z), z = H_{L+m} W_m + b_m
// (no residual), H_L the conv output (the projection then reads H_{L+M}):
//     dz = dH * act'(z),  dW_m[ci][co] = sum_s H_{L+m}[s][ci] dz[s][co],
//     db_m = sum_s dz[s],  dH_{L+m}[s] = W_m dz[s].
// Conv stack, l = L .. 1, with H_l = H_{l-1} + act(z_l), z_l = conv_l(H_{l-1}) + b_l:
//     dz = dH_l * act'(z_l)                 (z_l recomputed from the cached H_{l-1})
//     dK_l[t][ci][co] = sum_s dz[s][co] H_{l-1}[s + off_t][ci],   db_l = sum_s dz[s]
//     dH_{l-1}[s] = dH_l[s] + sum_t K_l[t] dz[s - off_t]          (transposed conv)
// Embedding: dE[o] = sum over sites with occupation o of dH_0 (one shared
// table), or dE_s[n_s] = dH_0[s] (per-site tables).
//
// All arithmetic in FP64 on the cached features (FP32 or FP64); the conv
// weights are the values the forward uses (rounded to its precision).  With
// BF16 conv inputs the rounding of the activations is not differentiated
// (its derivative is zero almost everywhere); the gradient is the one of the
// unrounded network at the same weights.
//
// One workgroup per walker: H_{l-1} of the walker lives in LDS when N C
// doubles fit (two workgroups per CU at 16x16, C = 32), else in a global
// scratch; dz and dH are global scratch (per walker 2 N C doubles, which do
// not stay in L2 with hundreds of walkers in flight: their re-reads bound the
// kernel); the site neighbours per tap are a table in LDS.  dW and the three products of
// each layer (z, dK, the transposed conv) run on the FP64 matrix cores
// (16 x 16 x 4 tiles); the sums over sites for db, db_l and dE are spread
// over the workgroup and combined in LDS.
#include "svmc_launch.h"

namespace svmc {

SVMC_DEV int grad_nbr(const LatDev& lt, int s, int dx, int dy) {
  int x = s % lt.Lx + dx, y = s / lt.Lx + dy;
  if (lt.pbc_x) x = imod(x, lt.Lx); else if (x < 0 || x >= lt.Lx) return -1;
  if (lt.pbc_y) y = imod(y, lt.Ly); else if (y < 0 || y >= lt.Ly) return -1;
  return x + lt.Lx * y;
}

SVMC_DEV double act_deriv(int act, double z) {
  if (act == ACT_TANH) {
    const double t = tanh(z);
    return 1.0 - t * t;
  }
  const double sg = 1.0 / (1.0 + exp(-z));
  return sg * (1.0 + z * (1.0 - sg));
}

template <class Tf>
__global__ __launch_bounds__(256) void k_grad(const LatDev* __restrict__ lats, int nlats, Bufs bf, GradArgs ga) {
  constexpr int NTH = 256;
  const long long w = ga.w_begin + blockIdx.x;
  int li = 0;
  while (li + 1 < nlats && w >= lats[li + 1].w0) ++li;
  const LatDev lt = lats[li];
  const long long wl = w - lt.w0;
  const int N = lt.N, nm = lt.nmax, C = ga.C, L = ga.L, NC = N * C;
  const int tid = threadIdx.x;
  double* row = ga.rows + (long long)blockIdx.x * ga.nparams;
  extern __shared__ __attribute__((aligned(16))) double glds[];
  __shared__ double gred[4 * NTH];   // partial sums of the reductions below
  double* hp = ga.lds ? glds : ga.hs + (long long)blockIdx.x * ga.ncmax;
  double* dz = ga.dzs + (long long)blockIdx.x * ga.ncmax;
  double* dH = ga.dH + (long long)blockIdx.x * ga.ncmax;
  // neighbour of site s at tap t (offset (t % 3 - 1, t / 3 - 1)), -1 off an open edge
  int16_t* nbt = (int16_t*)(ga.lds ? glds + ga.ncmax : glds);
  const bool bad = (bf.flags[w] & (1 | 2 | 8)) != 0;
  for (long long p = tid; p < ga.nparams; p += NTH) row[p] = bad ? NAN : 0.0;
  if (bad) return;
  const int8_t* occ = bf.occ + lt.occ_off + wl * N;
  const int16_t* lab = bf.lab + lt.lab_off + wl * 2LL * N;
  const int16_t* pos = bf.pos + lt.pos_off + wl * 2LL * nm;
  const Tf* feat = (const Tf*)bf.feat + lt.feat_off + wl * (long long)(L + ga.M) * NC;
  const Tf* HL = feat + (long long)(L + ga.M - 1) * NC;     // the projection's input
  const double* PTw = bf.PT + lt.pt_off + wl * 2LL * nm * C;
  const int n0 = lt.n[0], n1 = lt.n[1];
  for (int e = tid; e < 9 * N; e += NTH) {
    const int t = e / N, s = e - t * N;
    nbt[e] = (int16_t)grad_nbr(lt, s, t % 3 - 1, t / 3 - 1);
  }
  __syncthreads();

  // ---- projection and dH_L
  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp == 0 ? n0 : n1;
    const double* Y = bf.inv + lt.inv_off + wl * 2LL * nm * nm + (long long)sp * nm * nm;
    const int16_t* ps = pos + sp * nm;
    double* dW = row + lt.poff + (sp ? (long long)C * n0 : 0LL);
    double* db = row + lt.poff + (long long)C * (n0 + n1) + (sp ? n0 : 0);
    // dW[c][m] = sum_k H_L[pos_k][c] Y[m][k] on the FP64 matrix cores: tiles of
    // 16 channels x 16 orbitals, K over the electrons, four k-steps in flight
    {
      const int wave = tid >> 6, lane = tid & 63, lj = lane & 15, lk = lane >> 4;
      const int nrt = (C + 15) / 16, nmt = (n + 15) / 16;
      for (int tt = wave; tt < nrt * nmt; tt += NTH / 64) {
        const int tc = tt / nmt, tm = tt - tc * nmt;
        const int c = 16 * tc + lj, m = 16 * tm + lj;
        const double* Ym = Y + (long long)(m < n ? m : 0) * nm;
        v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < n; k0 += 16) {
          double a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + lk;
            a[u] = (k < n && c < C) ? (double)HL[(long long)ps[k] * C + c] : 0.0;
            b[u] = (k < n && m < n) ? Ym[k] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) mfma(acc, a[u], b[u]);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int co = 16 * tc + lk + 4 * v;
          if (co < C && m < n) dW[co * n + m] = acc[v];
        }
      }
    }
    // db[m] = sum_k Y[m][k]: each row summed in `parts` interleaved pieces
    if (n > 0) {
      const int parts = n < NTH ? NTH / n : 1;
      for (int m0 = 0; m0 < n; m0 += NTH) {
        const int m = m0 + tid % n, part = tid / n;
        double acc = 0.0;
        if (part < parts && m < n) {
          const double* Ym = Y + (long long)m * nm;
          for (int k = part; k < n; k += parts) acc += Ym[k];
        }
        gred[tid] = acc;
        __syncthreads();
        if (tid < n && m0 + tid < n) {
          double t = 0.0;
          for (int q = 0; q < parts; ++q) t += gred[q * n + tid];
          db[m0 + tid] = t;
        }
        __syncthreads();
      }
    }
  }
  for (int e = tid; e < NC; e += NTH) {
    const int s = e / C, c = e % C;
    double v = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
      const int k = lab[sp * N + s];
      if (k >= 0) v += PTw[((long long)sp * nm + k) * C + c];
    }
    dH[e] = v;
  }
  __syncthreads();

  // ---- site-wise layers, last first
  for (int m = ga.M - 1; m >= 0; --m) {
    const double* Wm = ga.MW + (long long)m * C * C;
    const double* bm = ga.MB + (long long)m * C;
    for (int e = tid; e < NC; e += NTH) hp[e] = (double)feat[(long long)(L - 1 + m) * NC + e];
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, lj = lane & 15, lk = lane >> 4;
    const int nct = (C + 15) / 16, ntr = (N + 15) / 16, ksc = C / 4;
    constexpr int GQ = 8;            // k-steps over the channels at most (C <= 32)
    // (1) z = H W + b, dz = dH * act'(z): tiles of 16 sites x 16 outputs
    for (int tt = wave; tt < ntr * nct; tt += NTH / 64) {
      const int ti = tt / nct, tj = tt - ti * nct;
      const int si = 16 * ti + lj, co = 16 * tj + lj;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      // input channel ksc * lk + u at k-step u (contiguous H runs, as in the conv)
      const double* hrow = hp + (si < N ? si : 0) * C + ksc * lk;
      double hv[GQ];
#pragma unroll
      for (int u = 0; u < GQ; ++u) hv[u] = hrow[u];
#pragma unroll
      for (int u = 0; u < GQ; ++u) {
        if (u >= ksc) break;                        // uniform
        const int ci = ksc * lk + u;
        const double a = si < N ? hv[u] : 0.0;
        const double b = co < C ? Wm[ci * C + co] : 0.0;
        mfma(acc, a, b);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = 16 * ti + lk + 4 * v;
        if (so < N && co < C) dz[so * C + co] = dH[so * C + co] * act_deriv(ga.act, acc[v] + bm[co]);
      }
    }
    __syncthreads();
    // (2) dW_m[ci][co] = sum_s H[s][ci] dz[s][co]: tiles of 16 inputs x 16 outputs, K over the sites
    double* dW = row + ga.off_mlpw + (long long)m * C * C;
    for (int tt = wave; tt < nct * nct; tt += NTH / 64) {
      const int tci = tt / nct, tco = tt - tci * nct;
      const int ci = 16 * tci + lj, co = 16 * tco + lj;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      for (int s0 = 0; s0 < N; s0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int sk = s0 + 4 * u + lk;
          a[u] = (sk < N && ci < C) ? hp[sk * C + ci] : 0.0;
          b[u] = (sk < N && co < C) ? dz[sk * C + co] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) mfma(acc, a[u], b[u]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cio = 16 * tci + lk + 4 * v;
        if (cio < C && co < C) dW[(long long)cio * C + co] = acc[v];
      }
    }
    {
      // db_m[co] = sum_s dz[s][co]
      const int parts = NTH / C, co = tid % C, part = tid / C;
      double acc = 0.0;
      for (int s = part; s < N; s += parts) acc += dz[s * C + co];
      gred[tid] = acc;
      __syncthreads();
      if (tid < C) {
        double t = 0.0;
        for (int q = 0; q < parts; ++q) t += gred[q * C + tid];
        row[ga.off_mlpb + (long long)m * C + tid] = t;
      }
    }
    // (3) dH[s][ci] = sum_co W_m[ci][co] dz[s][co]
    for (int tt = wave; tt < ntr * nct; tt += NTH / 64) {
      const int ti = tt / nct, tj = tt - ti * nct;
      const int si = 16 * ti + lj, ci = 16 * tj + lj;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      // k-step u takes channel ksc * lk + u in lane group lk, as in the
      // transposed conv: each lane's operands are contiguous runs
      const double* drow = dz + (si < N ? si : 0) * C + ksc * lk;
      const double* wrow = Wm + (ci < C ? ci : 0) * C + ksc * lk;
      double dv[GQ], wv[GQ];
#pragma unroll
      for (int u = 0; u < GQ; ++u) {
        dv[u] = drow[u];
        wv[u] = wrow[u];
      }
#pragma unroll
      for (int u = 0; u < GQ; ++u)
        if (u < ksc) mfma(acc, si < N ? dv[u] : 0.0, ci < C ? wv[u] : 0.0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = 16 * ti + lk + 4 * v;
        if (so < N && ci < C) dH[so * C + ci] = acc[v];
      }
    }
    __syncthreads();
  }

  // ---- conv stack, last layer first
  for (int l = L; l >= 1; --l) {
    const double* Kl = ga.K + (long long)(l - 1) * 9 * C * C;
    const double* bl = ga.B + (long long)(l - 1) * C;
    for (int e = tid; e < NC; e += NTH)
      hp[e] = l >= 2 ? (double)feat[(long long)(l - 2) * NC + e]
                     : ga.E[lt.emb_off + (long long)(e / C) * lt.emb_ss + occ[e / C] * C + e % C];
    __syncthreads();
    // The three products of the layer on the FP64 matrix cores (16 x 16 x 4
    // tiles; A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k, result
    // row l / 16 + 4 v, column l % 16 in slot v of lane l).  Tiles are dealt
    // to the wavefronts in the same order in (1) and (3), so the thread that
    // writes an element of dH is the one that reads it in the next layer.
    const int wave = tid >> 6, lane = tid & 63, lj = lane & 15, lk = lane >> 4;
    const int nct = (C + 15) / 16, ntr = (N + 15) / 16, ksc = C / 4;
    constexpr int GQ = 8;            // k-steps per tap at most (C <= 32)
    // (1) z = conv(H_{l-1}) + b, dz = dH * act'(z): tiles of 16 sites x 16 outputs
    for (int tt = wave; tt < ntr * nct; tt += NTH / 64) {
      const int ti = tt / nct, tj = tt - ti * nct;
      const int si = 16 * ti + lj, co = 16 * tj + lj;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      // operands of tap t + 1 are requested before the products of tap t
      double a[2][GQ], b[2][GQ];
      auto load = [&](int t, double (&aa)[GQ], double (&bb)[GQ]) {
        // k-step u takes input channel ksc * lk + u in lane group lk: the
        // H_{l-1} operands of a lane are a contiguous run (wide reads)
        const int nb = si < N ? nbt[t * N + si] : -1;
        const double* hrow = hp + (nb >= 0 ? nb : 0) * C + ksc * lk;
        const double* kt = Kl + (long long)t * C * C + co + ksc * lk * C;
        double hv[GQ];
#pragma unroll
        for (int u = 0; u < GQ; ++u) hv[u] = hrow[u];
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
          const bool ok = u < ksc;
          aa[u] = (ok && nb >= 0) ? hv[u] : 0.0;
          bb[u] = (ok && co < C) ? kt[u * C] : 0.0;
        }
      };
      load(0, a[0], b[0]);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        if (t + 1 < 9) load(t + 1, a[(t + 1) & 1], b[(t + 1) & 1]);
#pragma unroll
        for (int u = 0; u < GQ; ++u)
          if (u < ksc) mfma(acc, a[t & 1][u], b[t & 1][u]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = 16 * ti + lk + 4 * v;
        if (so < N && co < C) dz[so * C + co] = dH[so * C + co] * act_deriv(ga.act, acc[v] + bl[co]);
      }
    }
    __syncthreads();
    // (2) dK[t][ci][co] = sum_s H_{l-1}[nb(s, t)][ci] dz[s][co]: tiles of 16
    // inputs x 16 outputs, K over the sites.  A wavefront holds the tiles of
    // all taps of its group (every tap when there are at least as many tiles
    // as wavefronts), so each block of dz is read once per group rather than
    // once per tap; each tap's accumulator takes the same products in the
    // same order as in a loop over single taps.
    double* dK = row + ga.off_convw + (long long)(l - 1) * 9 * C * C;
    {
      const int ntl = nct * nct;
      const int tg = ntl >= NTH / 64 ? 1 : (NTH / 64) / ntl;      // tap groups per tile
      const int gs = (9 + tg - 1) / tg;                            // taps per group
      for (int it = wave; it < ntl * tg; it += NTH / 64) {
        const int r2 = it / tg, g = it - r2 * tg, tci = r2 / nct, tco = r2 - tci * nct;
        const int t0 = g * gs, t1 = min(9, t0 + gs);
        const int ci = 16 * tci + lj, co = 16 * tco + lj;
        v4d acc[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int s0 = 0; s0 < N; s0 += 16) {
          double b[4];                              // this block of dz, shared by the taps
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int sk = s0 + 4 * u + lk;
            b[u] = (sk < N && co < C) ? dz[sk * C + co] : 0.0;
          }
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            if (t < t0 || t >= t1) continue;      // uniform
            double a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int sk = s0 + 4 * u + lk;
              const int nb = sk < N ? nbt[t * N + sk] : -1;
              a[u] = (nb >= 0 && ci < C) ? hp[nb * C + ci] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) mfma(acc[t], a[u], b[u]);
          }
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          if (t < t0 || t >= t1) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int cio = 16 * tci + lk + 4 * v;
            if (cio < C && co < C) dK[((long long)t * C + cio) * C + co] = acc[t][v];
          }
        }
      }
    }
    {
      // db_l[co] = sum_s dz[s][co]: NTH / C interleaved pieces per channel
      const int parts = NTH / C, co = tid % C, part = tid / C;
      double acc = 0.0;
      for (int s = part; s < N; s += parts) acc += dz[s * C + co];
      gred[tid] = acc;
      __syncthreads();
      if (tid < C) {
        double t = 0.0;
        for (int q = 0; q < parts; ++q) t += gred[q * C + tid];
        row[ga.off_convb + (long long)(l - 1) * C + tid] = t;
      }
    }
    // (3) dH_{l-1}[s][ci] = dH_l[s][ci] + sum_t sum_co K[t][ci][co] dz[s - off_t][co]
    for (int tt = wave; tt < ntr * nct; tt += NTH / 64) {
      const int ti = tt / nct, tj = tt - ti * nct;
      const int si = 16 * ti + lj, ci = 16 * tj + lj;
      v4d acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = 16 * ti + lk + 4 * v;
        acc[v] = (so < N && ci < C) ? dH[so * C + ci] : 0.0;
      }
      double a[2][GQ], b[2][GQ];
      // k-step u takes channel ksc * lk + u in lane group lk: each lane's
      // channels are consecutive, so its operands of a tap are contiguous
      // runs (wide loads; the sum over channels in another order)
      auto load = [&](int t, double (&aa)[GQ], double (&bb)[GQ]) {
        const int src = si < N ? nbt[(8 - t) * N + si] : -1;      // tap 8 - t: the opposite offset
        const double* drow = dz + (src >= 0 ? src : 0) * C + ksc * lk;
        const double* kt = Kl + ((long long)t * C + (ci < C ? ci : 0)) * C + ksc * lk;
        double dv[GQ], kv[GQ];
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
          dv[u] = drow[u];
          kv[u] = kt[u];
        }
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
          const bool ok = u < ksc;
          aa[u] = (ok && src >= 0) ? dv[u] : 0.0;
          bb[u] = (ok && ci < C) ? kv[u] : 0.0;
        }
      };
      load(0, a[0], b[0]);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        if (t + 1 < 9) load(t + 1, a[(t + 1) & 1], b[(t + 1) & 1]);
#pragma unroll
        for (int u = 0; u < GQ; ++u)
          if (u < ksc) mfma(acc, a[t & 1][u], b[t & 1][u]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = 16 * ti + lk + 4 * v;
        if (so < N && ci < C) dH[so * C + ci] = acc[v];
      }
    }
    __syncthreads();
  }

  // ---- embedding
  if (lt.emb_ss) {
    // per-site tables: dE_s[o][c] = dH_0[s][c] for the site's own occupation o
    for (int e = tid; e < NC; e += NTH) {
      const int s = e / C, c = e - s * C;
      row[lt.emb_off + (long long)s * lt.emb_ss + occ[s] * C + c] = dH[e];
    }
  } else {
    // dE[o][c] = sum over sites with occupation o of dH_0[s][c]: NTH / C
    // interleaved pieces of the sites per channel, four bins each
    const int parts = NTH / C, c = tid % C, part = tid / C;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = part; s < N; s += parts) {
      const double v = dH[s * C + c];
      const int o = occ[s];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += (o == q) ? v : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) gred[q * NTH + tid] = acc[q];
    __syncthreads();
    if (tid < 4 * C) {
      const int o = tid / C, cc = tid % C;
      double t = 0.0;
      for (int q = 0; q < parts; ++q) t += gred[o * NTH + q * C + cc];
      row[tid] = t;
    }
  }
}

// out[p] (+)= sum_w vjp[w] rows[w][p] over the walkers of one chunk, walker
// order fixed; flagged walkers are skipped.
__global__ void k_grad_reduce(const double* __restrict__ rows, long long cnt, long long nparams,
                              const double* __restrict__ vjp, const int32_t* __restrict__ flags, double* out,
                              int first) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= nparams) return;
  double acc = first ? 0.0 : out[p];
  for (long long w = 0; w < cnt; ++w)
    if (!(flags[w] & (1 | 2 | 8))) acc = fma(vjp[w], rows[w * nparams + p], acc);
  out[p] = acc;
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)nb), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

size_t grad_tab_bytes(long long nsmax) { return (size_t)((9 * nsmax * 2 + 15) & ~15LL); }
size_t grad_smem(long long ncmax, long long nsmax) {
  // k_grad also holds 4 * 256 doubles of static LDS for its reductions
  const size_t b = (size_t)ncmax * sizeof(double) + grad_tab_bytes(nsmax);
  return b + 4 * 256 * sizeof(double) <= 160 * 1024 ? b : 0;
}

hipError_t launch_grad(int prec, const LatDev* lats_dev, int nlats, long long cnt, const Bufs& bf,
                       const GradArgs& ga, hipStream_t st) {
  if (cnt == 0) return hipSuccess;
  const size_t smem = ga.lds ? grad_smem(ga.ncmax, ga.nsmax) : grad_tab_bytes(ga.nsmax);
  if (prec == PREC_F64) {
    hipError_t e = hipFuncSetAttribute((const void*)k_grad<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad<double>, dim3((unsigned)cnt), dim3(256), smem, st, lats_dev, nlats, bf, ga);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_grad<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad<float>, dim3((unsigned)cnt), dim3(256), smem, st, lats_dev, nlats, bf, ga);
  }
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* rows, long long cnt, long long nparams, const double* vjp,
                              const int32_t* flags, double* out, int first, hipStream_t st) {
  const unsigned nb = (unsigned)((nparams + 255) / 256);
  hipLaunchKernelGGL(k_grad_reduce, dim3(nb), dim3(256), 0, st, rows, cnt, nparams, vjp, flags, out, first);
  return hipGetLastError();
}

}  // namespace svmc
