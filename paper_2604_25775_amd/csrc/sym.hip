// Symmetry-projected amplitudes (App. B, symmetrized wavefunction):
//   psi_sym(n) = sum over g of Pi(n, g) chi_g psi(g n),
// g a lattice symmetry (site permutation, optionally with the two spins
// exchanged) and U_g |n> = Pi(n, g) |g n> on Fock states (creation operators
// mapped site by site, then put back into canonical order: spin-up block
// first, ascending site).
//
// When every g commutes with the Hamiltonian, the local energy of psi_sym
// is a weighted mean of the copies' local energies:
//   E_sym(n) = <n|H P|psi> / <n|P|psi> = <n|P H|psi> / <n|P|psi>
//            = sum_g w_g E_loc(g n),   w_g = Pi(n, g) chi_g psi(g n) / psi_sym(n)
// (P = sum_g chi_g U_g^dagger), so the copies g n are ordinary walkers of
// the batch (walker k n_G + g holds g n_k) and their local energies come
// from the low-rank kernels.  Here: the expansion of a batch into its
// copies, and the combination (fermion signs, weights, log-sum-exp).
#include "hop.h"
#include "svmc_launch.h"

namespace svmc {

// occupation code of a site after g: the two spin bits exchanged under flip
SVMC_DEV int sym_code(int o, int flip) { return flip ? (((o & 1) << 1) | ((o >> 1) & 1)) : o; }

// out[(k n_G + g) N + perm_g[s]] = sym_code(in[k N + s]); grid (W, n_G)
static __global__ void k_sym_expand(int N, int nG, const int32_t* __restrict__ perm, const int32_t* __restrict__ flip,
                                    const int8_t* __restrict__ in, int8_t* __restrict__ out) {
  const long long k = blockIdx.x;
  const int g = blockIdx.y;
  const int8_t* o = in + k * N;
  int8_t* d = out + (k * nG + g) * (long long)N;
  const int32_t* p = perm + (long long)g * N;
  for (int s = threadIdx.x; s < N; s += blockDim.x) d[p[s]] = (int8_t)sym_code(o[s], flip[g]);
}

hipError_t launch_sym_expand(int N, int nG, const int32_t* perm, const int32_t* flip, long long W, const int8_t* in,
                             int8_t* out, hipStream_t st) {
  if (W == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_expand, dim3((unsigned)W, (unsigned)nG), dim3(256), 0, st, N, nG, perm, flip, in, out);
  return hipGetLastError();
}

// Pi(n, g) of copy g of symmetric walker k (256 threads; every thread gets
// the result) and whether copy g is the image of copy 0 (o0: copy 0's
// occupation).  Pi is the sign of sorting the mapped creation operators of
// n into canonical order: the inversions within each spin's list (sites
// s < s' of that spin with perm[s] > perm[s']) and, under flip, every
// (up, down) pair (the up block now follows the down block).
SVMC_DEV double sym_pi_of(const LatDev& lt, const int32_t* p, int fl, const int8_t* o0, const int8_t* og, int* red,
                          bool& image) {
  const int N = lt.N, tid = threadIdx.x;
  int inv = 0, mism = 0;
  for (int s = tid; s < N; s += 256) {
    const int o = o0[s], ps = p[s];
    mism |= og[ps] != sym_code(o, fl);
    for (int sp = 0; sp < 2; ++sp) {
      if (!((o >> sp) & 1)) continue;
      for (int s2 = s + 1; s2 < N; ++s2) inv += ((o0[s2] >> sp) & 1) && p[s2] < ps;
    }
  }
  inv = wave_sum_i(inv);
  mism = wave_sum_i(mism);
  if ((tid & 63) == 0) {
    red[tid >> 6] = inv;
    red[4 + (tid >> 6)] = mism;
  }
  __syncthreads();
  const int inversions = red[0] + red[1] + red[2] + red[3];
  image = (red[4] + red[5] + red[6] + red[7]) == 0;
  __syncthreads();
  const long long blocks = fl ? (long long)lt.n[0] * lt.n[1] : 0;
  return ((inversions + blocks) & 1) ? -1.0 : 1.0;
}

// One workgroup per symmetric walker k (copies w = k n_G + g of the batch,
// copy 0 = n itself).  e, sg, la: the copies' local energies, signs and
// log|psi|.  Outputs E_sym, sign and log|psi_sym| of walker k; a walker
// whose copies are not the images of copy 0, or holds a wrong electron
// count, gets NaN and flag 16 on copy 0.
static __global__ __launch_bounds__(256) void k_sym_combine(LatDev lt, int nG, const int32_t* __restrict__ perm,
                                                            const int32_t* __restrict__ flip,
                                                            const double* __restrict__ chi, Bufs bf,
                                                            const double* __restrict__ e,
                                                            const double* __restrict__ sg,
                                                            const double* __restrict__ la, double* eloc,
                                                            double* sign_out, double* logabs_out, double* wts) {
  const long long k = blockIdx.x;
  const int N = lt.N, tid = threadIdx.x;
  const long long w0 = lt.w0 + k * nG;               // global index of copy 0
  const int8_t* o0 = bf.occ + lt.occ_off + k * nG * (long long)N;
  __shared__ int red[8];
  // thread 0's running sums: weights and weights * E, both scaled by
  // exp(-lmax), lmax the largest log|psi(g n)| over the copies with psi != 0
  double lmax = -INFINITY, acc_w = 0.0, acc_e = 0.0;
  bool bad = false;
  if (tid == 0)
    for (int g = 0; g < nG; ++g)
      if (sg[w0 + g] != 0.0) lmax = fmax(lmax, la[w0 + g]);
  for (int g = 0; g < nG; ++g) {
    bool image;
    const double pi = sym_pi_of(lt, perm + (long long)g * N, flip[g], o0, o0 + (long long)g * N, red, image);
    if (tid == 0) {
      bad |= !image || (bf.flags[w0 + g] & 8) != 0;
      const double s = sg[w0 + g];
      double a = 0.0;
      if (s != 0.0) {
        a = pi * chi[g] * s * exp(la[w0 + g] - lmax);
        acc_w += a;
        acc_e += a * e[w0 + g];
      }
      if (wts) wts[w0 + g] = a;
    }
  }
  if (tid == 0) {
    const double tot = acc_w;
    if (bad) atomicOr(bf.flags + w0, 16);
    eloc[k] = (bad || tot == 0.0) ? NAN : acc_e / tot;
    if (sign_out) sign_out[k] = bad ? NAN : (tot > 0.0 ? 1.0 : (tot < 0.0 ? -1.0 : 0.0));
    if (logabs_out) logabs_out[k] = bad ? NAN : (tot == 0.0 ? -INFINITY : lmax + log(fabs(tot)));
    // w_g = Pi chi psi(g n) / psi_sym(n): d log|psi_sym| = sum_g w_g d log|psi(g n)|
    if (wts)
      for (int g = 0; g < nG; ++g) wts[w0 + g] = (bad || tot == 0.0) ? NAN : wts[w0 + g] / tot;
  }
}

// ---------------------------------------------------------------------------
// Symmetric sampling of |psi_sym|^2.  Per proposal step: k_sym_draw draws
// the move of each symmetric walker (the Philox block of the ordinary
// sampler, counter (k, step)) and maps it to every copy; the proposal
// kernel computes each copy's in-place ratio R_g of its mapped move
// (ratio-only pass); k_sym_decide forms
//   psi_sym(n') / psi_sym(n) = jw_n(h) sum_g a_g R_g / sum_g a_g,
//   a_g = Pi(n, g) chi_g psi(g n),
// (because Pi(n', g) = Pi(n, g) jw_n(h) jw_gn(g h)), accepts iff
// u < ratio^2; the proposal kernel then commits the accepted copies.
// The sampler keeps each copy's determinants in label order (labels stay
// with their electrons), whose sign is psi's canonical sign times the
// parity par_g of the labels' site order, so the factor kept per copy is
// Q_g = Pi(n, g) par_g: then a_g = Q_g chi_g (label-order psi(g n)), and
// along an accepted hop par_g changes by jw_gn(g h), so Q_g changes by
// jw_n(h) alone.  k_sym_signs computes Q_g at the start.
// ---------------------------------------------------------------------------
static __global__ __launch_bounds__(256) void k_sym_signs(LatDev lt, int nG, const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ flip, Bufs bf, double* q) {
  const long long k = blockIdx.x;
  const int N = lt.N, nm = lt.nmax, tid = threadIdx.x;
  const long long w0 = lt.w0 + k * nG;
  const int8_t* o0 = bf.occ + lt.occ_off + k * nG * (long long)N;
  __shared__ int red[8];
  for (int g = 0; g < nG; ++g) {
    bool image;
    const double v = sym_pi_of(lt, perm + (long long)g * N, flip[g], o0, o0 + (long long)g * N, red, image);
    // parity of the labels' site order: label pairs a < b with pos[a] > pos[b]
    const int16_t* pos = bf.pos + lt.pos_off + (w0 - lt.w0 + g) * 2LL * nm;
    int inv = 0;
    for (int sp = 0; sp < 2; ++sp) {
      const int n = lt.n[sp];
      for (int a = tid; a < n; a += 256)
        for (int b = a + 1; b < n; ++b) inv += pos[sp * nm + a] > pos[sp * nm + b];
    }
    inv = wave_sum_i(inv);
    if ((tid & 63) == 0) red[tid >> 6] = inv;
    __syncthreads();
    if (tid == 0) {
      q[w0 + g] = ((red[0] + red[1] + red[2] + red[3]) & 1) ? -v : v;
      if (!image) atomicOr(bf.flags + w0, 16);
    }
    __syncthreads();
  }
}

// one thread per symmetric walker
static __global__ void k_sym_draw(LatDev lt, int nG, const int32_t* __restrict__ perm,
                                  const int32_t* __restrict__ flip, Bufs bf, unsigned long long seed,
                                  unsigned long long step, int32_t* move, double* u_out) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= lt.nw / nG) return;
  const int N = lt.N, nm = lt.nmax, n_up = lt.n[0], ne = lt.n[0] + lt.n[1];
  const long long w0 = lt.w0 + k * nG;
  int32_t* mv = move + w0;
  bool ok = ne > 0 && !(bf.flags[w0] & (1 | 2 | 8 | 16));
  int sp = 0, i = 0, j = -1;
  if (ok) {
    unsigned long long ctr[4] = {(unsigned long long)k, step, 0ULL, 0ULL};
    philox4x64_10(ctr, seed, 0ULL);
    const int e = (int)__umul64hi(ctr[0], (unsigned long long)ne);
    const int d = (int)(ctr[1] >> 62);
    u_out[k] = (double)(ctr[2] >> 11) * 0x1.0p-53;
    sp = e < n_up ? 0 : 1;
    const int lab = sp == 0 ? e : e - n_up;
    const int8_t* o0 = bf.occ + lt.occ_off + (w0 - lt.w0) * N;
    i = bf.pos[lt.pos_off + (w0 - lt.w0) * 2LL * nm + sp * nm + lab];
    j = conn_target(lt, i, d);
    ok = j >= 0 && (lt.tj ? o0[j] == 0 : !((o0[j] >> sp) & 1));
  }
  for (int g = 0; g < nG; ++g) {
    int code = -1;
    if (ok) {
      const int32_t* p = perm + (long long)g * N;
      const int ig = p[i], jg = p[j];
      for (int d2 = 0; d2 < 4; ++d2)
        if (conn_target(lt, ig, d2) == jg) code = (ig << 4) | ((sp ^ flip[g]) << 3) | d2;
    }
    mv[g] = code;
  }
}

// one 64-thread workgroup per symmetric walker; copies g dealt to the lanes
static __global__ __launch_bounds__(64) void k_sym_decide(LatDev lt, int nG, const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ flip,
                                                          const double* __restrict__ chi, Bufs bf,
                                                          const int32_t* __restrict__ move,
                                                          const double* __restrict__ ratio,
                                                          const double* __restrict__ u, double* pi, int32_t* acc) {
  const long long k = blockIdx.x;
  const int N = lt.N, lane = threadIdx.x;
  const long long w0 = lt.w0 + k * nG;
  if (move[w0] < 0) {
    for (int g = lane; g < nG; g += 64) acc[w0 + g] = 0;
    return;
  }
  // label-order log|psi| and sign of a copy, as the sampler keeps them
  auto logpsi = [&](long long w) { return bf.ld[2 * w] + bf.ld[2 * w + 1]; };
  auto sgn = [&](long long w) { return bf.sg[2 * w] * bf.sg[2 * w + 1]; };
  double lmax = -INFINITY;
  for (int g = lane; g < nG; g += 64)
    if (sgn(w0 + g) != 0.0) lmax = fmax(lmax, logpsi(w0 + g));
  for (int o = 32; o >= 1; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  double num = 0.0, den = 0.0;
  for (int g = lane; g < nG; g += 64) {
    const double s = sgn(w0 + g);
    if (s == 0.0) continue;
    const double a = pi[w0 + g] * chi[g] * s * exp(logpsi(w0 + g) - lmax);
    num += a * ratio[w0 + g];
    den += a;
  }
  num = wave_sum_d(num);
  den = wave_sum_d(den);
  const double r = den != 0.0 ? num / den : 0.0;
  const bool accept = u[k] < r * r;
  // Q_g changes by jw_n(h): electrons of the moving spin strictly between
  // the move's two sites in copy 0
  const int8_t* o0 = bf.occ + lt.occ_off + (w0 - lt.w0) * N;
  const int m0 = move[w0], i0 = m0 >> 4, sp0 = (m0 >> 3) & 1, j0 = conn_target(lt, i0, m0 & 7);
  int cnt = 0;
  for (int s = min(i0, j0) + 1 + lane; s < max(i0, j0); s += 64) cnt += (o0[s] >> sp0) & 1;
  cnt = wave_sum_i(cnt);
  for (int g = lane; g < nG; g += 64) {
    acc[w0 + g] = accept ? 1 : 0;
    if (accept && (cnt & 1)) pi[w0 + g] = -pi[w0 + g];
  }
}

hipError_t launch_sym_signs(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const Bufs& bf,
                            double* pi, hipStream_t st) {
  const long long K = lt.nw / nG;
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_signs, dim3((unsigned)K), dim3(256), 0, st, lt, nG, perm, flip, bf, pi);
  return hipGetLastError();
}

hipError_t launch_sym_draw(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const Bufs& bf,
                           unsigned long long seed, unsigned long long step, int32_t* move, double* u,
                           hipStream_t st) {
  const long long K = lt.nw / nG;
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_draw, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, lt, nG, perm, flip, bf, seed,
                     step, move, u);
  return hipGetLastError();
}

hipError_t launch_sym_decide(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const double* chi,
                             const Bufs& bf, const int32_t* move, const double* ratio, const double* u, double* pi,
                             int32_t* acc, hipStream_t st) {
  const long long K = lt.nw / nG;
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_decide, dim3((unsigned)K), dim3(64), 0, st, lt, nG, perm, flip, chi, bf, move, ratio, u,
                     pi, acc);
  return hipGetLastError();
}

hipError_t launch_sym_combine(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const double* chi,
                              const Bufs& bf, const double* e, const double* sg, const double* la, double* eloc,
                              double* sign_out, double* logabs_out, double* wts, hipStream_t st) {
  const long long K = lt.nw / nG;
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_combine, dim3((unsigned)K), dim3(256), 0, st, lt, nG, perm, flip, chi, bf, e, sg, la, eloc,
                     sign_out, logabs_out, wts);
  return hipGetLastError();
}

}  // namespace svmc
