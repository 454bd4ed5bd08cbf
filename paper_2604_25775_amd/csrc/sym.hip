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
                                                            double* sign_out, double* logabs_out) {
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
    const int32_t* p = perm + (long long)g * N;
    const int fl = flip[g];
    const int8_t* og = o0 + (long long)g * N;
    // copy g must be the image of copy 0; inversions of the mapped up and
    // down operator lists (pairs s < s' of one spin with perm[s] > perm[s'])
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
    if (tid == 0) {
      const int inversions = red[0] + red[1] + red[2] + red[3];
      bad |= (red[4] + red[5] + red[6] + red[7]) != 0 || (bf.flags[w0 + g] & 8) != 0;
      // under flip every (up, down) pair of the list is out of order
      const long long blocks = fl ? (long long)lt.n[0] * lt.n[1] : 0;
      const double pi = ((inversions + blocks) & 1) ? -1.0 : 1.0;
      const double s = sg[w0 + g];
      if (s != 0.0) {
        const double a = pi * chi[g] * s * exp(la[w0 + g] - lmax);
        acc_w += a;
        acc_e += a * e[w0 + g];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double tot = acc_w;
    if (bad) atomicOr(bf.flags + w0, 16);
    eloc[k] = (bad || tot == 0.0) ? NAN : acc_e / tot;
    if (sign_out) sign_out[k] = bad ? NAN : (tot > 0.0 ? 1.0 : (tot < 0.0 ? -1.0 : 0.0));
    if (logabs_out) logabs_out[k] = bad ? NAN : (tot == 0.0 ? -INFINITY : lmax + log(fabs(tot)));
  }
}

hipError_t launch_sym_combine(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const double* chi,
                              const Bufs& bf, const double* e, const double* sg, const double* la, double* eloc,
                              double* sign_out, double* logabs_out, hipStream_t st) {
  const long long K = lt.nw / nG;
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sym_combine, dim3((unsigned)K), dim3(256), 0, st, lt, nG, perm, flip, chi, bf, e, sg, la, eloc,
                     sign_out, logabs_out);
  return hipGetLastError();
}

}  // namespace svmc
