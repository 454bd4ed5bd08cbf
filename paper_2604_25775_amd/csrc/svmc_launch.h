// Host-side launchers of the scalevmc kernels (implemented in the .hip files,
// called from api.cpp).  All are asynchronous on `st`.
#pragma once
#include <hip/hip_runtime.h>
#include "svmc_dev.h"

// Supported (precision, channels) pairs of the templated conv kernels.
#define SVMC_FOR_EACH_PREC_C(X) \
  X(PREC_F64, 8) X(PREC_F64, 16) X(PREC_F64, 24) X(PREC_F64, 32) \
  X(PREC_F32, 8) X(PREC_F32, 16) X(PREC_F32, 24) X(PREC_F32, 32) \
  X(PREC_BF16, 8) X(PREC_BF16, 16) X(PREC_BF16, 24) X(PREC_BF16, 32) \
  X(PREC_BF16X3, 8) X(PREC_BF16X3, 16) X(PREC_BF16X3, 24) X(PREC_BF16X3, 32) \
  X(PREC_F16X2, 8) X(PREC_F16X2, 16) X(PREC_F16X2, 24) X(PREC_F16X2, 32)

namespace svmc {

// setup.hip
hipError_t launch_labels(const LatDev& lt, const Bufs& bf, hipStream_t st);
hipError_t launch_forward(int prec, const LatDev& lt, const Bufs& bf, const ModelDev& md, void* h0tmp,
                          hipStream_t st);
// Walkers a refresh launch works on: all walkers of the lattice (list null),
// or the global walker indices list[0 .. *count) that belong to it.
struct WalkerSel {
  const int32_t* list;
  const int32_t* count;
};
// Walker of slot z: 0 = no more slots, 1 = walker wl (lattice-local), 2 = skip.
SVMC_DEV int pick_walker(const WalkerSel& s, const LatDev& lt, long long z, long long& wl) {
  if (s.list) {
    if (z >= *(const volatile int32_t*)s.count) return 0;
    const long long w = s.list[z];
    if (w < lt.w0 || w >= lt.w0 + lt.nw) return 2;
    wl = w - lt.w0;
    return 1;
  }
  if (z >= lt.nw) return 0;
  wl = z;
  return 1;
}
// Orbital rows from the last of the `planes` cached feature planes (conv
// layers, then site-wise layers).
hipError_t launch_rows(int prec, const LatDev& lt, const Bufs& bf, int planes, int C, hipStream_t st,
                       WalkerSel sel = WalkerSel{nullptr, nullptr});
hipError_t launch_gj(const LatDev& lt, const Bufs& bf, hipStream_t st, WalkerSel sel = WalkerSel{nullptr, nullptr});
hipError_t launch_gp(int prec, const LatDev& lt, const Bufs& bf, int planes, int C, hipStream_t st,
                     WalkerSel sel = WalkerSel{nullptr, nullptr});
hipError_t launch_logpsi(const LatDev& lt, const Bufs& bf, double* sign, double* logabs, hipStream_t st);

// sym.hip: copies of a batch under a symmetry group, and the symmetric
// amplitude and local energy from the copies' values
hipError_t launch_sym_expand(int N, int nG, const int32_t* perm, const int32_t* flip, long long W, const int8_t* in,
                             int8_t* out, hipStream_t st);
hipError_t launch_sym_combine(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const double* chi,
                              const Bufs& bf, const double* e, const double* sg, const double* la, double* eloc,
                              double* sign_out, double* logabs_out, double* wts, hipStream_t st);
hipError_t launch_sym_signs(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const Bufs& bf,
                            double* pi, hipStream_t st);
hipError_t launch_sym_draw(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const Bufs& bf,
                           unsigned long long seed, unsigned long long step, int32_t* move, double* u,
                           hipStream_t st);
hipError_t launch_sym_decide(const LatDev& lt, int nG, const int32_t* perm, const int32_t* flip, const double* chi,
                             const Bufs& bf, const int32_t* move, const double* ratio, const double* u, double* pi,
                             int32_t* acc, hipStream_t st);

// eloc.hip: low-rank local energies over all walkers of all lattices in one launch
struct ElocOut {
  double* eloc;
  int32_t* nhops;
  int32_t* code;
  double* ratio;
  int stride;       // row stride of code/ratio
  double* part;     // [W][slices] partial sums (scratch)
  int slices;       // workgroups per walker
  int row_form_max; // hops whose spins both change at most this many rows (0, 8 or 16) use the row form
};
size_t eloc_lowrank_smem(const LatDev* lats_host, int nlats, int prec, int L, int C, bool rows_only);
// Allocation-free local energies: the per-slice partial sums live in a fixed
// device array of kNoAllocPartials doubles (8 MiB) per device.
// noalloc_scratch_init looks its address up for device `dev` (which must be
// current) once; noalloc_scratch returns it (null before the lookup).
constexpr long long kNoAllocPartials = 1LL << 20;
hipError_t noalloc_scratch_init(int dev);
double* noalloc_scratch(int dev);
hipError_t launch_eloc_lowrank(int prec, const ModelDev& md, const LatDev* lats_dev, const LatDev* lats_host,
                               int nlats, long long W, const Bufs& bf, const ElocOut& out, hipStream_t st);

// sweep.hip: Metropolis sweeps, step-synchronous across walkers: per proposal
// index q one launch of the proposal kernel (all walkers) and one of the
// Woodbury update (walkers that accepted)
struct StepArgs {
  unsigned long long seed, step0;
  const unsigned long long* step0_dev;   // if non-null, step0 is read from here
  long long q;                           // proposal index of this step
  int n_sweeps;
  int64_t* n_accept;     // [W] incremented by accepted moves (may be null)
  char* stage;           // [W][stage_stride] accepted-move staging
  long long stage_stride;
  int32_t* acc_list;     // [W] walkers that accepted at this step
  int32_t* count;        // their number (zero on entry)
  int32_t* count_next;   // cleared for the next step
  int32_t* due_list;     // [W] walkers that reached refresh_every (batch refresh)
  int32_t* due_count;    // their number since the last batch refresh
  int32_t* urgent_list;  // [W] walkers to rebuild before their next proposal
  int32_t* urgent_count; // their number (cleared by the host sequence each step)
  int refresh_every;
  // symmetric sampling (sym.hip drives it): 0 = draw and decide in the
  // proposal kernel; 1 = the move of walker w is sym_move[w] ((i << 4) |
  // (spin << 3) | d, or -1 for none) and only its ratio is written to
  // sym_ratio[w]; 2 = the same move, accepted iff sym_acc[w] != 0
  int sym_mode = 0;
  const int32_t* sym_move = nullptr;
  double* sym_ratio = nullptr;
  const int32_t* sym_acc = nullptr;
};
struct StepSizes {
  size_t smem_propose, smem_update, stage_bytes;
};
StepSizes step_sizes(const LatDev* lats_host, int nlats, int prec, int L, int C);
hipError_t launch_sweep_step(int prec, const ModelDev& md, const LatDev* lats_dev, const LatDev* lats_host,
                             int nlats, long long W, const Bufs& bf, const StepArgs& sa, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, long long n, int32_t v, hipStream_t st);
hipError_t launch_drift(const LatDev& lt, const Bufs& bf, WalkerSel sel, hipStream_t st);
hipError_t launch_clear_nacc(const LatDev& lt, const Bufs& bf, WalkerSel sel, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, long long n, int64_t v, hipStream_t st);

// grad.hip: d log|psi| / d theta, one row per walker
struct GradArgs {
  int L, C, act, lds;     // lds: H_{l-1} of a walker in LDS (else hs)
  int M;                  // site-wise layers after the conv stack
  const double* K;        // [L][9][C][C] conv weights as the forward uses them
  const double* B;        // [L][C]
  const double* E;        // [4][C]
  const double* MW;       // [M][C][C] site-wise weights as the forward uses them
  const double* MB;       // [M][C]
  long long nparams, off_convw, off_convb, off_mlpw, off_mlpb;
  long long w_begin;      // first walker of the launch
  long long ncmax;        // per-walker scratch stride (max N * C)
  long long nsmax;        // sites of the largest lattice (neighbour table in LDS)
  double* rows;           // [cnt][nparams]
  double* dH;             // [cnt][ncmax]
  double* hs;             // [cnt][ncmax] when !lds
  double* dzs;            // [cnt][ncmax]
};
size_t grad_smem(long long ncmax, long long nsmax);   // 0 when H_{l-1} and the table do not fit in LDS
hipError_t launch_grad(int prec, const LatDev* lats_dev, int nlats, long long cnt, const Bufs& bf,
                       const GradArgs& ga, hipStream_t st);
hipError_t launch_grad_reduce(const double* rows, long long cnt, long long nparams, const double* vjp,
                              const int32_t* flags, double* out, int first, hipStream_t st);
// dst[i] = (float)src[i], i < n (round to nearest)
hipError_t launch_to_f32(const double* src, float* dst, long long n, hipStream_t st);

// full.hip: full-recompute comparison path, batched over configurations
// (each walker's own and its hop configurations) in chunks of `chunk`.
struct FullScratch {
  long long chunk;        // configurations per chunk
  int32_t* cnt;           // [W] hops per walker
  long long* off;         // [W + 1] configuration offsets
  int8_t* occ;            // [chunk][N]
  void* feat;             // [chunk][L][N][C] features (Tf)
  void* h0;               // [chunk][N][C] embedding (Tf)
  int32_t *cfg_w, *cfg_h; // [chunk] walker, hop index (-1: own configuration)
  double* cfg_jw;         // [chunk] JW sign of the hop
  double *ld, *sg;        // [chunk][2] log|det|, sign per spin (canonical)
  double* ref;            // [W][2] log|psi|, sign of each walker's own configuration
  // N_sigma > 128 (cold-setup kernels): labels, rows, inverses, flags
  int16_t *lab, *pos;
  double *M, *inv;
  int32_t *flags, *nacc;
};
// bytes of chunk storage per configuration
size_t full_config_bytes(const LatDev& lt, int L, int C, int tfb);
hipError_t launch_eloc_full(int prec, const ModelDev& md, const LatDev& lt, const Bufs& bf, const ElocOut& out,
                            double* ratio_tmp, int stride, const FullScratch& fs, hipStream_t st);

// Per-(precision, channels) instances; each is compiled in its own
// translation unit (the build defines SVMC_INST_P / SVMC_INST_C).
#define SVMC_DECL_INST(P_, C_)                                                                          \
  hipError_t eloc_lowrank_##P_##_##C_(const ModelDev& md, const LatDev* lats_dev, int nlats, long long W, \
                                      const Bufs& bf, const ElocOut& out, size_t smem, hipStream_t st);   \
  hipError_t forward_##P_##_##C_(const LatDev& lt, const Bufs& bf, const ModelDev& md, void* h0tmp,       \
                                 hipStream_t st);                                                         \
  hipError_t sweep_step_##P_##_##C_(const ModelDev& md, const LatDev* lats_dev, int nlats, long long W,   \
                                    const Bufs& bf, const StepArgs& sa, size_t smem_p, size_t smem_u,     \
                                    int upd_blocks, hipStream_t st);
SVMC_FOR_EACH_PREC_C(SVMC_DECL_INST)
#undef SVMC_DECL_INST

#define SVMC_CAT3_(a, b, c) a##b##_##c
#define SVMC_CAT3(a, b, c) SVMC_CAT3_(a, b, c)

}  // namespace svmc
