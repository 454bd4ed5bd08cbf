// Host side of the scalevmc C ABI: argument validation, parameter packing,
// device buffers and kernel sequencing.  Declarations and the contract of
// every entry point are in include/scalevmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "scalevmc.h"
#include "svmc_launch.h"

using namespace svmc;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) { p = nullptr; return e; }
    bytes = n;
    return hipSuccess;
  }
  template <class T> T* as() const { return (T*)p; }
};

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// x rounded toward zero to FP16 (the device's round-toward-zero conversion):
// 11 significant bits in FP16's normal range, multiples of 2^-24 below it,
// the largest finite FP16 value above it.  x finite.
float f16_rtz(float x) {
  const float a = std::fabs(x);
  float r;
  if (a >= 0x1p-14f) {
    uint32_t u;
    std::memcpy(&u, &a, 4);
    u &= 0xffffe000u;
    std::memcpy(&r, &u, 4);
    if (r > 65504.0f) r = 65504.0f;
  } else {
    r = std::trunc(a * 0x1p24f) * 0x1p-24f;
  }
  return std::copysign(r, x);
}
// FP16 pair value hi + lo of x (hi = f16_rtz(x), lo = f16_rtz(x - hi))
float f16_pair(float x) {
  const float h = f16_rtz(x);
  return h + f16_rtz(x - h);
}

}  // namespace

// Bound on the connected configurations of one walker: every electron hops
// in at most 4 (t' = 0) or 8 directions; in the t-J model every lone up
// electron also exchanges with at most 4 down neighbours.
static int lattice_max_hops(const svmc_lattice& l) {
  return (l.n_up + l.n_dn) * (l.tp != 0.0 ? 8 : 4) + (l.tj ? 4 * std::min(l.n_up, l.n_dn) : 0);
}

struct svmc_ctx {
  std::vector<svmc_lattice> lats;
  svmc_model model{};
  int prec = 0, L = 0, C = 0;
  int nmlp = 0;            // site-wise layers after the conv stack
  long long emb_len = 0;   // length of the embedding block of theta
  std::string err;
  int64_t nparams = 0;
  bool have_params = false, have_walkers = false;
  bool prepared = false;   // G/P match the current walkers
  bool dets_fresh = false; // rows M, inverses and log|psi| rebuilt since the last move
  int eloc_slices = 8;     // workgroups per walker in the low-rank E_loc launch
  int row_form_max = 16;   // row-form determinants when both spins change at most this many rows
  int dev = 0;             // device current at svmc_create
  // parameters
  DevBuf Bpack, Bmlp, embed, bias;
  std::vector<DevBuf> base, W, b;    // per lattice
  // walkers
  std::vector<LatDev> ld;            // host copies of the descriptors
  DevBuf lats_dev;
  long long Wtot = 0;
  DevBuf occ, lab, pos, feat, inv, M, G, PT, ldet, sgn, flags, nacc;
  DevBuf ratio_tmp, eloc_part;
  // full-recompute path: configuration chunks
  DevBuf f_cnt, f_off, f_occ, f_feat, f_h0, f_cw, f_ch, f_jw, f_ld, f_sg, f_ref, f_lab, f_pos, f_M, f_inv, f_flags,
      f_nacc;
  DevBuf sw_stage, sw_list, sw_count;  // sweep: accepted-move staging, accepted walkers, their counts
  DevBuf gK, gB, gE;                 // conv weights, conv bias, embedding (FP64, forward's rounding)
  DevBuf gMW, gMB;                   // site-wise weights and biases (FP64, forward's rounding)
  DevBuf g_rows, g_dH, g_hs, g_dzs, g_vjp;  // gradient scratch
  // symmetry projection: group (site permutations, spin flips, characters)
  // and the copies' local energies, signs and log|psi|
  int sym_n = 0;
  DevBuf sym_perm, sym_flip, sym_chi, sym_e, sym_s, sym_l;
  DevBuf sym_move, sym_ratio, sym_acc, sym_u, sym_pi;   // symmetric sampling
  std::vector<int64_t> counts;

  svmc_status fail(svmc_status s, const std::string& m) {
    err = m;
    return s;
  }
  svmc_status hip(hipError_t e, const char* where) {
    if (e == hipSuccess) return SVMC_OK;
    err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SVMC_ERR_OOM : SVMC_ERR_HIP;
  }
  int tf_bytes() const { return prec == PREC_F64 ? 8 : 4; }
  // feature planes cached per walker: conv layers, then site-wise layers
  int planes() const { return L + nmlp; }
  ModelDev mdev() const {
    ModelDev m;
    m.L = L;
    m.C = C;
    m.act = model.act;
    m.M = nmlp;
    m.Bpack = Bpack.p;
    m.Bmlp = Bmlp.p;
    m.embed = embed.p;
    m.bias = bias.p;
    return m;
  }
  Bufs bufs() const {
    Bufs x;
    x.occ = occ.as<int8_t>();
    x.lab = lab.as<int16_t>();
    x.pos = pos.as<int16_t>();
    x.feat = feat.p;
    x.inv = inv.as<double>();
    x.M = M.as<double>();
    x.G = G.as<double>();
    x.PT = PT.as<double>();
    x.ld = ldet.as<double>();
    x.sg = sgn.as<double>();
    x.flags = flags.as<int32_t>();
    x.nacc = nacc.as<int32_t>();
    return x;
  }
  int max_hops() const {
    int m = 0;
    for (auto& l : lats) m = std::max(m, lattice_max_hops(l));
    return m;
  }
  int max_elec() const {
    int m = 0;
    for (auto& l : lats) m = std::max(m, std::max(l.n_up, l.n_dn));
    return m;
  }
};

static svmc_status check_lattice(const svmc_lattice& l, std::string& why) {
  if (l.Lx < 1 || l.Ly < 1) { why = "lattice dimensions must be >= 1"; return SVMC_ERR_INVALID_ARG; }
  if ((l.pbc_x && l.Lx < 3) || (l.pbc_y && l.Ly < 3)) {
    why = "a periodic axis needs length >= 3";
    return SVMC_ERR_INVALID_ARG;
  }
  const long long N = (long long)l.Lx * l.Ly;
  if (N > 4096) { why = "more than 4096 sites"; return SVMC_ERR_UNSUPPORTED; }
  if (l.n_up < 0 || l.n_dn < 0 || l.n_up > N || l.n_dn > N) {
    why = "electron counts must lie in [0, N]";
    return SVMC_ERR_INVALID_ARG;
  }
  if (std::max(l.n_up, l.n_dn) > 512) { why = "more than 512 electrons per spin"; return SVMC_ERR_UNSUPPORTED; }
  if (!std::isfinite(l.t) || !std::isfinite(l.tp) || !std::isfinite(l.U) || !std::isfinite(l.J) ||
      !std::isfinite(l.h_pin)) {
    why = "non-finite Hamiltonian parameter";
    return SVMC_ERR_INVALID_ARG;
  }
  if (l.tj != 0 && l.tj != 1) { why = "tj must be 0 (Hubbard) or 1 (t-J)"; return SVMC_ERR_INVALID_ARG; }
  if (l.reserved != 0) { why = "svmc_lattice.reserved must be 0"; return SVMC_ERR_INVALID_ARG; }
  if (!l.tj && (l.J != 0.0 || l.h_pin != 0.0)) {
    why = "J and h_pin belong to the t-J model (tj = 1)";
    return SVMC_ERR_INVALID_ARG;
  }
  if (l.tj && N > 2048) { why = "t-J lattices hold at most 2048 sites"; return SVMC_ERR_UNSUPPORTED; }
  if (l.tj && l.n_up + l.n_dn > N) {
    why = "t-J: more electrons than sites (every site holds at most one)";
    return SVMC_ERR_INVALID_ARG;
  }
  return SVMC_OK;
}

extern "C" {

const char* svmc_status_string(svmc_status s) {
  switch (s) {
    case SVMC_OK: return "ok";
    case SVMC_ERR_INVALID_ARG: return "invalid argument";
    case SVMC_ERR_OOM: return "out of device memory";
    case SVMC_ERR_HIP: return "HIP runtime error";
    case SVMC_ERR_STATE: return "call out of order";
    case SVMC_ERR_UNSUPPORTED: return "unsupported shape";
  }
  return "unknown status";
}

const char* svmc_last_error(const svmc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

svmc_status svmc_create(const svmc_lattice* lats, int32_t n_lats, const svmc_model* m, svmc_ctx** out) {
  if (!out || !lats || !m || n_lats < 1 || n_lats > 8) return SVMC_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  for (int i = 0; i < n_lats; ++i) {
    svmc_status s = check_lattice(lats[i], why);
    if (s != SVMC_OK) return s;
  }
  if (m->n_conv < 1 || m->n_conv > 4) return SVMC_ERR_UNSUPPORTED;
  if (m->channels != 8 && m->channels != 16 && m->channels != 24 && m->channels != 32) return SVMC_ERR_UNSUPPORTED;
  if (m->act != SVMC_ACT_TANH && m->act != SVMC_ACT_SILU) return SVMC_ERR_INVALID_ARG;
  if (m->conv_prec < 0 || m->conv_prec > 4) return SVMC_ERR_INVALID_ARG;
  if (m->refresh_every < 1) return SVMC_ERR_INVALID_ARG;
  if (m->per_site_embed != 0 && m->per_site_embed != 1) return SVMC_ERR_INVALID_ARG;
  if (m->ksize != 3) return SVMC_ERR_UNSUPPORTED;
  if (m->n_mlp < 0) return SVMC_ERR_INVALID_ARG;
  if (m->n_mlp > 8) return SVMC_ERR_UNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SVMC_ERR_HIP;
  // address of this device's partial-sum array (allocation-free entry point)
  if (noalloc_scratch_init(dev) != hipSuccess) return SVMC_ERR_HIP;
  svmc_ctx* c = new svmc_ctx();
  c->dev = dev;
  c->lats.assign(lats, lats + n_lats);
  c->model = *m;
  c->prec = m->conv_prec;
  c->L = m->n_conv;
  c->C = m->channels;
  c->nmlp = m->n_mlp;
  c->emb_len = 4LL * c->C;
  if (m->per_site_embed) {
    c->emb_len = 0;
    for (auto& l : c->lats) c->emb_len += 4LL * l.Lx * l.Ly * c->C;
  }
  int64_t np = c->emb_len + 9LL * c->L * c->C * c->C + (int64_t)c->L * c->C +
               (int64_t)c->nmlp * (c->C * c->C + c->C);
  for (auto& l : c->lats) np += (int64_t)c->C * (l.n_up + l.n_dn) + l.n_up + l.n_dn;
  c->nparams = np;
  *out = c;
  return SVMC_OK;
}

svmc_status svmc_destroy(svmc_ctx* ctx) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  delete ctx;
  return SVMC_OK;
}

int64_t svmc_num_params(const svmc_ctx* ctx) { return ctx ? ctx->nparams : -1; }
int64_t svmc_num_walkers(const svmc_ctx* ctx) { return ctx ? ctx->Wtot : -1; }
int32_t svmc_max_hops(const svmc_ctx* ctx) { return ctx ? ctx->max_hops() : -1; }
int32_t svmc_max_electrons(const svmc_ctx* ctx) { return ctx ? ctx->max_elec() : -1; }

svmc_status svmc_set_params(svmc_ctx* ctx, const double* theta, const double* const* base, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!theta || !base) return ctx->fail(SVMC_ERR_INVALID_ARG, "null theta or base");
  for (size_t l = 0; l < ctx->lats.size(); ++l)
    if (!base[l]) return ctx->fail(SVMC_ERR_INVALID_ARG, "null base orbital pointer");
  const int L = ctx->L, C = ctx->C, P = ctx->prec;
  std::vector<double> th(ctx->nparams);
  svmc_status s;
  if ((s = ctx->hip(hipMemcpyAsync(th.data(), theta, th.size() * 8, hipMemcpyDeviceToHost, st), "theta copy")))
    return s;
  if ((s = ctx->hip(hipStreamSynchronize(st), "theta sync"))) return s;
  for (double v : th)
    if (!std::isfinite(v)) return ctx->fail(SVMC_ERR_INVALID_ARG, "non-finite parameter");
  const double* E = th.data();
  const long long EL = ctx->emb_len;
  const double* K = E + EL;
  const double* Bc = K + 9LL * L * C * C;
  const int NM = ctx->nmlp;
  const double* MW = Bc + (long long)L * C;           // site-wise weights [NM][C][C]
  const double* MB = MW + (long long)NM * C * C;      // site-wise biases [NM][C]
  const double* rest = MB + (long long)NM * C;
  // values the device uses: rnd for the embedding and conv bias (feature
  // type; BF16 in the BF16 modes), rnd_w for the conv weights (FP16 in F16X2)
  auto rnd = [&](double x) -> double {
    if (P == PREC_F64) return x;
    float f = (float)x;
    if (P == PREC_F32 || P == PREC_F16X2) return f;
    return bf16_to_f32(f32_to_bf16_rne(f));
  };
  auto rnd_w = [&](double x) -> double {
    if (P == PREC_F16X2) return (double)(float)(_Float16)(float)x;
    return rnd(x);
  };
  // the embedding is the layer-0 feature: an FP16 pair in F16X2
  auto rnd_e = [&](double x) -> double {
    if (P == PREC_F16X2) return (double)f16_pair((float)x);
    return rnd(x);
  };
  // embedding and conv bias in the feature type
  const int tfb = ctx->tf_bytes();
  std::vector<char> eb((size_t)EL * tfb), bb((size_t)(L + NM) * C * tfb);
  for (long long k = 0; k < EL; ++k) {
    if (tfb == 8) ((double*)eb.data())[k] = E[k];
    else ((float*)eb.data())[k] = (float)rnd_e(E[k]);
  }
  for (int k = 0; k < (L + NM) * C; ++k) {
    const double v = k < L * C ? Bc[k] : MB[k - L * C];
    if (tfb == 8) ((double*)bb.data())[k] = v;
    else ((float*)bb.data())[k] = (float)rnd(v);
  }
  // conv kernels as MFMA B fragments
  const bool bf = P == PREC_BF16 || P == PREC_BF16X3 || P == PREC_F16X2;
  const int KC = bf ? 32 : 4;
  const int Q = (9 * C + KC - 1) / KC, NT = (C + 15) / 16;
  const int per = bf ? 8 : 1;
  const size_t esz = P == PREC_F64 ? 8 : (P == PREC_F32 ? 4 : 2);
  std::vector<char> bp((size_t)L * Q * NT * 64 * per * esz, 0);
  for (int l = 0; l < L; ++l)
    for (int q = 0; q < Q; ++q)
      for (int nt = 0; nt < NT; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < per; ++e) {
            const int kap = bf ? 32 * q + 8 * (lane >> 4) + e : 4 * q + (lane >> 4);
            const int n = 16 * nt + (lane & 15);
            double v = 0.0;
            if (kap < 9 * C && n < C) {
              const int t = kap / C, c = kap % C;
              v = K[(((long long)l * 9 + t) * C + c) * C + n];
            }
            const size_t idx = ((((size_t)l * Q + q) * NT + nt) * 64 + lane) * per + e;
            if (P == PREC_F64) ((double*)bp.data())[idx] = v;
            else if (P == PREC_F32) ((float*)bp.data())[idx] = (float)v;
            else if (P == PREC_F16X2) ((_Float16*)bp.data())[idx] = (_Float16)(float)v;
            else ((uint16_t*)bp.data())[idx] = f32_to_bf16_rne((float)v);
          }
  // site-wise weights as B fragments of one tap: [m][q][nt][lane]
  const int QM = (C + KC - 1) / KC;
  std::vector<char> bpm((size_t)std::max(NM, 1) * QM * NT * 64 * per * esz, 0);
  for (int m = 0; m < NM; ++m)
    for (int q = 0; q < QM; ++q)
      for (int nt = 0; nt < NT; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < per; ++e) {
            const int kap = bf ? 32 * q + 8 * (lane >> 4) + e : 4 * q + (lane >> 4);
            const int n = 16 * nt + (lane & 15);
            const double v = (kap < C && n < C) ? MW[((long long)m * C + kap) * C + n] : 0.0;
            const size_t idx = ((((size_t)m * QM + q) * NT + nt) * 64 + lane) * per + e;
            if (P == PREC_F64) ((double*)bpm.data())[idx] = v;
            else if (P == PREC_F32) ((float*)bpm.data())[idx] = (float)v;
            else if (P == PREC_F16X2) ((_Float16*)bpm.data())[idx] = (_Float16)(float)v;
            else ((uint16_t*)bpm.data())[idx] = f32_to_bf16_rne((float)v);
          }
  // FP64 copies of what the forward uses, for the backward
  std::vector<double> gk(9ULL * L * C * C), gbias((size_t)L * C), ge((size_t)EL);
  std::vector<double> gmw((size_t)std::max(NM, 1) * C * C, 0.0), gmb((size_t)std::max(NM, 1) * C, 0.0);
  for (long long k = 0; k < (long long)NM * C * C; ++k) gmw[k] = rnd_w(MW[k]);
  for (long long k = 0; k < (long long)NM * C; ++k) gmb[k] = rnd(MB[k]);
  // (read by the gradient in runs of 8 doubles, like the conv weights: slack)
  if ((s = ctx->hip(ctx->gMW.ensure((gmw.size() + 8) * 8), "alloc")) ||
      (s = ctx->hip(ctx->gMB.ensure(gmb.size() * 8), "alloc")) ||
      (s = ctx->hip(hipMemcpy(ctx->gMW.p, gmw.data(), gmw.size() * 8, hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(hipMemcpy(ctx->gMB.p, gmb.data(), gmb.size() * 8, hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(ctx->Bmlp.ensure(bpm.size()), "alloc")) ||
      (s = ctx->hip(hipMemcpy(ctx->Bmlp.p, bpm.data(), bpm.size(), hipMemcpyHostToDevice), "upload")))
    return s;
  for (size_t k = 0; k < gk.size(); ++k) gk[k] = rnd_w(K[k]);
  for (size_t k = 0; k < gbias.size(); ++k) gbias[k] = rnd(Bc[k]);
  for (size_t k = 0; k < ge.size(); ++k) ge[k] = rnd_e(E[k]);
  // (the gradient reads the conv weights in runs of 8 doubles that may pass
  // the end of the array by up to 7 - C / 4 values, masked: 8 doubles of slack)
  if ((s = ctx->hip(ctx->gK.ensure((gk.size() + 8) * 8), "alloc")) ||
      (s = ctx->hip(ctx->gB.ensure(gbias.size() * 8), "alloc")) ||
      (s = ctx->hip(ctx->gE.ensure(ge.size() * 8), "alloc")) ||
      (s = ctx->hip(hipMemcpy(ctx->gK.p, gk.data(), gk.size() * 8, hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(hipMemcpy(ctx->gB.p, gbias.data(), gbias.size() * 8, hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(hipMemcpy(ctx->gE.p, ge.data(), ge.size() * 8, hipMemcpyHostToDevice), "upload")))
    return s;
  if ((s = ctx->hip(ctx->Bpack.ensure(bp.size()), "alloc")) || (s = ctx->hip(ctx->embed.ensure(eb.size()), "alloc")) ||
      (s = ctx->hip(ctx->bias.ensure(bb.size()), "alloc")))
    return s;
  if ((s = ctx->hip(hipMemcpy(ctx->Bpack.p, bp.data(), bp.size(), hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(hipMemcpy(ctx->embed.p, eb.data(), eb.size(), hipMemcpyHostToDevice), "upload")) ||
      (s = ctx->hip(hipMemcpy(ctx->bias.p, bb.data(), bb.size(), hipMemcpyHostToDevice), "upload")))
    return s;
  // per lattice: projection (padded to nmax columns) and base orbitals
  const size_t nl = ctx->lats.size();
  ctx->base.resize(nl);
  ctx->W.resize(nl);
  ctx->b.resize(nl);
  const double* cur = rest;
  for (size_t l = 0; l < nl; ++l) {
    const svmc_lattice& lt = ctx->lats[l];
    const int N = lt.Lx * lt.Ly, n0 = lt.n_up, n1 = lt.n_dn, nm = std::max(std::max(n0, n1), 1);
    std::vector<double> w(2LL * C * nm, 0.0), bv(2LL * nm, 0.0);
    for (int c = 0; c < C; ++c)
      for (int k = 0; k < n0; ++k) w[(size_t)c * nm + k] = cur[(size_t)c * n0 + k];
    cur += (size_t)C * n0;
    for (int c = 0; c < C; ++c)
      for (int k = 0; k < n1; ++k) w[(size_t)C * nm + (size_t)c * nm + k] = cur[(size_t)c * n1 + k];
    cur += (size_t)C * n1;
    for (int k = 0; k < n0; ++k) bv[k] = cur[k];
    cur += n0;
    for (int k = 0; k < n1; ++k) bv[nm + k] = cur[k];
    cur += n1;
    if ((s = ctx->hip(ctx->W[l].ensure(w.size() * 8), "alloc")) || (s = ctx->hip(ctx->b[l].ensure(bv.size() * 8), "alloc")) ||
        (s = ctx->hip(ctx->base[l].ensure(2ULL * N * nm * 8), "alloc")))
      return s;
    if ((s = ctx->hip(hipMemcpy(ctx->W[l].p, w.data(), w.size() * 8, hipMemcpyHostToDevice), "upload")) ||
        (s = ctx->hip(hipMemcpy(ctx->b[l].p, bv.data(), bv.size() * 8, hipMemcpyHostToDevice), "upload")) ||
        (s = ctx->hip(hipMemsetAsync(ctx->base[l].p, 0, 2ULL * N * nm * 8, st), "memset")))
      return s;
    if (n0 && (s = ctx->hip(hipMemcpy2DAsync(ctx->base[l].p, nm * 8, base[l], n0 * 8, n0 * 8, N,
                                             hipMemcpyDeviceToDevice, st), "base copy")))
      return s;
    if (n1 && (s = ctx->hip(hipMemcpy2DAsync((char*)ctx->base[l].p + (size_t)N * nm * 8, nm * 8,
                                             base[l] + (size_t)N * n0, n1 * 8, n1 * 8, N,
                                             hipMemcpyDeviceToDevice, st), "base copy")))
      return s;
  }
  ctx->have_params = true;
  ctx->have_walkers = false;
  return SVMC_OK;
}

// Rebuild orbital rows and inverses from the cached features (every lattice).
static svmc_status rebuild_dets(svmc_ctx* ctx, hipStream_t st) {
  const Bufs bf = ctx->bufs();
  svmc_status s;
  for (auto& lt : ctx->ld) {
    if ((s = ctx->hip(launch_rows(ctx->prec, lt, bf, ctx->planes(), ctx->C, st), "rows"))) return s;
    if ((s = ctx->hip(launch_gj(lt, bf, st), "inverse"))) return s;
  }
  ctx->prepared = false;
  ctx->dets_fresh = true;
  return SVMC_OK;
}

// Low-rank precompute: G = M Phi^-1 and P^T from the current features and
// inverses (inverses first rebuilt if moves made them stale); the rows M of
// every site are not formed (G = (base + b) Phi^-1 + H_L P).
static svmc_status prepare(svmc_ctx* ctx, hipStream_t st) {
  svmc_status s;
  if (!ctx->dets_fresh && (s = rebuild_dets(ctx, st))) return s;
  const Bufs bf = ctx->bufs();
  for (auto& lt : ctx->ld)
    if ((s = ctx->hip(launch_gp(ctx->prec, lt, bf, ctx->planes(), ctx->C, st), "G/P precompute"))) return s;
  ctx->prepared = true;
  return SVMC_OK;
}

svmc_status svmc_load_walkers(svmc_ctx* ctx, const int64_t* counts, const int8_t* occ, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_params) return ctx->fail(SVMC_ERR_STATE, "svmc_set_params must come first");
  if (!counts || !occ) return ctx->fail(SVMC_ERR_INVALID_ARG, "null counts or occ");
  const size_t nl = ctx->lats.size();
  long long Wt = 0;
  for (size_t l = 0; l < nl; ++l) {
    if (counts[l] < 0) return ctx->fail(SVMC_ERR_INVALID_ARG, "negative walker count");
    Wt += counts[l];
  }
  if (Wt < 1) return ctx->fail(SVMC_ERR_INVALID_ARG, "no walkers");
  const int L = ctx->L, C = ctx->C, tfb = ctx->tf_bytes();
  std::vector<LatDev> d(nl);
  long long w0 = 0, o_occ = 0, o_lab = 0, o_pos = 0, o_feat = 0, o_inv = 0, o_m = 0, o_pt = 0;
  long long poff = ctx->emb_len + 9LL * L * C * C + (long long)L * C + (long long)ctx->nmlp * (C * C + C);
  long long emb_off = 0;
  size_t h0max = 0;
  for (size_t l = 0; l < nl; ++l) {
    const svmc_lattice& s = ctx->lats[l];
    LatDev& x = d[l];
    x.Lx = s.Lx; x.Ly = s.Ly; x.pbc_x = s.pbc_x ? 1 : 0; x.pbc_y = s.pbc_y ? 1 : 0;
    x.N = s.Lx * s.Ly;
    x.n[0] = s.n_up; x.n[1] = s.n_dn;
    x.nmax = std::max(std::max(s.n_up, s.n_dn), 1);
    x.nd = s.tp != 0.0 ? 8 : 4;
    x.maxhops = lattice_max_hops(s);
    const int G = 2 * L + 4;
    x.torus_x = (x.pbc_x && s.Lx < G) ? 1 : 0;
    x.torus_y = (x.pbc_y && s.Ly < G) ? 1 : 0;
    x.Gx = x.torus_x ? s.Lx : G;
    x.Gy = x.torus_y ? s.Ly : G;
    x.t = s.t; x.tp = s.tp; x.U = s.U;
    x.tj = s.tj; x.J = s.J; x.hpin = s.h_pin;
    x.w0 = w0; x.nw = counts[l];
    x.occ_off = o_occ; x.lab_off = o_lab; x.pos_off = o_pos; x.feat_off = o_feat;
    x.inv_off = o_inv; x.m_off = o_m; x.g_off = o_m; x.pt_off = o_pt;
    x.base = ctx->base[l].as<double>();
    x.W = ctx->W[l].as<double>();
    x.b = ctx->b[l].as<double>();
    x.poff = poff;
    poff += (long long)C * (s.n_up + s.n_dn) + s.n_up + s.n_dn;
    x.emb_off = ctx->model.per_site_embed ? emb_off : 0;
    x.emb_ss = ctx->model.per_site_embed ? 4 * C : 0;
    emb_off += 4LL * x.N * C;
    const long long nw = counts[l], N = x.N, nm = x.nmax;
    w0 += nw;
    o_occ += nw * N;
    o_lab += nw * 2 * N;
    o_pos += nw * 2 * nm;
    o_feat += nw * (long long)ctx->planes() * N * C;
    o_inv += nw * 2 * nm * nm;
    o_m += nw * 2 * N * nm;
    o_pt += nw * 2 * nm * C;
    h0max = std::max(h0max, (size_t)(nw * N * C * tfb));
  }
  svmc_status s;
  ctx->have_walkers = false;
  if ((s = ctx->hip(ctx->occ.ensure(o_occ), "alloc occ")) || (s = ctx->hip(ctx->lab.ensure(o_lab * 2), "alloc")) ||
      (s = ctx->hip(ctx->pos.ensure(o_pos * 2), "alloc")) || (s = ctx->hip(ctx->feat.ensure(o_feat * tfb), "alloc feat")) ||
      (s = ctx->hip(ctx->inv.ensure(o_inv * 8), "alloc inv")) ||
      (s = ctx->hip(ctx->M.ensure(std::max((size_t)o_m * 8, h0max)), "alloc M")) ||
      (s = ctx->hip(ctx->G.ensure(o_m * 8), "alloc G")) || (s = ctx->hip(ctx->PT.ensure((o_pt + 8) * 8), "alloc PT")) ||   // slack: the update reads P^T rows in runs
      (s = ctx->hip(ctx->ldet.ensure(Wt * 16), "alloc")) || (s = ctx->hip(ctx->sgn.ensure(Wt * 16), "alloc")) ||
      (s = ctx->hip(ctx->flags.ensure(Wt * 4), "alloc")) || (s = ctx->hip(ctx->nacc.ensure(Wt * 4), "alloc")) ||
      (s = ctx->hip(ctx->lats_dev.ensure(nl * sizeof(LatDev)), "alloc")))
    return s;
  ctx->ld = d;
  ctx->Wtot = Wt;
  ctx->counts.assign(counts, counts + nl);
  if ((s = ctx->hip(hipMemcpyAsync(ctx->lats_dev.p, d.data(), nl * sizeof(LatDev), hipMemcpyHostToDevice, st),
                    "descriptors")))
    return s;
  if ((s = ctx->hip(hipMemcpyAsync(ctx->occ.p, occ, o_occ, hipMemcpyDeviceToDevice, st), "occ copy"))) return s;
  const Bufs bf = ctx->bufs();
  const ModelDev md = ctx->mdev();
  for (auto& lt : ctx->ld) {
    if ((s = ctx->hip(launch_labels(lt, bf, st), "labels"))) return s;
    if ((s = ctx->hip(launch_forward(ctx->prec, lt, bf, md, ctx->M.p, st), "forward"))) return s;
  }
  if ((s = rebuild_dets(ctx, st))) return s;
  // descriptor copy must finish before the host vector can change
  if ((s = ctx->hip(hipStreamSynchronize(st), "load sync"))) return s;
  ctx->have_walkers = true;
  return SVMC_OK;
}

svmc_status svmc_log_psi(svmc_ctx* ctx, double* sign, double* logabs, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!sign && !logabs) return ctx->fail(SVMC_ERR_INVALID_ARG, "no output");
  const Bufs bf = ctx->bufs();
  svmc_status s;
  for (auto& lt : ctx->ld)
    if ((s = ctx->hip(launch_logpsi(lt, bf, sign, logabs, st), "logpsi"))) return s;
  return SVMC_OK;
}

svmc_status svmc_prepare(svmc_ctx* ctx, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  return prepare(ctx, st);
}

svmc_status svmc_local_energy(svmc_ctx* ctx, svmc_path path, double* eloc, int32_t* n_hops, int32_t* hop_code,
                              double* ratio, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!eloc) return ctx->fail(SVMC_ERR_INVALID_ARG, "eloc is null");
  if ((hop_code == nullptr) != (ratio == nullptr))
    return ctx->fail(SVMC_ERR_INVALID_ARG, "hop_code and ratio must both be given or both be NULL");
  ElocOut out;
  out.eloc = eloc;
  out.nhops = n_hops;
  out.code = hop_code;
  out.ratio = ratio;
  out.stride = ctx->max_hops();
  out.part = nullptr;
  out.slices = 1;
  out.row_form_max = ctx->row_form_max;
  const Bufs bf = ctx->bufs();
  const ModelDev md = ctx->mdev();
  svmc_status s;
  if (path == SVMC_PATH_LOWRANK) {
    if (!ctx->prepared && (s = prepare(ctx, st))) return s;
    out.slices = ctx->eloc_slices;
    if ((s = ctx->hip(ctx->eloc_part.ensure((size_t)ctx->Wtot * out.slices * 8), "alloc"))) return s;
    out.part = ctx->eloc_part.as<double>();
    return ctx->hip(launch_eloc_lowrank(ctx->prec, md, ctx->lats_dev.as<LatDev>(), ctx->ld.data(),
                                        (int)ctx->ld.size(), ctx->Wtot, bf, out, st),
                    "low-rank local energy");
  }
  if (path != SVMC_PATH_FULL) return ctx->fail(SVMC_ERR_INVALID_ARG, "unknown path");
  const int stride = ctx->max_hops();
  if ((s = ctx->hip(ctx->ratio_tmp.ensure((size_t)ctx->Wtot * stride * 8), "alloc"))) return s;
  // chunk storage: configurations per chunk from a 2 GiB budget for the
  // largest lattice (at least one walker's worth of configurations)
  const int tfb = ctx->tf_bytes(), L = ctx->planes(), C = ctx->C;   // L: feature planes
  size_t per = 0;
  long long nmx = 1, Nmx = 1, wmx = 1;
  for (auto& lt : ctx->ld) {
    per = std::max(per, full_config_bytes(lt, L, C, tfb));
    nmx = std::max<long long>(nmx, lt.nmax);
    Nmx = std::max<long long>(Nmx, lt.N);
    wmx = std::max<long long>(wmx, lt.nw);
  }
  long long chunk = std::max<long long>((2LL << 30) / (long long)per, (long long)ctx->max_hops() + 1);
  chunk = std::min<long long>(chunk, 1LL << 20);
  FullScratch fs;
  fs.chunk = chunk;
  const bool big = nmx > 128;
  if ((s = ctx->hip(ctx->f_cnt.ensure((size_t)wmx * 4), "alloc")) ||
      (s = ctx->hip(ctx->f_off.ensure((size_t)(wmx + 1) * 8), "alloc")) ||
      (s = ctx->hip(ctx->f_occ.ensure((size_t)chunk * Nmx), "alloc")) ||
      (s = ctx->hip(ctx->f_feat.ensure((size_t)chunk * L * Nmx * C * tfb), "alloc")) ||
      (s = ctx->hip(ctx->f_h0.ensure((size_t)chunk * Nmx * C * tfb), "alloc")) ||
      (s = ctx->hip(ctx->f_cw.ensure((size_t)chunk * 4), "alloc")) ||
      (s = ctx->hip(ctx->f_ch.ensure((size_t)chunk * 4), "alloc")) ||
      (s = ctx->hip(ctx->f_jw.ensure((size_t)chunk * 8), "alloc")) ||
      (s = ctx->hip(ctx->f_ld.ensure((size_t)chunk * 16), "alloc")) ||
      (s = ctx->hip(ctx->f_sg.ensure((size_t)chunk * 16), "alloc")) ||
      (s = ctx->hip(ctx->f_ref.ensure((size_t)wmx * 16), "alloc")))
    return s;
  if (big && ((s = ctx->hip(ctx->f_lab.ensure((size_t)chunk * 2 * Nmx * 2), "alloc")) ||
              (s = ctx->hip(ctx->f_pos.ensure((size_t)chunk * 2 * nmx * 2), "alloc")) ||
              (s = ctx->hip(ctx->f_M.ensure((size_t)chunk * 2 * Nmx * nmx * 8), "alloc")) ||
              (s = ctx->hip(ctx->f_inv.ensure((size_t)chunk * 2 * nmx * nmx * 8), "alloc")) ||
              (s = ctx->hip(ctx->f_flags.ensure((size_t)chunk * 4), "alloc")) ||
              (s = ctx->hip(ctx->f_nacc.ensure((size_t)chunk * 4), "alloc"))))
    return s;
  fs.cnt = ctx->f_cnt.as<int32_t>();
  fs.off = ctx->f_off.as<long long>();
  fs.occ = ctx->f_occ.as<int8_t>();
  fs.feat = ctx->f_feat.p;
  fs.h0 = ctx->f_h0.p;
  fs.cfg_w = ctx->f_cw.as<int32_t>();
  fs.cfg_h = ctx->f_ch.as<int32_t>();
  fs.cfg_jw = ctx->f_jw.as<double>();
  fs.ld = ctx->f_ld.as<double>();
  fs.sg = ctx->f_sg.as<double>();
  fs.ref = ctx->f_ref.as<double>();
  fs.lab = ctx->f_lab.as<int16_t>();
  fs.pos = ctx->f_pos.as<int16_t>();
  fs.M = ctx->f_M.as<double>();
  fs.inv = ctx->f_inv.as<double>();
  fs.flags = ctx->f_flags.as<int32_t>();
  fs.nacc = ctx->f_nacc.as<int32_t>();
  for (auto& lt : ctx->ld)
    if ((s = ctx->hip(launch_eloc_full(ctx->prec, md, lt, bf, out, ctx->ratio_tmp.as<double>() + lt.w0 * stride,
                                       stride, fs, st),
                      "full-recompute local energy")))
      return s;
  return SVMC_OK;
}

svmc_status svmc_local_energy_noalloc(svmc_ctx* ctx, double* eloc, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!eloc) return ctx->fail(SVMC_ERR_INVALID_ARG, "eloc is null");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->dev)
    return ctx->fail(SVMC_ERR_INVALID_ARG, "the context's device must be current");
  double* part = noalloc_scratch(dev);
  if (!part) return ctx->fail(SVMC_ERR_STATE, "partial-sum array not set up on this device");
  if ((long long)ctx->Wtot * ctx->eloc_slices > kNoAllocPartials)
    return ctx->fail(SVMC_ERR_UNSUPPORTED, "walkers x slices exceeds the fixed partial-sum array (2^20 entries)");
  ElocOut out;
  out.eloc = eloc;
  out.nhops = nullptr;
  out.code = nullptr;
  out.ratio = nullptr;
  out.stride = ctx->max_hops();
  out.slices = ctx->eloc_slices;
  out.row_form_max = ctx->row_form_max;
  out.part = part;
  svmc_status s;
  if (!ctx->prepared && (s = prepare(ctx, st))) return s;
  return ctx->hip(launch_eloc_lowrank(ctx->prec, ctx->mdev(), ctx->lats_dev.as<LatDev>(), ctx->ld.data(),
                                      (int)ctx->ld.size(), ctx->Wtot, ctx->bufs(), out, st),
                  "low-rank local energy (no allocation)");
}

svmc_status svmc_refresh(svmc_ctx* ctx, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  const Bufs bf = ctx->bufs();
  svmc_status s;
  if (ctx->prepared)
    for (auto& lt : ctx->ld)
      if ((s = ctx->hip(launch_drift(lt, bf, WalkerSel{nullptr, nullptr}, st), "drift check"))) return s;
  if ((s = rebuild_dets(ctx, st))) return s;
  return prepare(ctx, st);
}

// Sweep workspace (allocated outside any capture) and the step loop shared by
// svmc_sweep and svmc_sweep_async.
static svmc_status sweep_workspace(svmc_ctx* ctx, bool capturing, StepSizes& z) {
  z = step_sizes(ctx->ld.data(), (int)ctx->ld.size(), ctx->prec, ctx->L, ctx->C);
  if (z.smem_propose > 160 * 1024 || z.smem_update > 160 * 1024)
    return ctx->fail(SVMC_ERR_UNSUPPORTED, "sweep workspace exceeds 160 KiB of LDS");
  const size_t stage = (size_t)ctx->Wtot * z.stage_bytes, list = (size_t)ctx->Wtot * 4;
  if (ctx->sw_stage.bytes < stage || ctx->sw_list.bytes < 3 * list || ctx->sw_count.bytes < 16) {
    if (capturing) return ctx->fail(SVMC_ERR_STATE, "call svmc_sweep_async once outside capture first (allocates)");
    svmc_status s;
    if ((s = ctx->hip(ctx->sw_stage.ensure(stage), "alloc")) ||
        (s = ctx->hip(ctx->sw_list.ensure(3 * list), "alloc")) || (s = ctx->hip(ctx->sw_count.ensure(16), "alloc")))
      return s;
  }
  return SVMC_OK;
}

// Proposal steps between batch refreshes: a walker that reaches
// refresh_every accepted moves is rebuilt at most this many steps later.
constexpr int kRefreshBatch = 8;

// FP64 rebuild of the listed walkers (drift check first), their accept
// counters cleared, then the list emptied.
static svmc_status refresh_list(svmc_ctx* ctx, const Bufs& bf, WalkerSel sel, int32_t* count, hipStream_t st) {
  svmc_status s;
  for (auto& lt : ctx->ld) {
    if ((s = ctx->hip(launch_drift(lt, bf, sel, st), "drift check")) ||
        (s = ctx->hip(launch_rows(ctx->prec, lt, bf, ctx->planes(), ctx->C, st, sel), "rows")) ||
        (s = ctx->hip(launch_gj(lt, bf, st, sel), "inverse")) ||
        (s = ctx->hip(launch_gp(ctx->prec, lt, bf, ctx->planes(), ctx->C, st, sel), "G/P precompute")) ||
        (s = ctx->hip(launch_clear_nacc(lt, bf, sel, st), "clear")))
      return s;
  }
  return ctx->hip(launch_fill_i32(count, 1, 0, st), "list reset");
}

static svmc_status sweep_steps(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed, uint64_t step0,
                               const uint64_t* step0_dev, int64_t* n_accept, const StepSizes& z, hipStream_t st,
                               bool sym = false) {
  const int every = ctx->model.refresh_every;
  const Bufs bf = ctx->bufs();
  const ModelDev md = ctx->mdev();
  StepArgs sa;
  sa.seed = seed;
  sa.step0 = step0;
  sa.step0_dev = (const unsigned long long*)step0_dev;
  sa.n_sweeps = n_sweeps;
  sa.n_accept = n_accept;
  sa.stage = ctx->sw_stage.as<char>();
  sa.stage_stride = (long long)z.stage_bytes;
  sa.acc_list = ctx->sw_list.as<int32_t>();
  sa.due_list = ctx->sw_list.as<int32_t>() + ctx->Wtot;
  sa.urgent_list = ctx->sw_list.as<int32_t>() + 2 * ctx->Wtot;
  sa.refresh_every = every;
  int32_t* cnt = ctx->sw_count.as<int32_t>();     // [2] accepted (per step parity), due, urgent
  sa.due_count = cnt + 2;
  sa.urgent_count = cnt + 3;
  long long qmax = 0;
  for (auto& lt : ctx->ld) qmax = std::max(qmax, (long long)n_sweeps * lt.N);
  ctx->dets_fresh = false;
  svmc_status s;
  if ((s = ctx->hip(launch_fill_i32(cnt, 4, 0, st), "counter reset"))) return s;
  const int nG = ctx->sym_n;
  if (sym) {
    // symmetric sampling: moves drawn per symmetric walker and mapped to its
    // copies, a ratio-only pass, the decision on psi_sym, then the commit
    const size_t W = (size_t)ctx->Wtot;
    if ((s = ctx->hip(ctx->sym_move.ensure(W * 4), "alloc")) || (s = ctx->hip(ctx->sym_ratio.ensure(W * 8), "alloc")) ||
        (s = ctx->hip(ctx->sym_acc.ensure(W * 4), "alloc")) || (s = ctx->hip(ctx->sym_u.ensure(W * 8), "alloc")) ||
        (s = ctx->hip(ctx->sym_pi.ensure(W * 8), "alloc")))
      return s;
    if ((s = ctx->hip(launch_sym_signs(ctx->ld[0], nG, ctx->sym_perm.as<int32_t>(), ctx->sym_flip.as<int32_t>(), bf,
                                       ctx->sym_pi.as<double>(), st),
                      "symmetry signs")))
      return s;
    sa.sym_move = ctx->sym_move.as<int32_t>();
    sa.sym_ratio = ctx->sym_ratio.as<double>();
    sa.sym_acc = ctx->sym_acc.as<int32_t>();
  }
  // per proposal index: every walker proposes, the walkers that accepted are
  // updated, and walkers that reached `every` accepted moves are rebuilt in
  // FP64 before their next proposal
  for (long long q = 0; q < qmax; ++q) {
    sa.q = q;
    sa.count = cnt + (q & 1);
    sa.count_next = cnt + ((q + 1) & 1);
    if (sym) {
      const int32_t* perm = ctx->sym_perm.as<int32_t>();
      const int32_t* flip = ctx->sym_flip.as<int32_t>();
      sa.sym_mode = 1;
      if ((s = ctx->hip(launch_sym_draw(ctx->ld[0], nG, perm, flip, bf, seed, step0 + (uint64_t)q,
                                        ctx->sym_move.as<int32_t>(), ctx->sym_u.as<double>(), st),
                        "symmetric draw")) ||
          (s = ctx->hip(launch_sweep_step(ctx->prec, md, ctx->lats_dev.as<LatDev>(), ctx->ld.data(),
                                          (int)ctx->ld.size(), ctx->Wtot, bf, sa, st),
                        "symmetric ratios")) ||
          (s = ctx->hip(launch_sym_decide(ctx->ld[0], nG, perm, flip, ctx->sym_chi.as<double>(), bf,
                                          ctx->sym_move.as<int32_t>(), ctx->sym_ratio.as<double>(),
                                          ctx->sym_u.as<double>(), ctx->sym_pi.as<double>(),
                                          ctx->sym_acc.as<int32_t>(), st),
                        "symmetric decision")))
        return s;
      sa.sym_mode = 2;
    }
    if ((s = ctx->hip(launch_sweep_step(ctx->prec, md, ctx->lats_dev.as<LatDev>(), ctx->ld.data(),
                                        (int)ctx->ld.size(), ctx->Wtot, bf, sa, st),
                      "sweep step")))
      return s;
    // urgent rebuilds (almost always none) after every step; walkers that
    // reached refresh_every together every kRefreshBatch steps and at the end
    if ((s = refresh_list(ctx, bf, WalkerSel{sa.urgent_list, sa.urgent_count}, sa.urgent_count, st))) return s;
    if ((q + 1) % kRefreshBatch == 0 || q + 1 == qmax)
      if ((s = refresh_list(ctx, bf, WalkerSel{sa.due_list, sa.due_count}, sa.due_count, st))) return s;
  }
  return SVMC_OK;
}

svmc_status svmc_sweep(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed, uint64_t step0, int64_t* n_accept,
                       hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (n_sweeps < 0) return ctx->fail(SVMC_ERR_INVALID_ARG, "negative sweep count");
  if (n_sweeps == 0) return SVMC_OK;
  if (ctx->model.refresh_every < 1) return ctx->fail(SVMC_ERR_INVALID_ARG, "refresh_every must be >= 1");
  for (auto& lt : ctx->ld)
    if ((long long)n_sweeps * lt.N > (1LL << 40)) return ctx->fail(SVMC_ERR_INVALID_ARG, "too many sweeps");
  StepSizes z;
  svmc_status s;
  if ((s = sweep_workspace(ctx, false, z))) return s;
  if (!ctx->prepared && (s = prepare(ctx, st))) return s;
  return sweep_steps(ctx, n_sweeps, seed, step0, nullptr, n_accept, z, st);
}

svmc_status svmc_sweep_sym(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed, uint64_t step0, int64_t* n_accept,
                           hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (ctx->sym_n == 0) return ctx->fail(SVMC_ERR_STATE, "no symmetry group set");
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (ctx->Wtot % ctx->sym_n) return ctx->fail(SVMC_ERR_INVALID_ARG, "walker count is not a multiple of the group order");
  if (n_sweeps < 0) return ctx->fail(SVMC_ERR_INVALID_ARG, "negative sweep count");
  if (n_sweeps == 0) return SVMC_OK;
  if ((long long)n_sweeps * ctx->ld[0].N > (1LL << 40)) return ctx->fail(SVMC_ERR_INVALID_ARG, "too many sweeps");
  StepSizes z;
  svmc_status s;
  if ((s = sweep_workspace(ctx, false, z))) return s;
  if (!ctx->prepared && (s = prepare(ctx, st))) return s;
  return sweep_steps(ctx, n_sweeps, seed, step0, nullptr, n_accept, z, st, true);
}

svmc_status svmc_sweep_async(svmc_ctx* ctx, int32_t n_sweeps, uint64_t seed, const uint64_t* step0_dev,
                             int64_t* n_accept, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (n_sweeps < 0) return ctx->fail(SVMC_ERR_INVALID_ARG, "negative sweep count");
  if (!step0_dev) return ctx->fail(SVMC_ERR_INVALID_ARG, "step0_dev is null");
  if (ctx->model.refresh_every < 1) return ctx->fail(SVMC_ERR_INVALID_ARG, "refresh_every must be >= 1");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return ctx->fail(SVMC_ERR_HIP, "capture query");
  const bool capturing = cap != hipStreamCaptureStatusNone;
  StepSizes z;
  svmc_status s;
  if ((s = sweep_workspace(ctx, capturing, z))) return s;
  // G and P must be current when the work runs: a captured precompute would
  // be replayed against stale inverses, so capture needs them ready
  if (!ctx->prepared) {
    if (capturing) return ctx->fail(SVMC_ERR_STATE, "call svmc_prepare before capturing svmc_sweep_async");
    if ((s = prepare(ctx, st))) return s;
  }
  if (n_sweeps == 0) return SVMC_OK;
  return sweep_steps(ctx, n_sweeps, seed, 0, step0_dev, n_accept, z, st);
}

svmc_status svmc_get_state(svmc_ctx* ctx, int8_t* occ, int16_t* pos, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!occ) return ctx->fail(SVMC_ERR_INVALID_ARG, "occ is null");
  svmc_status s;
  size_t tot = 0;
  for (auto& lt : ctx->ld) tot += (size_t)lt.nw * lt.N;
  if ((s = ctx->hip(hipMemcpyAsync(occ, ctx->occ.p, tot, hipMemcpyDeviceToDevice, st), "occ copy"))) return s;
  if (pos) {
    const int E = ctx->max_elec();
    if ((s = ctx->hip(hipMemsetAsync(pos, 0xff, (size_t)ctx->Wtot * 2 * E * 2, st), "memset"))) return s;
    for (auto& lt : ctx->ld) {
      if (lt.nw == 0) continue;
      // [nw][2][nmax] -> [nw][2][E]
      if ((s = ctx->hip(hipMemcpy2DAsync(pos + lt.w0 * 2 * E, (size_t)E * 2, ctx->pos.as<int16_t>() + lt.pos_off,
                                         (size_t)lt.nmax * 2, (size_t)lt.nmax * 2, (size_t)lt.nw * 2,
                                         hipMemcpyDeviceToDevice, st),
                        "pos copy")))
        return s;
    }
  }
  return SVMC_OK;
}

svmc_status svmc_grad_logpsi(svmc_ctx* ctx, const double* vjp_w, void* out_v, svmc_prec out_prec,
                             hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!out_v) return ctx->fail(SVMC_ERR_INVALID_ARG, "out is null");
  if (out_prec != SVMC_FP64 && out_prec != SVMC_FP32)
    return ctx->fail(SVMC_ERR_INVALID_ARG, "out_prec must be SVMC_FP64 or SVMC_FP32");
  const bool f32 = out_prec == SVMC_FP32;
  svmc_status s;
  // fresh inverses (rows, Phi^-1) and P = W Phi^-1 of the current walkers
  if (!ctx->dets_fresh && (s = rebuild_dets(ctx, st))) return s;
  if (!ctx->prepared && (s = prepare(ctx, st))) return s;
  long long ncmax = 0, nsmax = 0;
  for (auto& lt : ctx->ld) {
    ncmax = std::max(ncmax, (long long)lt.N * ctx->C);
    nsmax = std::max(nsmax, (long long)lt.N);
  }
  const long long W = ctx->Wtot, np = ctx->nparams;
  const bool jac = vjp_w == nullptr;
  // walkers per launch: bounded scratch (rows only in the VJP mode)
  long long chunk = std::min<long long>(W, jac ? 4096 : 1024);
  const size_t smem = grad_smem(ncmax, nsmax);
  GradArgs ga;
  ga.L = ctx->L;
  ga.C = ctx->C;
  ga.act = ctx->model.act;
  ga.lds = smem > 0 ? 1 : 0;
  ga.K = ctx->gK.as<double>();
  ga.B = ctx->gB.as<double>();
  ga.E = ctx->gE.as<double>();
  ga.M = ctx->nmlp;
  ga.MW = ctx->gMW.as<double>();
  ga.MB = ctx->gMB.as<double>();
  ga.nparams = np;
  ga.off_convw = ctx->emb_len;
  ga.off_convb = ga.off_convw + 9LL * ctx->L * ctx->C * ctx->C;
  ga.off_mlpw = ga.off_convb + (long long)ctx->L * ctx->C;
  ga.off_mlpb = ga.off_mlpw + (long long)ctx->nmlp * ctx->C * ctx->C;
  ga.ncmax = ncmax;
  ga.nsmax = nsmax;
  if ((s = ctx->hip(ctx->g_dH.ensure((size_t)chunk * ncmax * 8), "alloc gradient scratch"))) return s;
  // (dz is read in runs of 8 doubles: 8 doubles of slack past the last walker)
  if ((s = ctx->hip(ctx->g_dzs.ensure(((size_t)chunk * ncmax + 8) * 8), "alloc gradient scratch"))) return s;
  if (!ga.lds && (s = ctx->hip(ctx->g_hs.ensure(((size_t)chunk * ncmax + 8) * 8), "alloc gradient scratch")))
    return s;
  // rows are formed in FP64: in the caller's buffer for an FP64 Jacobian, else
  // in scratch (then summed for the VJP, or rounded to FP32)
  const bool direct = jac && !f32;
  if (!direct && (s = ctx->hip(ctx->g_rows.ensure((size_t)chunk * np * 8), "alloc gradient rows"))) return s;
  if (!jac && f32 && (s = ctx->hip(ctx->g_vjp.ensure((size_t)np * 8), "alloc gradient sum"))) return s;
  ga.dH = ctx->g_dH.as<double>();
  ga.hs = ga.lds ? nullptr : ctx->g_hs.as<double>();
  ga.dzs = ctx->g_dzs.as<double>();
  const Bufs bf = ctx->bufs();
  for (long long b0 = 0; b0 < W; b0 += chunk) {
    const long long cnt = std::min(chunk, W - b0);
    ga.w_begin = b0;
    ga.rows = direct ? (double*)out_v + b0 * np : ctx->g_rows.as<double>();
    if ((s = ctx->hip(launch_grad(ctx->prec, ctx->lats_dev.as<LatDev>(), (int)ctx->ld.size(), cnt, bf, ga, st),
                      "gradient")))
      return s;
    if (jac && f32 && (s = ctx->hip(launch_to_f32(ga.rows, (float*)out_v + b0 * np, cnt * np, st), "FP32 rows")))
      return s;
    double* sum = f32 ? ctx->g_vjp.as<double>() : (double*)out_v;
    if (!jac && (s = ctx->hip(launch_grad_reduce(ga.rows, cnt, np, vjp_w + b0, bf.flags + b0, sum, b0 == 0, st),
                              "gradient reduction")))
      return s;
  }
  if (!jac && f32) return ctx->hip(launch_to_f32(ctx->g_vjp.as<double>(), (float*)out_v, np, st), "FP32 sum");
  return SVMC_OK;
}

// Site of lattice l at direction d from s, or -1 off an open edge (host).
static int host_target(const svmc_lattice& l, int s, int d) {
  static const int dx[8] = {1, -1, 0, 0, 1, 1, -1, -1}, dy[8] = {0, 0, 1, -1, 1, -1, 1, -1};
  int x = s % l.Lx + dx[d], y = s / l.Lx + dy[d];
  if (l.pbc_x) x = ((x % l.Lx) + l.Lx) % l.Lx; else if (x < 0 || x >= l.Lx) return -1;
  if (l.pbc_y) y = ((y % l.Ly) + l.Ly) % l.Ly; else if (y < 0 || y >= l.Ly) return -1;
  return x + l.Lx * y;
}

svmc_status svmc_set_symmetry(svmc_ctx* ctx, int32_t n_g, const int32_t* perm, const int32_t* flip, const double* chi) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (n_g == 0) {
    ctx->sym_n = 0;
    return SVMC_OK;
  }
  if (ctx->lats.size() != 1) return ctx->fail(SVMC_ERR_UNSUPPORTED, "symmetry projection needs a one-lattice context");
  if (n_g < 0 || !perm || !flip || !chi) return ctx->fail(SVMC_ERR_INVALID_ARG, "bad group description");
  const svmc_lattice& l = ctx->lats[0];
  const int N = l.Lx * l.Ly, nd = l.tp != 0.0 ? 8 : 4;
  for (int g = 0; g < n_g; ++g) {
    const int32_t* p = perm + (size_t)g * N;
    std::vector<char> seen((size_t)N, 0);
    for (int s = 0; s < N; ++s) {
      if (p[s] < 0 || p[s] >= N || seen[(size_t)p[s]]) return ctx->fail(SVMC_ERR_INVALID_ARG, "perm is not a permutation");
      seen[(size_t)p[s]] = 1;
    }
    if (flip[g] != 0 && flip[g] != 1) return ctx->fail(SVMC_ERR_INVALID_ARG, "flip must be 0 or 1");
    if (flip[g] && l.n_up != l.n_dn) return ctx->fail(SVMC_ERR_INVALID_ARG, "spin flip needs n_up == n_dn");
    if (!std::isfinite(chi[g])) return ctx->fail(SVMC_ERR_INVALID_ARG, "non-finite character");
    if (g == 0) {
      bool id = !flip[0];
      for (int s = 0; s < N; ++s) id = id && p[s] == s;
      if (!id) return ctx->fail(SVMC_ERR_INVALID_ARG, "the first group element must be the identity");
    }
    // a symmetry of the Hamiltonian: bonds go to bonds of the same kind
    // (nearest / next-nearest), and the t-J pinning field is kept
    for (int s = 0; s < N; ++s)
      for (int d = 0; d < nd; ++d) {
        const int j = host_target(l, s, d);
        if (j < 0) continue;
        bool found = false;
        for (int d2 = (d < 4 ? 0 : 4); d2 < (d < 4 ? 4 : 8) && !found; ++d2) found = host_target(l, p[s], d2) == p[j];
        if (!found) return ctx->fail(SVMC_ERR_INVALID_ARG, "a group element does not map bonds to bonds");
      }
    if (l.tj && l.h_pin != 0.0)
      for (int s = 0; s < N; ++s) {
        auto field = [&](int q) { return q % l.Lx == 0 ? ((q / l.Lx) & 1 ? -1 : 1) : 0; };
        if (field(p[s]) * (flip[g] ? -1 : 1) != field(s))
          return ctx->fail(SVMC_ERR_INVALID_ARG, "a group element does not keep the pinning field");
      }
  }
  svmc_status st;
  if ((st = ctx->hip(ctx->sym_perm.ensure((size_t)n_g * N * 4), "alloc")) ||
      (st = ctx->hip(ctx->sym_flip.ensure((size_t)n_g * 4), "alloc")) ||
      (st = ctx->hip(ctx->sym_chi.ensure((size_t)n_g * 8), "alloc")))
    return st;
  if ((st = ctx->hip(hipMemcpy(ctx->sym_perm.p, perm, (size_t)n_g * N * 4, hipMemcpyHostToDevice), "copy")) ||
      (st = ctx->hip(hipMemcpy(ctx->sym_flip.p, flip, (size_t)n_g * 4, hipMemcpyHostToDevice), "copy")) ||
      (st = ctx->hip(hipMemcpy(ctx->sym_chi.p, chi, (size_t)n_g * 8, hipMemcpyHostToDevice), "copy")))
    return st;
  ctx->sym_n = n_g;
  return SVMC_OK;
}

svmc_status svmc_sym_expand(svmc_ctx* ctx, int64_t W, const int8_t* occ, int8_t* out, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (ctx->sym_n == 0) return ctx->fail(SVMC_ERR_STATE, "no symmetry group set");
  if (W < 0 || (W > 0 && (!occ || !out))) return ctx->fail(SVMC_ERR_INVALID_ARG, "bad batch");
  const svmc_lattice& l = ctx->lats[0];
  return ctx->hip(launch_sym_expand(l.Lx * l.Ly, ctx->sym_n, ctx->sym_perm.as<int32_t>(), ctx->sym_flip.as<int32_t>(),
                                    W, occ, out, st),
                  "symmetry expansion");
}

svmc_status svmc_local_energy_sym(svmc_ctx* ctx, double* eloc, double* sign, double* logabs, double* weights,
                                  hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (ctx->sym_n == 0) return ctx->fail(SVMC_ERR_STATE, "no symmetry group set");
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!eloc) return ctx->fail(SVMC_ERR_INVALID_ARG, "eloc is null");
  if (ctx->Wtot % ctx->sym_n) return ctx->fail(SVMC_ERR_INVALID_ARG, "walker count is not a multiple of the group order");
  svmc_status s;
  const size_t W = (size_t)ctx->Wtot;
  if ((s = ctx->hip(ctx->sym_e.ensure(W * 8), "alloc")) || (s = ctx->hip(ctx->sym_s.ensure(W * 8), "alloc")) ||
      (s = ctx->hip(ctx->sym_l.ensure(W * 8), "alloc")))
    return s;
  if ((s = svmc_local_energy(ctx, SVMC_PATH_LOWRANK, ctx->sym_e.as<double>(), nullptr, nullptr, nullptr, st))) return s;
  if ((s = svmc_log_psi(ctx, ctx->sym_s.as<double>(), ctx->sym_l.as<double>(), st))) return s;
  return ctx->hip(launch_sym_combine(ctx->ld[0], ctx->sym_n, ctx->sym_perm.as<int32_t>(), ctx->sym_flip.as<int32_t>(),
                                     ctx->sym_chi.as<double>(), ctx->bufs(), ctx->sym_e.as<double>(),
                                     ctx->sym_s.as<double>(), ctx->sym_l.as<double>(), eloc, sign, logabs, weights,
                                     st),
                  "symmetric local energy");
}

svmc_status svmc_walker_flags(svmc_ctx* ctx, int32_t* flags, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  if (!flags) return ctx->fail(SVMC_ERR_INVALID_ARG, "flags is null");
  return ctx->hip(hipMemcpyAsync(flags, ctx->flags.p, (size_t)ctx->Wtot * 4, hipMemcpyDeviceToDevice, st), "flags");
}

svmc_status svmc_set_launch(svmc_ctx* ctx, const svmc_launch* ln) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ln) return ctx->fail(SVMC_ERR_INVALID_ARG, "launch is null");
  if (ln->slices < 1 || ln->slices > 64) return ctx->fail(SVMC_ERR_INVALID_ARG, "slices must lie in 1..64");
  if (ln->row_form_max != 0 && ln->row_form_max != 8 && ln->row_form_max != 16)
    return ctx->fail(SVMC_ERR_INVALID_ARG, "row_form_max must be 0, 8 or 16");
  ctx->eloc_slices = ln->slices;
  ctx->row_form_max = ln->row_form_max;
  return SVMC_OK;
}

svmc_status svmc_get_launch(const svmc_ctx* ctx, svmc_launch* ln) {
  if (!ctx || !ln) return SVMC_ERR_INVALID_ARG;
  ln->slices = ctx->eloc_slices;
  ln->row_form_max = ctx->row_form_max;
  return SVMC_OK;
}

svmc_status svmc_tune(svmc_ctx* ctx, const char* cache_path, int32_t* slices_out, hipStream_t st) {
  if (!ctx) return SVMC_ERR_INVALID_ARG;
  if (!ctx->have_walkers) return ctx->fail(SVMC_ERR_STATE, "no walkers loaded");
  // shape key
  std::ostringstream key;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return ctx->fail(SVMC_ERR_HIP, "device query");
  key << "dev=" << prop.gcnArchName << " L=" << ctx->L << " C=" << ctx->C << " M=" << ctx->nmlp
      << " prec=" << ctx->prec;
  for (size_t l = 0; l < ctx->lats.size(); ++l) {
    const svmc_lattice& a = ctx->lats[l];
    key << " lat=" << a.Lx << "x" << a.Ly << ":" << a.pbc_x << a.pbc_y << ":" << a.n_up << "+" << a.n_dn
        << ":" << (a.tp != 0.0 ? 8 : 4) << (a.tj ? ":tJ" : "") << ":" << ctx->counts[l];
  }
  const std::string k = key.str();
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const std::string tag = "scalevmc-tune v2 | " + k + " | slices=";
      if (line.compare(0, tag.size(), tag) == 0) {
        int s = 0, r = -1;
        if (std::sscanf(line.c_str() + tag.size(), "%d rowform=%d", &s, &r) == 2 && s >= 1 && s <= 64 &&
            (r == 0 || r == 8 || r == 16)) {
          ctx->eloc_slices = s;
          ctx->row_form_max = r;
          if (slices_out) *slices_out = s;
          return SVMC_OK;
        }
      }
    }
  }
  svmc_status s;
  DevBuf eo;
  if ((s = ctx->hip(eo.ensure((size_t)ctx->Wtot * 8), "alloc"))) return s;
  hipEvent_t e0, e1;
  if ((s = ctx->hip(hipEventCreate(&e0), "event")) || (s = ctx->hip(hipEventCreate(&e1), "event"))) return s;
  const int cand[7] = {1, 2, 4, 8, 16, 24, 32};
  const int forms[3] = {0, 8, 16};
  int best = ctx->eloc_slices, best_rf = ctx->row_form_max;
  float best_ms = 1e30f, tv[21];
  int nv = 0;
  std::ostringstream times;
  for (int v = 0; v < 21 && !s; ++v) {
    const int c = cand[v % 7], rf = forms[v / 7];
    ctx->eloc_slices = c;
    ctx->row_form_max = rf;
    // one untimed call, then two timed
    if ((s = svmc_local_energy(ctx, SVMC_PATH_LOWRANK, eo.as<double>(), nullptr, nullptr, nullptr, st))) break;
    if ((s = ctx->hip(hipEventRecord(e0, st), "event"))) break;
    for (int r = 0; r < 2 && !s; ++r)
      s = svmc_local_energy(ctx, SVMC_PATH_LOWRANK, eo.as<double>(), nullptr, nullptr, nullptr, st);
    if (s) break;
    if ((s = ctx->hip(hipEventRecord(e1, st), "event")) || (s = ctx->hip(hipEventSynchronize(e1), "event sync")))
      break;
    float ms = 0.0f;
    if ((s = ctx->hip(hipEventElapsedTime(&ms, e0, e1), "event time"))) break;
    ms *= 0.5f;
    times << " " << c << "/" << rf << ":" << ms;
    tv[nv++] = ms;
    best_ms = std::min(best_ms, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // among the shapes within 0.5 % of the fastest (timing noise), the
  // fewest slices per walker, then the largest row-form limit: the choice
  // does not flip between runs on differences the timer cannot resolve
  if (!s) {
    bool have = false;
    for (int v = 0; v < nv; ++v) {
      const int c = cand[v % 7], rf = forms[v / 7];
      if (tv[v] > 1.005f * best_ms) continue;
      if (!have || c < best || (c == best && rf > best_rf)) {
        best = c;
        best_rf = rf;
        have = true;
      }
    }
  }
  ctx->eloc_slices = best;
  ctx->row_form_max = best_rf;
  if (s) return s;
  if (slices_out) *slices_out = best;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    if (out)
      out << "scalevmc-tune v2 | " << k << " | slices=" << best << " rowform=" << best_rf << " | ms (slices/rowform)"
          << times.str() << "\n";
  }
  return SVMC_OK;
}

}  // extern "C"
