// Host entries of the real-valued path: plaintext packing/encoding, encryption
// of the encrypted operand, decryption + decoding + lazy rotate-and-sum.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "capi_internal.hpp"
#include "encode.hpp"

using namespace pvfl;

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

namespace {
struct EncHost {
  EncTabs et{};
  CrtTabs crt{};
  std::vector<void*> allocs;
  ~EncHost() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

pvfl_status upload(EncHost* h, const void* src, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(PVFL_E_NOMEM, "encoder table allocation");
  h->allocs.push_back(p);
  if (hipMemcpy(p, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return fail(PVFL_E_DEVICE, "table upload");
  *out = p;
  return PVFL_OK;
}

pvfl_status enc_tables(pvfl_ctx* c, EncHost** out) {
  if (c->enc_tabs) {
    *out = (EncHost*)c->enc_tabs;
    return PVFL_OK;
  }
  std::unique_ptr<EncHost> h(new EncHost());
  const int N = c->N, M = N / 2;
  std::vector<uint32_t> slot2f(M);
  uint64_t e = 1;
  for (int j = 0; j < M; ++j) {
    slot2f[j] = (uint32_t)((e - 1) / 4);
    e = e * 5 % (2 * (uint64_t)N);
  }
  const long double PI = 3.141592653589793238462643383279502884L;
  std::vector<double2> tw(M / 2), twist(M);
  for (int t = 0; t < M / 2; ++t) {
    const long double ang = -2.0L * PI * (long double)t / (long double)M;
    tw[t] = make_double2((double)std::cos(ang), (double)std::sin(ang));
  }
  for (int k = 0; k < M; ++k) {
    const long double ang = PI * (long double)k / (long double)N;
    twist[k] = make_double2((double)std::cos(ang), (double)std::sin(ang));
  }
  std::vector<double> ginv(kMaxLimbs * kMaxLimbs, 0.0);
  for (int i = 0; i < c->n_q; ++i)
    for (int j = 0; j < i; ++j) ginv[j * kMaxLimbs + i] = centred(invm(c->primes[j] % c->primes[i], c->primes[i]), c->primes[i]);
  std::vector<uint32_t> f2slot(M);
  for (int j = 0; j < M; ++j) f2slot[slot2f[j]] = (uint32_t)j;
  void *d_s2f, *d_f2s, *d_tw, *d_twist, *d_g;
  pvfl_status st;
  if ((st = upload(h.get(), slot2f.data(), sizeof(uint32_t) * M, &d_s2f)) != PVFL_OK) return st;
  if ((st = upload(h.get(), f2slot.data(), sizeof(uint32_t) * M, &d_f2s)) != PVFL_OK) return st;
  if ((st = upload(h.get(), tw.data(), sizeof(double2) * (M / 2), &d_tw)) != PVFL_OK) return st;
  if ((st = upload(h.get(), twist.data(), sizeof(double2) * M, &d_twist)) != PVFL_OK) return st;
  if ((st = upload(h.get(), ginv.data(), sizeof(double) * ginv.size(), &d_g)) != PVFL_OK) return st;
  h->et = EncTabs{(const uint32_t*)d_s2f, (const uint32_t*)d_f2s, (const double2*)d_tw, (const double2*)d_twist};
  h->crt = CrtTabs{c->tabs.mods, (const double*)d_g};
  c->enc_tabs = h.release();
  c->enc_tabs_free = [](void* p) { delete (EncHost*)p; };
  *out = (EncHost*)c->enc_tabs;
  return PVFL_OK;
}

}  // namespace

namespace pvfl {
EncodeArgs geometry_of(const pvfl_plan* p, const double* X, int64_t ld) {
  EncodeArgs a{};
  const pvfl_plan_info& I = p->info;
  a.kind = I.kind;
  a.m = I.m;
  a.n = I.n;
  a.ld = (int)ld;
  a.X = X;
  a.slots = p->ctx->N / 2;
  a.mprime = std::max(1, I.mprime);
  a.col_blocks = I.col_blocks;
  a.pack = std::max(1, p->opts.pack);
  a.n_out = I.n_out;
  a.n_out_cts = I.ct_out;
  switch (I.kind) {
    case PVFL_PLAN_HYBRID: a.bm = p->bm; a.bn = p->bn; a.bsgs = p->opts.bsgs; break;
    case PVFL_PLAN_DIAG:
    case PVFL_PLAN_CTMAT: a.bm = I.m_pad; a.bn = I.n_pad; a.width = std::max(I.m_pad, I.n_pad); break;
    case PVFL_PLAN_ROW: a.bm = I.m_pad; a.bn = I.n_pad; break;
    case PVFL_PLAN_COL: a.bm = p->bm; a.bn = p->bn; a.n_out_cts = I.ct_out; break;
  }
  auto lg = [](int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
  };
  a.lbn = lg(a.bn);
  a.lmp = lg(a.mprime);
  a.lw = lg(std::max(1, a.width));
  return a;
}

pvfl_status enc_tables_for(pvfl_ctx* c, EncTabs* et, CrtTabs* crt) {
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  if (et) *et = h->et;
  if (crt) *crt = h->crt;
  return PVFL_OK;
}
}  // namespace pvfl

extern "C" pvfl_status pvfl_encode_pt(const pvfl_plan* p, const double* X, int64_t ld, void* pt, void* stream) {
  return pvfl_encode_pt_scaled(p, X, ld, 1.0, pt, stream);
}

extern "C" pvfl_status pvfl_encode_pt_scaled(const pvfl_plan* p, const double* X, int64_t ld, double coef, void* pt,
                                             void* stream) {
  if (!p || !X || !pt) return fail(PVFL_E_INVALID, "null argument");
  if (!std::isfinite(coef)) return fail(PVFL_E_INVALID, "coef must be finite");
  pvfl_ctx* c = p->ctx;
  const int need_ld = p->info.kind == PVFL_PLAN_CTMAT ? p->info.n_out : p->info.n;
  if (ld < need_ld) return fail(PVFL_E_SHAPE, "leading dimension smaller than the row length");
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  EncodeArgs a = geometry_of(p, X, ld);
  a.scale = p->pt_scale * coef;
  if (p->info.kind == PVFL_PLAN_ROW) a.ind_scale = (double)c->primes[p->lv - 1];
  LimbMap map = qp_map(c, p->lv, p->info.pt_limbs > p->lv + 1);
  KernelTimer kt(c, stream, PVFL_TIMING_ENCODE, 8.0 * (double)p->info.n_pts * map.n * c->N);
  HIP_TRY(launch_encode_pt(launch_ctx(c, stream), a, h->et, map, p->info.n_pts, (double*)pt));
  kt.stop();
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_encrypt(const pvfl_plan* p, const pvfl_sk* sk, const double* v, int64_t ld, uint64_t seed,
                                    void* ct, void* stream) {
  if (!p || !sk || !v || !ct) return fail(PVFL_E_INVALID, "null argument");
  pvfl_ctx* c = p->ctx;
  if (p->info.kind == PVFL_PLAN_CTMAT && ld < p->info.n) return fail(PVFL_E_SHAPE, "leading dimension too small");
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  const int nct = p->info.ct_in, N = c->N, lv = p->lv;
  double* scratch;
  if ((st = ctx_scratch(c, sizeof(int64_t) * (size_t)nct * N, &scratch)) != PVFL_OK) return st;
  int64_t* msg = (int64_t*)scratch;
  EncodeArgs a = geometry_of(p, v, ld);
  a.scale = std::pow(2.0, c->log2_scale);
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_encode_ct(L, a, h->et, nct, msg));
  HIP_TRY(launch_encrypt(L, msg, nct, sk->s, seed, lv, (double*)ct));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_encrypt_pk(const pvfl_plan* p, const pvfl_pk* pk, const double* v, int64_t ld,
                                       uint64_t seed, void* ct, void* stream) {
  if (!p || !pk || !v || !ct) return fail(PVFL_E_INVALID, "null argument");
  pvfl_ctx* c = p->ctx;
  if (pk->ctx != c) return fail(PVFL_E_INVALID, "public key belongs to another context");
  if (p->info.kind == PVFL_PLAN_CTMAT && ld < p->info.n) return fail(PVFL_E_SHAPE, "leading dimension too small");
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  const int nct = p->info.ct_in, N = c->N, lv = p->lv;
  double* scratch;
  if ((st = ctx_scratch(c, sizeof(int64_t) * (size_t)nct * N, &scratch)) != PVFL_OK) return st;
  int64_t* msg = (int64_t*)scratch;
  EncodeArgs a = geometry_of(p, v, ld);
  a.scale = std::pow(2.0, c->log2_scale);
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_encode_ct(L, a, h->et, nct, msg));
  HIP_TRY(launch_encrypt_pk(L, msg, nct, pk->pk, c->n_q, seed, lv, (double*)ct));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_decrypt_decode(const pvfl_plan* p, const pvfl_sk* sk, const void* ct, double* y,
                                           void* stream) {
  if (!p || !sk || !ct || !y) return fail(PVFL_E_INVALID, "null argument");
  pvfl_ctx* c = p->ctx;
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  const int nct = p->info.ct_out, N = c->N, lv = p->info.out_level;
  double* scratch;
  const size_t res_n = (size_t)nct * (lv + 1) * N, z_n = (size_t)nct * (N / 2);
  if ((st = ctx_scratch(c, sizeof(double) * (res_n + z_n), &scratch)) != PVFL_OK) return st;
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_decrypt_f64(L, (const double*)ct, nct, sk->s, lv, scratch));
  HIP_TRY(launch_decode(L, scratch, nct, lv, h->crt, h->et, std::pow(2.0, -p->info.out_log2_scale), scratch + res_n));
  EncodeArgs a = geometry_of(p, nullptr, 0);
  const int count = p->info.kind == PVFL_PLAN_CTMAT ? p->info.m * p->info.n_out : p->info.m;
  HIP_TRY(launch_readout(L, scratch + res_n, a, p->opts.ras_in_ct, count, y));
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// cleartexts at the output scale (Sec. 5.2: Eq. 4's cleartext term, Alg. 2's
// masks) and the masking party's rotate-and-sum
// ---------------------------------------------------------------------------
namespace {
// exponent e with output scale = 2^e * Delta, or -1 when it is not a
// non-negative integer (a plan with a rescale)
int out_shift(const pvfl_plan* p) {
  const double e = p->info.out_log2_scale - p->ctx->log2_scale;
  const double r = std::nearbyint(e);
  if (p->info.kind == PVFL_PLAN_ROW || std::fabs(e - r) > 1e-9 || r < 0 || r > 1000) return -1;
  return (int)r;
}
double pow2_mod_centred(int e, uint64_t q) {
  unsigned __int128 x = 1;
  for (int i = 0; i < e; ++i) x = (x * 2) % q;
  const uint64_t r = (uint64_t)x;
  return r > q / 2 ? (double)r - (double)q : (double)r;
}
}  // namespace

extern "C" size_t pvfl_bytes_pt_out(const pvfl_plan* p) {
  return p ? sizeof(double) * (size_t)p->info.ct_out * (p->info.out_level + 1) * p->ctx->N : 0;
}

extern "C" pvfl_status pvfl_encode_out(const pvfl_plan* p, const double* v, int32_t mode, void* pt, void* stream) {
  if (!p || !v || !pt) return fail(PVFL_E_INVALID, "null argument");
  if (mode != PVFL_OUT_ROWS && mode != PVFL_OUT_SLOTS) return fail(PVFL_E_INVALID, "unknown mode");
  const int e = out_shift(p);
  if (e < 0) return fail(PVFL_E_PLAN, "the plan's output scale is not 2^e times the context scale (ROW rescales)");
  pvfl_ctx* c = p->ctx;
  EncHost* h;
  pvfl_status st = enc_tables(c, &h);
  if (st != PVFL_OK) return st;
  EncodeArgs a = geometry_of(p, nullptr, 0);
  a.scale = std::pow(2.0, c->log2_scale);
  const int lv = p->info.out_level;
  const LimbMap map = qp_map(c, lv, false);
  OutFactors fac{};
  for (int l = 0; l < map.n; ++l) fac.f[l] = pow2_mod_centred(e, c->primes[map.idx[l]]);
  HIP_TRY(launch_encode_out(launch_ctx(c, stream), a, v, mode, p->opts.ras_in_ct, fac, h->et, map, p->info.ct_out,
                            (double*)pt));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_out_add_pt(const pvfl_plan* p, const void* ct, const void* pt, int32_t sign, void* out,
                                       void* stream) {
  if (!p || !ct || !pt || !out) return fail(PVFL_E_INVALID, "null argument");
  if (sign != 1 && sign != -1) return fail(PVFL_E_INVALID, "sign must be +1 or -1");
  pvfl_ctx* c = p->ctx;
  HIP_TRY(launch_out_add_pt(launch_ctx(c, stream), (const double*)ct, (const double*)pt, (double)sign, p->info.ct_out,
                            p->info.out_level, c->N, (double*)out));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_lazy_ras(const pvfl_plan* p, const double* slots, double* y, void* stream) {
  if (!p || !slots || !y) return fail(PVFL_E_INVALID, "null argument");
  EncodeArgs a = geometry_of(p, nullptr, 0);
  const int count = p->info.kind == PVFL_PLAN_CTMAT ? p->info.m * p->info.n_out : p->info.m;
  HIP_TRY(launch_readout(launch_ctx(p->ctx, stream), slots, a, p->opts.ras_in_ct, count, y));
  return PVFL_OK;
}
