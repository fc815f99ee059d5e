// Host side of the C ABI in include/pvfl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pvfl.h"
#include "capi_internal.hpp"

using namespace pvfl;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
extern "C" const char* pvfl_last_error(void) { return g_err.c_str(); }

namespace pvfl {
pvfl_status fail(pvfl_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
pvfl_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorName(e) + " (" + std::to_string((int)e) + "): " +
          hipGetErrorString(e);
  return PVFL_E_DEVICE;
}
}  // namespace pvfl

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

// ---------------------------------------------------------------------------
// host modular arithmetic (exact, 128-bit products)
// ---------------------------------------------------------------------------
namespace pvfl {
u64 mulm(u64 a, u64 b, u64 q) { return (u64)((unsigned __int128)a * b % q); }
u64 powm(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mulm(r, a, q);
    a = mulm(a, a, q);
  }
  return r;
}
u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); }
double centred(u64 x, u64 q) {
  x %= q;
  return x > q / 2 ? (double)x - (double)q : (double)x;
}
static bool probable_prime(u64 n) {
  if (n < 2) return false;
  static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 b : bases)
    if (n % b == 0) return n == b;
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (u64 b : bases) {
    u64 x = powm(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}
static u64 primitive_2n_root(u64 q, int N) {
  const u64 e = (q - 1) / (2 * (u64)N);
  for (u64 x = 2;; ++x) {
    const u64 w = powm(x, e, q);
    if (powm(w, (u64)N, q) == q - 1) return w;
  }
}
static int bit_reverse(int x, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
  return r;
}
}  // namespace pvfl

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
pvfl_ctx::~pvfl_ctx() {
  for (auto& t : timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  if (enc_tabs && enc_tabs_free) enc_tabs_free(enc_tabs);
  if (scratch) (void)hipFree(scratch);
  for (void* p : dev_allocs) (void)hipFree(p);
}

static pvfl_status dev_upload(pvfl_ctx* c, const void* host, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(PVFL_E_NOMEM, "hipMalloc of context tables failed");
  c->dev_allocs.push_back(p);
  HIP_TRY(hipMemcpy(p, host, bytes, hipMemcpyHostToDevice));
  *out = p;
  return PVFL_OK;
}

namespace pvfl {
// basis of level lv: q_0..q_lv then p_0..p_{alpha-1}; limb r -> prime index
LimbMap qp_map(const pvfl_ctx* c, int lv, bool with_p) {
  LimbMap m{};
  m.n = 0;
  for (int i = 0; i <= lv; ++i) m.idx[m.n++] = i;
  if (with_p)
    for (int k = 0; k < c->alpha; ++k) m.idx[m.n++] = c->n_q + k;
  return m;
}
LimbMap key_limb_map(const pvfl_ctx* c, int lv) {
  return qp_map(c, lv, true);  // key limbs follow the context's prime order
}
LaunchCtx launch_ctx(const pvfl_ctx* c, void* stream) { return LaunchCtx{(hipStream_t)stream, c->tabs, c->logN}; }
}  // namespace pvfl

static void build_ks_level(const pvfl_ctx* c, int lv, KsLevel& kl) {
  std::memset(&kl, 0, sizeof(kl));
  const int alpha = c->alpha;
  kl.lv = lv;
  kl.alpha = alpha;
  kl.beta = (lv + 1 + alpha - 1) / alpha;
  kl.K = lv + 1 + alpha;
  kl.n_q_total = c->n_q;
  const std::vector<u64>& P = c->primes;
  auto prime_of_limb = [&](int r) { return r <= lv ? r : c->n_q + (r - lv - 1); };
  // ModUp
  for (int i = 0; i <= lv; ++i) {
    const int j = i / alpha;
    const int lo = j * alpha, hi = std::min(lo + alpha - 1, lv);
    u64 prod = 1;
    for (int k = lo; k <= hi; ++k)
      if (k != i) prod = mulm(prod, P[k] % P[i], P[i]);
    kl.up_inv_hat[i] = centred(invm(prod, P[i]), P[i]);
  }
  int nt = 0;
  for (int j = 0; j < kl.beta; ++j) {
    const int lo = j * alpha, hi = std::min(lo + alpha - 1, lv);
    for (int r = 0; r < kl.K; ++r) {
      KsTask& t = kl.up_task[nt++];
      t.digit = j;
      t.limb = r;
      t.prime = prime_of_limb(r);
      if (r <= lv && r >= lo && r <= hi) {
        t.nsrc = 0;
        t.src0 = r;
        continue;
      }
      t.nsrc = hi - lo + 1;
      t.src0 = lo;
      const u64 tr = P[t.prime];
      for (int u = 0; u < t.nsrc; ++u) {
        u64 prod = 1;
        for (int k = lo; k <= hi; ++k)
          if (k != lo + u) prod = mulm(prod, P[k] % tr, tr);
        t.hat[u] = centred(prod, tr);
      }
    }
  }
  kl.n_tasks = nt;
  // ModDown
  u64 Pmod[kMaxLimbs];
  for (int r = 0; r < kl.K; ++r) {
    const u64 m = P[prime_of_limb(r)];
    u64 pm = 1;
    for (int k = 0; k < alpha; ++k) pm = mulm(pm, P[c->n_q + k] % m, m);
    Pmod[r] = pm;
    // floor(P/2) = (P - 1)/2 since P is odd
    const u64 half = mulm((pm + m - 1) % m, invm(2, m), m);
    kl.down_half[r] = (double)half;
  }
  for (int k = 0; k < alpha; ++k) {
    const u64 pk = P[c->n_q + k];
    u64 prod = 1;
    for (int k2 = 0; k2 < alpha; ++k2)
      if (k2 != k) prod = mulm(prod, P[c->n_q + k2] % pk, pk);
    kl.down_inv_hat[k] = centred(invm(prod, pk), pk);
    for (int i = 0; i <= lv; ++i) {
      u64 h = 1;
      for (int k2 = 0; k2 < alpha; ++k2)
        if (k2 != k) h = mulm(h, P[c->n_q + k2] % P[i], P[i]);
      kl.down_hat[k * kMaxLimbs + i] = centred(h, P[i]);
    }
  }
  for (int i = 0; i <= lv; ++i) {
    kl.down_pinv[i] = centred(invm(Pmod[i], P[i]), P[i]);
    kl.p_mod[i] = centred(Pmod[i], P[i]);
  }
}

extern "C" pvfl_status pvfl_context_create(const pvfl_params* prm, int device, pvfl_ctx** out) {
  if (!prm || !out) return fail(PVFL_E_INVALID, "null argument");
  *out = nullptr;
  if (prm->log_n < 12 || prm->log_n > 15) return fail(PVFL_E_INVALID, "log_n must be 12..15");
  if (prm->n_q < 1 || prm->n_p < 1 || prm->n_p > (uint32_t)kMaxAlpha || prm->n_q + prm->n_p > (uint32_t)kMaxLimbs)
    return fail(PVFL_E_INVALID, "unsupported prime counts");
  const int N = 1 << prm->log_n;
  std::unique_ptr<pvfl_ctx> c(new pvfl_ctx());
  c->logN = (int)prm->log_n;
  c->N = N;
  c->n_q = (int)prm->n_q;
  c->alpha = (int)prm->n_p;
  c->log2_scale = prm->log2_scale;
  c->device = device;
  for (uint32_t i = 0; i < prm->n_q; ++i) c->primes.push_back(prm->q[i]);
  for (uint32_t i = 0; i < prm->n_p; ++i) c->primes.push_back(prm->p[i]);
  for (size_t i = 0; i < c->primes.size(); ++i) {
    const u64 q = c->primes[i];
    if (q >= (1ull << 48) || q < 3 || (q - 1) % (2 * (u64)N) != 0 || !probable_prime(q))
      return fail(PVFL_E_INVALID, "prime " + std::to_string(i) + " is not an NTT-friendly prime below 2^48");
    for (size_t k = 0; k < i; ++k)
      if (c->primes[k] == q) return fail(PVFL_E_INVALID, "primes must be distinct");
  }
  if (hipSetDevice(device) != hipSuccess) return fail(PVFL_E_DEVICE, "hipSetDevice failed");
  const int nm = (int)c->primes.size();
  std::vector<ModQ> mods(nm);
  std::vector<double> fwd((size_t)nm * N), inv((size_t)nm * N), ninv(nm), two32(nm);
  for (int pi = 0; pi < nm; ++pi) {
    const u64 q = c->primes[pi];
    mods[pi] = ModQ{(double)q, 1.0 / (double)q};
    const u64 psi = primitive_2n_root(q, N);
    const u64 psi_inv = invm(psi, q);
    for (int k = 0; k < N; ++k) {
      const int e = bit_reverse(k, c->logN);
      fwd[(size_t)pi * N + k] = centred(powm(psi, (u64)e, q), q);
      inv[(size_t)pi * N + k] = centred(powm(psi_inv, (u64)e, q), q);
    }
    ninv[pi] = centred(invm((u64)N % q, q), q);
    two32[pi] = centred((1ull << 32) % q, q);
    if (c->logN == 15) {
      // split layout: half h's 2^14-point table at h * N/2 (entry (1 << lg) + g is
      // the full table's (1 << (lg + 1)) + (h << lg) + g), the first stage's
      // twiddle at index 0
      const int H = N / 2;
      std::vector<double> f(N, 0.0), iv(N, 0.0);
      double* fr = &fwd[(size_t)pi * N];
      double* ir = &inv[(size_t)pi * N];
      f[0] = fr[1];
      iv[0] = ir[1];
      for (int h = 0; h < 2; ++h)
        for (int k = 1; k < H; ++k) {
          int lg = 0;
          while ((2 << lg) <= k) ++lg;
          const int src = (1 << (lg + 1)) + (h << lg) + (k - (1 << lg));
          f[(size_t)h * H + k] = fr[src];
          iv[(size_t)h * H + k] = ir[src];
        }
      std::copy(f.begin(), f.end(), fr);
      std::copy(iv.begin(), iv.end(), ir);
    }
  }
  // orbit order t -> bit-reversed index
  std::vector<uint32_t> perm(N);
  c->log5.assign(2 * N, -1);
  {
    u64 e = 1;
    for (int t = 0; t < N / 2; ++t) {
      c->log5[e] = t;
      const u64 eneg = (2 * (u64)N - e) % (2 * N);
      perm[t] = (uint32_t)bit_reverse((int)((e - 1) / 2), c->logN);
      perm[t + N / 2] = (uint32_t)bit_reverse((int)((eneg - 1) / 2), c->logN);
      e = e * 5 % (2 * (u64)N);
    }
  }
  pvfl_status st;
  void *d_mods, *d_fwd, *d_inv, *d_ninv, *d_two32, *d_perm;
  if ((st = dev_upload(c.get(), mods.data(), sizeof(ModQ) * nm, &d_mods)) != PVFL_OK) return st;
  if ((st = dev_upload(c.get(), fwd.data(), sizeof(double) * fwd.size(), &d_fwd)) != PVFL_OK) return st;
  if ((st = dev_upload(c.get(), inv.data(), sizeof(double) * inv.size(), &d_inv)) != PVFL_OK) return st;
  if ((st = dev_upload(c.get(), ninv.data(), sizeof(double) * nm, &d_ninv)) != PVFL_OK) return st;
  if ((st = dev_upload(c.get(), two32.data(), sizeof(double) * nm, &d_two32)) != PVFL_OK) return st;
  if ((st = dev_upload(c.get(), perm.data(), sizeof(uint32_t) * N, &d_perm)) != PVFL_OK) return st;
  c->tabs = DevTabs{(const ModQ*)d_mods, (const double*)d_fwd, (const double*)d_inv, (const double*)d_ninv,
                    (const double*)d_two32, (const uint32_t*)d_perm, c->logN};
  c->mods_host = mods;
  // key-switching constants of every level
  c->ks_host.resize(c->n_q);
  for (int lv = 0; lv < c->n_q; ++lv) {
    build_ks_level(c.get(), lv, c->ks_host[lv]);
    if (c->ks_host[lv].n_tasks > kMaxTasks) return fail(PVFL_E_INVALID, "too many ModUp tasks");
  }
  void* d_ks;
  if ((st = dev_upload(c.get(), c->ks_host.data(), sizeof(KsLevel) * c->n_q, &d_ks)) != PVFL_OK) return st;
  c->ks_dev = (const KsLevel*)d_ks;
  // P mod q_i per level 0 row (same for every level), for P*c
  {
    std::vector<double> pm(c->n_q);
    for (int i = 0; i < c->n_q; ++i) pm[i] = c->ks_host[c->n_q - 1].p_mod[i];
    void* d;
    if ((st = dev_upload(c.get(), pm.data(), sizeof(double) * c->n_q, &d)) != PVFL_OK) return st;
    c->pmod_dev = (const double*)d;
  }
  // rescale constants
  c->rescale.resize(c->n_q);
  for (int lv = 1; lv < c->n_q; ++lv) {
    RescaleArgs& ra = c->rescale[lv];
    std::memset(&ra, 0, sizeof(ra));
    const u64 ql = c->primes[lv];
    ra.half_mod_last = (double)(ql / 2);
    for (int i = 0; i < lv; ++i) {
      ra.half_mod[i] = centred((ql / 2) % c->primes[i], c->primes[i]);
      ra.inv_last[i] = centred(invm(ql % c->primes[i], c->primes[i]), c->primes[i]);
    }
  }
  if ((st = noalloc_scratch_init(device)) != PVFL_OK) return st;
  HIP_TRY(hipDeviceSynchronize());
  *out = c.release();
  return PVFL_OK;
}

extern "C" void pvfl_context_destroy(pvfl_ctx* c) { delete c; }

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
pvfl_sk::~pvfl_sk() {
  if (s) (void)hipFree(s);
}
pvfl_rotkeys::~pvfl_rotkeys() {}  // the key memory is the caller's

extern "C" pvfl_status pvfl_keygen(pvfl_ctx* c, uint64_t seed, pvfl_sk** out) {
  if (!c || !out) return fail(PVFL_E_INVALID, "null argument");
  std::unique_ptr<pvfl_sk> sk(new pvfl_sk());
  sk->ctx = c;
  const size_t bytes = sizeof(double) * c->primes.size() * c->N;
  if (hipMalloc((void**)&sk->s, bytes) != hipSuccess) return fail(PVFL_E_NOMEM, "secret key allocation");
  HIP_TRY(launch_keygen(launch_ctx(c, nullptr), seed, sk->s, (int)c->primes.size()));
  HIP_TRY(hipDeviceSynchronize());
  *out = sk.release();
  return PVFL_OK;
}
extern "C" void pvfl_sk_destroy(pvfl_sk* sk) { delete sk; }

pvfl_pk::~pvfl_pk() {
  if (pk) (void)hipFree(pk);
}
extern "C" pvfl_status pvfl_pk_gen(pvfl_ctx* c, const pvfl_sk* sk, uint64_t seed, pvfl_pk** out) {
  if (!c || !sk || !out) return fail(PVFL_E_INVALID, "null argument");
  if (sk->ctx != c) return fail(PVFL_E_INVALID, "secret key belongs to another context");
  std::unique_ptr<pvfl_pk> pk(new pvfl_pk());
  pk->ctx = c;
  const int nl = c->n_q;
  if (hipMalloc((void**)&pk->pk, sizeof(double) * 2 * (size_t)nl * c->N) != hipSuccess)
    return fail(PVFL_E_NOMEM, "public key allocation");
  HIP_TRY(launch_pk_gen(launch_ctx(c, nullptr), sk->s, seed, nl, pk->pk));
  HIP_TRY(hipDeviceSynchronize());
  *out = pk.release();
  return PVFL_OK;
}
extern "C" void pvfl_pk_destroy(pvfl_pk* pk) { delete pk; }
extern "C" pvfl_status pvfl_pk_export(const pvfl_pk* pk, uint64_t* out, void* stream) {
  if (!pk || !out) return fail(PVFL_E_INVALID, "null argument");
  const pvfl_ctx* c = pk->ctx;
  LimbMap m = qp_map(c, c->n_q - 1, false);
  HIP_TRY(launch_ntt(launch_ctx(c, stream), NttOp::ExportU64, pk->pk, out, 2 * m.n, m));
  return PVFL_OK;
}

// Key memory: [count][beta][2][L+1+alpha][N] doubles, then the rotation ->
// key-index table (N/2 ints), 256-byte aligned.
static size_t rotkey_stride(const pvfl_ctx* c) {
  const int beta = (c->n_q + c->alpha - 1) / c->alpha;
  return (size_t)beta * 2 * c->primes.size() * c->N;
}
static size_t rotkey_table_off(const pvfl_ctx* c, int count) {
  return ((sizeof(double) * rotkey_stride(c) * (size_t)std::max(count, 0)) + 255) & ~(size_t)255;
}
extern "C" size_t pvfl_bytes_rotkeys(const pvfl_ctx* c, int32_t count) {
  if (!c || count < 0) return 0;
  return rotkey_table_off(c, count) + sizeof(int) * (size_t)(c->N / 2);
}

extern "C" pvfl_status pvfl_rotkeys_gen(pvfl_ctx* c, const pvfl_sk* sk, const uint32_t* galois, int32_t count,
                                        uint64_t seed, void* keys_dev, size_t keys_bytes, pvfl_rotkeys** out) {
  if (!c || !sk || !out || (count > 0 && !galois) || count < 0) return fail(PVFL_E_INVALID, "bad argument");
  *out = nullptr;
  if (sk->ctx != c) return fail(PVFL_E_INVALID, "secret key belongs to another context");
  std::unique_ptr<pvfl_rotkeys> rk(new pvfl_rotkeys());
  rk->ctx = c;
  const int N = c->N;
  rk->key_limbs = (int)c->primes.size();
  rk->beta = (c->n_q + c->alpha - 1) / c->alpha;
  rk->key_stride = rotkey_stride(c);
  rk->slot_of_rot.assign(N / 2, -1);
  for (int k = 0; k < count; ++k) {
    const uint32_t g = galois[k];
    if (g >= (uint32_t)(2 * N) || c->log5[g] < 0)
      return fail(PVFL_E_INVALID, "Galois element " + std::to_string(g) + " is not a power of 5 mod 2N");
    const int rot = c->log5[g];
    if (rk->slot_of_rot[rot] >= 0) continue;
    rk->slot_of_rot[rot] = (int)rk->galois.size();
    rk->galois.push_back(g);
    rk->rot.push_back(rot);
  }
  const int nk = (int)rk->galois.size();
  const size_t need = pvfl_bytes_rotkeys(c, nk);
  if (!keys_dev) return fail(PVFL_E_INVALID, "the keys need a device buffer of pvfl_bytes_rotkeys bytes");
  if (keys_bytes < need)
    return fail(PVFL_E_SHAPE, "key buffer of " + std::to_string(keys_bytes) + " bytes, the keys need " +
                                  std::to_string(need));
  if (((uintptr_t)keys_dev & 255) != 0) return fail(PVFL_E_INVALID, "the key buffer must be 256-byte aligned");
  rk->keys = (double*)keys_dev;
  rk->slot_of_rot_dev = (int*)((char*)keys_dev + rotkey_table_off(c, nk));
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpy(rk->slot_of_rot_dev, rk->slot_of_rot.data(), sizeof(int) * (N / 2), hipMemcpyHostToDevice));
  RotKeyArgs ka{};
  ka.n_limbs = rk->key_limbs;
  ka.beta = rk->beta;
  ka.alpha = c->alpha;
  ka.n_q = c->n_q;
  for (int r = 0; r < rk->key_limbs; ++r) {
    const u64 m = c->primes[r];
    u64 pm = 1;
    for (int k = 0; k < c->alpha; ++k) pm = mulm(pm, c->primes[c->n_q + k] % m, m);
    ka.P_mod[r] = centred(pm, m);
  }
  // bounded launches, the keys of each passed by value
  for (int k0 = 0; k0 < nk; k0 += kKeysPerLaunch) {
    const int cnt = std::min(kKeysPerLaunch, nk - k0);
    RotKeyList list{};
    for (int u = 0; u < cnt; ++u) {
      list.rot[u] = rk->rot[k0 + u];
      list.galois[u] = rk->galois[k0 + u];
    }
    HIP_TRY(launch_rotkey_gen(launch_ctx(c, nullptr), sk->s, list, cnt, seed, ka,
                              rk->keys + (size_t)k0 * rk->key_stride));
  }
  HIP_TRY(hipDeviceSynchronize());
  *out = rk.release();
  return PVFL_OK;
}
extern "C" void pvfl_rotkeys_destroy(pvfl_rotkeys* k) { delete k; }

extern "C" pvfl_status pvfl_sk_export(const pvfl_sk* sk, uint64_t* out, void* stream) {
  if (!sk || !out) return fail(PVFL_E_INVALID, "null argument");
  const pvfl_ctx* c = sk->ctx;
  LimbMap m = qp_map(c, c->n_q - 1, true);
  HIP_TRY(launch_ntt(launch_ctx(c, stream), NttOp::ExportU64, sk->s, out, m.n, m));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_rotkeys_export(const pvfl_rotkeys* k, int32_t index, uint64_t* out, void* stream) {
  if (!k || !out || index < 0 || index >= (int)k->galois.size()) return fail(PVFL_E_INVALID, "bad key index");
  const pvfl_ctx* c = k->ctx;
  LimbMap m = qp_map(c, c->n_q - 1, true);
  HIP_TRY(launch_ntt(launch_ctx(c, stream), NttOp::ExportU64, k->keys + (size_t)index * k->key_stride, out,
                     k->beta * 2 * m.n, m));
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// integer-level entries
// ---------------------------------------------------------------------------
static bool bad_level(const pvfl_ctx* c, int lv) { return lv < 0 || lv >= c->n_q; }

extern "C" pvfl_status pvfl_pt_import(pvfl_ctx* c, int32_t level, int32_t with_p, const int64_t* m, int32_t count,
                                      void* pt, void* stream) {
  if (!c || !m || !pt || count < 0) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  LimbMap map = qp_map(c, level, with_p != 0);
  HIP_TRY(launch_ntt(launch_ctx(c, stream), NttOp::ImportI64, m, pt, count * map.n, map));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_encrypt_coeffs(pvfl_ctx* c, const pvfl_sk* sk, int32_t level, const int64_t* m,
                                           uint64_t seed, void* ct, void* stream) {
  if (!c || !sk || !m || !ct) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  HIP_TRY(launch_encrypt(launch_ctx(c, stream), m, 1, sk->s, seed, level, (double*)ct));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_encrypt_coeffs_pk(pvfl_ctx* c, const pvfl_pk* pk, int32_t level, const int64_t* m,
                                              uint64_t seed, void* ct, void* stream) {
  if (!c || !pk || !m || !ct) return fail(PVFL_E_INVALID, "null argument");
  if (pk->ctx != c) return fail(PVFL_E_INVALID, "public key belongs to another context");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  HIP_TRY(launch_encrypt_pk(launch_ctx(c, stream), m, 1, pk->pk, c->n_q, seed, level, (double*)ct));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_export_coeffs(pvfl_ctx* c, int32_t level, int32_t with_p, const void* poly,
                                          int32_t count, uint64_t* out, void* stream) {
  if (!c || !poly || !out || count < 0) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  LimbMap map = qp_map(c, level, with_p != 0);
  HIP_TRY(launch_ntt(launch_ctx(c, stream), NttOp::ExportU64, poly, out, count * map.n, map));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_decrypt_coeffs(pvfl_ctx* c, const pvfl_sk* sk, int32_t level, const void* ct,
                                           uint64_t* out, void* stream) {
  if (!c || !sk || !ct || !out) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  HIP_TRY(launch_decrypt_u64(launch_ctx(c, stream), (const double*)ct, sk->s, level, out));
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// single operations
// ---------------------------------------------------------------------------
namespace pvfl {
// per-context scratch for single operations (grown on demand, stream-ordered use)
pvfl_status ctx_scratch(pvfl_ctx* c, size_t bytes, double** out) {
  if (c->scratch_bytes < bytes) {
    if (c->scratch) (void)hipFree(c->scratch);
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    if (hipMalloc((void**)&c->scratch, bytes) != hipSuccess) return fail(PVFL_E_NOMEM, "scratch allocation");
    c->scratch_bytes = bytes;
  }
  *out = c->scratch;
  return PVFL_OK;
}

// key switch of the hoisted digits of c1 (or of an already-rotated c1 with
// rot = 0), then ModDown; writes (v0, v1) to v [2][lv+1][N].
pvfl_status keyswitch_digits(pvfl_ctx* c, const pvfl_rotkeys* keys, int lv, const double* digits, int rot_digits,
                             int key_rot, double* u, double* ydown, double* v, void* stream) {
  const int slot = keys->slot_of_rot[key_rot];
  if (slot < 0) return fail(PVFL_E_NOKEY, "missing rotation key for rotation " + std::to_string(key_rot));
  const KsLevel& kl = c->ks_host[lv];
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_key_inner(L, digits, kl.beta, kl.K, c->N, rot_digits, keys->keys + (size_t)slot * keys->key_stride,
                           keys->key_limbs, qp_map(c, lv, true), key_limb_map(c, lv), u));
  HIP_TRY(launch_moddown(L, u, 2, lv, c->alpha, c->ks_dev + lv, ydown, v));
  return PVFL_OK;
}
}  // namespace pvfl

extern "C" pvfl_status pvfl_rotate(pvfl_ctx* c, const pvfl_rotkeys* keys, int32_t level, const void* ct_v,
                                   uint32_t galois, int32_t hoisted, void* out_v, void* stream) {
  if (!c || !keys || !ct_v || !out_v) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  const int N = c->N;
  if (galois >= (uint32_t)(2 * N) || c->log5[galois] < 0) return fail(PVFL_E_INVALID, "Galois element not in <5>");
  const int rot = c->log5[galois];
  if (keys->slot_of_rot[rot] < 0) return fail(PVFL_E_NOKEY, "missing rotation key");
  const KsLevel& kl = c->ks_host[level];
  const size_t Q = (size_t)(level + 1) * N;
  const size_t need = (size_t)kl.beta * kl.K * N + Q + 2 * (size_t)kl.K * N + 2 * (size_t)c->alpha * N + 2 * Q + 2 * Q;
  double* ws;
  pvfl_status st = ctx_scratch(c, need * sizeof(double), &ws);
  if (st != PVFL_OK) return st;
  double* digits = ws;
  double* yup = digits + (size_t)kl.beta * kl.K * N;
  double* u = yup + Q;
  double* ydown = u + 2 * (size_t)kl.K * N;
  double* v = ydown + 2 * (size_t)c->alpha * N;
  double* rct = v + 2 * Q;
  const double* ct = (const double*)ct_v;
  double* out = (double*)out_v;
  LaunchCtx L = launch_ctx(c, stream);
  if (hoisted) {
    HIP_TRY(launch_modup(L, ct, 0, 1, level, c->ks_dev + level, kl.n_tasks, yup, digits, 0));
    if ((st = keyswitch_digits(c, keys, level, digits, rot, rot, u, ydown, v, stream)) != PVFL_OK) return st;
    HIP_TRY(launch_automorph(L, ct, level + 1, N, rot, rct));
  } else {
    HIP_TRY(launch_automorph(L, ct, 2 * (level + 1), N, rot, rct));
    HIP_TRY(launch_modup(L, rct, 0, 1, level, c->ks_dev + level, kl.n_tasks, yup, digits, 0));
    if ((st = keyswitch_digits(c, keys, level, digits, 0, rot, u, ydown, v, stream)) != PVFL_OK) return st;
  }
  // out = (phi(c0) + v0, v1)
  HIP_TRY(launch_ct_add(L, rct, v, level, N, out));  // adds both halves; fix c1 below
  HIP_TRY(hipMemcpyAsync(out + Q, v + Q, Q * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_rescale(pvfl_ctx* c, int32_t level, const void* ct, void* out, void* stream) {
  if (!c || !ct || !out) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level) || level < 1) return fail(PVFL_E_LEVEL, "rescale needs level >= 1");
  HIP_TRY(launch_rescale(launch_ctx(c, stream), (const double*)ct, 2, level, c->rescale[level], (double*)out));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_ct_mul_pt(pvfl_ctx* c, int32_t level, const void* ct, const void* pt, void* out,
                                      void* stream) {
  if (!c || !ct || !pt || !out) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  HIP_TRY(launch_ct_mul_pt(launch_ctx(c, stream), (const double*)ct, (const double*)pt, level, c->N, (double*)out));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_ct_add(pvfl_ctx* c, int32_t level, const void* a, const void* b, void* out, void* stream) {
  if (!c || !a || !b || !out) return fail(PVFL_E_INVALID, "null argument");
  if (bad_level(c, level)) return fail(PVFL_E_LEVEL, "level out of range");
  HIP_TRY(launch_ct_add(launch_ctx(c, stream), (const double*)a, (const double*)b, level, c->N, (double*)out));
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
extern "C" pvfl_status pvfl_timing_enable(pvfl_ctx* c, int32_t enable) {
  if (!c) return fail(PVFL_E_INVALID, "null argument");
  c->timing_on = enable != 0;
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_timing_read(pvfl_ctx* c, int32_t cls, double* total_ms, int64_t* launches, double* bytes) {
  if (!c || !total_ms || !launches || !bytes) return fail(PVFL_E_INVALID, "null argument");
  double ms = 0, by = 0;
  int64_t n = 0;
  std::vector<pvfl_ctx::Timed> keep;
  for (auto& t : c->timed) {
    if (t.cls != cls) {
      keep.push_back(t);
      continue;
    }
    HIP_TRY(hipEventSynchronize(t.stop));
    float e = 0;
    HIP_TRY(hipEventElapsedTime(&e, t.start, t.stop));
    ms += e;
    by += t.bytes;
    ++n;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  c->timed.swap(keep);
  *total_ms = ms;
  *launches = n;
  *bytes = by;
  return PVFL_OK;
}
