// Batched execution of many independent products (host side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <vector>

#include "batch.hpp"
#include "capi_internal.hpp"

using namespace pvfl;

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

namespace pvfl {
pvfl_status enc_tables_for(pvfl_ctx* c, EncTabs* et, CrtTabs* crt);  // codec.cpp
EncodeArgs geometry_of(const pvfl_plan* p, const double* X, int64_t ld);  // codec.cpp
}  // namespace pvfl

struct pvfl_batch {
  pvfl_ctx* ctx = nullptr;
  const pvfl_rotkeys* keys = nullptr;
  int count = 0, pg = 4, CH = 64, vec = 1, lv = 0, K = 0, beta = 0, max_rows = 0;
  int n_enc_work = 0, n_work = 0, n_slots = 0;
  double inv_scale = 1.0;
  // every device pointer below lies in the caller's workspace
  BatchProd* prods = nullptr;
  EncodeArgs* args_pt = nullptr;
  EncodeArgs* args_ct = nullptr;
  int2* enc_work = nullptr;
  DiagGroup* groups = nullptr;
  DiagWork* work = nullptr;
  DiagTask* tasks = nullptr;
  int n_tasks = 0;
  const double** ct_tab = nullptr;
  double** ct_out_tab = nullptr;
  double** out_tab = nullptr;
  double *digits = nullptr, *yup = nullptr, *pc = nullptr, *part = nullptr, *acc = nullptr, *ydown = nullptr;
  double *res = nullptr, *z = nullptr;
  int64_t* msg = nullptr;
  double key_bytes = 0, key_bytes_min = 0, pt_bytes = 0;
  // captured whole-step graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const pvfl_sk* graph_sk = nullptr;
  uint64_t graph_seed = 0;
  hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
  hipStream_t cap_stream2 = nullptr;  // second branch of the captured graph
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool has_X = false, has_v = false, has_y = false;
  ~pvfl_batch() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (cap_stream2) (void)hipStreamDestroy(cap_stream2);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};

namespace {

struct BatchOpts {
  int group, chunk, vec, order;
};

pvfl_status read_opts(const pvfl_batch_opts* opts, BatchOpts* o) {
  const pvfl_batch_opts dflt{2, 32, 1, 1};
  const pvfl_batch_opts x = opts ? *opts : dflt;
  if (x.group != 1 && x.group != 2 && x.group != 4) return fail(PVFL_E_INVALID, "group must be 1, 2 or 4");
  if (x.vec != 1 && x.vec != 2) return fail(PVFL_E_INVALID, "vec must be 1 or 2");
  if (x.chunk > 1024) return fail(PVFL_E_INVALID, "chunk must be at most 1024");
  if (x.chunk < 1) return fail(PVFL_E_INVALID, "chunk must be positive");
  *o = BatchOpts{x.group, x.chunk, x.vec, x.chunk_major};
  return PVFL_OK;
}

// the plans a batch accepts: lazy, hoisted HYBRID (or DIAG without in-ciphertext
// RaS) plans of one context, level and plaintext scale, one input and one output
pvfl_status check_plans(pvfl_ctx* c, int count, const pvfl_plan* const* plans) {
  if (!c || !plans || count < 1) return fail(PVFL_E_INVALID, "bad argument");
  const pvfl_plan* p0 = plans[0];
  if (!p0) return fail(PVFL_E_INVALID, "null plan");
  if (p0->beta > 4) return fail(PVFL_E_PLAN, "batched kernel supports up to 4 digits");
  for (int k = 0; k < count; ++k) {
    const pvfl_plan* p = plans[k];
    if (!p || p->ctx != c) return fail(PVFL_E_INVALID, "plan belongs to another context");
    const bool ok_kind = p->opts.kind == PVFL_PLAN_HYBRID || (p->opts.kind == PVFL_PLAN_DIAG && p->ras_rots.empty());
    if (!ok_kind || !p->opts.lazy_moddown || p->info.ct_in != 1 || p->info.ct_out != 1 || p->info.bsgs != 0)
      return fail(PVFL_E_PLAN, "batched products must be lazy, hoisted HYBRID/DIAG plans with one input and one "
                               "output ciphertext");
    if (p->lv != p0->lv) return fail(PVFL_E_LEVEL, "batched products must share the level");
    if (p->pt_scale != p0->pt_scale) return fail(PVFL_E_PLAN, "batched products must share the plaintext scale");
  }
  return PVFL_OK;
}

// Work schedule of the fused kernel: groups of products with similar m'
// (descending), chunked diagonal ranges, and the task list of workgroups.
struct Schedule {
  std::vector<DiagGroup> groups;
  std::vector<DiagWork> work;
  std::vector<DiagTask> tasks;
  std::vector<int> part0;  // first partial-sum slot of each product
  int n_slots = 0;
  double key_reads = 0;    // rotation keys streamed (once per group and diagonal)
  int max_mp = 0;
};

Schedule make_schedule(const std::vector<int>& mprime, int K, int N, const BatchOpts& o) {
  Schedule S;
  const int count = (int)mprime.size();
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int z) { return mprime[a] > mprime[z]; });
  for (int g0 = 0; g0 < count; g0 += o.group) {
    DiagGroup G{};
    G.np = std::min(o.group, count - g0);
    int mx = 0;
    for (int u = 0; u < G.np; ++u) {
      G.prod[u] = order[g0 + u];
      mx = std::max(mx, mprime[G.prod[u]]);
    }
    for (int i0 = 0; i0 < mx; i0 += o.chunk)
      S.work.push_back(DiagWork{(int)S.groups.size(), i0, std::min(i0 + o.chunk, mx), 0});
    S.key_reads += std::max(0, mx - 1);
    S.groups.push_back(G);
    S.max_mp = std::max(S.max_mp, mx);
  }
  // Chunk-major order: work items of every group for diagonals [0, CH) first,
  // then [CH, 2 CH), ...  Blocks are dispatched round-robin over the 8 XCDs by
  // linear block index; the blocks of one (tile, limb) for consecutive work
  // items are (N/256)*K apart, a multiple of 8, so they land on the same XCD
  // and read the same rotation-key lines from its L2.
  if (o.order == 1)
    std::stable_sort(S.work.begin(), S.work.end(), [](const DiagWork& a, const DiagWork& z) { return a.i0 < z.i0; });
  // task list: for each chunk (in order), tile, limb: the work items of that
  // chunk, so that consecutive tasks read the same rotation-key tile
  const int ntile = N / (256 * o.vec);
  size_t w0 = 0;
  while (w0 < S.work.size()) {
    size_t w1 = w0;
    while (w1 < S.work.size() && S.work[w1].i0 == S.work[w0].i0) ++w1;
    if (o.order != 1) w1 = w0 + 1;
    for (int tile = 0; tile < ntile; ++tile)
      for (int r = 0; r < K; ++r)
        for (size_t wi = w0; wi < w1; ++wi) S.tasks.push_back(DiagTask{(int)wi, tile, r, 0});
    w0 = w1;
  }
  S.part0.resize(count);
  for (int k = 0; k < count; ++k) {
    S.part0[k] = S.n_slots;
    S.n_slots += (mprime[k] + o.chunk - 1) / o.chunk;
  }
  return S;
}

// Byte offsets of everything a batch keeps in device memory, carved from one
// workspace in this order (each piece 256-byte aligned): the tables of the
// launches, then the buffers of the phases.
struct Layout {
  size_t prods, args_pt, args_ct, enc_work, groups, work, tasks, ct_tab, ct_out_tab, out_tab;
  size_t digits, yup, pc, part, acc, ydown, msg, res, z;
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t o = total;
    total += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return o;
  }
};

Layout make_layout(const pvfl_ctx* c, int count, int n_enc_work, const Schedule& S, int lv, int K, int beta) {
  const size_t N = c->N, KN = (size_t)K * N, Q = (size_t)(lv + 1) * N, cn = (size_t)count;
  Layout L{};
  L.prods = L.take(sizeof(BatchProd) * cn);
  L.args_pt = L.take(sizeof(EncodeArgs) * cn);
  L.args_ct = L.take(sizeof(EncodeArgs) * cn);
  L.enc_work = L.take(sizeof(int2) * (size_t)n_enc_work);
  L.groups = L.take(sizeof(DiagGroup) * S.groups.size());
  L.work = L.take(sizeof(DiagWork) * S.work.size());
  L.tasks = L.take(sizeof(DiagTask) * S.tasks.size());
  L.ct_tab = L.take(sizeof(double*) * cn);
  L.ct_out_tab = L.take(sizeof(double*) * cn);
  L.out_tab = L.take(sizeof(double*) * cn);
  L.digits = L.take(sizeof(double) * cn * beta * KN);
  L.yup = L.take(sizeof(double) * cn * Q);
  L.pc = L.take(sizeof(double) * cn * 2 * Q);
  L.part = L.take(sizeof(double) * (size_t)S.n_slots * 2 * KN);
  L.acc = L.take(sizeof(double) * cn * 2 * KN);
  L.ydown = L.take(sizeof(double) * cn * 2 * c->alpha * N);
  L.msg = L.take(sizeof(int64_t) * cn * N);
  L.res = L.take(sizeof(double) * cn * Q);
  L.z = L.take(sizeof(double) * cn * (N / 2));
  return L;
}

template <class T>
pvfl_status upload(const std::vector<T>& v, char* base, size_t off) {
  if (v.empty()) return PVFL_OK;
  const hipError_t e = hipMemcpy(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e == hipSuccess ? PVFL_OK : hip_fail(e, "batch table upload");
}

int total_pts(int count, const pvfl_plan* const* plans) {
  int n = 0;
  for (int k = 0; k < count; ++k) n += plans[k]->info.n_pts;
  return n;
}

std::vector<int> mprimes_of(int count, const pvfl_plan* const* plans) {
  std::vector<int> mp(count);
  for (int k = 0; k < count; ++k) mp[k] = plans[k]->info.mprime;
  return mp;
}

}  // namespace

extern "C" pvfl_status pvfl_batch_workspace_bytes(pvfl_ctx* c, int32_t count, const pvfl_plan* const* plans,
                                                  const pvfl_batch_opts* opts, size_t* bytes) {
  if (!bytes) return fail(PVFL_E_INVALID, "null argument");
  *bytes = 0;
  BatchOpts o;
  pvfl_status st = read_opts(opts, &o);
  if (st != PVFL_OK) return st;
  if ((st = check_plans(c, count, plans)) != PVFL_OK) return st;
  const pvfl_plan* p0 = plans[0];
  const Schedule S = make_schedule(mprimes_of(count, plans), p0->K, c->N, o);
  *bytes = make_layout(c, count, total_pts(count, plans), S, p0->lv, p0->K, p0->beta).total;
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_batch_create(pvfl_ctx* c, int32_t count, const pvfl_plan* const* plans,
                                         const double* const* X_dev, const int64_t* ldx, const double* const* v_dev,
                                         void* const* pt_dev, void* const* ct_dev, void* const* out_dev,
                                         double* const* y_dev, const pvfl_rotkeys* keys, const pvfl_batch_opts* opts,
                                         void* ws_dev, size_t ws_bytes, pvfl_batch** out) {
  if (!out) return fail(PVFL_E_INVALID, "bad argument");
  *out = nullptr;
  if (!pt_dev || !ct_dev || !out_dev) return fail(PVFL_E_INVALID, "bad argument");
  BatchOpts o;
  pvfl_status st = read_opts(opts, &o);
  if (st != PVFL_OK) return st;
  if ((st = check_plans(c, count, plans)) != PVFL_OK) return st;
  std::unique_ptr<pvfl_batch> b(new pvfl_batch());
  b->ctx = c;
  b->keys = keys;
  b->count = count;
  b->pg = o.group;
  b->vec = o.vec;
  b->CH = o.chunk;
  const pvfl_plan* p0 = plans[0];
  b->lv = p0->lv;
  b->K = p0->K;
  b->beta = p0->beta;
  const int N = c->N;
  std::vector<BatchProd> prods(count);
  std::vector<EncodeArgs> apt(count), act(count);
  std::vector<int2> encw;
  std::vector<const double*> ct_tab(count);
  std::vector<double*> ct_out_tab(count), out_tab(count);
  for (int k = 0; k < count; ++k) {
    const pvfl_plan* p = plans[k];
    if (!p->galois.empty()) {
      if (!keys || keys->ctx != c) return fail(PVFL_E_NOKEY, "batch needs rotation keys");
      for (uint32_t g : p->galois)
        if (keys->slot_of_rot[c->log5[g]] < 0) return fail(PVFL_E_NOKEY, "missing rotation key");
    }
    if ((X_dev && !X_dev[k]) || (v_dev && !v_dev[k]) || (y_dev && !y_dev[k]) || !pt_dev[k] || !ct_dev[k] || !out_dev[k])
      return fail(PVFL_E_INVALID, "null buffer for product " + std::to_string(k));
    if (X_dev && ldx && ldx[k] < p->info.n)
      return fail(PVFL_E_SHAPE, "product " + std::to_string(k) + ": leading dimension smaller than the row length");
    BatchProd& B = prods[k];
    B.ct = (const double*)ct_dev[k];
    B.ct_out = (double*)ct_dev[k];
    B.pt = (const double*)pt_dev[k];
    B.pt_out = (double*)pt_dev[k];
    B.out = (double*)out_dev[k];
    B.y = y_dev ? y_dev[k] : nullptr;
    B.mprime = p->info.mprime;
    apt[k] = geometry_of(p, X_dev ? X_dev[k] : nullptr, ldx ? ldx[k] : p->info.n);
    apt[k].scale = p->pt_scale;
    act[k] = geometry_of(p, v_dev ? v_dev[k] : nullptr, p->info.n);
    act[k].scale = std::pow(2.0, c->log2_scale);
    for (int j = 0; j < p->info.n_pts; ++j) encw.push_back(make_int2(k, j));
    ct_tab[k] = B.ct;
    ct_out_tab[k] = B.ct_out;
    out_tab[k] = B.out;
    b->max_rows = std::max(b->max_rows, p->info.m);
    b->pt_bytes += 8.0 * (double)p->info.n_pts * b->K * N;
  }
  b->inv_scale = std::pow(2.0, -p0->info.out_log2_scale);
  b->has_X = X_dev != nullptr;
  b->has_v = v_dev != nullptr;
  b->has_y = y_dev != nullptr;
  const Schedule S = make_schedule(mprimes_of(count, plans), b->K, N, o);
  for (int k = 0; k < count; ++k) prods[k].part0 = S.part0[k];
  b->key_bytes = S.key_reads * 8.0 * 2 * b->beta * b->K * N;
  // algorithmic minimum: every distinct rotation key of the batch streamed once
  b->key_bytes_min = std::max(0, S.max_mp - 1) * 8.0 * 2 * b->beta * b->K * N;
  b->n_tasks = (int)S.tasks.size();
  b->n_slots = S.n_slots;
  b->n_work = (int)S.work.size();
  b->n_enc_work = (int)encw.size();
  const Layout L = make_layout(c, count, b->n_enc_work, S, b->lv, b->K, b->beta);
  if (!ws_dev) return fail(PVFL_E_INVALID, "the batch needs a workspace of pvfl_batch_workspace_bytes bytes");
  if (ws_bytes < L.total)
    return fail(PVFL_E_SHAPE, "workspace of " + std::to_string(ws_bytes) + " bytes, the batch needs " +
                                  std::to_string(L.total));
  if (((uintptr_t)ws_dev & 255) != 0) return fail(PVFL_E_INVALID, "the workspace must be 256-byte aligned");
  char* base = (char*)ws_dev;
  if ((st = upload(prods, base, L.prods)) != PVFL_OK) return st;
  if ((st = upload(apt, base, L.args_pt)) != PVFL_OK) return st;
  if ((st = upload(act, base, L.args_ct)) != PVFL_OK) return st;
  if ((st = upload(encw, base, L.enc_work)) != PVFL_OK) return st;
  if ((st = upload(S.groups, base, L.groups)) != PVFL_OK) return st;
  if ((st = upload(S.work, base, L.work)) != PVFL_OK) return st;
  if ((st = upload(S.tasks, base, L.tasks)) != PVFL_OK) return st;
  if ((st = upload(ct_tab, base, L.ct_tab)) != PVFL_OK) return st;
  if ((st = upload(ct_out_tab, base, L.ct_out_tab)) != PVFL_OK) return st;
  if ((st = upload(out_tab, base, L.out_tab)) != PVFL_OK) return st;
  b->prods = (BatchProd*)(base + L.prods);
  b->args_pt = (EncodeArgs*)(base + L.args_pt);
  b->args_ct = (EncodeArgs*)(base + L.args_ct);
  b->enc_work = (int2*)(base + L.enc_work);
  b->groups = (DiagGroup*)(base + L.groups);
  b->work = (DiagWork*)(base + L.work);
  b->tasks = (DiagTask*)(base + L.tasks);
  b->ct_tab = (const double**)(base + L.ct_tab);
  b->ct_out_tab = (double**)(base + L.ct_out_tab);
  b->out_tab = (double**)(base + L.out_tab);
  b->digits = (double*)(base + L.digits);
  b->yup = (double*)(base + L.yup);
  b->pc = (double*)(base + L.pc);
  b->part = (double*)(base + L.part);
  b->acc = (double*)(base + L.acc);
  b->ydown = (double*)(base + L.ydown);
  b->msg = (int64_t*)(base + L.msg);
  b->res = (double*)(base + L.res);
  b->z = (double*)(base + L.z);
  *out = b.release();
  return PVFL_OK;
}

extern "C" void pvfl_batch_destroy(pvfl_batch* b) { delete b; }

extern "C" pvfl_status pvfl_batch_encode(pvfl_batch* b, void* stream) {
  if (!b) return fail(PVFL_E_INVALID, "null argument");
  if (!b->has_X) return fail(PVFL_E_INVALID, "batch was created without plaintext matrices");
  pvfl_ctx* c = b->ctx;
  EncTabs et;
  CrtTabs crt;
  pvfl_status st = enc_tables_for(c, &et, &crt);
  if (st != PVFL_OK) return st;
  KernelTimer kt(c, stream, PVFL_TIMING_ENCODE, b->pt_bytes);
  HIP_TRY(launch_encode_pt_batch(launch_ctx(c, stream), b->args_pt, b->enc_work, b->n_enc_work, b->prods, et,
                                 qp_map(c, b->lv, true)));
  kt.stop();
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_batch_encrypt(pvfl_batch* b, const pvfl_sk* sk, uint64_t seed, void* stream) {
  if (!b || !sk) return fail(PVFL_E_INVALID, "null argument");
  if (!b->has_v) return fail(PVFL_E_INVALID, "batch was created without input vectors");
  pvfl_ctx* c = b->ctx;
  EncTabs et;
  CrtTabs crt;
  pvfl_status st = enc_tables_for(c, &et, &crt);
  if (st != PVFL_OK) return st;
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_encode_ct_batch(L, b->args_ct, b->count, et, b->msg));
  HIP_TRY(launch_encrypt(L, b->msg, b->count, sk->s, seed, b->lv, nullptr, b->ct_out_tab));
  return PVFL_OK;
}

// ModUp of every input ciphertext into digits, and P c0 (no plaintexts needed)
static pvfl_status batch_modup(pvfl_batch* b, void* stream) {
  pvfl_ctx* c = b->ctx;
  const int N = c->N, lv = b->lv, K = b->K;
  const size_t KN = (size_t)K * N, Q = (size_t)(lv + 1) * N;
  const KsLevel& kl = c->ks_host[lv];
  LaunchCtx L = launch_ctx(c, stream);
  {
    KernelTimer kt(c, stream, PVFL_TIMING_MODUP, 8.0 * (double)b->count * (Q + (size_t)b->beta * KN));
    HIP_TRY(launch_modup(L, nullptr, 0, b->count, lv, c->ks_dev + lv, kl.n_tasks, b->yup, b->digits,
                         (size_t)b->beta * KN, b->ct_tab));
    kt.stop();
  }
  HIP_TRY(launch_scale_by_p(L, nullptr, lv, N, c->pmod_dev, b->pc, b->count, b->ct_tab));
  return PVFL_OK;
}

// fused product over the digits and plaintexts, partial sums, ModDown
static pvfl_status batch_product(pvfl_batch* b, void* stream) {
  pvfl_ctx* c = b->ctx;
  const int N = c->N, lv = b->lv, K = b->K;
  const size_t KN = (size_t)K * N, Q = (size_t)(lv + 1) * N;
  LaunchCtx L = launch_ctx(c, stream);
  BatchDiagArgs a{};
  a.N = N;
  a.K = K;
  a.lv = lv;
  a.CH = b->CH;
  a.mods = c->tabs.mods;
  const LimbMap lp = qp_map(c, lv, true);
  for (int r = 0; r < K; ++r) a.limb_prime[r] = a.key_limb[r] = lp.idx[r];
  a.prods = b->prods;
  a.groups = b->groups;
  a.work = b->work;
  a.tasks = b->tasks;
  a.n_tasks = b->n_tasks;
  a.per_xcd = (b->n_tasks + 7) / 8;
  if (b->keys) {
    a.keys = b->keys->keys;
    a.key_limbs = b->keys->key_limbs;
    a.key_stride = b->keys->key_stride;
    a.slot_of_rot = b->keys->slot_of_rot_dev;
  }
  a.digits = b->digits;
  a.dig_stride = (size_t)b->beta * KN;
  a.pc = b->pc;
  a.pc_stride = 2 * Q;
  a.part = b->part;
  {
    // algorithmic bytes: each distinct rotation key once, every plaintext once, digits and P*c once,
    // and each product's 2K-limb accumulator written once (the chunk partial sums the kernel
    // writes instead are an intermediate of this kernel's own design, not counted)
    const double bytes = b->key_bytes_min + b->pt_bytes + 8.0 * (double)b->count * ((size_t)b->beta * KN + 2 * Q) +
                         8.0 * (double)b->count * 2 * KN;
    KernelTimer kt(c, stream, PVFL_TIMING_DIAG, bytes);
    HIP_TRY(launch_diag_batch(L, a, b->pg, b->beta, b->vec));
    kt.stop();
  }
  HIP_TRY(launch_sum_partials_batch(L, b->part, b->prods, b->count, b->CH, K, N, lp, b->acc));
  {
    KernelTimer kt(c, stream, PVFL_TIMING_MODDOWN, 8.0 * (double)b->count * (2 * KN + 2 * Q));
    HIP_TRY(launch_moddown(L, b->acc, 2 * b->count, lv, c->alpha, c->ks_dev + lv, b->ydown, nullptr, b->out_tab));
    kt.stop();
  }
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_batch_matmul(pvfl_batch* b, void* stream) {
  if (!b) return fail(PVFL_E_INVALID, "null argument");
  pvfl_status st = batch_modup(b, stream);
  return st != PVFL_OK ? st : batch_product(b, stream);
}

extern "C" pvfl_status pvfl_batch_decrypt(pvfl_batch* b, const pvfl_sk* sk, void* stream) {
  if (!b || !sk) return fail(PVFL_E_INVALID, "null argument");
  if (!b->has_y) return fail(PVFL_E_INVALID, "batch was created without result buffers");
  pvfl_ctx* c = b->ctx;
  EncTabs et;
  CrtTabs crt;
  pvfl_status st = enc_tables_for(c, &et, &crt);
  if (st != PVFL_OK) return st;
  LaunchCtx L = launch_ctx(c, stream);
  HIP_TRY(launch_decrypt_f64(L, nullptr, b->count, sk->s, b->lv, b->res, (const double* const*)b->out_tab));
  if (c->logN <= 14) {  // the slots never leave LDS
    HIP_TRY(launch_decode_readout_batch(L, b->res, b->count, b->lv, crt, et, b->inv_scale, b->args_ct, b->prods));
  } else {
    HIP_TRY(launch_decode(L, b->res, b->count, b->lv, crt, et, b->inv_scale, b->z));
    HIP_TRY(launch_readout_batch(L, b->z, b->args_ct, b->prods, b->count, b->max_rows, c->N / 2));
  }
  return PVFL_OK;
}

static pvfl_status run_phases(pvfl_batch* b, const pvfl_sk* sk, uint64_t seed, void* stream) {
  pvfl_status st;
  if ((st = pvfl_batch_encode(b, stream)) != PVFL_OK) return st;
  if ((st = pvfl_batch_encrypt(b, sk, seed, stream)) != PVFL_OK) return st;
  if ((st = pvfl_batch_matmul(b, stream)) != PVFL_OK) return st;
  return pvfl_batch_decrypt(b, sk, stream);
}

// The same phases as two branches: encryption and ModUp of the inputs on s2
// run beside the plaintext encode on s1 (they share no buffer); s1 waits for
// both before the fused product.
static pvfl_status run_phases_forked(pvfl_batch* b, const pvfl_sk* sk, uint64_t seed, hipStream_t s1, hipStream_t s2) {
  pvfl_status st;
  HIP_TRY(hipEventRecord(b->ev_fork, s1));
  HIP_TRY(hipStreamWaitEvent(s2, b->ev_fork, 0));
  if ((st = pvfl_batch_encrypt(b, sk, seed, s2)) != PVFL_OK) return st;
  if ((st = batch_modup(b, s2)) != PVFL_OK) return st;
  HIP_TRY(hipEventRecord(b->ev_join, s2));
  if ((st = pvfl_batch_encode(b, s1)) != PVFL_OK) return st;
  HIP_TRY(hipStreamWaitEvent(s1, b->ev_join, 0));
  if ((st = batch_product(b, s1)) != PVFL_OK) return st;
  return pvfl_batch_decrypt(b, sk, s1);
}

extern "C" pvfl_status pvfl_batch_run(pvfl_batch* b, const pvfl_sk* sk, uint64_t seed, int32_t use_graph,
                                      void* stream) {
  if (!b || !sk) return fail(PVFL_E_INVALID, "null argument");
  if (!use_graph) return run_phases(b, sk, seed, stream);
  if (!b->has_X || !b->has_v || !b->has_y) return fail(PVFL_E_INVALID, "batch was created without input/output buffers");
  if (!b->graph_exec || b->graph_sk != sk || b->graph_seed != seed) {
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
    pvfl_status st = enc_tables_for(b->ctx, nullptr, nullptr);  // tables are created outside the capture
    if (st != PVFL_OK) return st;
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    const bool timing = b->ctx->timing_on;
    b->ctx->timing_on = false;  // no event records inside the captured graph
    if (!b->cap_stream2) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream2, hipStreamNonBlocking));
    if (!b->ev_fork) HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    if (!b->ev_join) HIP_TRY(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    st = run_phases_forked(b, sk, seed, b->cap_stream, b->cap_stream2);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    b->ctx->timing_on = timing;
    if (st != PVFL_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
    b->graph_sk = sk;
    b->graph_seed = seed;
  }
  HIP_TRY(hipGraphLaunch(b->graph_exec, (hipStream_t)stream));
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_batch_info(const pvfl_batch* b, int64_t* n_work_items, double* key_bytes,
                                       double* pt_bytes) {
  if (!b) return fail(PVFL_E_INVALID, "null argument");
  if (n_work_items) *n_work_items = b->n_work;
  if (key_bytes) *key_bytes = b->key_bytes;
  if (pt_bytes) *pt_bytes = b->pt_bytes;
  return PVFL_OK;
}
