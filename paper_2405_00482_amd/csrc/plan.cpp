// Plans of the packed-HE matrix product and their execution.
//
// HYBRID (Sec. 4): Eq. 5 diagonals applied blockwise to the Eq. 6 packed
// matrix, input partitioning when m or n exceed N' = N/2 slots, lazy
// rotate-and-sum after decryption.  With m, n zero-padded to powers of two
// (Sec. 3) and S = N':
//   bm = min(m, S), bn = min(n, S), m' = max(1, bm bn / S), G = S / bn,
//   row blocks m/S (outputs), column blocks n/S (inputs, summed),
//   diagonal i < m' of block (b, c) at slot g bn + j holds
//   X[b S + g m' + (j mod m'), c S + (i + j) mod bn].
// DIAG (Sec. 4.1): Eq. 5 alone, min(m,n) diagonals over max(m,n) slots, with
// the final rotate-and-sum either inside the ciphertext (O3) or lazy.
// ROW (Sec. 3.1): per row, Mult, log2 n rotate-and-sum steps, indicator,
// placement rotation, two rescales.
// CTMAT (Alg. 3): the encrypted matrix arrives as its Eq. 5 diagonals; each
// output is sum_i [[e_i]] * w_i with no rotation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>

#include "capi_internal.hpp"

using namespace pvfl;

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return hip_fail(_e, #expr);          \
  } while (0)

static int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
static int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

pvfl_plan::~pvfl_plan() {
  if (iota_dev) (void)hipFree(iota_dev);
  if (rot_dev) (void)hipFree(rot_dev);
}

static uint32_t galois_rotl(int i, int N) {
  const int half = N / 2;
  i = ((i % half) + half) % half;
  uint64_t g = 1;
  for (int k = 0; k < i; ++k) g = g * 5 % (2 * (uint64_t)N);
  return (uint32_t)g;
}

extern "C" pvfl_status pvfl_plan_create(pvfl_ctx* c, const pvfl_plan_opts* o, pvfl_plan** out) {
  if (!c || !o || !out) return fail(PVFL_E_INVALID, "null argument");
  *out = nullptr;
  if (o->m < 1 || o->n < 1) return fail(PVFL_E_SHAPE, "m and n must be positive");
  std::unique_ptr<pvfl_plan> p(new pvfl_plan());
  p->ctx = c;
  p->opts = *o;
  const int N = c->N, S = N / 2;
  const int lv = o->level < 0 ? c->n_q - 1 : o->level;
  if (lv >= c->n_q) return fail(PVFL_E_LEVEL, "level out of range");
  p->lv = lv;
  p->K = lv + 1 + c->alpha;
  p->beta = (lv + 1 + c->alpha - 1) / c->alpha;
  p->pt_scale = std::ldexp(1.0, 0) * std::pow(2.0, o->pt_log2_scale > 0 ? o->pt_log2_scale : c->log2_scale);
  pvfl_plan_info& I = p->info;
  std::memset(&I, 0, sizeof(I));
  I.kind = o->kind;
  I.m = o->m;
  I.n = o->n;
  I.n_out = o->n_out;
  I.m_pad = pow2_ceil(o->m);
  I.n_pad = pow2_ceil(o->n);
  I.in_level = lv;
  I.out_level = lv;
  const double lds = c->log2_scale + std::log2(p->pt_scale);
  I.out_log2_scale = lds;
  const bool lazy = o->lazy_moddown != 0;
  if (o->bsgs != 0 && o->kind != PVFL_PLAN_HYBRID) return fail(PVFL_E_PLAN, "bsgs applies to HYBRID plans only");
  const bool o3 = o->unhoisted != 0;
  if (o3 && o->kind != PVFL_PLAN_HYBRID && o->kind != PVFL_PLAN_DIAG)
    return fail(PVFL_E_PLAN, "unhoisted rotations apply to HYBRID and DIAG plans only");
  if (o3 && (lazy || o->bsgs != 0))
    return fail(PVFL_E_PLAN, "unhoisted rotations need per-rotation ModDown and no baby-step/giant-step split");
  switch (o->kind) {
    case PVFL_PLAN_HYBRID: {
      const int mp = I.m_pad, np = I.n_pad;
      I.row_blocks = std::max(1, mp / S);
      I.col_blocks = std::max(1, np / S);
      p->bm = std::min(mp, S);
      p->bn = std::min(np, S);
      I.mprime = std::max(1, (int)((int64_t)p->bm * p->bn / S));
      I.groups = S / p->bn;
      for (int b = 0; b < I.row_blocks; ++b)
        for (int cb = 0; cb < I.col_blocks; ++cb)
          for (int i = 0; i < I.mprime; ++i)
            p->terms.push_back(Term{cb, i, (b * I.col_blocks + cb) * I.mprime + i, b});
      I.n_pts = (int)p->terms.size();
      I.ct_in = I.col_blocks;
      I.ct_out = I.row_blocks;
      I.n_mult = I.n_pts;
      I.n_add = I.n_pts - I.row_blocks;
      if (o->bsgs != 0) {
        const int bs = o->bsgs;
        if (!lazy) return fail(PVFL_E_PLAN, "the baby-step/giant-step schedule needs lazy ModDown");
        if (bs < 2 || (bs & (bs - 1)) != 0 || 2 * bs > I.mprime)
          return fail(PVFL_E_PLAN, "bsgs must be a power of two with 2 <= bsgs <= m'/2");
        const int g = I.mprime / bs;
        for (int k = 1; k < bs; ++k) p->galois.push_back(galois_rotl(k, N));
        for (int j = 1; j < g; ++j) p->galois.push_back(galois_rotl(j * bs, N));
        I.bsgs = bs;
        I.n_hstrot = (int64_t)I.col_blocks * (bs - 1);
        I.n_rot = (int64_t)I.row_blocks * I.col_blocks * (g - 1);
        I.n_modup = I.col_blocks + (int)I.n_rot;
        I.n_moddown = I.row_blocks * I.col_blocks * g + (int)I.n_rot;
      } else if (o3) {
        // every (row block, column block, diagonal i > 0) term rotates its input ciphertext by i
        for (int i = 1; i < I.mprime; ++i) p->galois.push_back(galois_rotl(i, N));
        I.n_rot = (int64_t)I.row_blocks * I.col_blocks * (I.mprime - 1);
        I.n_hstrot = 0;
        I.n_modup = I.n_moddown = (int)I.n_rot;
      } else {
        for (int i = 1; i < I.mprime; ++i) p->galois.push_back(galois_rotl(i, N));
        I.n_rot = 0;
        I.n_hstrot = (int64_t)I.col_blocks * (I.mprime - 1);
        I.n_modup = I.mprime > 1 ? I.col_blocks : 0;
        I.n_moddown = lazy ? (I.mprime > 1 || c->alpha > 1 ? I.row_blocks : 0) : (int)I.n_hstrot * I.row_blocks;
      }
      break;
    }
    case PVFL_PLAN_DIAG: {
      const int mp = I.m_pad, np = I.n_pad;
      if (mp > S || np > S) return fail(PVFL_E_SHAPE, "DIAG needs m, n <= N/2 (no partitioning)");
      const int nd = std::min(mp, np);
      I.mprime = nd;
      I.groups = 1;
      I.row_blocks = I.col_blocks = 1;
      p->bm = mp;
      p->bn = np;
      for (int i = 0; i < nd; ++i) p->terms.push_back(Term{0, i, i, 0});
      I.n_pts = nd;
      I.ct_in = I.ct_out = 1;
      for (int i = 1; i < nd; ++i) p->galois.push_back(galois_rotl(i, N));
      if (mp < np && o->ras_in_ct)
        for (int k = mp; k < np; k *= 2) {
          p->ras_rots.push_back(k);
          p->galois.push_back(galois_rotl(k, N));
        }
      I.n_mult = nd;
      I.n_rot = (int64_t)p->ras_rots.size();
      I.n_add = nd - 1 + I.n_rot;
      I.n_hstrot = nd - 1;
      I.n_modup = (nd > 1 ? 1 : 0) + (int)I.n_rot;
      I.n_moddown = (lazy ? (nd > 1 || c->alpha > 1 ? 1 : 0) : nd - 1) + (int)I.n_rot;
      if (o3) {  // Table 2, GALA's diagonal: the nd - 1 diagonal rotations become O3
        I.n_rot += nd - 1;
        I.n_hstrot = 0;
        I.n_modup = I.n_moddown = (int)I.n_rot;
      }
      break;
    }
    case PVFL_PLAN_ROW: {
      const int np = I.n_pad;
      if (np > S || o->m > S) return fail(PVFL_E_SHAPE, "ROW needs m, n <= N/2");
      if (lv < 2) return fail(PVFL_E_LEVEL, "ROW consumes two levels (two rescales)");
      I.mprime = 1;
      I.row_blocks = I.col_blocks = 1;
      I.n_pts = o->m + 1;  // one row plaintext per row, then the indicator
      I.ct_in = I.ct_out = 1;
      const int logn = ilog2(np);
      for (int k = 0; k < logn; ++k) p->ras_rots.push_back(1 << k);
      for (int k : p->ras_rots) p->galois.push_back(galois_rotl(k, N));
      for (int r = 1; r < o->m; ++r) p->galois.push_back(galois_rotl(-r, N));
      I.n_mult = 2 * (int64_t)o->m;
      I.n_rot = (int64_t)o->m * logn + o->m - 1;
      I.n_add = I.n_rot;
      I.n_hstrot = 0;
      I.n_modup = I.n_moddown = (int)I.n_rot;
      I.out_level = lv - 2;
      I.out_log2_scale = lds - std::log2((double)c->primes[lv]);
      break;
    }
    case PVFL_PLAN_COL: {
      // row blocks of N/2 rows; input ciphertext j carries y_j in every slot
      if (o->n > 65536) return fail(PVFL_E_SHAPE, "COL sends one ciphertext per column: n <= 65536");
      I.mprime = 1;
      I.row_blocks = std::max(1, (I.m_pad + S - 1) / S);
      I.col_blocks = 1;
      p->bm = std::min(I.m_pad, S);
      p->bn = I.n_pad;
      I.ct_in = o->n;
      I.ct_out = I.row_blocks;
      I.n_pts = I.ct_in * I.ct_out;
      I.n_mult = I.n_pts;
      I.n_add = (int64_t)(o->n - 1) * I.row_blocks;
      break;
    }
    case PVFL_PLAN_CTMAT: {
      const int mp = I.m_pad, np = I.n_pad;
      const int width = std::max(mp, np);
      const int pack = std::max(1, o->pack);
      if (o->n_out < 1) return fail(PVFL_E_SHAPE, "CTMAT needs n_out >= 1");
      if ((int64_t)width * pack > S) return fail(PVFL_E_SHAPE, "CTMAT needs pack * max(m,n) <= N/2");
      I.mprime = std::min(mp, np);
      I.groups = pack;
      I.row_blocks = I.col_blocks = 1;
      I.ct_in = I.mprime;
      I.ct_out = (o->n_out + pack - 1) / pack;
      I.n_pts = I.ct_in * I.ct_out;
      p->bm = mp;
      p->bn = np;
      I.n_mult = I.n_pts;
      I.n_add = I.n_pts - I.ct_out;
      break;
    }
    default:
      return fail(PVFL_E_PLAN, "unknown plan kind");
  }
  std::sort(p->galois.begin(), p->galois.end());
  p->galois.erase(std::unique(p->galois.begin(), p->galois.end()), p->galois.end());
  I.n_galois = (int)p->galois.size();
  I.pt_limbs = (lazy && (o->kind == PVFL_PLAN_HYBRID || o->kind == PVFL_PLAN_DIAG)) ? p->K : lv + 1;
  // fused-kernel chunking: aim for >= 4096 workgroups per launch
  const int mprime = std::max(1, I.mprime);
  const int per_chunk = (N / 256) * p->K;
  int target = std::max(1, std::min(64, 4096 / std::max(1, per_chunk)));
  p->chunk = std::max(1, (mprime + target - 1) / target);
  p->nchunk = (mprime + p->chunk - 1) / p->chunk;
  std::vector<int> iota(mprime);
  for (int i = 0; i < mprime; ++i) iota[i] = i;
  if (hipMalloc((void**)&p->iota_dev, sizeof(int) * mprime) != hipSuccess) return fail(PVFL_E_NOMEM, "plan tables");
  HIP_TRY(hipMemcpy(p->iota_dev, iota.data(), sizeof(int) * mprime, hipMemcpyHostToDevice));
  if (I.bsgs) {
    // chunks never straddle a giant step; enough of them to fill the chip
    const int g = mprime / I.bsgs;
    int per = 1;
    while (per < I.bsgs && (int64_t)g * per < target) per *= 2;
    p->chunks_per_giant = per;
    p->chunk = I.bsgs / per;
    p->nchunk = g * per;
    for (int i = 0; i < mprime; ++i) iota[i] = i % I.bsgs;
    if (hipMalloc((void**)&p->rot_dev, sizeof(int) * mprime) != hipSuccess) return fail(PVFL_E_NOMEM, "plan tables");
    HIP_TRY(hipMemcpy(p->rot_dev, iota.data(), sizeof(int) * mprime, hipMemcpyHostToDevice));
  }
  *out = p.release();
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_plan_get_info(const pvfl_plan* p, pvfl_plan_info* out) {
  if (!p || !out) return fail(PVFL_E_INVALID, "null argument");
  *out = p->info;
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_plan_galois(const pvfl_plan* p, uint32_t* out, int32_t cap) {
  if (!p || (!out && cap > 0)) return fail(PVFL_E_INVALID, "null argument");
  if (cap < (int)p->galois.size()) return fail(PVFL_E_INVALID, "output too small");
  std::copy(p->galois.begin(), p->galois.end(), out);
  return PVFL_OK;
}

extern "C" void pvfl_plan_destroy(pvfl_plan* p) { delete p; }

extern "C" size_t pvfl_bytes_ct_in(const pvfl_plan* p) {
  return p ? sizeof(double) * 2 * (size_t)(p->lv + 1) * p->ctx->N * p->info.ct_in : 0;
}
extern "C" size_t pvfl_bytes_ct_out(const pvfl_plan* p) {
  return p ? sizeof(double) * 2 * (size_t)(p->info.out_level + 1) * p->ctx->N * p->info.ct_out : 0;
}
extern "C" size_t pvfl_bytes_pt(const pvfl_plan* p) {
  return p ? sizeof(double) * (size_t)p->info.pt_limbs * p->ctx->N * p->info.n_pts : 0;
}

// workspace layout (doubles), per plan kind
static size_t ws_doubles(const pvfl_plan* p, int count = 1) {
  const pvfl_ctx* c = p->ctx;
  const size_t N = c->N, Q = (size_t)(p->lv + 1) * N, KN = (size_t)p->K * N;
  const size_t digits = (size_t)p->beta * KN;
  const size_t ydown = 2 * (size_t)c->alpha * N;
  switch (p->opts.kind) {
    case PVFL_PLAN_HYBRID:
    case PVFL_PLAN_DIAG:
      if (p->opts.lazy_moddown) {
        // every term (count of them) brings col_blocks input ciphertexts
        const size_t CB = (size_t)count * p->info.col_blocks, g = p->info.bsgs ? p->nchunk / p->chunks_per_giant : 1;
        const size_t bsgs = p->info.bsgs ? g * 2 * Q + digits + 2 * Q + Q : 0;
        // + 4Q at the end: in-ciphertext RaS temporaries
        return CB * digits + Q + CB * 2 * Q + CB * p->nchunk * 2 * KN + g * 2 * KN + g * ydown + bsgs + 4 * Q;
      }
      // + Q: the rotated c1 of an unhoisted rotation; + 4Q at the end: in-ciphertext RaS temporaries
      return digits + Q + 2 * KN + ydown + 2 * Q + Q + 4 * Q;
    case PVFL_PLAN_ROW:
      return 8 * Q;
    case PVFL_PLAN_CTMAT:
    case PVFL_PLAN_COL:
      return 0;
  }
  return 0;
}
extern "C" size_t pvfl_bytes_workspace(const pvfl_plan* p) { return p ? sizeof(double) * std::max<size_t>(ws_doubles(p), 1) : 0; }
extern "C" size_t pvfl_bytes_workspace_sum(const pvfl_plan* p, int32_t count) {
  return p && count >= 1 ? sizeof(double) * std::max<size_t>(ws_doubles(p, count), 1) : 0;
}

// the caller's workspace (plans with no workspace -- CTMAT, COL -- take NULL)
static pvfl_status get_ws(const pvfl_plan* p, void* ws, size_t ws_bytes, double** out, int count = 1) {
  *out = (double*)ws;
  if (ws_doubles(p, count) == 0) return PVFL_OK;
  const size_t need = pvfl_bytes_workspace_sum(p, count);
  if (!ws) return fail(PVFL_E_INVALID, "the plan needs a workspace of " + std::to_string(need) + " bytes");
  if (ws_bytes < need) return fail(PVFL_E_SHAPE, "workspace too small");
  return PVFL_OK;
}

static pvfl_status check_keys(const pvfl_plan* p, const pvfl_rotkeys* keys) {
  if (p->galois.empty()) return PVFL_OK;
  if (!keys) return fail(PVFL_E_NOKEY, "plan needs rotation keys");
  if (keys->ctx != p->ctx) return fail(PVFL_E_INVALID, "keys belong to another context");
  for (uint32_t g : p->galois)
    if (keys->slot_of_rot[p->ctx->log5[g]] < 0)
      return fail(PVFL_E_NOKEY, "missing rotation key for Galois element " + std::to_string(g));
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// diagonal products (HYBRID, DIAG)
// ---------------------------------------------------------------------------
// `count` terms, each an input ciphertext set cts[k] and its plaintexts pts[k]
// laid out by the plan, summed over Q u P before the ModDown (count > 1: Eq. 4)
static pvfl_status run_diag_lazy(const pvfl_plan* p, int count, const double* const* cts, const double* const* ptss,
                                 const pvfl_rotkeys* keys, double* out, double* ws, void* stream) {
  pvfl_ctx* c = p->ctx;
  const int N = c->N, lv = p->lv, K = p->K;
  const int CB1 = p->info.col_blocks, CB = count * CB1, RB = p->info.row_blocks;
  const int bs = p->info.bsgs, g = bs ? p->nchunk / p->chunks_per_giant : 1;
  const size_t Q = (size_t)(lv + 1) * N, KN = (size_t)K * N, DG = (size_t)p->beta * KN;
  const KsLevel& kl = c->ks_host[lv];
  // workspace, in the order ws_doubles counts it
  // input x = k * CB1 + cb: column block cb of term k
  auto ct_of = [&](int x) { return cts[x / CB1] + (size_t)(x % CB1) * 2 * (lv + 1) * N; };
  auto pt_of = [&](int b, int x) {
    return ptss[x / CB1] + (size_t)(b * CB1 + x % CB1) * std::max(1, p->info.mprime) * K * N;
  };
  double* digits = ws;                                  // [CB][beta][K][N]
  double* yup = digits + CB * DG;                       // [lv+1][N]
  double* pc = yup + Q;                                 // [CB][2][lv+1][N]: P*c of every input
  double* part = pc + CB * 2 * Q;                       // [CB][nchunk][2][K][N]
  double* acc = part + (size_t)CB * p->nchunk * 2 * KN; // [g][2][K][N]
  double* ydown = acc + (size_t)g * 2 * KN;             // [2g][alpha][N]
  double* cj = ydown + (size_t)2 * g * c->alpha * N;    // BSGS: [g][2][lv+1][N] giant-step inner sums
  double* dig2 = cj + (bs ? g * 2 * Q : 0);             // BSGS: digits of one inner sum
  double* v = dig2 + (bs ? DG : 0);                     // BSGS: key-switched part [2][lv+1][N]
  double* rct = v + (bs ? 2 * Q : 0);                   // BSGS: phi(c0) [lv+1][N]
  LaunchCtx L = launch_ctx(c, stream);
  const int mprime = p->info.mprime;
  if (mprime == 1 && c->alpha == 1) {
    // no rotation and one special prime: ModDown(P * c * pt) is c * pt exactly
    // (the base conversion of a single residue is exact), so skip Q u P; the
    // Q limbs of a Q u P plaintext come first.  With alpha > 1 the fast base
    // conversion may add P, and the Q u P form's result differs by one.
    for (int b = 0; b < RB; ++b) {
      double* ob = out + (size_t)b * 2 * Q;
      HIP_TRY(launch_fill_zero(L, ob, 2 * Q));
      for (int cb = 0; cb < CB; ++cb) {
        const double* ct = ct_of(cb);
        HIP_TRY(launch_eager_term(L, ct, ct + Q, nullptr, 0, pt_of(b, cb), lv, N, ob));
      }
    }
    return PVFL_OK;
  }
  // one ModUp and one P*c per input ciphertext, shared by every row block
  for (int cb = 0; cb < CB; ++cb) {
    const double* ct = ct_of(cb);
    if (mprime > 1) {
      KernelTimer kt(c, stream, PVFL_TIMING_MODUP, 8.0 * (double)(Q + DG));
      HIP_TRY(launch_modup(L, ct, 0, 1, lv, c->ks_dev + lv, kl.n_tasks, yup, digits + cb * DG, 0));
      kt.stop();
    }
    HIP_TRY(launch_scale_by_p(L, ct, lv, N, c->pmod_dev, pc + cb * 2 * Q));
  }
  DiagArgs a{};
  a.N = N;
  a.K = K;
  a.lv = lv;
  a.beta = p->beta;
  a.mprime = mprime;
  a.chunk = p->chunk;
  a.mods = c->tabs.mods;
  const LimbMap lp = qp_map(c, lv, true);
  const LimbMap qm = qp_map(c, lv, false);
  for (int r = 0; r < K; ++r) {
    a.limb_prime[r] = lp.idx[r];
    a.key_limb[r] = lp.idx[r];
  }
  a.pt_index = p->iota_dev;
  a.rot = bs ? p->rot_dev : p->iota_dev;
  if (keys) {
    a.keys = keys->keys;
    a.key_limbs = keys->key_limbs;
    a.key_stride = keys->key_stride;
    a.slot_of_rot = keys->slot_of_rot_dev;
  }
  // algorithmic bytes of one fused launch: every key and plaintext limb once,
  // digits and P*c once, partials written
  const int n_keys = bs ? bs - 1 : mprime - 1;
  const double diag_bytes = 8.0 * ((double)n_keys * 2 * p->beta * KN + (double)mprime * KN + (double)DG + 2.0 * Q +
                                   (double)p->nchunk * 2 * KN);
  for (int b = 0; b < RB; ++b) {
    double* ob = out + (size_t)b * 2 * Q;
    if (bs) HIP_TRY(launch_fill_zero(L, ob, 2 * Q));
    int z = 0;
    for (int cb = 0; cb < CB; ++cb) {
      a.digits = digits + cb * DG;
      a.pc = pc + cb * 2 * Q;
      a.pt = pt_of(b, cb);
      a.part = part + (size_t)z * 2 * KN;
      {
        KernelTimer kt(c, stream, PVFL_TIMING_DIAG, diag_bytes);
        HIP_TRY(launch_diag_lazy(L, a, p->nchunk));
        kt.stop();
      }
      if (!bs) {
        z += p->nchunk;
        continue;
      }
      // every giant step's inner sum (its chunks added) down to Q at once, then
      // rotated by j*bs and added
      HIP_TRY(launch_sum_partials(L, a.part, p->chunks_per_giant, K, N, lp, acc, g));
      {
        KernelTimer kt(c, stream, PVFL_TIMING_MODDOWN, 8.0 * (double)g * (2 * KN + 2 * Q));
        HIP_TRY(launch_moddown(L, acc, 2 * g, lv, c->alpha, c->ks_dev + lv, ydown, cj));
        kt.stop();
      }
      HIP_TRY(launch_add_limbs(L, ob, cj, 2 * (lv + 1), N, qm, ob));
      for (int j = 1; j < g; ++j) {
        const double* cjj = cj + (size_t)j * 2 * Q;
        const int rot = j * bs;
        HIP_TRY(launch_modup(L, cjj, 0, 1, lv, c->ks_dev + lv, kl.n_tasks, yup, dig2, 0));
        pvfl_status st = keyswitch_digits(c, keys, lv, dig2, rot, rot, acc, ydown, v, stream);  // acc reused: summed above
        if (st != PVFL_OK) return st;
        HIP_TRY(launch_automorph(L, cjj, lv + 1, N, rot, rct));
        HIP_TRY(launch_add_limbs(L, ob, rct, lv + 1, N, qm, ob));
        HIP_TRY(launch_add_limbs(L, ob, v, 2 * (lv + 1), N, qm, ob));
      }
    }
    if (bs) continue;
    HIP_TRY(launch_sum_partials(L, part, z, K, N, lp, acc));
    {
      KernelTimer kt(c, stream, PVFL_TIMING_MODDOWN, 8.0 * (double)(2 * KN + 2 * Q));
      HIP_TRY(launch_moddown(L, acc, 2, lv, c->alpha, c->ks_dev + lv, ydown, ob));
      kt.stop();
    }
  }
  return PVFL_OK;
}

static pvfl_status run_diag_eager(const pvfl_plan* p, const double* ct_in, const double* pts, const pvfl_rotkeys* keys,
                                  double* out, double* ws, void* stream) {
  pvfl_ctx* c = p->ctx;
  const int N = c->N, lv = p->lv, K = p->K;
  const size_t Q = (size_t)(lv + 1) * N, KN = (size_t)K * N;
  const KsLevel& kl = c->ks_host[lv];
  double* digits = ws;
  double* yup = digits + (size_t)p->beta * KN;
  double* u = yup + Q;
  double* ydown = u + 2 * KN;
  double* v = ydown + 2 * (size_t)c->alpha * N;
  // an unhoisted rotation's phi_i(c1) sits at rct + Q = v + 2Q, past v: ModUp reads
  // only the c1 half of the ciphertext it is given
  double* rct = v + Q;
  LaunchCtx L = launch_ctx(c, stream);
  const int mprime = p->info.mprime;
  const bool o3 = p->opts.unhoisted != 0;
  for (int b = 0; b < p->info.row_blocks; ++b) {
    double* acc = out + (size_t)b * 2 * Q;
    HIP_TRY(launch_fill_zero(L, acc, 2 * Q));
    for (int cb = 0; cb < p->info.col_blocks; ++cb) {
      const double* ct = ct_in + (size_t)cb * 2 * Q;
      if (mprime > 1 && !o3) HIP_TRY(launch_modup(L, ct, 0, 1, lv, c->ks_dev + lv, kl.n_tasks, yup, digits, 0));
      for (int i = 0; i < mprime; ++i) {
        const double* pt = pts + ((size_t)(b * p->info.col_blocks + cb) * mprime + i) * Q;
        if (i == 0) {
          HIP_TRY(launch_eager_term(L, ct, ct + Q, nullptr, 0, pt, lv, N, acc));
        } else {
          if (o3) {
            // O3: the automorphism first, then this rotation's own ModUp (Sec. 2)
            HIP_TRY(launch_automorph(L, ct + Q, lv + 1, N, i, rct + Q));
            HIP_TRY(launch_modup(L, rct, 0, 1, lv, c->ks_dev + lv, kl.n_tasks, yup, digits, 0));
          }
          pvfl_status st = keyswitch_digits(c, keys, lv, digits, o3 ? 0 : i, i, u, ydown, v, stream);
          if (st != PVFL_OK) return st;
          HIP_TRY(launch_eager_term(L, ct, nullptr, v, i, pt, lv, N, acc));
        }
      }
    }
  }
  return PVFL_OK;
}

// in-ciphertext rotate-and-sum (DIAG, m < n): ct += RotL(ct, k) for each k
static pvfl_status run_ras_in_ct(const pvfl_plan* p, const pvfl_rotkeys* keys, double* ct, double* tmp, void* stream) {
  pvfl_ctx* c = p->ctx;
  const size_t Q = (size_t)(p->lv + 1) * c->N;
  for (int k : p->ras_rots) {
    pvfl_status st = pvfl_rotate(c, keys, p->lv, ct, galois_rotl(k, c->N), 0, tmp, stream);
    if (st != PVFL_OK) return st;
    HIP_TRY(launch_ct_add(launch_ctx(c, stream), ct, tmp, p->lv, c->N, ct));
  }
  (void)Q;
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// ROW (Sec. 3.1)
// ---------------------------------------------------------------------------
static pvfl_status run_row(const pvfl_plan* p, const double* ct, const double* pts, const pvfl_rotkeys* keys,
                           double* out, double* ws, void* stream) {
  pvfl_ctx* c = p->ctx;
  const int N = c->N, lv = p->lv;
  const size_t Q2 = (size_t)(lv + 1) * N, Q1 = (size_t)lv * N, Q0 = (size_t)(lv - 1) * N;
  double* t2 = ws;              // product at lv
  double* t1 = t2 + 2 * Q2;     // after the first rescale (lv - 1)
  double* r1 = t1 + 2 * Q2;     // rotation temporary
  double* t0 = r1 + 2 * Q2;     // after the indicator rescale (lv - 2)
  LaunchCtx L = launch_ctx(c, stream);
  const int m = p->info.m;
  const double* ind = pts + (size_t)m * Q2;  // indicator plaintext (level lv - 1 limbs used)
  HIP_TRY(launch_fill_zero(L, out, 2 * Q0));
  pvfl_status st;
  for (int r = 0; r < m; ++r) {
    HIP_TRY(launch_ct_mul_pt(L, ct, pts + (size_t)r * Q2, lv, N, t2));
    HIP_TRY(launch_rescale(L, t2, 2, lv, c->rescale[lv], t1));
    for (int k : p->ras_rots) {
      if ((st = pvfl_rotate(c, keys, lv - 1, t1, galois_rotl(k, N), 0, r1, stream)) != PVFL_OK) return st;
      HIP_TRY(launch_ct_add(L, t1, r1, lv - 1, N, t1));
    }
    // the indicator plaintext is stored with lv+1 limbs; its first lv are used here
    HIP_TRY(launch_ct_mul_pt(L, t1, ind, lv - 1, N, r1));
    HIP_TRY(launch_rescale(L, r1, 2, lv - 1, c->rescale[lv - 1], t0));
    if (r > 0) {
      if ((st = pvfl_rotate(c, keys, lv - 2, t0, galois_rotl(-r, N), 0, r1, stream)) != PVFL_OK) return st;
      HIP_TRY(launch_ct_add(L, out, r1, lv - 2, N, out));
    } else {
      HIP_TRY(launch_ct_add(L, out, t0, lv - 2, N, out));
    }
  }
  (void)Q1;
  return PVFL_OK;
}

// ---------------------------------------------------------------------------
// entry point
// ---------------------------------------------------------------------------
extern "C" pvfl_status pvfl_matmul_ct_pt(const pvfl_plan* p, const void* ct_v, const void* pt_v,
                                         const pvfl_rotkeys* keys, void* out_v, void* ws_v, size_t ws_bytes,
                                         void* stream) {
  if (!p || !ct_v || !pt_v || !out_v) return fail(PVFL_E_INVALID, "null argument");
  pvfl_status st = check_keys(p, keys);
  if (st != PVFL_OK) return st;
  double* ws = nullptr;
  if ((st = get_ws(p, ws_v, ws_bytes, &ws)) != PVFL_OK) return st;
  const double* ct = (const double*)ct_v;
  const double* pt = (const double*)pt_v;
  double* out = (double*)out_v;
  switch (p->opts.kind) {
    case PVFL_PLAN_HYBRID:
    case PVFL_PLAN_DIAG: {
      st = p->opts.lazy_moddown ? run_diag_lazy(p, 1, &ct, &pt, keys, out, ws, stream)
                                : run_diag_eager(p, ct, pt, keys, out, ws, stream);
      if (st != PVFL_OK) return st;
      if (p->opts.kind == PVFL_PLAN_DIAG && !p->ras_rots.empty()) {
        const size_t Q = (size_t)(p->lv + 1) * p->ctx->N;
        double* tmp = ws + ws_doubles(p) - 4 * Q;
        return run_ras_in_ct(p, keys, out, tmp, stream);
      }
      return PVFL_OK;
    }
    case PVFL_PLAN_ROW:
      return run_row(p, ct, pt, keys, out, ws, stream);
    case PVFL_PLAN_CTMAT:
    case PVFL_PLAN_COL: {
      // both are out[k] = sum_i ct[i] * pt[i][k] (COL: i = column j, k = row block)
      LaunchCtx L = launch_ctx(p->ctx, stream);
      HIP_TRY(launch_ctmat(L, ct, pt, p->info.ct_in, p->info.ct_out, p->lv, p->ctx->N, out));
      return PVFL_OK;
    }
  }
  return fail(PVFL_E_PLAN, "unknown plan kind");
}

// ---------------------------------------------------------------------------
// The allocation-free product.  Its workspace is a fixed array in device
// memory: each device the library runs on holds one copy for the life of the
// process.  In host code `scratch` only names the symbol; the address of a
// device's copy comes from hipGetSymbolAddress, looked up once per device when
// a context is created there, and only that address reaches kernels.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocBytes = size_t(64) << 20;
static constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kNoAllocDevices] = {};

namespace pvfl {
// with `device` current (pvfl_context_create)
pvfl_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoAllocDevices) return fail(PVFL_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return PVFL_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_scratch_dev[device] = (double*)ptr;
  return PVFL_OK;
}
}  // namespace pvfl

extern "C" size_t pvfl_noalloc_max_bytes(void) { return kNoAllocBytes; }

extern "C" pvfl_status pvfl_matmul_ct_pt_noalloc(const pvfl_plan* p, const void* ct_v, const void* pt_v,
                                                 const pvfl_rotkeys* keys, void* out_v, void* stream) {
  if (!p || !ct_v || !pt_v || !out_v) return fail(PVFL_E_INVALID, "null argument");
  if (p->opts.kind == PVFL_PLAN_ROW || (p->opts.kind == PVFL_PLAN_DIAG && !p->ras_rots.empty()))
    return fail(PVFL_E_PLAN, "the allocation-free product takes HYBRID, DIAG (lazy rotate-and-sum), CTMAT and COL "
                             "plans; ROW and in-ciphertext rotate-and-sum run single rotations with their own scratch");
  const size_t need = ws_doubles(p) * sizeof(double);
  if (need > kNoAllocBytes)
    return fail(PVFL_E_SHAPE, "the plan's workspace (" + std::to_string(need) + " bytes) exceeds the " +
                                  std::to_string(kNoAllocBytes) + "-byte fixed scratch array; use pvfl_matmul_ct_pt");
  pvfl_status st = check_keys(p, keys);
  if (st != PVFL_OK) return st;
  const int dev = p->ctx->device;
  double* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ws = (dev >= 0 && dev < kNoAllocDevices) ? g_scratch_dev[dev] : nullptr;
  }
  if (!ws) return fail(PVFL_E_DEVICE, "no scratch address for the plan's device");
  const double* ct = (const double*)ct_v;
  const double* pt = (const double*)pt_v;
  double* out = (double*)out_v;
  t_timing_off = true;
  switch (p->opts.kind) {
    case PVFL_PLAN_HYBRID:
    case PVFL_PLAN_DIAG:
      st = p->opts.lazy_moddown ? run_diag_lazy(p, 1, &ct, &pt, keys, out, ws, stream)
                                : run_diag_eager(p, ct, pt, keys, out, ws, stream);
      break;
    default: {
      LaunchCtx L = launch_ctx(p->ctx, stream);
      const hipError_t e = launch_ctmat(L, ct, pt, p->info.ct_in, p->info.ct_out, p->lv, p->ctx->N, out);
      st = e == hipSuccess ? PVFL_OK : hip_fail(e, "launch_ctmat");
    }
  }
  t_timing_off = false;
  return st;
}

// Eq. 4: the terms of one layout summed over Q u P, one ModDown per output
extern "C" pvfl_status pvfl_matmul_ct_pt_sum(const pvfl_plan* p, int32_t count, const void* const* cts_v,
                                             const void* const* pts_v, const pvfl_rotkeys* keys, void* out_v,
                                             void* ws_v, size_t ws_bytes, void* stream) {
  if (!p || !cts_v || !pts_v || !out_v) return fail(PVFL_E_INVALID, "null argument");
  if (count < 1) return fail(PVFL_E_INVALID, "count must be positive");
  if ((p->opts.kind != PVFL_PLAN_HYBRID && p->opts.kind != PVFL_PLAN_DIAG) || !p->opts.lazy_moddown ||
      p->info.bsgs != 0 || (p->opts.kind == PVFL_PLAN_DIAG && !p->ras_rots.empty()))
    return fail(PVFL_E_PLAN, "the summed product needs a HYBRID or DIAG plan with lazy ModDown, no baby-step/giant-step "
                             "split and no in-ciphertext rotate-and-sum");
  std::vector<const double*> cts(count), pts(count);
  for (int k = 0; k < count; ++k) {
    if (!cts_v[k] || !pts_v[k]) return fail(PVFL_E_INVALID, "null term buffer");
    cts[k] = (const double*)cts_v[k];
    pts[k] = (const double*)pts_v[k];
  }
  pvfl_status st = check_keys(p, keys);
  if (st != PVFL_OK) return st;
  double* ws = nullptr;
  if ((st = get_ws(p, ws_v, ws_bytes, &ws, count)) != PVFL_OK) return st;
  return run_diag_lazy(p, count, cts.data(), pts.data(), keys, (double*)out_v, ws, stream);
}

// ---------------------------------------------------------------------------
// Transposed diagonal conversion (Sec. 5.3, Eq. 7): [[A]] as Eq. 5 diagonals ->
// [[A^T]] as Eq. 5 diagonals, e'_i = RotL(e_k, r) (see transpose_step)
// ---------------------------------------------------------------------------
namespace {
// diagonal i of A^T is diagonal k of A rotated left by r slots
void transpose_step(const pvfl_plan* p, int i, int* k, int* r) {
  const int lo = p->info.mprime, mp = p->info.m_pad, np = p->info.n_pad, hi = std::max(mp, np);
  *k = (lo - i) % lo;
  if (mp >= np)
    *r = i;
  else
    *r = i == 0 ? 0 : hi - lo + i;
}

pvfl_status transpose_check(const pvfl_plan* p) {
  if (p->opts.kind != PVFL_PLAN_CTMAT) return fail(PVFL_E_PLAN, "the conversion takes a CTMAT plan");
  const int width = std::max(p->info.m_pad, p->info.n_pad);
  if ((int64_t)std::max(1, p->opts.pack) * width != p->ctx->N / 2)
    return fail(PVFL_E_PLAN, "the conversion needs pack * max(m, n) = N/2 (every block holding the diagonal)");
  return PVFL_OK;
}
}  // namespace

extern "C" pvfl_status pvfl_ctmat_transpose_galois(const pvfl_plan* p, uint32_t* out, int32_t cap, int32_t* count) {
  if (!p || !count || (!out && cap > 0)) return fail(PVFL_E_INVALID, "null argument");
  pvfl_status st = transpose_check(p);
  if (st != PVFL_OK) return st;
  std::vector<uint32_t> g;
  for (int i = 0; i < p->info.mprime; ++i) {
    int k, r;
    transpose_step(p, i, &k, &r);
    if (r) g.push_back(galois_rotl(r, p->ctx->N));
  }
  std::sort(g.begin(), g.end());
  g.erase(std::unique(g.begin(), g.end()), g.end());
  *count = (int32_t)g.size();
  if ((int32_t)g.size() > cap) return fail(PVFL_E_SHAPE, "buffer too small");
  std::copy(g.begin(), g.end(), out);
  return PVFL_OK;
}

extern "C" pvfl_status pvfl_ctmat_transpose(const pvfl_plan* p, const void* ct_in, const pvfl_rotkeys* keys,
                                            void* ct_out, void* stream) {
  if (!p || !ct_in || !ct_out) return fail(PVFL_E_INVALID, "null argument");
  pvfl_status st = transpose_check(p);
  if (st != PVFL_OK) return st;
  if (ct_in == ct_out) return fail(PVFL_E_INVALID, "the conversion cannot run in place");
  pvfl_ctx* c = p->ctx;
  const size_t Q = (size_t)(p->lv + 1) * c->N;
  for (int i = 0; i < p->info.mprime; ++i) {
    int k, r;
    transpose_step(p, i, &k, &r);
    const double* src = (const double*)ct_in + (size_t)k * 2 * Q;
    double* dst = (double*)ct_out + (size_t)i * 2 * Q;
    if (r == 0) {
      HIP_TRY(hipMemcpyAsync(dst, src, 2 * Q * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    } else {
      if (!keys) return fail(PVFL_E_NOKEY, "the conversion needs rotation keys");
      if ((st = pvfl_rotate(c, keys, p->lv, src, galois_rotl(r, c->N), 0, dst, stream)) != PVFL_OK) return st;
    }
  }
  return PVFL_OK;
}
