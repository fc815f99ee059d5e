/*
 * pvfl.h -- C ABI of the MI355X (gfx950) library for the packed-HE
 * ciphertext x plaintext matrix product of PackVFL (arXiv 2405.00482).
 *
 * Problem statement (Sec. 3, Eq. 1): a party holding the plaintext matrix X
 * computes X [[y]] = [[X y]] on a vector y that the key owner encrypted; the
 * result goes back to the key owner, who only decrypts it (characteristic C3,
 * Sec. 4).  The matrix form [[A]] W of Alg. 3 (Sec. 5.3) is also supported.
 * The encryption is RNS-CKKS (the paper's implementation uses Lattigo CKKS,
 * Sec. 7) with hybrid key switching.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns pvfl_status (0 = OK, < 0 = error) and never
 *   throws; pvfl_last_error() returns a message for the calling thread.
 * - Arguments are validated (shapes, levels, key coverage) before any work is
 *   enqueued; on error nothing is launched.
 * - Device buffers ("_dev") are caller-owned device memory (e.g. from
 *   torch), sized with the pvfl_bytes_* queries; the library never frees them.
 *   Host arrays are only read during the call.  Handles (pvfl_ctx, pvfl_sk,
 *   pvfl_rotkeys, pvfl_plan) are opaque, owned by the library, and released
 *   with the matching destroy call; destroying a handle twice is undefined.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   work is enqueued on it and the call returns without waiting, except the
 *   handle-creating calls, which synchronise.
 * - Residue storage.  A "poly" of L limbs is double[L][N]: limb i holds the
 *   residues modulo prime i of the basis, each an integer held exactly in an
 *   IEEE-754 binary64 with |x| <= q_i, in the evaluation (NTT) domain, in the
 *   slot-orbit order (index t is the evaluation at psi^(5^t) for t < N/2 and
 *   at psi^(-5^(t-N/2)) otherwise).  A ciphertext at level l is double[2][l+1][N]
 *   (c0 then c1).  Basis order: q_0..q_l, then the special primes p_0..p_{a-1}.
 *   Use pvfl_export_coeffs to read residues back as canonical uint64
 *   coefficient-domain values.
 * - All primes must be below 2^48 and congruent to 1 mod 2N.
 */
#ifndef PVFL_H
#define PVFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PVFL_OK = 0,
  PVFL_E_INVALID = -1, /* bad argument or parameter set */
  PVFL_E_SHAPE = -2,   /* shape or buffer size does not match the plan */
  PVFL_E_LEVEL = -3,   /* ciphertext level too low for the plan */
  PVFL_E_NOKEY = -4,   /* a rotation key the plan needs is missing */
  PVFL_E_NOMEM = -5,   /* device allocation failed */
  PVFL_E_DEVICE = -6,  /* HIP runtime error */
  PVFL_E_PLAN = -7     /* plan kind cannot serve this request */
} pvfl_status;

typedef struct pvfl_ctx pvfl_ctx;
typedef struct pvfl_sk pvfl_sk;
typedef struct pvfl_pk pvfl_pk;
typedef struct pvfl_rotkeys pvfl_rotkeys;
typedef struct pvfl_plan pvfl_plan;

/* RNS-CKKS parameter set.  q: n_q ciphertext primes (level L = n_q - 1);
 * p: n_p special primes of the key-switching modulus P (alpha = n_p, so the
 * digit count at level l is ceil((l+1)/alpha)).  Copied by the library. */
typedef struct {
  uint32_t log_n;      /* ring degree N = 2^log_n, 12..15 */
  uint32_t n_q;
  uint32_t n_p;
  const uint64_t* q;
  const uint64_t* p;
  double log2_scale;   /* default encoding scale Delta = 2^log2_scale */
} pvfl_params;

/* Plan kinds (Sec. 3-5). */
enum {
  PVFL_PLAN_HYBRID = 0, /* Eq. 5 diagonals + Eq. 6 input packing + partitioning + lazy RaS (Sec. 4) */
  PVFL_PLAN_DIAG = 1,   /* Eq. 5 alone over max(m,n) slots (Sec. 4.1) */
  PVFL_PLAN_ROW = 2,    /* row-order (naive) method (Sec. 3.1) */
  PVFL_PLAN_CTMAT = 3,  /* [[A]] W with A sent as Eq. 5 diagonals (Alg. 3) */
  PVFL_PLAN_COL = 4     /* column-order method (Sec. 3.1): n input ciphertexts, [[y_j]] replicated over every
                           slot, times column j of X; no rotation (Table 2: n Mult, n-1 Add) */
};

typedef struct {
  int32_t kind;          /* PVFL_PLAN_* */
  int32_t m, n;          /* X is m x n (plaintext) for HYBRID/DIAG/ROW; A is m x n (encrypted) for CTMAT */
  int32_t n_out;         /* CTMAT: columns of W (n x n_out); ignored otherwise */
  int32_t level;         /* ciphertext level; -1 = the top level L */
  int32_t lazy_moddown;  /* 1: one ModDown per output ciphertext (Q u P accumulation); 0: per rotation (Alg. 1 literal) */
  int32_t ras_in_ct;     /* DIAG with m < n: 1 = rotate-and-sum inside the ciphertext, 0 = lazy RaS after decryption */
  int32_t pack;          /* CTMAT: columns of W per plaintext (1 = Alg. 3 literal) */
  double pt_log2_scale;  /* plaintext scale exponent; <= 0 means the context's default */
  int32_t bsgs;          /* HYBRID with lazy ModDown: baby-step size b (power of two, 2 <= b <= m'/2) of a
                            baby-step/giant-step split of the diagonal sum (Halevi-Shoup 2018; not in the paper):
                            b - 1 hoisted baby rotations, m'/b - 1 giant rotations per block, each giant inner
                            sum brought down by its own ModDown.  0 = every rotation hoisted (Sec. 4, O4). */
  int32_t unhoisted;     /* HYBRID/DIAG with per-rotation ModDown (lazy_moddown = 0, bsgs = 0): 1 = every rotation
                            is a complete O3 rotation of the input ciphertext (Sec. 2; automorphism, then its own
                            ModUp, key inner product and ModDown), the cost profile of GALA's method in Table 2
                            (m'-1 Rot, 0 HstRot); 0 = hoisted rotations sharing one ModUp (Sec. 4, O4). */
} pvfl_plan_opts;

typedef struct {
  int32_t kind, m, n, n_out, m_pad, n_pad;
  int32_t mprime;        /* diagonals per block (m' of Eq. 6) */
  int32_t groups;        /* N' / n per ciphertext (input packing) */
  int32_t row_blocks, col_blocks;
  int32_t n_pts, pt_limbs, ct_in, ct_out, in_level, out_level, n_galois;
  int64_t n_add, n_mult, n_rot, n_hstrot; /* Table 2 / Table 3 counts of this plan */
  double out_log2_scale;
  int32_t bsgs;          /* baby-step size (0 = none) */
  int32_t n_modup;       /* digit decompositions (ModUp) one product runs */
  int32_t n_moddown;     /* ModDowns of a ciphertext one product runs */
} pvfl_plan_info;

const char* pvfl_last_error(void);

/* Context: parameters, transform tables and key-switching constants on the
 * given HIP device.  Synchronises. */
pvfl_status pvfl_context_create(const pvfl_params* params, int device, pvfl_ctx** out);
void pvfl_context_destroy(pvfl_ctx* ctx);

/* Secret key: uniform ternary s drawn from the Philox4x32-10 stream
 * (seed, 0x01<<56), kept on the device transformed for every prime. */
pvfl_status pvfl_keygen(pvfl_ctx* ctx, uint64_t seed, pvfl_sk** out);
void pvfl_sk_destroy(pvfl_sk* sk);

/* Public key (the public-key form of RLWE encryption; Alg. 2's parties
 * encrypt with the key owner's public key): pk = (b, a) = (-a s + e, a) over
 * the L+1 ciphertext primes, a uniform per limb from the stream
 * (seed, 0x06<<56 | limb), e CBD(21) from (seed, 0x07<<56).  Synchronises.
 * pvfl_pk_export: canonical uint64 coefficient residues [2][L+1][N] (b, a).
 * pvfl_encrypt_pk: pvfl_encrypt with the public key: v ternary from
 *   (seed + k, 0x08<<56), c0 = v b + m + e0, c1 = v a + e1 with e0, e1 CBD(21)
 *   from (seed + k, 0x09<<56) and (seed + k, 0x0A<<56), ciphertext k.  Its
 *   noise v e + e0 + e1 s is about sqrt(N) times that of secret-key
 *   encryption.  Errors as pvfl_encrypt, PVFL_E_INVALID for a key of another
 *   context.
 * pvfl_encrypt_coeffs_pk: the same on integer coefficients m_dev [N] at
 *   `level` (seed used as is), for bit-exact parity. */
pvfl_status pvfl_pk_gen(pvfl_ctx* ctx, const pvfl_sk* sk, uint64_t seed, pvfl_pk** out);
void pvfl_pk_destroy(pvfl_pk* pk);
pvfl_status pvfl_pk_export(const pvfl_pk* pk, uint64_t* out_dev, void* stream);

/* Rotation keys (hybrid key switching) for `count` Galois elements, each a
 * power of 5 modulo 2N (RotL by i slots is 5^i, Sec. 3.1's rotation).  The
 * keys live in the caller's device buffer keys_dev (256-byte aligned, at
 * least pvfl_bytes_rotkeys(ctx, count) bytes): count * beta * 2 * (L+1+alpha)
 * * N doubles, then a table of N/2 ints mapping a rotation to its key.  The
 * buffer must stay allocated and unchanged until pvfl_rotkeys_destroy; the
 * library never frees it.  Repeated elements get one key.  Errors:
 * PVFL_E_INVALID (element not a power of 5, NULL or misaligned buffer, key of
 * another context), PVFL_E_SHAPE (buffer too small).  Synchronises. */
size_t pvfl_bytes_rotkeys(const pvfl_ctx* ctx, int32_t count);
pvfl_status pvfl_rotkeys_gen(pvfl_ctx* ctx, const pvfl_sk* sk, const uint32_t* galois, int32_t count, uint64_t seed,
                             void* keys_dev, size_t keys_bytes, pvfl_rotkeys** out);
void pvfl_rotkeys_destroy(pvfl_rotkeys* keys);

/* Plans (Sec. 4 and 5): layout, partitioning, rotation list, op counts. */
pvfl_status pvfl_plan_create(pvfl_ctx* ctx, const pvfl_plan_opts* opts, pvfl_plan** out);
pvfl_status pvfl_plan_get_info(const pvfl_plan* plan, pvfl_plan_info* out);
/* writes the plan's Galois elements (info.n_galois of them) */
pvfl_status pvfl_plan_galois(const pvfl_plan* plan, uint32_t* out, int32_t cap);
void pvfl_plan_destroy(pvfl_plan* plan);

size_t pvfl_bytes_ct_in(const pvfl_plan* plan);    /* all input ciphertexts */
size_t pvfl_bytes_ct_out(const pvfl_plan* plan);   /* all output ciphertexts */
size_t pvfl_bytes_pt(const pvfl_plan* plan);       /* all diagonal plaintexts */
size_t pvfl_bytes_workspace(const pvfl_plan* plan);

/* The hot path.
 * pvfl_matmul_ct_pt: out = the plan's product of the input ciphertexts and
 *   the encoded plaintexts (Alg. 1 loop: sum_i pt_i * HstRotL(ct, i)).  ws is
 *   the caller's device workspace of at least pvfl_bytes_workspace bytes (NULL
 *   is accepted only by plans that need none: CTMAT, COL).  Errors:
 *   PVFL_E_NOKEY, PVFL_E_SHAPE (workspace too small), PVFL_E_INVALID (no
 *   workspace). */
pvfl_status pvfl_matmul_ct_pt(const pvfl_plan* plan, const void* ct_dev, const void* pt_dev, const pvfl_rotkeys* keys,
                              void* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Allocation-free variant of pvfl_matmul_ct_pt, for callers that cannot
 * allocate device memory while they run: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It runs the same kernels
 * with the same results, but its workspace is a fixed array of
 * pvfl_noalloc_max_bytes() bytes (64 MiB) in device memory, one copy per
 * device, held until the process ends; the call allocates and frees nothing
 * and creates no runtime objects (kernel timing is skipped).  The caller
 * still passes ct_dev, pt_dev and out_dev as for pvfl_matmul_ct_pt.
 * Every workspace element a call reads was written earlier in the same call,
 * so the array's previous contents never matter.  All calls on one device
 * share its array: calls that overlap in time on one device (different
 * streams, or host threads without ordering) race and must not be issued.
 * Plans: HYBRID, DIAG with lazy rotate-and-sum, CTMAT and COL.  Errors as
 * pvfl_matmul_ct_pt, plus PVFL_E_PLAN for ROW and in-ciphertext
 * rotate-and-sum plans and PVFL_E_SHAPE when the plan's workspace
 * (pvfl_bytes_workspace) exceeds the array, before anything is enqueued. */
pvfl_status pvfl_matmul_ct_pt_noalloc(const pvfl_plan* plan, const void* ct_dev, const void* pt_dev,
                                      const pvfl_rotkeys* keys, void* out_dev, void* stream);
size_t pvfl_noalloc_max_bytes(void);

/* Real-valued path (canonical-embedding encoding, Sec. 2.2).
 * pvfl_encode_pt: pack the plaintext matrix into the plan's diagonal
 *   plaintexts (Eq. 5 / Eq. 6 layout; for CTMAT the matrix is W, n x n_out)
 *   and encode them at the plan's plaintext scale.  X_dev is row-major with
 *   row stride ld (elements).  Every slot value times the scale must stay
 *   below 2^50 in magnitude.  pt_dev holds pvfl_bytes_pt bytes.
 * pvfl_encrypt: the key owner's side: build the plan's input ciphertexts from
 *   v_dev (the vector y, replicated with period n over the slots, Sec. 4.1;
 *   for CTMAT the m x n matrix A as its Eq. 5 diagonals, row stride ld) at the
 *   context scale, secret-key encrypted; ciphertext k uses seed + k.
 * pvfl_decrypt_decode: decrypt the plan's output ciphertexts, lift by CRT,
 *   decode, and apply the lazy rotate-and-sum of Sec. 4.3: y_dev receives m
 *   values (CTMAT: the m x n_out product, row-major).  Uses the context's
 *   scratch memory: calls on one context must be ordered on one stream. */
pvfl_status pvfl_encode_pt(const pvfl_plan* plan, const double* X_dev, int64_t ld, void* pt_dev, void* stream);
pvfl_status pvfl_encrypt(const pvfl_plan* plan, const pvfl_sk* sk, const double* v_dev, int64_t ld, uint64_t seed,
                         void* ct_dev, void* stream);
pvfl_status pvfl_decrypt_decode(const pvfl_plan* plan, const pvfl_sk* sk, const void* ct_dev, double* y_dev,
                                void* stream);
pvfl_status pvfl_encrypt_pk(const pvfl_plan* plan, const pvfl_pk* pk, const double* v_dev, int64_t ld, uint64_t seed,
                            void* ct_dev, void* stream);

/* Multiplication-level reduction (Sec. 5.2, Eq. 4) and the shares of the
 * result (Alg. 2).  Eq. 4 rewrites CAESAR's gradient [[g_B]] = (q0 1 - y)^T X
 * + (q1 X)^T [[z]] + (q2 X)^T [[z^3]]: two ciphertext-plaintext products that
 * share one layout and one multiplicative level, plus a cleartext term.
 *
 * pvfl_encode_pt_scaled: pvfl_encode_pt of coef * X (the q1 X and q2 X of
 *   Eq. 4); same layout and errors.
 * pvfl_matmul_ct_pt_sum: out = sum_{k < count} (product of cts[k] and pts[k]),
 *   every term laid out by `plan`, which must be HYBRID or DIAG with lazy
 *   ModDown and no baby-step/giant-step split: the terms accumulate over
 *   Q u P and each output ciphertext takes one ModDown.  cts[k], pts[k]:
 *   device buffers of pvfl_bytes_ct_in / pvfl_bytes_pt bytes (host array of
 *   count device pointers); ws: the caller's device workspace of at least
 *   pvfl_bytes_workspace_sum(plan, count) bytes.  Errors: PVFL_E_PLAN for
 *   other plans, PVFL_E_INVALID for count < 1, PVFL_E_NOKEY, PVFL_E_SHAPE.
 * pvfl_encode_out: a cleartext as a plaintext at the plan's output level and
 *   scale (HYBRID, DIAG or CTMAT; no rescale in the plan), layout
 *   [ct_out][out_level+1][N] (evaluation domain, pvfl_bytes_pt_out bytes).
 *   The values are encoded at the context scale Delta and the residues
 *   multiplied by 2^e mod q, e = output exponent - log2(Delta), an integer.
 *   mode PVFL_OUT_ROWS: v_dev holds the plan's m output values (CTMAT: the
 *   m x n_out product, row-major); each is split into equal parts over the
 *   slots that the lazy rotate-and-sum of its row adds up, halving it once per
 *   rotate-and-sum level (the cleartext inverse RaS of Sec. 5.2), so that
 *   pvfl_decrypt_decode of ct + pt returns the product plus v.
 *   mode PVFL_OUT_SLOTS: v_dev holds N/2 slot values per output ciphertext,
 *   [ct_out][N/2], placed as they are (a mask in the slot domain).
 * pvfl_out_add_pt: out = ct + sign * pt on the plan's output ciphertexts
 *   (sign +1 or -1; c1 copied): O1 with a plaintext, e.g. the masking party
 *   subtracting its random slots (Alg. 2).  out may equal ct.
 * pvfl_lazy_ras: the lazy rotate-and-sum of Sec. 4.3 over cleartext slot
 *   vectors [ct_out][N/2] -> the plan's m outputs: the masking party's share
 *   of the result (Alg. 2, last step). */
enum { PVFL_OUT_ROWS = 0, PVFL_OUT_SLOTS = 1 };
pvfl_status pvfl_encode_pt_scaled(const pvfl_plan* plan, const double* X_dev, int64_t ld, double coef, void* pt_dev,
                                  void* stream);
pvfl_status pvfl_matmul_ct_pt_sum(const pvfl_plan* plan, int32_t count, const void* const* cts_dev,
                                  const void* const* pts_dev, const pvfl_rotkeys* keys, void* out_dev, void* ws_dev,
                                  size_t ws_bytes, void* stream);
size_t pvfl_bytes_workspace_sum(const pvfl_plan* plan, int32_t count);
size_t pvfl_bytes_pt_out(const pvfl_plan* plan);
pvfl_status pvfl_encode_out(const pvfl_plan* plan, const double* v_dev, int32_t mode, void* pt_dev, void* stream);
pvfl_status pvfl_out_add_pt(const pvfl_plan* plan, const void* ct_dev, const void* pt_dev, int32_t sign,
                            void* out_dev, void* stream);
pvfl_status pvfl_lazy_ras(const pvfl_plan* plan, const double* slots_dev, double* y_dev, void* stream);

/* Integer-level entry points (exact residues; used for bit-exact parity).
 * m_dev: int64 coefficient vectors [count][N] on the device.
 * pvfl_pt_import: plaintexts [count][limbs][N] with limbs = level+1 (+alpha if with_p).
 * pvfl_encrypt_coeffs: secret-key encryption at `level`; noise and `a` drawn
 *   from the Philox streams (seed, 0x03<<56) and (seed, 0x02<<56 | limb).
 * pvfl_export_coeffs: evaluation-domain polys [count][limbs][N] -> canonical
 *   uint64 coefficient residues, same layout.
 * pvfl_decrypt_coeffs: c0 + c1 s as canonical uint64 residues [level+1][N]. */
pvfl_status pvfl_pt_import(pvfl_ctx* ctx, int32_t level, int32_t with_p, const int64_t* m_dev, int32_t count,
                           void* pt_dev, void* stream);
pvfl_status pvfl_encrypt_coeffs(pvfl_ctx* ctx, const pvfl_sk* sk, int32_t level, const int64_t* m_dev, uint64_t seed,
                                void* ct_dev, void* stream);
pvfl_status pvfl_encrypt_coeffs_pk(pvfl_ctx* ctx, const pvfl_pk* pk, int32_t level, const int64_t* m_dev,
                                   uint64_t seed, void* ct_dev, void* stream);
pvfl_status pvfl_export_coeffs(pvfl_ctx* ctx, int32_t level, int32_t with_p, const void* poly_dev, int32_t count,
                               uint64_t* out_dev, void* stream);
pvfl_status pvfl_decrypt_coeffs(pvfl_ctx* ctx, const pvfl_sk* sk, int32_t level, const void* ct_dev, uint64_t* out_dev,
                                void* stream);
/* secret key and rotation keys as canonical uint64 coefficient residues:
 * sk -> [L+1+alpha][N];  key k -> [beta_L][2 (b, a)][L+1+alpha][N] */
pvfl_status pvfl_sk_export(const pvfl_sk* sk, uint64_t* out_dev, void* stream);
pvfl_status pvfl_rotkeys_export(const pvfl_rotkeys* keys, int32_t index, uint64_t* out_dev, void* stream);

/* Single operations on one ciphertext at `level` (O1-O4 of Sec. 2.2).
 * pvfl_rotate: RotL by the Galois element (O3: automorphism, then ModUp, key
 *   product, ModDown; hoisted = 1 gives O4's order: ModUp of c1 first, the
 *   automorphism applied to the extended digits).
 * pvfl_rescale: divide by q_level with rounding; out has level-1.
 * pvfl_ct_mul_pt / pvfl_ct_add: slot-wise product / sum. */
pvfl_status pvfl_rotate(pvfl_ctx* ctx, const pvfl_rotkeys* keys, int32_t level, const void* ct_dev, uint32_t galois,
                        int32_t hoisted, void* out_dev, void* stream);
pvfl_status pvfl_rescale(pvfl_ctx* ctx, int32_t level, const void* ct_dev, void* out_dev, void* stream);
pvfl_status pvfl_ct_mul_pt(pvfl_ctx* ctx, int32_t level, const void* ct_dev, const void* pt_dev, void* out_dev,
                           void* stream);
pvfl_status pvfl_ct_add(pvfl_ctx* ctx, int32_t level, const void* a_dev, const void* b_dev, void* out_dev, void* stream);

/* Batched form: many independent products of uneven shapes sharing one
 * context, level, plaintext scale and rotation-key set.  Every phase of the
 * path runs as one launch over all products, and the fused rotation x
 * diagonal kernel streams each rotation key once per group of `group`
 * products (products are grouped by their diagonal count m').  Products must
 * be lazy-ModDown HYBRID (or DIAG without in-ciphertext RaS) plans with one
 * input and one output ciphertext.  The buffers named at creation are the
 * caller's (arrays of `count` device pointers): X_dev[k] (row stride ldx[k]),
 * v_dev[k] (the encrypted vector), pt_dev[k], ct_dev[k], out_dev[k] sized by
 * the plan queries, y_dev[k] (m_k doubles); X_dev/v_dev/y_dev may be NULL when
 * only pvfl_batch_matmul is used.  So is the workspace ws_dev (256-byte
 * aligned, at least pvfl_batch_workspace_bytes bytes for the same plans and
 * options): the batch keeps its launch tables and every intermediate there
 * and allocates no device memory.  The buffers must outlive the batch.
 * opts (NULL = defaults {2, 32, 1, 1}): see pvfl_batch_opts.
 * pvfl_batch_encrypt: product k uses seed + k.
 * pvfl_batch_run: encode, encrypt, matmul, decrypt in order; with use_graph
 *   the sequence is captured once into a HIP graph (per sk and seed) and
 *   replayed.  Kernel timing is not recorded inside a captured graph. */
typedef struct {
  int32_t group;        /* products sharing one key stream per work item: 1, 2 or 4 */
  int32_t chunk;        /* diagonals per work item (one partial sum each), 1..1024 */
  int32_t vec;          /* evaluation indices per thread: 1 or 2 */
  int32_t chunk_major;  /* 1: work items ordered by diagonal chunk first, so that work items
                           running together share rotation-key lines in L2; 0: product-major */
} pvfl_batch_opts;
typedef struct pvfl_batch pvfl_batch;
pvfl_status pvfl_batch_workspace_bytes(pvfl_ctx* ctx, int32_t count, const pvfl_plan* const* plans,
                                       const pvfl_batch_opts* opts, size_t* bytes);
pvfl_status pvfl_batch_create(pvfl_ctx* ctx, int32_t count, const pvfl_plan* const* plans,
                              const double* const* X_dev, const int64_t* ldx, const double* const* v_dev,
                              void* const* pt_dev, void* const* ct_dev, void* const* out_dev, double* const* y_dev,
                              const pvfl_rotkeys* keys, const pvfl_batch_opts* opts, void* ws_dev, size_t ws_bytes,
                              pvfl_batch** out);
pvfl_status pvfl_batch_encode(pvfl_batch* batch, void* stream);
pvfl_status pvfl_batch_encrypt(pvfl_batch* batch, const pvfl_sk* sk, uint64_t seed, void* stream);
pvfl_status pvfl_batch_matmul(pvfl_batch* batch, void* stream);
pvfl_status pvfl_batch_decrypt(pvfl_batch* batch, const pvfl_sk* sk, void* stream);
pvfl_status pvfl_batch_run(pvfl_batch* batch, const pvfl_sk* sk, uint64_t seed, int32_t use_graph, void* stream);
/* work items of the fused kernel and its algorithmic key / plaintext bytes */
pvfl_status pvfl_batch_info(const pvfl_batch* batch, int64_t* n_work_items, double* key_bytes, double* pt_bytes);
void pvfl_batch_destroy(pvfl_batch* batch);

/* Transposed diagonal conversion (Sec. 5.3, Eq. 7).  plan: a CTMAT plan of
 * [[A]] (m x n) with pack * max(m_pad, n_pad) = N/2, so that every slot block
 * holds the diagonal and a rotation is cyclic over max(m, n).  ct_in: the
 * plan's input ciphertexts (min(m, n) Eq. 5 diagonals of A); ct_out (same
 * size, not overlapping ct_in) receives the Eq. 5 diagonals of A^T, the
 * input of a CTMAT plan of shape n x m with the same pack.  Diagonal i of A^T
 * is diagonal k of A rotated left by r (unhoisted rotation): with
 * lo = min(m_pad, n_pad), k = (lo - i) mod lo and r = i when m_pad >= n_pad,
 * r = max - lo + i (0 for i = 0) otherwise -- the printed equation's RotR by
 * max - min + i does not reproduce A^T for tall matrices.
 * pvfl_ctmat_transpose_galois lists the Galois elements the keys must hold. */
pvfl_status pvfl_ctmat_transpose_galois(const pvfl_plan* plan, uint32_t* out, int32_t cap, int32_t* count);
pvfl_status pvfl_ctmat_transpose(const pvfl_plan* plan, const void* ct_in, const pvfl_rotkeys* keys, void* ct_out,
                                 void* stream);

/* Latency-model network of the plan selector: a 3-layer perceptron
 * y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 in FP32 (n_in <= 64 inputs,
 * hidden <= 64), trained on measured plan latencies by hand-written HIP
 * forward, backward and Adam kernels.  Parameters are one FP32 vector laid out
 * W1[hidden][n_in], b1, W2[hidden][hidden], b2, w3, b3 (He-uniform init from
 * seed, zero biases).  x: [batch][n_in], t and y: [batch] device arrays.
 * pvfl_mlp_grad: gradient of the mean squared error (1/B) sum (y - t)^2 into
 *   grad_dev (n_params floats) and the loss into loss_dev (either may be NULL).
 * pvfl_mlp_train_step: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8). */
typedef struct pvfl_mlp pvfl_mlp;
pvfl_status pvfl_mlp_create(int32_t n_in, int32_t hidden, int32_t max_batch, uint64_t seed, pvfl_mlp** out);
int32_t pvfl_mlp_num_params(const pvfl_mlp* mlp);
pvfl_status pvfl_mlp_get_params(const pvfl_mlp* mlp, float* out_dev, void* stream);
pvfl_status pvfl_mlp_set_params(pvfl_mlp* mlp, const float* in_dev, void* stream);
pvfl_status pvfl_mlp_forward(const pvfl_mlp* mlp, const float* x_dev, int32_t batch, float* y_dev, void* stream);
pvfl_status pvfl_mlp_grad(pvfl_mlp* mlp, const float* x_dev, const float* t_dev, int32_t batch, float* grad_dev,
                          float* loss_dev, void* stream);
pvfl_status pvfl_mlp_train_step(pvfl_mlp* mlp, const float* x_dev, const float* t_dev, int32_t batch, float lr,
                                float* loss_dev, void* stream);
void pvfl_mlp_destroy(pvfl_mlp* mlp);

/* Plan selection.  Two operand forms (Sec. 5):
 *   PVFL_OPERAND_CT_VEC: X (m x n, plaintext) times an encrypted vector.  The
 *     candidates are every valid HYBRID / DIAG / ROW plan with lazy or
 *     per-rotation ModDown and every baby-step size (Sec. 3-4), batch 1.
 *   PVFL_OPERAND_CT_MAT: [[A]] (m x n, encrypted) times W (n x n_out).  The
 *     candidates are Alg. 3 (CTMAT) with every column-packing factor, batch 1,
 *     and the per-row form: W^T times each encrypted row of A as a lazy
 *     HYBRID or DIAG plan of shape n_out x n, batch m, sharing one set of
 *     plaintexts.
 * pvfl_plan_candidates: writes up to cap candidates, *count = how many exist.
 * pvfl_plan_features: the PVFL_PLAN_FEATURES-long feature vector of a plan run
 *   `batch` times (log2 N, l+1, alpha, beta, K, log2 m, log2 n, log2 m', kind
 *   one-hot (HYBRID, DIAG, ROW, CTMAT), lazy, in-ciphertext RaS, BSGS flag and
 *   log2 b, log2 pack, log2 batch, log2(1+count) of Mult, Add, Rot, HstRot,
 *   ModUp, ModDown (per product), encoded limbs, keys, blocks).
 * pvfl_plan_analytic_ms: sum over the PVFL_COST_TERMS counts (Mult, Add, Rot,
 *   HstRot, ModUp, ModDown -- each times batch -- encoded plaintext limbs, 1)
 *   of count x costs[i].
 * pvfl_planner_create: a learned latency model -- a pvfl_mlp over features
 *   standardised by (x - x_mean) / x_std predicting (ln ms - y_mean) / y_std.
 *   The network is borrowed and must outlive the planner.
 * pvfl_plan_choose: the candidate of least predicted latency, by the network
 *   when costs is NULL, else by the analytic model.  Synchronises `stream`. */
#define PVFL_PLAN_FEATURES 27
#define PVFL_COST_TERMS 8
enum { PVFL_OPERAND_CT_VEC = 0, PVFL_OPERAND_CT_MAT = 1 };
typedef struct {
  pvfl_plan_opts opts;
  int32_t batch;  /* products the candidate runs with these options (rows of A for the per-row form) */
} pvfl_candidate;
typedef struct pvfl_planner pvfl_planner;
pvfl_status pvfl_plan_candidates(pvfl_ctx* ctx, int32_t operand, int32_t m, int32_t n, int32_t n_out, int32_t level,
                                 pvfl_candidate* out, int32_t cap, int32_t* count);
int32_t pvfl_plan_num_features(void);
pvfl_status pvfl_plan_features(const pvfl_plan* plan, int32_t batch, float* out, int32_t cap);
pvfl_status pvfl_plan_analytic_ms(const pvfl_plan* plan, int32_t batch, const double* costs, double* ms);
pvfl_status pvfl_planner_create(pvfl_mlp* mlp, const float* x_mean, const float* x_std, float y_mean, float y_std,
                                pvfl_planner** out);
pvfl_status pvfl_plan_choose(pvfl_planner* planner, pvfl_ctx* ctx, int32_t operand, int32_t m, int32_t n,
                             int32_t n_out, int32_t level, const double* costs, pvfl_candidate* chosen,
                             double* predicted_ms, void* stream);
void pvfl_planner_destroy(pvfl_planner* planner);

/* Optional kernel timing for measurement.  When enabled, every launch of the
 * timed kernel classes is bracketed by HIP events recorded on the launch's
 * stream; pvfl_timing_read waits for the recorded events of one class, returns
 * the summed elapsed time, the launch count and the summed algorithmic bytes
 * (each key, plaintext and ciphertext limb counted once per launch), and
 * forgets them.  Timing adds an event pair per launch; leave it off otherwise. */
enum {
  PVFL_TIMING_DIAG = 0,    /* fused hoisted-rotation x diagonal kernel */
  PVFL_TIMING_ENCODE = 1,  /* plaintext packing + encoding + NTTs */
  PVFL_TIMING_MODUP = 2,   /* ModUp of an input ciphertext */
  PVFL_TIMING_MODDOWN = 3  /* ModDown of an output ciphertext */
};
pvfl_status pvfl_timing_enable(pvfl_ctx* ctx, int32_t enable);
pvfl_status pvfl_timing_read(pvfl_ctx* ctx, int32_t kernel_class, double* total_ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* PVFL_H */
