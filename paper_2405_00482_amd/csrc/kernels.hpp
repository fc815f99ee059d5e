// Kernel argument structures and launcher declarations shared by the HIP
// kernels and the host side of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_core.hpp"

namespace pvfl {

constexpr int kMaxLimbs = 24;   // primes of Q_L u P
constexpr int kMaxTasks = 128;  // ModUp (digit, limb) tasks per level
constexpr int kMaxAlpha = 4;    // special primes

// counter-based generator streams (top byte = purpose)
constexpr uint64_t kStreamSecret = 0x01ull << 56;
constexpr uint64_t kStreamEncA = 0x02ull << 56;  // | limb
constexpr uint64_t kStreamEncE = 0x03ull << 56;
constexpr uint64_t kStreamKeyA = 0x04ull << 56;  // | j<<40 | r<<24 | g
constexpr uint64_t kStreamKeyE = 0x05ull << 56;  // | j<<40 | g
constexpr uint64_t kStreamPkA = 0x06ull << 56;   // | limb: public key a
constexpr uint64_t kStreamPkE = 0x07ull << 56;   // public key error
constexpr uint64_t kStreamPkV = 0x08ull << 56;   // public-key encryption: ternary v
constexpr uint64_t kStreamPkE0 = 0x09ull << 56;  // public-key encryption: e0
constexpr uint64_t kStreamPkE1 = 0x0Aull << 56;  // public-key encryption: e1

struct LimbMap {
  int n;
  int idx[kMaxLimbs];
};

struct LaunchCtx {
  hipStream_t stream;
  DevTabs tb;
  int logN;
};

enum class NttOp { Fwd, Inv, ImportI64, ExportU64 };

struct KsTask {
  int digit, limb, prime, nsrc, src0;
  double hat[kMaxAlpha];  // [Q_j / q_src]_{prime}
};

// key-switching constants of one level l (device resident)
struct KsLevel {
  int lv, alpha, beta, K, n_q_total, n_tasks;
  double up_inv_hat[kMaxLimbs];              // limb i <= l: [(Q_j/q_i)^-1]_{q_i}, j = digit of i
  KsTask up_task[kMaxTasks];
  double down_inv_hat[kMaxAlpha];            // [(P/p_k)^-1]_{p_k}
  double down_hat[kMaxAlpha * kMaxLimbs];    // [k][i]: [P/p_k]_{q_i}
  double down_pinv[kMaxLimbs];               // [P^-1]_{q_i}
  double down_half[kMaxLimbs];               // floor(P/2) mod limb r of Q_l u P
  double p_mod[kMaxLimbs];                   // P mod q_i, centred
};

struct RotKeyArgs {
  int n_limbs, beta, alpha, n_q;
  double P_mod[kMaxLimbs];
};

// Up to kKeysPerLaunch rotation keys of one generation launch, passed by
// value: rotation amount and Galois element of each.
constexpr int kKeysPerLaunch = 64;
struct RotKeyList {
  int rot[kKeysPerLaunch];
  uint32_t galois[kKeysPerLaunch];
};

struct RescaleArgs {
  double half_mod_last;            // floor(q_l / 2)
  double half_mod[kMaxLimbs];      // floor(q_l / 2) mod q_i
  double inv_last[kMaxLimbs];      // q_l^-1 mod q_i
};

struct DiagArgs {
  int N, K, lv, beta, mprime, chunk, key_limbs;
  size_t key_stride;
  const ModQ* mods;
  int limb_prime[kMaxLimbs];
  int key_limb[kMaxLimbs];
  const double* pt;        // [n_pts][K][N]
  const int* pt_index;     // [mprime]
  const int* rot;          // [mprime] rotation amount of diagonal i (0: the unrotated P*c term)
  const int* slot_of_rot;  // [N/2] rotation amount -> key index
  const double* keys;
  const double* digits;    // [beta][K][N]
  const double* pc;        // [2][lv+1][N]: P*c0, P*c1
  double* part;            // [nchunk][2][K][N]
};

hipError_t launch_ntt(const LaunchCtx& L, NttOp op, const void* in, void* out, int nblocks, LimbMap map);
hipError_t launch_keygen(const LaunchCtx& L, uint64_t seed, double* sk, int n_mod);
// nct ciphertexts [nct][2][lv+1][N] from messages [nct][N]; ciphertext c uses seed + c
// public key (b, a) = (-a s + e, a) over the nl = L+1 ciphertext primes: pk [2][nl][N]
hipError_t launch_pk_gen(const LaunchCtx& L, const double* sk, uint64_t seed, int nl, double* pk);
// public-key encryption at level lv: c = v (b, a) + (m + e0, e1); pk_stride = limbs per pk half
hipError_t launch_encrypt_pk(const LaunchCtx& L, const int64_t* msg, int nct, const double* pk, int pk_nl,
                             uint64_t seed, int lv, double* ct);
hipError_t launch_encrypt(const LaunchCtx& L, const int64_t* msg, int nct, const double* sk, uint64_t seed, int lv,
                          double* ct, double* const* ct_tab = nullptr);
hipError_t launch_decrypt_u64(const LaunchCtx& L, const double* ct, const double* sk, int lv, uint64_t* out);
hipError_t launch_decrypt_f64(const LaunchCtx& L, const double* ct, int nct, const double* sk, int lv, double* out,
                              const double* const* ct_tab = nullptr);
hipError_t launch_rotkey_gen(const LaunchCtx& L, const double* sk, const RotKeyList& list, int nkeys, uint64_t seed,
                             const RotKeyArgs& ka, double* keys);
// ModUp of the c1 halves of nct ciphertexts (ct + c*ct_stride); y holds
// [nct][lv+1][N] coefficient scratch; digits of ciphertext c at digits + c*dig_stride
hipError_t launch_modup(const LaunchCtx& L, const double* ct, size_t ct_stride, int nct, int lv, const KsLevel* kl_dev,
                        int n_tasks, double* y, double* digits, size_t dig_stride,
                        const double* const* ct_tab = nullptr);
// out_tab (optional): output of poly x at out_tab[x/2] + (x%2)*(lv+1)*N
hipError_t launch_moddown(const LaunchCtx& L, const double* u, int npoly, int lv, int alpha, const KsLevel* kl_dev,
                          double* y, double* out, double* const* out_tab = nullptr);
hipError_t launch_rescale(const LaunchCtx& L, const double* in, int npoly, int lv, const RescaleArgs& ra, double* out);
hipError_t launch_diag_lazy(const LaunchCtx& L, const DiagArgs& a, int nchunk);
// part[y][nchunk][2][K][N] summed over the chunks into acc[y][2][K][N], y < ngroups
hipError_t launch_sum_partials(const LaunchCtx& L, const double* part, int nchunk, int K, int N, LimbMap limb_prime,
                               double* acc, int ngroups = 1);
// Alg. 3: out[k] = sum_i ct[i] * pt[i][k]   (ct [nct][2][lv+1][N], pt [nct][nout][lv+1][N])
hipError_t launch_ctmat(const LaunchCtx& L, const double* ct, const double* pt, int nct, int nout, int lv, int N,
                        double* out);
hipError_t launch_fill_zero(const LaunchCtx& L, double* p, size_t n);
hipError_t launch_add_limbs(const LaunchCtx& L, const double* a, const double* b, int nlimbs, int N, LimbMap map,
                            double* out);
// acc (ct at lv) += (c0[shift rot] + v0, v1) * pt   (v0 = v1 = null: (c0, c1) unshifted)
hipError_t launch_eager_term(const LaunchCtx& L, const double* c0, const double* c1, const double* v, int rot, const double* pt,
                             int lv, int N, double* acc);
hipError_t launch_scale_by_p(const LaunchCtx& L, const double* ct, int lv, int N, const double* pmod_dev, double* out,
                             int nct = 1, const double* const* ct_tab = nullptr);
hipError_t launch_ct_mul_pt(const LaunchCtx& L, const double* ct, const double* pt, int lv, int N, double* out);
hipError_t launch_ct_add(const LaunchCtx& L, const double* a, const double* b, int lv, int N, double* out);
hipError_t launch_automorph(const LaunchCtx& L, const double* in, int npoly_limbs, int N, int rot, double* out);
hipError_t launch_key_inner(const LaunchCtx& L, const double* digits, int beta, int K, int N, int rot, const double* key,
                            int key_limbs, LimbMap limb_prime, LimbMap key_limb, double* u);

}  // namespace pvfl
