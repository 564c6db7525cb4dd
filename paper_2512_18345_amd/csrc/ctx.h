// Context (per ring degree N): device-resident tables and the launchers'
// view of them.  Internal to the library; the public surface is ckks.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ckks.h"

namespace ckks {

constexpr int kTileLog = 12;            // elements per NTT work-group tile
constexpr int kTile = 1 << kTileLog;
constexpr int kBlockLog = 8;            // pass-2 line length (N = N1 * 256)
constexpr int kWG = 256;                // threads per work-group
constexpr int kMinLogN = 12, kMaxLogN = 16;
constexpr int kMaxPrimes = 64;
constexpr int kMaxAlpha = 16;           // digit size / special-prime count

// Per-prime constants (device).
struct ModC {
  uint32_t q;
  uint32_t mu32;        // floor(2^32 / q)
  uint32_t mu_hi, mu_lo;  // floor(2^64 / q)
  uint32_t ninv, ninv_s;  // N^-1 mod q and its Shoup companion
};

// What a kernel needs to find a prime's tables.  Every twiddle is stored as
// (w, floor(w 2^32 / q)).
//  * column pass: tw / itw [nprimes][N1], index m + i < N1 -> psi^(+-brv_logN(m + i));
//  * block pass (after the twist below the 256-word block transform is the same
//    for every block): ctw / ictw [nprimes][256], index 2^s + g ->
//    psi^(+-(N / 2^s) brv_s(g));
//  * twist of block b: twist / itwist [nprimes][N1][32], entries j < 16 are
//    rho_b^(+-j) and 16 + h are rho_b^(+-16 h), rho_b = psi^(2 brv_logN1(b) + 1);
//    the block pass multiplies element j of block b by rho_b^j before the
//    forward network (by rho_b^-j after the inverse one);
//  * whole-limb transforms of small rings (N = 2^kSrLog only, else null):
//    ftw / fitw [nprimes][N], index m + i < N -> psi^(+-brv_logN(m + i)).
constexpr int kSrLog = 12;
struct DevTab {
  const ModC* mod;   // [nprimes]
  const uint2* tw;
  const uint2* itw;
  const uint2* ctw;
  const uint2* ictw;
  const uint2* twist;
  const uint2* itwist;
  const uint2* ftw;
  const uint2* fitw;
  int logN;
  int L_max;
  __host__ __device__ int logN1() const { return logN - 8; }
  __device__ const uint2* col_tw(int pi) const { return tw + ((size_t)pi << logN1()); }
  __device__ const uint2* col_itw(int pi) const { return itw + ((size_t)pi << logN1()); }
  __device__ const uint2* blk_tw(int pi) const { return ctw + ((size_t)pi << 8); }
  __device__ const uint2* blk_itw(int pi) const { return ictw + ((size_t)pi << 8); }
  __device__ const uint2* blk_twist(int pi, int b) const {
    return twist + ((((size_t)pi << logN1()) + b) << 5);
  }
  __device__ const uint2* blk_itwist(int pi, int b) const {
    return itwist + ((((size_t)pi << logN1()) + b) << 5);
  }
  __device__ const uint2* full_tw(int pi) const { return ftw + ((size_t)pi << logN); }
  __device__ const uint2* full_itw(int pi) const { return fitw + ((size_t)pi << logN); }
};

// Rows of a launch: row r of the data is prime index pidx(r).
struct RowMap {
  int L;       // rows [0, L) are q_0..q_{L-1}
  int L_max;   // rows >= L are p_{r - L}, prime index L_max + (r - L)
  __host__ __device__ int pidx(int r) const { return r < L ? r : L_max + (r - L); }
};

struct Ctx {
  int device;
  int logN, N;
  int L_max, k, dnum, alpha;
  std::vector<uint32_t> primes;  // q_0..q_{L_max-1}, p_0..p_{k-1}
  // host copies used to build launches
  std::vector<ModC> h_mod;

  // device tables
  ModC* d_mod = nullptr;
  uint2* d_tw = nullptr;      // [nprimes][N1]
  uint2* d_itw = nullptr;
  uint2* d_ctw = nullptr;     // [nprimes][256]
  uint2* d_ictw = nullptr;
  uint2* d_twist = nullptr;   // [nprimes][N1][32]
  uint2* d_itwist = nullptr;
  uint2* d_ftw = nullptr;     // [nprimes][N], N = 2^kSrLog only
  uint2* d_fitw = nullptr;
  // ModUp at level L (1-based): per Q row i < L, (N^-1 * (D_j/q_i)^-1, Shoup) where j = i / alpha.
  uint2* d_modup_scale = nullptr;     // [L_max + 1][L_max]
  // ModUp BConv tables at level L, digit j: T[r][i] = (D_j / q_{j alpha + i}) mod prime(r),
  // r over the L + k ModUp rows.  Offsets into one buffer.
  uint32_t* d_modup_T = nullptr;
  std::vector<size_t> modup_T_off;    // index (L * beta_max + j)
  uint32_t* d_modup_T_off = nullptr;  // device copy of modup_T_off
  // ModDown: P rows scale (N^-1 * (P/p_m)^-1, Shoup) indexed m; T_down[i][m] = (P/p_m) mod q_i;
  // P^-1 mod q_i with Shoup.
  uint2* d_moddown_scale = nullptr;   // [k]
  uint32_t* d_moddown_T = nullptr;    // [L_max][k]
  uint2* d_pinv = nullptr;            // [L_max]
  // Rescale at level L: q_{L-1}^-1 mod q_i (Shoup), i < L - 1.
  uint2* d_rescale_inv = nullptr;     // [L_max + 1][L_max]

  // kernel tracing (ckks_trace_begin / ckks_trace_end)
  struct Trace {
    int stage = 0;
    std::vector<hipEvent_t> starts, stops;
    int count = 0;
  };
  mutable Trace trace;

  // Kernel schedule of the key-switching pipeline (ckks_ctx_set_schedule /
  // ckks_ctx_tune): BConv output rows per work-group for ModUp and ModDown
  // (2, 4, 6 or 12), and the largest inner-product grid that uses one thread
  // group per digit (0: never).  Results do not depend on it.
  // Kernel schedule: launch shapes only, results are bitwise the same under
  // every schedule.  ntt_shape bits (kShape*): NTT tile and radix choices.
  struct Sched {
    int up_rows = 12, down_rows = 6, small_grid = 128, ntt_shape = 0;
  };
  Sched sched;
  // The start / stop events for the next launch of a traced stage (both null
  // when the stage is not traced or the capacity is used up).  Launchers pass
  // them to hipExtLaunchKernel, which records them at the dispatch's own
  // start and end.
  void trace_take(int stage, hipEvent_t* t0, hipEvent_t* t1) const {
    *t0 = *t1 = nullptr;
    if (trace.stage == stage && trace.count < (int)trace.starts.size()) {
      *t0 = trace.starts[trace.count];
      *t1 = trace.stops[trace.count++];
    }
  }

  DevTab tab() const {
    return DevTab{d_mod, d_tw, d_itw, d_ctw, d_ictw, d_twist, d_itwist, d_ftw, d_fitw, logN, L_max};
  }
  RowMap rows(int L) const { return RowMap{L, L_max}; }
  int beta(int L) const { return (L + alpha - 1) / alpha; }
  int beta_max() const { return beta(L_max); }
};

// Host-side table construction (params.cpp).  Returns "" or an error message.
std::string build_tables(Ctx& c, const uint32_t* q, const uint32_t* p, int* code);
void free_tables(Ctx& c);

}  // namespace ckks

struct ckks_ctx {
  ckks::Ctx c;
};
