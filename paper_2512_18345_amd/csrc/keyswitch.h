// Job-table key-switching pipeline (keyswitch.hip).
//
// A launch sequence processes up to 65535 independent jobs (grid.z = job);
// each job is a key-switch, an HMult, an HRot, or one rotation of a hoisted
// group, at its own level L.  The same nine kernels serve a single call and a
// batch, so batching adds work-groups to every launch instead of launches.
#pragma once
#include <hip/hip_runtime.h>

#include "arith.h"
#include "ctx.h"

namespace ckks {

enum KsKind : int {
  KS_PLAIN = 0,  // a = d [L][N]; out = KS(d)
  KS_HMULT = 1,  // a = ct1, b = ct2 [2][L][N]; out = (d0 + KS_0(d2), d1 + KS_1(d2))
  KS_HROT = 2,   // a = ct [2][L][N]; out = (sigma(c0) + KS_0(sigma(c1)), KS_1(sigma(c1)))
  KS_HOIST = 3,  // a = ct, b = ModUp(c1) [beta][L + k][N]; out as HROT but from sigma(ModUp(c1))
  KS_MODUP = 4,  // ModUp alone (the shared ModUp of hoisted rotations): a = d [L][N] (evaluation
                 // domain), out = M [beta][L + k][N] (every row, the digit rows copied), ws = [L][N]
};

struct __align__(16) KsJob {
  int kind;
  int L;
  uint32_t gal;        // Galois element 5^rot mod 2N (HROT, HOIST)
  int pad;
  const uint32_t* a;
  const uint32_t* b;
  const uint32_t* key;  // [beta_max][2][L_max + k][N]
  uint32_t* out;        // [2][L][N]
  uint32_t* ws;         // ks_ws_words(c, L) words of scratch (ks_hoist_ws_words for KS_HOIST)
};

struct __align__(16) RsJob {
  int L;
  int pad[3];
  const uint32_t* a;  // [2][L][N]
  uint32_t* out;      // [2][L - 1][N]
  uint32_t* ws;       // rs_ws_words(c, L) words
  const void* pad2;
};

constexpr int kInlineJobs = 16;

// NTT shape bits of Ctx::Sched::ntt_shape (whole-line column tiles and the
// ModUp INTT block pass; small grids keep their own shapes):
constexpr int kShapeFwdRadix8 = 1;   // forward column passes: 8 elements / thread, radix-8 phases (else 16, radix-16)
constexpr int kShapeInvRadix16 = 2;  // inverse column passes: 16 elements / thread, radix-16 phases (else 8, radix-8)
constexpr int kShapeK1Radix16 = 4;   // ModUp INTT block pass: 16 elements / thread on 256 threads (else 8 on 512)
constexpr int kShapeWholeLimb = 8;   // N = 2^kSrLog: two kernels with whole limbs in LDS instead of nine
constexpr int kShapeAll = 15;
constexpr int kSrGroups = 4;  // whole-limb key-switch: digit groups of its first kernel, at most

// Rows of the key inner product a K5 launch covers.
enum KsPart : int { KS_PART_ALL = 0, KS_PART_P = 1, KS_PART_Q = 2 };

// Complementary pipelining resources: a side stream and two events (fork,
// join).  side == nullptr runs the pipeline on one stream.  The Q-row inner
// product runs on the side stream either beside the P-row one (p_first =
// false: both start after ModUp) or after it (p_first = true: the Q rows
// overlap only the ModDown chain).
struct KsSplit {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool p_first = false;
};

// Jobs either inline in the kernel arguments (n <= kInlineJobs) or in a device
// table written only by the host.  get() returns the job by value through
// scalar loads, so every field is work-group uniform.
template <class J>
struct JobArg {
  const J* table;
  J inl[kInlineJobs];
  __device__ __forceinline__ J get(int z) const {
    if (table) return ldc(table + z);
    return inl[z];
  }
};

size_t ks_ws_words(const Ctx& c, int L);        // any job kind
size_t ks_hoist_ws_words(const Ctx& c, int L);  // KS_HOIST jobs only (no ModUp scratch)
size_t rs_ws_words(const Ctx& c, int L);

// Enqueue the key-switching pipeline for njobs jobs whose largest level is
// Lmax under kernel schedule sc (the context's, or a batch's own).
// with_modup: some job is not KS_HOIST (stage 1 runs); with_hoist: some job
// is KS_HOIST.
hipError_t ks_launch(const Ctx& c, const Ctx::Sched& sc, const JobArg<KsJob>& jobs, int njobs, int Lmax,
                     bool with_modup, bool with_hoist, hipStream_t st, const KsSplit& sp = KsSplit{});
// Enqueue the ModUp of njobs KS_MODUP jobs (K1-K4 and the block pass of the
// new rows: M ends fully in the evaluation domain, canonical).
hipError_t ks_modup_launch(const Ctx& c, const Ctx::Sched& sc, const JobArg<KsJob>& jobs, int njobs, int Lmax,
                           hipStream_t st);
// Enqueue rescale (drop the top prime) for njobs jobs.
hipError_t rs_launch(const Ctx& c, const JobArg<RsJob>& jobs, int njobs, int Lmax, hipStream_t st);

}  // namespace ckks
