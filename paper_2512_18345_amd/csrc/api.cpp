// C-ABI entry points (include/ckks.h): argument checks, workspace layout and
// the order of kernel launches for each operation.  Every step of every
// operation runs in the gfx950 kernels of kernels.hip; this file only
// validates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "keyswitch.h"
#include "kernels.h"

using namespace ckks;

// Key-switching scratch of ckks_hmult_noalloc, for callers that cannot
// allocate: 128 MiB per device, enough for an HMult at N = 2^16 with L = 36,
// k = 12, dnum = 3 (102 MiB).  Host code never uses the array's name as an
// address: each device's copy is reached through the pointer that
// hipGetSymbolAddress returns on that device (g_scratch_ptr).
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(CKKS_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define CKKS_TRY(expr, where)                        \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Device address of `scratch` on each device, set once per device by
// ckks_ctx_create with that device current.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_setup(int device) {
  if (device >= kMaxScratchDevices) return 0;  // ckks_hmult_noalloc refuses such devices
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return 0;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
  g_scratch_ptr[device] = p;
  return 0;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

constexpr size_t kAlign = 256;
size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace.
struct WS {
  char* base;
  size_t size, used = 0;
  uint32_t* take(size_t words) {
    uint32_t* p = reinterpret_cast<uint32_t*>(base + used);
    used += round_up(words * 4);
    return p;
  }
};

size_t words(const Ctx& c, size_t rows) { return rows * (size_t)c.N; }

size_t ws_modup(const Ctx& c, int L) { return round_up(words(c, L) * 4); }
size_t ws_moddown(const Ctx& c, int L) { return round_up(words(c, c.k) * 4) + round_up(words(c, L) * 4); }
size_t ws_keyswitch(const Ctx& c, int L) { return round_up(ks_ws_words(c, L) * 4); }
size_t ws_hoisted(const Ctx& c, int L) {
  // the shared ModUp output and its scratch, plus one KS_HOIST scratch per
  // rotation of a chunk of up to kInlineJobs rotations
  return round_up(words(c, (size_t)c.beta(L) * (L + c.k)) * 4) + ws_modup(c, L) +
         (size_t)kInlineJobs * round_up(ks_hoist_ws_words(c, L) * 4);
}
size_t ws_bytes(const Ctx& c, int op, int L) {
  switch (op) {
    case CKKS_OP_NTT: return 0;
    case CKKS_OP_MODUP: return ws_modup(c, L);
    case CKKS_OP_MODDOWN: return ws_moddown(c, L);
    case CKKS_OP_KEYSWITCH:
    case CKKS_OP_HMULT:
    case CKKS_OP_HROT: return ws_keyswitch(c, L);
    case CKKS_OP_HROT_HOISTED: return ws_hoisted(c, L);
    case CKKS_OP_RESCALE: return round_up(rs_ws_words(c, L) * 4);
    default: return 0;
  }
}

int check_level(const ckks_ctx* ctx, int L, int lo = 1) {
  if (!ctx) return fail(CKKS_EINVAL, "null context");
  if (L < lo || L > ctx->c.L_max)
    return fail(CKKS_EINVAL, "level L=" + std::to_string(L) + " outside [" + std::to_string(lo) +
                                 ", " + std::to_string(ctx->c.L_max) + "]");
  return CKKS_OK;
}

int check_ws(const Ctx& c, int op, int L, const void* ws, size_t ws_bytes_given) {
  const size_t need = ws_bytes(c, op, L);
  if (need && !ws) return fail(CKKS_EINVAL, "null workspace");
  if (ws_bytes_given < need)
    return fail(CKKS_ENOMEM, "workspace of " + std::to_string(ws_bytes_given) + " bytes < " +
                                 std::to_string(need) + " needed");
  return CKKS_OK;
}

uint32_t galois(const Ctx& c, int rot) {
  const uint64_t two_n = 2ull * c.N;
  const uint64_t half = (uint64_t)c.N / 2;
  uint64_t e = ((int64_t)rot % (int64_t)half + (int64_t)half) % half;
  uint64_t g = 1, b = 5;
  while (e) {
    if (e & 1) g = g * b % two_n;
    b = b * b % two_n;
    e >>= 1;
  }
  return (uint32_t)g;
}

// ---- compositions ---------------------------------------------------------

// ModDown of a [L + k][N] into out [L][N] (+ add if non-null); x: [k][N], z: [L][N] scratch.
int moddown_impl(const Ctx& c, const uint32_t* a, int L, const uint32_t* add, uint32_t* out,
                 uint32_t* x, uint32_t* z, hipStream_t st) {
  const size_t N = c.N;
  CKKS_TRY(launch_intt(c, a + (size_t)L * N, x, c.k, RowMap{0, c.L_max}, 0, 0, c.d_moddown_scale,
                       c.L_max, st),
           "ModDown INTT");
  CKKS_TRY(launch_bconv(c, c.rows(L), x, c.k, z, L, 0, 0, c.d_moddown_T, c.k, st), "ModDown BConv");
  CKKS_TRY(launch_ntt(c, z, z, L, c.rows(L), 0, 0, st), "ModDown NTT");
  CKKS_TRY(launch_moddown_combine(c, L, a, z, add, out, st), "ModDown combine");
  return CKKS_OK;
}

// One job through the fused pipeline.
int run_one(const Ctx& c, int kind, int L, uint32_t gal, const uint32_t* a, const uint32_t* b,
            const uint32_t* key, uint32_t* out, void* ws, hipStream_t st) {
  JobArg<KsJob> ja{};
  ja.table = nullptr;
  ja.inl[0] = KsJob{kind, L, gal, 0, a, b, key, out, (uint32_t*)ws};
  CKKS_TRY(ks_launch(c, c.sched, ja, 1, L, true, false, st), "key-switching pipeline");
  return CKKS_OK;
}

}  // namespace

namespace ckks {
int api_fail(int code, const std::string& msg) { return fail(code, msg); }
uint32_t api_galois(const Ctx& c, int rot) { return galois(c, rot); }
}  // namespace ckks

constexpr int kMaxBranches = 4;

struct ckks_batch {
  const Ctx* c = nullptr;
  int n_ks = 0, n_rs = 0, Lmax_rs = 0;
  std::vector<int> L_ks;  // levels of the key-switching jobs in table order (non-increasing)
  KsJob* d_ks = nullptr;
  RsJob* d_rs = nullptr;
  // host copies of the tables: launch groups of at most kInlineJobs jobs
  // carry their jobs in the kernel arguments (no table read at kernel start)
  std::vector<KsJob> h_ks;
  std::vector<RsJob> h_rs;
  void* d_ws = nullptr;
  size_t bytes = 0;
  bool use_graph = false;
  ckks_batch_plan plan{0, 1, 1, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  // branch 0 is the launch stream; branches 1.. and every branch's side
  // stream (complementary pipelining) belong to the batch
  hipStream_t branch[kMaxBranches] = {};
  hipStream_t side[kMaxBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxBranches] = {};
  std::vector<hipEvent_t> gev;  // fork / join events of the split, two per launch group
  std::vector<std::pair<ckks_batch_plan, float>> tune_log;  // last ckks_batch_tune: plan, us
  Ctx::Sched sched;  // kernel schedule of this batch's launches (the context's at creation)
};

namespace {

// Key-switching jobs are kept in non-increasing level order, so a launch
// group of consecutive jobs has a tight largest level.  Group g (B jobs)
// runs on branch g mod S; the rescale jobs run on the last branch; all
// branches fork from and join back to the launch stream.
hipError_t batch_enqueue(ckks_batch* b, hipStream_t st) {
  const Ctx& c = *b->c;
  const int S = b->plan.streams;
  const int B = b->plan.jobs_per_launch > 0 ? std::min(b->plan.jobs_per_launch, b->n_ks) : b->n_ks;
  auto on = [&](int br) { return br == 0 ? st : b->branch[br]; };
  hipError_t e;
  if (S > 1) {
    if ((e = hipEventRecord(b->fork, st)) != hipSuccess) return e;
    for (int br = 1; br < S; ++br)
      if ((e = hipStreamWaitEvent(b->branch[br], b->fork, 0)) != hipSuccess) return e;
  }
  int group = 0;
  for (int s0 = 0; s0 < b->n_ks; s0 += B, ++group) {
    const int br = group % S;
    JobArg<KsJob> ka{};
    const int cnt = std::min(B, b->n_ks - s0);
    if (cnt <= kInlineJobs) {
      ka.table = nullptr;
      for (int t = 0; t < cnt; ++t) ka.inl[t] = b->h_ks[s0 + t];
    } else {
      ka.table = b->d_ks + s0;
    }
    if (b->plan.split && b->gev.size() < 2 * (size_t)group + 2) return hipErrorInvalidValue;
    const KsSplit sp = b->plan.split
                           ? KsSplit{b->side[br], b->gev[2 * group], b->gev[2 * group + 1], b->plan.split == 2}
                           : KsSplit{};
    if ((e = ks_launch(c, b->sched, ka, cnt, b->L_ks[s0], true, false, on(br), sp)) !=
        hipSuccess)
      return e;
  }
  if (b->n_rs) {
    JobArg<RsJob> ra{};
    if (b->n_rs <= kInlineJobs) {
      ra.table = nullptr;
      for (int t = 0; t < b->n_rs; ++t) ra.inl[t] = b->h_rs[t];
    } else {
      ra.table = b->d_rs;
    }
    if ((e = rs_launch(c, ra, b->n_rs, b->Lmax_rs, on(S - 1))) != hipSuccess) return e;
  }
  if (S > 1) {
    for (int br = 1; br < S; ++br) {
      if ((e = hipEventRecord(b->join[br], b->branch[br])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st, b->join[br], 0)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

int batch_groups(const ckks_batch* b, const ckks_batch_plan& p) {
  if (b->n_ks == 0) return 0;
  const int B = p.jobs_per_launch > 0 ? std::min(p.jobs_per_launch, b->n_ks) : b->n_ks;
  return (b->n_ks + B - 1) / B;
}

// Two events per launch group, so no event is recorded twice in one launch
// sequence (in particular not inside one graph capture).
hipError_t batch_events(ckks_batch* b, const ckks_batch_plan& p) {
  const size_t need = 2 * (size_t)batch_groups(b, p);
  while (b->gev.size() < need) {
    hipEvent_t ev;
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    b->gev.push_back(ev);
  }
  return hipSuccess;
}

void batch_drop_graph(ckks_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Capture the batch's launch sequence under its current plan and schedule.
// The new graph replaces the old one only once it is instantiated; on failure
// the batch keeps the graph it had.
hipError_t batch_capture(ckks_batch* b) {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t le = batch_enqueue(b, b->capture);
  e = hipStreamEndCapture(b->capture, &graph);
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return e;
  }
  batch_drop_graph(b);
  b->graph = graph;
  b->exec = exec;
  return hipSuccess;
}

void batch_free(ckks_batch* b) {
  batch_drop_graph(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  for (int i = 0; i < kMaxBranches; ++i) {
    if (b->branch[i]) (void)hipStreamDestroy(b->branch[i]);
    if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
    if (b->join[i]) (void)hipEventDestroy(b->join[i]);
  }
  for (hipEvent_t ev : b->gev) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->d_ks) (void)hipFree(b->d_ks);
  if (b->d_rs) (void)hipFree(b->d_rs);
  if (b->d_ws) (void)hipFree(b->d_ws);
  delete b;
}

bool plan_ok(const ckks_batch_plan& p) {
  return p.jobs_per_launch >= 0 && p.streams >= 1 && p.streams <= kMaxBranches && p.split >= 0 &&
         p.split <= 2;
}

}  // namespace

extern "C" {

const char* ckks_last_error(void) { return g_err.c_str(); }

int ckks_ctx_create(ckks_ctx** out, int logN, const uint32_t* h_q, int L_max, const uint32_t* h_p,
                    int k, int dnum, int device) {
  if (!out || !h_q || !h_p) return fail(CKKS_EINVAL, "null argument");
  *out = nullptr;
  if (logN < kMinLogN || logN > kMaxLogN)
    return fail(CKKS_EUNSUPPORTED, "logN must be in [12, 16]");
  if (L_max < 1 || k < 1 || dnum < 1 || L_max + k > kMaxPrimes)
    return fail(CKKS_EINVAL, "need L_max >= 1, k >= 1, dnum >= 1, L_max + k <= 64");
  const int alpha = (L_max + dnum - 1) / dnum;
  if (alpha != k) return fail(CKKS_EINVAL, "digit size ceil(L_max / dnum) must equal k");
  if (alpha > kMaxAlpha) return fail(CKKS_EUNSUPPORTED, "digit size above 16");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(CKKS_EINVAL, "no such HIP device");
  DeviceGuard g(device);
  if (!g.ok) return fail(CKKS_EHIP, "hipSetDevice failed");
  if (const int rc = scratch_setup(device)) return rc;
  ckks_ctx* ctx = new (std::nothrow) ckks_ctx;
  if (!ctx) return fail(CKKS_ENOMEM, "host allocation failed");
  Ctx& c = ctx->c;
  c.device = device;
  c.logN = logN;
  c.N = 1 << logN;
  c.L_max = L_max;
  c.k = k;
  c.dnum = dnum;
  c.alpha = alpha;
  int code = CKKS_OK;
  const std::string err = build_tables(c, h_q, h_p, &code);
  if (code != CKKS_OK) {
    free_tables(c);
    delete ctx;
    return fail(code, err);
  }
  // small rings run the key-switch on whole limbs by default
  if (c.logN == kSrLog) c.sched.ntt_shape = kShapeWholeLimb;
  *out = ctx;
  return CKKS_OK;
}

int ckks_ctx_destroy(ckks_ctx* ctx) {
  if (!ctx) return CKKS_OK;
  DeviceGuard g(ctx->c.device);
  free_tables(ctx->c);
  delete ctx;
  return CKKS_OK;
}

size_t ckks_workspace_bytes(const ckks_ctx* ctx, int op, int L) {
  if (!ctx || L < 1 || L > ctx->c.L_max) return 0;
  return ws_bytes(ctx->c, op, L);
}

static int ntt_common(const ckks_ctx* ctx, uint32_t* a, int L, int with_P, void* stream, bool inv) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!a) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  DeviceGuard g(c.device);
  const int rows = L + (with_P ? c.k : 0);
  const hipStream_t st = (hipStream_t)stream;
  if (inv)
    CKKS_TRY(launch_intt(c, a, a, rows, c.rows(L), 0, 0, nullptr, 0, st), "INTT");
  else
    CKKS_TRY(launch_ntt(c, a, a, rows, c.rows(L), 0, 0, st), "NTT");
  return CKKS_OK;
}

int ckks_ntt(const ckks_ctx* ctx, uint32_t* a, int L, int with_P, void* stream) {
  return ntt_common(ctx, a, L, with_P, stream, false);
}

int ckks_intt(const ckks_ctx* ctx, uint32_t* a, int L, int with_P, void* stream) {
  return ntt_common(ctx, a, L, with_P, stream, true);
}

int ckks_automorph(const ckks_ctx* ctx, const uint32_t* in, uint32_t* out, int rows, int rot,
                   void* stream) {
  if (!ctx) return fail(CKKS_EINVAL, "null context");
  if (!in || !out || rows < 1) return fail(CKKS_EINVAL, "bad automorphism arguments");
  if (in == out) return fail(CKKS_EINVAL, "automorphism output aliases its input");
  const Ctx& c = ctx->c;
  DeviceGuard g(c.device);
  CKKS_TRY(launch_automorph(c, in, out, rows, galois(c, rot), (hipStream_t)stream), "automorphism");
  return CKKS_OK;
}

int ckks_tensor(const ckks_ctx* ctx, const uint32_t* ct1, const uint32_t* ct2, int L, uint32_t* out,
                void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!ct1 || !ct2 || !out) return fail(CKKS_EINVAL, "null data pointer");
  DeviceGuard g(ctx->c.device);
  CKKS_TRY(launch_tensor(ctx->c, ct1, ct2, L, out, (hipStream_t)stream), "tensor");
  return CKKS_OK;
}

int ckks_pmult_sum(const ckks_ctx* ctx, const uint32_t* const* h_cts, const uint32_t* const* h_pts,
                   int nb, int L, uint32_t* out, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!h_cts || !h_pts || !out || nb < 1 || nb > 16) return fail(CKKS_EINVAL, "bad pmult_sum arguments");
  for (int b = 0; b < nb; ++b)
    if (!h_cts[b] || !h_pts[b]) return fail(CKKS_EINVAL, "null ciphertext or plaintext pointer");
  DeviceGuard g(ctx->c.device);
  CKKS_TRY(launch_pmult_sum(ctx->c, h_cts, h_pts, nb, L, out, (hipStream_t)stream), "pmult_sum");
  return CKKS_OK;
}

int ckks_pmult_sums(const ckks_ctx* ctx, const uint32_t* const* h_cts, int nb, const uint32_t* const* h_pts,
                    int ng, int L, uint32_t* const* h_outs, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!h_cts || !h_pts || !h_outs || nb < 1 || nb > 16 || ng < 1 || ng > 8)
    return fail(CKKS_EINVAL, "bad pmult_sums arguments (1 <= nb <= 16, 1 <= ng <= 8)");
  for (int b = 0; b < nb; ++b)
    if (!h_cts[b]) return fail(CKKS_EINVAL, "null ciphertext pointer");
  for (int g = 0; g < ng; ++g) {
    if (!h_outs[g]) return fail(CKKS_EINVAL, "null output pointer");
    for (int b = 0; b < nb; ++b)
      if (!h_pts[g * nb + b]) return fail(CKKS_EINVAL, "null plaintext pointer");
  }
  DeviceGuard g(ctx->c.device);
  CKKS_TRY(launch_pmult_sums(ctx->c, h_cts, nb, h_pts, ng, L, h_outs, (hipStream_t)stream), "pmult_sums");
  return CKKS_OK;
}

int ckks_add(const ckks_ctx* ctx, const uint32_t* a, const uint32_t* b, int L, uint32_t* out,
             void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!a || !b || !out) return fail(CKKS_EINVAL, "null data pointer");
  DeviceGuard g(ctx->c.device);
  CKKS_TRY(launch_ct_add(ctx->c, a, b, L, out, (hipStream_t)stream), "add");
  return CKKS_OK;
}

int ckks_modup(const ckks_ctx* ctx, const uint32_t* d, int L, uint32_t* out, void* ws,
               size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!d || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_MODUP, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  JobArg<KsJob> mj{};
  mj.table = nullptr;
  mj.inl[0] = KsJob{KS_MODUP, L, 0, 0, d, nullptr, nullptr, out, (uint32_t*)ws};
  CKKS_TRY(ks_modup_launch(c, c.sched, mj, 1, L, (hipStream_t)stream), "ModUp");
  return CKKS_OK;
}

int ckks_inner_product(const ckks_ctx* ctx, const uint32_t* M, int L, const uint32_t* evk,
                       uint32_t* acc, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!M || !evk || !acc) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  DeviceGuard g(c.device);
  CKKS_TRY(launch_inner_product(c, c.rows(L), M, c.beta(L), L + c.k, evk, acc, (hipStream_t)stream),
           "inner product");
  return CKKS_OK;
}

int ckks_moddown(const ckks_ctx* ctx, const uint32_t* in, int L, uint32_t* out, void* ws,
                 size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!in || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_MODDOWN, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  WS w{(char*)ws, ws_bytes_given};
  uint32_t* x = w.take(words(c, c.k));
  uint32_t* z = w.take(words(c, L));
  return moddown_impl(c, in, L, nullptr, out, x, z, (hipStream_t)stream);
}

int ckks_keyswitch(const ckks_ctx* ctx, const uint32_t* d, int L, const uint32_t* evk,
                   uint32_t* out, void* ws, size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!d || !evk || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_KEYSWITCH, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  return run_one(c, KS_PLAIN, L, 0, d, nullptr, evk, out, ws, (hipStream_t)stream);
}

int ckks_hmult(const ckks_ctx* ctx, const uint32_t* ct1, const uint32_t* ct2, int L,
               const uint32_t* rlk, uint32_t* out, void* ws, size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!ct1 || !ct2 || !rlk || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_HMULT, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  return run_one(c, KS_HMULT, L, 0, ct1, ct2, rlk, out, ws, (hipStream_t)stream);
}

int ckks_hmult_noalloc(const ckks_ctx* ctx, const uint32_t* ct1, const uint32_t* ct2, int L,
                       const uint32_t* rlk, uint32_t* out, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!ct1 || !ct2 || !rlk || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  const size_t need = ws_bytes(c, CKKS_OP_HMULT, L);
  if (need > kScratchBytes)
    return fail(CKKS_ENOMEM, "HMult at L=" + std::to_string(L) + " needs " + std::to_string(need) +
                                 " bytes of scratch; the static scratch holds " +
                                 std::to_string(kScratchBytes));
  void* ws = scratch_ptr(c.device);
  if (!ws) return fail(CKKS_EUNSUPPORTED, "no static scratch on device " + std::to_string(c.device));
  DeviceGuard g(c.device);
  return run_one(c, KS_HMULT, L, 0, ct1, ct2, rlk, out, ws, (hipStream_t)stream);
}

int ckks_hrot(const ckks_ctx* ctx, const uint32_t* ct, int L, int rot, const uint32_t* rotk,
              uint32_t* out, void* ws, size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!ct || !rotk || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_HROT, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  return run_one(c, KS_HROT, L, galois(c, rot), ct, nullptr, rotk, out, ws, (hipStream_t)stream);
}

int ckks_hrot_many(const ckks_ctx* ctx, const uint32_t* const* h_cts, int L, const int* h_rots,
                   const uint32_t* const* h_rotks, uint32_t* const* h_outs, int n, void* ws,
                   size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!h_cts || !h_rots || !h_rotks || !h_outs || n < 1 || n > kInlineJobs)
    return fail(CKKS_EINVAL, "bad rotation-list arguments (1 <= n <= 16)");
  for (int i = 0; i < n; ++i)
    if (!h_cts[i] || !h_rotks[i] || !h_outs[i]) return fail(CKKS_EINVAL, "null ciphertext, key or output pointer");
  const Ctx& c = ctx->c;
  const size_t per = ws_bytes(c, CKKS_OP_HROT, L);
  if (!ws) return fail(CKKS_EINVAL, "null workspace");
  if (ws_bytes_given < per * n)
    return fail(CKKS_ENOMEM, "workspace of " + std::to_string(ws_bytes_given) + " bytes < " +
                                 std::to_string(per * n) + " needed (n times the HRot workspace)");
  DeviceGuard g(c.device);
  // the jobs of one launch sequence, each with its own slice of the workspace
  JobArg<KsJob> ja{};
  ja.table = nullptr;
  for (int i = 0; i < n; ++i)
    ja.inl[i] = KsJob{KS_HROT, L, galois(c, h_rots[i]), 0, h_cts[i], nullptr, h_rotks[i], h_outs[i],
                      (uint32_t*)((char*)ws + per * i)};
  CKKS_TRY(ks_launch(c, c.sched, ja, n, L, true, false, (hipStream_t)stream), "key-switching pipeline");
  return CKKS_OK;
}

int ckks_hrot_hoisted(const ckks_ctx* ctx, const uint32_t* ct, int L, const int* h_rots, int n,
                      const uint32_t* const* h_rotks, uint32_t* const* h_outs, void* ws,
                      size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (!ct || !h_rots || !h_rotks || !h_outs || n < 1)
    return fail(CKKS_EINVAL, "bad hoisted-rotation arguments");
  for (int i = 0; i < n; ++i)
    if (!h_rotks[i] || !h_outs[i]) return fail(CKKS_EINVAL, "null key or output pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_HROT_HOISTED, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  const hipStream_t st = (hipStream_t)stream;
  const size_t N = c.N;
  WS w{(char*)ws, ws_bytes_given};
  uint32_t* M = w.take(words(c, (size_t)c.beta(L) * (L + c.k)));
  uint32_t* y = w.take(words(c, L));
  // the shared ModUp of c1 through the fused stage-1 kernels
  JobArg<KsJob> mj{};
  mj.table = nullptr;
  mj.inl[0] = KsJob{KS_MODUP, L, 0, 0, ct + (size_t)L * N, nullptr, nullptr, M, y};
  CKKS_TRY(ks_modup_launch(c, c.sched, mj, 1, L, st), "hoisted ModUp");
  uint32_t* job_ws[kInlineJobs];
  for (int i = 0; i < kInlineJobs; ++i) job_ws[i] = w.take(ks_hoist_ws_words(c, L));
  for (int i0 = 0; i0 < n; i0 += kInlineJobs) {
    const int cnt = std::min(kInlineJobs, n - i0);
    JobArg<KsJob> ja{};
    ja.table = nullptr;
    for (int t = 0; t < cnt; ++t)
      ja.inl[t] = KsJob{KS_HOIST, L, galois(c, h_rots[i0 + t]), 0, ct, M, h_rotks[i0 + t],
                        h_outs[i0 + t], job_ws[t]};
    CKKS_TRY(ks_launch(c, c.sched, ja, cnt, L, false, true, st), "hoisted rotations");
  }
  return CKKS_OK;
}

int ckks_rescale(const ckks_ctx* ctx, const uint32_t* ct, int L, uint32_t* out, void* ws,
                 size_t ws_bytes_given, void* stream) {
  int rc = check_level(ctx, L, 2);
  if (rc) return rc;
  if (!ct || !out) return fail(CKKS_EINVAL, "null data pointer");
  const Ctx& c = ctx->c;
  if ((rc = check_ws(c, CKKS_OP_RESCALE, L, ws, ws_bytes_given))) return rc;
  DeviceGuard g(c.device);
  JobArg<RsJob> ja{};
  ja.table = nullptr;
  ja.inl[0] = RsJob{L, {0, 0, 0}, ct, out, (uint32_t*)ws, nullptr};
  CKKS_TRY(rs_launch(c, ja, 1, L, (hipStream_t)stream), "rescale");
  return CKKS_OK;
}

int ckks_ctx_get_schedule(const ckks_ctx* ctx, ckks_schedule* sched) {
  if (!ctx || !sched) return fail(CKKS_EINVAL, "null argument");
  const Ctx::Sched& s = ctx->c.sched;
  *sched = ckks_schedule{s.up_rows, s.down_rows, s.small_grid, s.ntt_shape};
  return CKKS_OK;
}

namespace {
bool sched_ok(const ckks_schedule& s) {
  auto rows_ok = [](int r) { return r == 2 || r == 4 || r == 6 || r == 12; };
  return rows_ok(s.bconv_up_rows) && rows_ok(s.bconv_down_rows) && s.small_grid >= 0 &&
         s.small_grid <= 65535 && s.ntt_shape >= 0 && s.ntt_shape <= kShapeAll;
}
}  // namespace

int ckks_ctx_set_schedule(ckks_ctx* ctx, const ckks_schedule* sched) {
  if (!ctx || !sched) return fail(CKKS_EINVAL, "null argument");
  if (!sched_ok(*sched))
    return fail(CKKS_EINVAL, "schedule needs rows in {2, 4, 6, 12}, 0 <= small_grid <= 65535, 0 <= ntt_shape <= 15");
  ctx->c.sched = Ctx::Sched{sched->bconv_up_rows, sched->bconv_down_rows, sched->small_grid, sched->ntt_shape};
  return CKKS_OK;
}

int ckks_ctx_tune(ckks_ctx* ctx, int L, int reps, void* stream, ckks_schedule* best, float* best_us) {
  int rc = check_level(ctx, L);
  if (rc) return rc;
  if (reps < 1 || reps > 1000) return fail(CKKS_EINVAL, "need 1 <= reps <= 1000");
  Ctx& c = ctx->c;
  DeviceGuard g(c.device);
  const hipStream_t st = (hipStream_t)stream;
  const size_t N = c.N;
  const size_t ct_b = 2 * (size_t)L * N * 4;
  const size_t key_b = (size_t)c.beta_max() * 2 * (c.L_max + c.k) * N * 4;
  const size_t ws_b = round_up(ks_ws_words(c, L) * 4);
  void *d_ct = nullptr, *d_key = nullptr, *d_out = nullptr, *d_ws = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto cleanup = [&]() {
    if (d_ct) (void)hipFree(d_ct);
    if (d_key) (void)hipFree(d_key);
    if (d_out) (void)hipFree(d_out);
    if (d_ws) (void)hipFree(d_ws);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  if (hipMalloc(&d_ct, 2 * ct_b) != hipSuccess || hipMalloc(&d_key, key_b) != hipSuccess ||
      hipMalloc(&d_out, ct_b) != hipSuccess || hipMalloc(&d_ws, ws_b) != hipSuccess) {
    cleanup();
    return fail(CKKS_ENOMEM, "tuning buffers");
  }
  hipError_t e = hipMemsetAsync(d_ct, 0, 2 * ct_b, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_key, 0, key_b, st);
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  const Ctx::Sched start = c.sched;
  Ctx::Sched top = start;
  float top_us = -1.f;
  const uint32_t* ct1 = (const uint32_t*)d_ct;
  const uint32_t* ct2 = (const uint32_t*)((char*)d_ct + ct_b);
  for (int shape = 0; shape <= kShapeAll; ++shape)
  for (int up : {12, 6, 4, 2}) {
    if ((shape & kShapeWholeLimb) && c.logN != kSrLog) break;  // the bit means nothing there
    for (int down : {6, 12, 4, 2}) {
      for (int small : {128, 0, 1024}) {
        if (e != hipSuccess) break;
        c.sched = Ctx::Sched{up, down, small, shape};
        auto once = [&]() {
          return run_one(c, KS_HMULT, L, 0, ct1, ct2, (const uint32_t*)d_key, (uint32_t*)d_out, d_ws, st);
        };
        if (once() != CKKS_OK) {
          e = hipErrorUnknown;
          break;
        }
        if ((e = hipEventRecord(t0, st)) != hipSuccess) break;
        for (int r = 0; r < reps; ++r)
          if (once() != CKKS_OK) {
            e = hipErrorUnknown;
            break;
          }
        if (e != hipSuccess || (e = hipEventRecord(t1, st)) != hipSuccess ||
            (e = hipEventSynchronize(t1)) != hipSuccess)
          break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
        const float us = 1e3f * ms / reps;
        if (top_us < 0.f || us < top_us) {
          top_us = us;
          top = c.sched;
        }
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  c.sched = e == hipSuccess ? top : start;
  if (e != hipSuccess) return hip_fail(e, "timing candidate schedules");
  if (best) *best = ckks_schedule{top.up_rows, top.down_rows, top.small_grid, top.ntt_shape};
  if (best_us) *best_us = top_us;
  return CKKS_OK;
}

int ckks_batch_create(const ckks_ctx* ctx, const ckks_job* h_jobs, int n, int use_graph,
                      ckks_batch** out) {
  if (!ctx || !h_jobs || !out || n < 1 || n > 65535) return fail(CKKS_EINVAL, "bad batch arguments");
  *out = nullptr;
  const Ctx& c = ctx->c;
  std::vector<KsJob> ks;
  std::vector<RsJob> rs;
  std::vector<size_t> ks_off, rs_off;
  size_t ws = 0;
  int Lrs = 0;
  for (int i = 0; i < n; ++i) {
    const ckks_job& j = h_jobs[i];
    const int lo = j.op == CKKS_JOB_RESCALE ? 2 : 1;
    if (j.L < lo || j.L > c.L_max || !j.in0 || !j.out)
      return fail(CKKS_EINVAL, "job " + std::to_string(i) + ": bad level or null pointer");
    if (j.op == CKKS_JOB_RESCALE) {
      rs.push_back(RsJob{j.L, {0, 0, 0}, j.in0, j.out, nullptr, nullptr});
      rs_off.push_back(ws);
      ws += round_up(rs_ws_words(c, j.L) * 4);
      Lrs = std::max(Lrs, j.L);
    } else if (j.op == CKKS_JOB_KEYSWITCH || j.op == CKKS_JOB_HMULT || j.op == CKKS_JOB_HROT) {
      if (!j.key || (j.op == CKKS_JOB_HMULT && !j.in1))
        return fail(CKKS_EINVAL, "job " + std::to_string(i) + ": null key or second input");
      const int kind = j.op == CKKS_JOB_KEYSWITCH ? KS_PLAIN : j.op == CKKS_JOB_HMULT ? KS_HMULT : KS_HROT;
      ks.push_back(KsJob{kind, j.L, j.op == CKKS_JOB_HROT ? galois(c, j.rot) : 0u, 0, j.in0,
                         j.op == CKKS_JOB_HMULT ? j.in1 : nullptr, j.key, j.out, nullptr});
      ks_off.push_back(ws);
      ws += round_up(ks_ws_words(c, j.L) * 4);
    } else {
      return fail(CKKS_EINVAL, "job " + std::to_string(i) + ": unknown op");
    }
  }
  // Non-increasing level order; jobs of one level that share a key are adjacent.
  std::vector<int> order(ks.size());
  for (size_t i = 0; i < ks.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (ks[x].L != ks[y].L) return ks[x].L > ks[y].L;
    return ks[x].key < ks[y].key;
  });
  DeviceGuard g(c.device);
  ckks_batch* b = new (std::nothrow) ckks_batch;
  if (!b) return fail(CKKS_ENOMEM, "host allocation failed");
  b->c = &c;
  b->n_ks = (int)ks.size();
  b->n_rs = (int)rs.size();
  b->Lmax_rs = Lrs;
  b->use_graph = use_graph != 0;
  b->sched = ctx->c.sched;
  // complementary pipelining pays off only when a launch group holds several
  // jobs; a lone key-switch runs unsplit, as a single call does.  On a small
  // ring with the whole-limb schedule the unsplit launch (two kernels) is the
  // faster one until its first kernel needs about 800 work-groups: HMults at
  // N = 2^12, L = 4 (20 work-groups each) measured 1.4-2.3x faster unsplit for
  // 2-32 jobs and even at 48.
  const int Lks = ks.empty() ? 0 : ks[order[0]].L;
  const bool whole_limb = c.logN == kSrLog && (b->sched.ntt_shape & kShapeWholeLimb);
  const long sr_wgs = (long)(Lks + c.k) * std::min(c.beta(std::max(Lks, 1)), kSrGroups) * b->n_ks;
  b->plan.split = b->n_ks >= 2 && !(whole_limb && sr_wgs <= 800) ? 1 : 0;
  const size_t tab = round_up(sizeof(KsJob) * ks.size()) + round_up(sizeof(RsJob) * rs.size());
  if (hipMalloc(&b->d_ws, ws) != hipSuccess ||
      (!ks.empty() && hipMalloc(&b->d_ks, sizeof(KsJob) * ks.size()) != hipSuccess) ||
      (!rs.empty() && hipMalloc(&b->d_rs, sizeof(RsJob) * rs.size()) != hipSuccess)) {
    batch_free(b);
    return fail(CKKS_ENOMEM, "device allocation for the batch failed");
  }
  b->bytes = ws + tab;
  std::vector<KsJob> sorted;
  for (int i : order) {
    sorted.push_back(ks[i]);
    sorted.back().ws = (uint32_t*)((char*)b->d_ws + ks_off[i]);
    b->L_ks.push_back(ks[i].L);
  }
  for (size_t i = 0; i < rs.size(); ++i) rs[i].ws = (uint32_t*)((char*)b->d_ws + rs_off[i]);
  b->h_ks = sorted;
  b->h_rs = rs;
  if ((!ks.empty() && hipMemcpy(b->d_ks, sorted.data(), sizeof(KsJob) * ks.size(), hipMemcpyHostToDevice) != hipSuccess) ||
      (!rs.empty() && hipMemcpy(b->d_rs, rs.data(), sizeof(RsJob) * rs.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    batch_free(b);
    return fail(CKKS_EHIP, "copying the job table failed");
  }
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < kMaxBranches; ++i)
    ok = (i == 0 || hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking) == hipSuccess) &&
         hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) == hipSuccess;
  ok = ok && batch_events(b, b->plan) == hipSuccess;
  if (!ok) {
    batch_free(b);
    return fail(CKKS_EHIP, "creating the batch's streams / events failed");
  }
  if (b->use_graph) {
    hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = batch_capture(b);
    if (e != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "capturing the batch graph");
    }
  }
  *out = b;
  return CKKS_OK;
}

int ckks_batch_launch(ckks_batch* b, void* stream) {
  if (!b) return fail(CKKS_EINVAL, "null batch");
  DeviceGuard g(b->c->device);
  const hipStream_t st = (hipStream_t)stream;
  if (b->use_graph) {
    if (!b->exec) return fail(CKKS_EHIP, "the batch has no instantiated graph");
    CKKS_TRY(hipGraphLaunch(b->exec, st), "hipGraphLaunch");
  } else {
    CKKS_TRY(batch_enqueue(b, st), "batch launch");
  }
  return CKKS_OK;
}

int ckks_batch_get_plan(const ckks_batch* b, ckks_batch_plan* plan) {
  if (!b || !plan) return fail(CKKS_EINVAL, "null argument");
  *plan = b->plan;
  return CKKS_OK;
}

int ckks_batch_set_plan(ckks_batch* b, const ckks_batch_plan* plan) {
  if (!b || !plan) return fail(CKKS_EINVAL, "null argument");
  if (!plan_ok(*plan))
    return fail(CKKS_EINVAL, "plan needs jobs_per_launch >= 0, 1 <= streams <= 4, split in {0, 1, 2}");
  if (b->use_graph && plan->streams > 1)
    return fail(CKKS_EUNSUPPORTED, "a graph batch runs one branch (streams = 1)");
  DeviceGuard g(b->c->device);
  CKKS_TRY(batch_events(b, *plan), "creating the batch's events");
  const ckks_batch_plan old = b->plan;
  b->plan = *plan;
  b->plan.reserved = 0;
  if (b->use_graph) {
    const hipError_t e = batch_capture(b);
    if (e != hipSuccess) {
      b->plan = old;  // the old graph is still in place
      return hip_fail(e, "re-capturing the batch graph");
    }
  }
  return CKKS_OK;
}

int ckks_batch_get_schedule(const ckks_batch* b, ckks_schedule* sched) {
  if (!b || !sched) return fail(CKKS_EINVAL, "null argument");
  *sched = ckks_schedule{b->sched.up_rows, b->sched.down_rows, b->sched.small_grid, b->sched.ntt_shape};
  return CKKS_OK;
}

int ckks_batch_set_schedule(ckks_batch* b, const ckks_schedule* sched) {
  if (!b || !sched) return fail(CKKS_EINVAL, "null argument");
  if (!sched_ok(*sched))
    return fail(CKKS_EINVAL, "schedule needs rows in {2, 4, 6, 12} and 0 <= small_grid <= 65535");
  DeviceGuard g(b->c->device);
  const Ctx::Sched old = b->sched;
  b->sched = Ctx::Sched{sched->bconv_up_rows, sched->bconv_down_rows, sched->small_grid, sched->ntt_shape};
  if (b->use_graph) {
    const hipError_t e = batch_capture(b);
    if (e != hipSuccess) {
      b->sched = old;  // the old graph is still in place
      return hip_fail(e, "re-capturing the batch graph");
    }
  }
  return CKKS_OK;
}

int ckks_batch_tune(ckks_batch* b, int reps, void* stream, ckks_batch_plan* best, float* best_us) {
  if (!b || reps < 1 || reps > 1000) return fail(CKKS_EINVAL, "need a batch and 1 <= reps <= 1000");
  DeviceGuard g(b->c->device);
  const hipStream_t st = (hipStream_t)stream;
  std::vector<int> sizes{0};
  for (int B : {32, 16, 8, 4, 2})
    if (B < b->n_ks) sizes.push_back(B);
  hipEvent_t t0, t1;
  CKKS_TRY(hipEventCreate(&t0), "hipEventCreate");
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return fail(CKKS_EHIP, "hipEventCreate failed");
  }
  // one warm-up and `reps` timed launches of the batch as it stands
  // (re-captured first for a graph batch); microseconds per launch
  auto time_it = [&](float* us) -> hipError_t {
    hipError_t te = b->use_graph ? batch_capture(b) : hipSuccess;
    auto launch = [&]() { return b->use_graph ? hipGraphLaunch(b->exec, st) : batch_enqueue(b, st); };
    if (te == hipSuccess) te = launch();
    if (te == hipSuccess) te = hipEventRecord(t0, st);
    for (int r = 0; r < reps && te == hipSuccess; ++r) te = launch();
    if (te == hipSuccess) te = hipEventRecord(t1, st);
    if (te == hipSuccess) te = hipEventSynchronize(t1);
    float ms = 0.f;
    if (te == hipSuccess) te = hipEventElapsedTime(&ms, t0, t1);
    *us = 1e3f * ms / reps;
    return te;
  };
  const ckks_batch_plan start = b->plan;
  const Ctx::Sched start_sched = b->sched;
  ckks_batch_plan top = start;
  Ctx::Sched top_sched = start_sched;
  b->tune_log.clear();
  float top_us = -1.f;
  hipError_t e = hipSuccess;
  const int max_streams = b->use_graph ? 1 : kMaxBranches;
  // 1) launch plans under the batch's schedule
  for (int B : sizes) {
    const int groups = B ? (b->n_ks + B - 1) / B : 1;
    if ((e = batch_events(b, ckks_batch_plan{B, 1, 1, 0})) != hipSuccess) break;
    for (int S = 1; S <= max_streams && e == hipSuccess; ++S) {
      if (S > 1 && S > groups + (b->n_rs ? 1 : 0)) break;
      for (int split = 0; split <= 2 && e == hipSuccess; ++split) {
        b->plan = ckks_batch_plan{B, S, split, 0};
        float us = 0.f;
        if ((e = time_it(&us)) != hipSuccess) break;
        b->tune_log.emplace_back(b->plan, us);
        if (top_us < 0.f || us < top_us) {
          top_us = us;
          top = b->plan;
        }
      }
    }
  }
  // 2) kernel schedules under the best plan: a batch's grids are larger than
  // a single operation's, so the context's schedule need not suit it
  if (e == hipSuccess) {
    b->plan = top;
    e = batch_events(b, top);
    const int sh = start_sched.ntt_shape;
    const Ctx::Sched cands[] = {{12, 6, 128, sh}, {6, 4, 128, sh}, {4, 6, 128, sh}, {12, 12, 128, sh}};
    for (const Ctx::Sched& cs : cands) {
      if (e != hipSuccess) break;
      if (cs.up_rows == start_sched.up_rows && cs.down_rows == start_sched.down_rows &&
          cs.small_grid == start_sched.small_grid)
        continue;  // timed in the plan search
      b->sched = cs;
      float us = 0.f;
      if ((e = time_it(&us)) != hipSuccess) break;
      if (us < top_us) {
        top_us = us;
        top_sched = cs;
      }
    }
    // 3) NTT tile / radix shapes under the best plan and BConv schedule
    const Ctx::Sched base = top_sched;
    for (int shape = 0; shape <= kShapeAll && e == hipSuccess; ++shape) {
      if (shape == base.ntt_shape || ((shape & kShapeWholeLimb) && b->c->logN != kSrLog)) continue;
      b->sched = base;
      b->sched.ntt_shape = shape;
      float us = 0.f;
      if ((e = time_it(&us)) != hipSuccess) break;
      if (us < top_us) {
        top_us = us;
        top_sched = b->sched;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->plan = e == hipSuccess ? top : start;
  b->sched = e == hipSuccess ? top_sched : start_sched;
  hipError_t ce = batch_events(b, b->plan);
  if (ce == hipSuccess && b->use_graph) ce = batch_capture(b);
  if (e != hipSuccess) return hip_fail(e, "timing candidate plans");
  if (ce != hipSuccess) return hip_fail(ce, "re-capturing the batch graph");
  if (best) *best = top;
  if (best_us) *best_us = top_us;
  return CKKS_OK;
}

int ckks_batch_tune_log(const ckks_batch* b, ckks_batch_plan* plans, float* us, int cap, int* n) {
  if (!b || !n || cap < 0 || (cap > 0 && (!plans || !us))) return fail(CKKS_EINVAL, "bad arguments");
  *n = (int)b->tune_log.size();
  for (int i = 0; i < std::min(cap, *n); ++i) {
    plans[i] = b->tune_log[i].first;
    us[i] = b->tune_log[i].second;
  }
  return CKKS_OK;
}

size_t ckks_batch_device_bytes(const ckks_batch* b) { return b ? b->bytes : 0; }

int ckks_batch_destroy(ckks_batch* b) {
  if (!b) return CKKS_OK;
  DeviceGuard g(b->c->device);
  batch_free(b);
  return CKKS_OK;
}

int ckks_trace_begin(ckks_ctx* ctx, int stage, int capacity) {
  if (!ctx) return fail(CKKS_EINVAL, "null context");
  if (stage < CKKS_STAGE_INTT_BLOCKS || stage > CKKS_STAGE_NTT_IP_P || capacity < 1)
    return fail(CKKS_EINVAL, "bad trace stage or capacity");
  Ctx& c = ctx->c;
  if (c.trace.stage) return fail(CKKS_EINVAL, "a trace is already armed on this context");
  DeviceGuard g(c.device);
  c.trace.starts.assign(capacity, nullptr);
  c.trace.stops.assign(capacity, nullptr);
  for (int i = 0; i < capacity; ++i) {
    if (hipEventCreate(&c.trace.starts[i]) != hipSuccess ||
        hipEventCreate(&c.trace.stops[i]) != hipSuccess) {
      for (auto* v : {&c.trace.starts, &c.trace.stops})
        for (hipEvent_t ev : *v)
          if (ev) (void)hipEventDestroy(ev);
      c.trace = Ctx::Trace{};
      return fail(CKKS_EHIP, "hipEventCreate failed");
    }
  }
  c.trace.count = 0;
  c.trace.stage = stage;
  return CKKS_OK;
}

int ckks_trace_end(ckks_ctx* ctx, float* h_ms, int* count) {
  if (!ctx) return fail(CKKS_EINVAL, "null context");
  Ctx& c = ctx->c;
  if (!c.trace.stage) return fail(CKKS_EINVAL, "no trace armed");
  DeviceGuard g(c.device);
  int rc = CKKS_OK;
  const int n = c.trace.count;
  if (n > 0 && hipEventSynchronize(c.trace.stops[n - 1]) != hipSuccess) rc = fail(CKKS_EHIP, "event sync failed");
  for (int i = 0; i < n && rc == CKKS_OK; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.trace.starts[i], c.trace.stops[i]) != hipSuccess)
      rc = fail(CKKS_EHIP, "hipEventElapsedTime failed");
    else if (h_ms)
      h_ms[i] = ms;
  }
  if (count) *count = n;
  for (auto* v : {&c.trace.starts, &c.trace.stops})
    for (hipEvent_t ev : *v) (void)hipEventDestroy(ev);
  c.trace = Ctx::Trace{};
  return rc;
}

}  // extern "C"
