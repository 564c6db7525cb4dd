// Fused key-switching pipeline over a job table (see keyswitch.h).
//
// Key-switching has three stages (Fig. keysw): ModUp of every digit, the
// inner product with the evaluation key, ModDown of both components.  The NTT
// is row-parallel and BConv column-parallel, so they cannot share a kernel
// (Sec. III-D); what does fuse here is everything element-wise around them:
//
//  K1  INTT block pass of the input (loader forms d: d, c1*c1', or sigma(c1))
//  K2  INTT column pass + N^-1 (D_j/q_i)^-1 pre-multiply            -> y
//  K3  ModUp BConv, every digit in one launch                        -> z
//  K4  NTT column pass of every digit's new rows                     -> z
//  K5  NTT block pass fused with the inner product over the digits
//      (digit rows come straight from the loader; hoisted jobs gather
//      sigma(M) instead of transforming), then, for the P rows, the first
//      INTT pass of ModDown                                          -> acc
//  K6  INTT column pass of the P rows, N^-1 (P/p_m)^-1 pre-multiply  -> x
//  K7  ModDown BConv P -> Q, both components                        -> w
//  K8  NTT column pass of w
//  K9  NTT block pass fused with (acc - w) P^-1 plus the epilogue
//      term (d0 / d1 of HMult, sigma(c0) of HRot)                    -> out
//
// Every launch covers all jobs (grid.z) and all rows of a stage, which is
// what gives small levels enough work-groups (the batching argument of
// Sec. IV-A).  Rescale has its own four kernels (R1..R4).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "arith.h"
#include "ctx.h"
#include "keyswitch.h"
#include "ntt_tile.h"

namespace ckks {

namespace {

struct KsConst {
  DevTab T;
  int k, alpha, beta_max;
  const uint2* modup_scale;
  const uint32_t* modup_T;
  const uint32_t* modup_T_off;
  const uint2* moddown_scale;
  const uint32_t* moddown_T;
  const uint2* pinv;
  const uint2* rescale_inv;
};

KsConst make_const(const Ctx& c) {
  return KsConst{c.tab(), c.k, c.alpha, c.beta_max(), c.d_modup_scale, c.d_modup_T,
                 c.d_modup_T_off, c.d_moddown_scale, c.d_moddown_T, c.d_pinv, c.d_rescale_inv};
}

// Scratch layout of one job (rows of N words): acc [2][R], x [2][k], w [2][L],
// then, for jobs that run ModUp, y [L], z [beta][R] and de [L] (the eval-domain
// polynomial being switched, kept by K1 for the digit rows of K5); R = L + k.
struct KsView {
  uint32_t *y, *z, *de, *acc, *x, *w;
  int L, R, beta;
};

__device__ __forceinline__ KsView ks_view(const KsJob& J, const KsConst& K, size_t N) {
  KsView v;
  v.L = J.L;
  v.R = J.L + K.k;
  v.beta = (J.L + K.alpha - 1) / K.alpha;
  if (J.kind == KS_MODUP) {  // ModUp alone: y in the scratch, z is the output M
    v.y = J.ws;
    v.z = J.out;
    v.acc = v.x = v.w = v.de = nullptr;
    return v;
  }
  v.acc = J.ws;
  v.x = v.acc + (size_t)2 * v.R * N;
  v.w = v.x + (size_t)2 * K.k * N;
  v.y = v.w + (size_t)2 * v.L * N;
  v.z = v.y + (size_t)v.L * N;
  v.de = v.z + (size_t)v.beta * v.R * N;
  return v;
}

__device__ __forceinline__ int ks_pidx(int r, int L, int L_max) { return r < L ? r : L_max + (r - L); }

// Source index of the eval-domain automorphism: out[j] = in[auto_src(j)].
__device__ __forceinline__ uint32_t auto_src(uint32_t j, uint32_t g, int logN) {
  const uint32_t bj = __builtin_bitreverse32(j) >> (32 - logN);
  const uint32_t e = (g * (2u * bj + 1u)) & ((2u << logN) - 1u);
  return __builtin_bitreverse32((e - 1u) >> 1) >> (32 - logN);
}

__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const ModC& m) {
  return reduce64((uint64_t)a * b, m.q, m.mu_hi, m.mu_lo);
}

// The QPT quads (words base + blk_elem(kk) .. +3) of row r of the polynomial
// a job key-switches: d (PLAIN), c1 c1' (HMULT), sigma(c1) (HROT / HOIST).
// Every load of a quad is issued before any of them is used.
template <int QPT = 4, int T = kWG>
__device__ __forceinline__ void load_d16(const KsJob& J, int r, uint32_t base, size_t N, int logN,
                                         const ModC& m, uint4 d[QPT]) {
  if (J.kind == KS_PLAIN || J.kind == KS_MODUP) {
#pragma unroll
    for (int kk = 0; kk < QPT; ++kk) d[kk] = ld4(J.a + (size_t)r * N + base + blk_elem<T>(kk));
    return;
  }
  const size_t row1 = (size_t)(J.L + r) * N;
  if (J.kind == KS_HMULT) {
    uint4 x[QPT], y[QPT];
#pragma unroll
    for (int kk = 0; kk < QPT; ++kk) {
      x[kk] = ld4(J.a + row1 + base + blk_elem<T>(kk));
      y[kk] = ld4(J.b + row1 + base + blk_elem<T>(kk));
    }
#pragma unroll
    for (int kk = 0; kk < QPT; ++kk)
      d[kk] = make_uint4(mulmod(x[kk].x, y[kk].x, m), mulmod(x[kk].y, y[kk].y, m),
                         mulmod(x[kk].z, y[kk].z, m), mulmod(x[kk].w, y[kk].w, m));
    return;
  }
  const uint32_t* src = J.a + row1;
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const uint32_t n = base + blk_elem<T>(kk);
    d[kk] = make_uint4(ld1(src + auto_src(n, J.gal, logN)), ld1(src + auto_src(n + 1, J.gal, logN)),
                       ld1(src + auto_src(n + 2, J.gal, logN)), ld1(src + auto_src(n + 3, J.gal, logN)));
  }
}

// ============================================================================
// Stage 1: ModUp
// ============================================================================

// BPW blocks per work-group: 16 (a 4096-word tile, radix-16 phases) or, for
// small grids, 4 (a quarter tile, one quad per thread, radix-4 phases).
template <int LOGN1, int BPW, int EPT = (BPW == 16 ? 16 : 4)>
__global__ __launch_bounds__(BPW * 256 / EPT) void k1_intt_blks(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const int r = blockIdx.y;
  if (J.kind == KS_HOIST || r >= J.L) return;
  __shared__ __align__(16) uint32_t s[kLds];
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const ModC m = ldc(K.T.mod + r);
  const uint32_t q = m.q, q2 = 2 * q;
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(K.T.blk_itw(r), 256);  // (T >= 256)
  constexpr int T = BPW * 256 / EPT;  // threads
  constexpr int QPT = EPT / 4;        // quads per thread
  const int blk0 = blockIdx.x * BPW;
  const uint32_t base = blk0 * 256;
  const KsView V = ks_view(J, K, N);
  // the switched polynomial in the evaluation domain, kept for K5's digit
  // rows (a ModUp-only job keeps it as the digit row of its output M)
  uint32_t* de = J.kind == KS_MODUP ? V.z + ((size_t)(r / K.alpha) * V.R + r) * N + base
                                    : V.de + (size_t)r * N + base;
  // all loads first: a store to de could alias the next quad's source; the
  // twist factors of the epilogue are requested with them
  uint4 d[QPT];
  load_d16<QPT, T>(J, r, base, N, logN, m, d);
  Twist4 tfi[QPT];
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem<T>(kk);
    tfi[kk] = twist4_load(K.T.blk_itwist(r, blk0 + (e >> 8)), e & 255);
  }
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem<T>(kk);
    lds_blk4_store(s, e, d[kk]);
    if (J.kind != KS_PLAIN) st4(de + e, d[kk]);  // HMULT, HROT, MODUP
  }
  if constexpr (EPT == 16)
    tw_put_perm(stw, tww);
  else
    tw_put(stw, tww, 256);
  __syncthreads();
  if constexpr (EPT == 16)
    blk_stages<true>(s, PermTw{stw}, q, q2);
  else if constexpr (EPT == 8)
    blk_stages_r8<true, const uint2*, T>(s, stw, q, q2);
  else
    blk_stages_r4<true, const uint2*, T>(s, stw, q, q2);
  __syncthreads();
  uint32_t* y = V.y + (size_t)r * N + base;
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) st4(y + blk_elem<T>(kk), twist4(lds_blk4(s, blk_elem<T>(kk)), tfi[kk], q));
}

template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void k2_intt_cols(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const int r = blockIdx.y;
  if (J.kind == KS_HOIST || r >= J.L) return;
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  constexpr int C = ColGeom<LOGN1, CW, T>::C;
  const size_t N = (size_t)1 << K.T.logN;
  const uint32_t q = ldc(K.T.mod + r).q, q2 = 2 * q;
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_itw(r), ColGeom<LOGN1, CW, T>::N1);
  const uint2 sc = ldc(K.modup_scale + (size_t)J.L * K.T.L_max + r);
  const int col0 = blockIdx.x * C;
  uint32_t* row = ks_view(J, K, N).y + (size_t)r * N;
  load_cols<LOGN1, CW, T>(s, row, col0);
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, true, CW, T>(s, stw, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < ColGeom<LOGN1, CW, T>::QUADS; ++kk) {
    const int lin = (threadIdx.x + kk * T) * 4;
    const int pos = lin / C, c = lin & (C - 1);
    uint4 v = *reinterpret_cast<const uint4*>(s + lidx_col(pos, c, C));
    v.x = csub(mul_shoup(v.x, sc.x, sc.y, q), q);
    v.y = csub(mul_shoup(v.y, sc.x, sc.y, q), q);
    v.z = csub(mul_shoup(v.z, sc.x, sc.y, q), q);
    v.w = csub(mul_shoup(v.w, sc.x, sc.y, q), q);
    st4(row + pos * 256 + col0 + c, v);
  }
}

// ModUp BConv of digit j: z[j][r] = sum_i y[j alpha + i] T_{L,j}[r][i] mod prime(r) for every
// row r outside the digit.  Rows of a block: [g * RB, g * RB + RB); blockIdx.y = j * groups + g.
// Table columns past a partial digit are zero, so every input load is unconditional.
template <int ALPHA, int RB>
__global__ __launch_bounds__(kWG) void k3_bconv_up(KsConst K, JobArg<KsJob> JA, int groups) {
  const KsJob J = JA.get(blockIdx.z);
  if (J.kind == KS_HOIST) return;
  const int j = blockIdx.y / groups, g = blockIdx.y % groups;
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  if (j >= V.beta || g * RB >= V.R) return;
  const int lo = j * ALPHA, hi = min(lo + ALPHA, V.L);
  const size_t n = ((size_t)blockIdx.x * kWG + threadIdx.x) * 4;  // four coefficients per thread
  uint4 x[ALPHA];
#pragma unroll
  for (int i = 0; i < ALPHA; ++i) x[i] = ld4(V.y + (size_t)min(lo + i, V.L - 1) * N + n);
  const uint32_t* Tt = K.modup_T + ldc(K.modup_T_off + (size_t)V.L * K.beta_max + j);
  const int r1 = min(g * RB + RB, V.R);
  for (int r = g * RB; r < r1; ++r) {
    if (r >= lo && r < hi) continue;
    const ModC m = ldc(K.T.mod + ks_pidx(r, V.L, K.T.L_max));
    const uint32_t* t = Tt + (size_t)r * ALPHA;
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int i = 0; i < ALPHA; ++i) {
      const uint64_t ti = ldc(t + i);
      a0 += x[i].x * ti;
      a1 += x[i].y * ti;
      a2 += x[i].z * ti;
      a3 += x[i].w * ti;
    }
    st4(V.z + ((size_t)j * V.R + r) * N + n,
        make_uint4(reduce64(a0, m.q, m.mu_hi, m.mu_lo), reduce64(a1, m.q, m.mu_hi, m.mu_lo),
                   reduce64(a2, m.q, m.mu_hi, m.mu_lo), reduce64(a3, m.q, m.mu_hi, m.mu_lo)));
  }
}

template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void k4_ntt_cols(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  if (J.kind == KS_HOIST) return;
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  const int gr = blockIdx.y;
  const int j = gr / V.R, r = gr % V.R;
  if (j >= V.beta) return;
  const int lo = j * K.alpha, hi = min(lo + K.alpha, V.L);
  if (r >= lo && r < hi) return;
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_tw(pi), ColGeom<LOGN1, CW, T>::N1);
  const uint32_t q = ldc(K.T.mod + pi).q, q2 = 2 * q;
  const int col0 = blockIdx.x * ColGeom<LOGN1, CW, T>::C;
  uint32_t* row = V.z + (size_t)gr * N;
  load_cols<LOGN1, CW, T>(s, row, col0);
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, false, CW, T>(s, stw, q, q2);
  __syncthreads();
  store_cols<LOGN1, CW, T>(s, row, col0);
}

// ModUp-only jobs: the block pass of the new rows of M (K4 left them after the
// column pass), canonical output in place, so that M is wholly in the
// evaluation domain for the hoisted rotations' gathers.
template <int LOGN1>
__global__ __launch_bounds__(kWG) void km_ntt_blks(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  if (J.kind != KS_MODUP) return;
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  const int gr = blockIdx.y;
  const int j = gr / V.R, r = gr % V.R;
  if (j >= V.beta) return;
  const int lo = j * K.alpha, hi = min(lo + K.alpha, V.L);
  if (r >= lo && r < hi) return;
  __shared__ __align__(16) uint32_t s[kLds];
  __shared__ uint2 stw[256];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  const uint2 tww = tw_fetch(K.T.blk_tw(pi), 256);
  const uint32_t q = ldc(K.T.mod + pi).q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  uint32_t* row = V.z + (size_t)gr * N + blk0 * 256;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    lds_blk4_store(s, e, twist4(ld4(row + e), K.T.blk_twist(pi, blk0 + (e >> 8)), e & 255, q));
  }
  tw_put_perm(stw, tww);
  __syncthreads();
  blk_stages<false>(s, PermTw{stw}, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    st4(row + e, canon4(lds_blk4(s, e), q, q2));
  }
}

// ============================================================================
// Stage 2: NTT block pass + inner product (+ first INTT pass of ModDown on P rows)
// ============================================================================
// HOIST selects the variant for hoisted-rotation jobs (gather of sigma(M), no
// transform; each rotation brings its own key, streamed with the
// non-temporal hint); the other variant serves every other job kind.
template <int LOGN1, bool HOIST>
__global__ __launch_bounds__(kWG) void k5_ntt_blks_ip(KsConst K, JobArg<KsJob> JA, int part) {
  const KsJob J = JA.get(blockIdx.z);
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const KsView V = ks_view(J, K, N);
  const int r = blockIdx.y + (part == KS_PART_P ? V.L : 0);
  if (r >= V.R || (part == KS_PART_Q && r >= V.L) || (J.kind == KS_HOIST) != HOIST) return;
  __shared__ __align__(16) uint32_t s[kLds];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  __shared__ uint2 stw[256], stwi[256];
  // twiddles: requested now, stored to LDS after the first tile's loads
  const uint2 tww = HOIST ? make_uint2(0, 0) : tw_fetch(K.T.blk_tw(pi), 256);
  const uint2 twwi = r >= V.L ? tw_fetch(K.T.blk_itw(pi), 256) : make_uint2(0, 0);
  bool tw_staged = false;
  const ModC m = ldc(K.T.mod + pi);
  const uint32_t q = m.q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t base = blk0 * 256;
  const size_t KR = (size_t)K.T.L_max + K.k;  // key rows
  uint64_t a0[16], a1[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) a0[i] = a1[i] = 0;

  for (int j = 0; j < V.beta; ++j) {
    const int lo = j * K.alpha, hi = min(lo + K.alpha, V.L);
    uint4 v[4];
    if (HOIST) {
      // hoisted rotation: sigma_g applied to the shared ModUp rows (a gather)
      const uint32_t* Mrow = J.b + ((size_t)j * V.R + r) * N;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const uint32_t n = base + blk_elem(kk);
        v[kk] = make_uint4(ld1(Mrow + auto_src(n, J.gal, logN)), ld1(Mrow + auto_src(n + 1, J.gal, logN)),
                           ld1(Mrow + auto_src(n + 2, J.gal, logN)), ld1(Mrow + auto_src(n + 3, J.gal, logN)));
      }
    } else if (r >= lo && r < hi) {
      // digit rows are the switched polynomial itself (kept by K1 unless it is the input)
      const uint32_t* drow = (J.kind == KS_PLAIN ? J.a : V.de) + (size_t)r * N + base;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) v[kk] = ld4(drow + blk_elem(kk));
    } else {
      const uint32_t* zrow = V.z + ((size_t)j * V.R + r) * N + base;
      __syncthreads();  // the previous digit's tile has been read
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int e = blk_elem(kk);
        lds_blk4_store(s, e, twist4(ld4(zrow + e),
                                    K.T.blk_twist(pi, blk0 + (e >> 8)), e & 255, q));
      }
      if (!tw_staged) {
        tw_put_perm(stw, tww);
        tw_staged = true;
      }
      __syncthreads();
      blk_stages<false>(s, PermTw{stw}, q, q2);
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) v[kk] = canon4(lds_blk4(s, blk_elem(kk)), q, q2);
    }
    const uint32_t* k0 = J.key + ((size_t)j * 2 * KR + pi) * N + base;
    const uint32_t* k1 = k0 + KR * N;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint4 e0 = HOIST ? ld4nt(k0 + blk_elem(kk)) : ld4(k0 + blk_elem(kk));
      a0[4 * kk + 0] += (uint64_t)v[kk].x * e0.x;
      a0[4 * kk + 1] += (uint64_t)v[kk].y * e0.y;
      a0[4 * kk + 2] += (uint64_t)v[kk].z * e0.z;
      a0[4 * kk + 3] += (uint64_t)v[kk].w * e0.w;
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint4 e1 = HOIST ? ld4nt(k1 + blk_elem(kk)) : ld4(k1 + blk_elem(kk));
      a1[4 * kk + 0] += (uint64_t)v[kk].x * e1.x;
      a1[4 * kk + 1] += (uint64_t)v[kk].y * e1.y;
      a1[4 * kk + 2] += (uint64_t)v[kk].z * e1.z;
      a1[4 * kk + 3] += (uint64_t)v[kk].w * e1.w;
    }
    // Each product of canonical words is below q^2 < 2^60, so 16 of them fit
    // a 64-bit sum; chains of more digits (digit size 1 allows up to 63) fold
    // the sums back below q after every eighth digit.
    if ((j & 7) == 7) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        a0[i] = reduce64(a0[i], q, m.mu_hi, m.mu_lo);
        a1[i] = reduce64(a1[i], q, m.mu_hi, m.mu_lo);
      }
    }
  }

  // one reduction per output (the overflow-free accumulation of Sec. III-C2)
  uint32_t r0[16], r1[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    r0[i] = reduce64(a0[i], q, m.mu_hi, m.mu_lo);
    r1[i] = reduce64(a1[i], q, m.mu_hi, m.mu_lo);
  }
  uint32_t* acc0 = V.acc + (size_t)r * N + base;
  uint32_t* acc1 = V.acc + ((size_t)V.R + r) * N + base;
  if (r < V.L) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int e = blk_elem(kk);
      st4(acc0 + e, make_uint4(r0[4 * kk], r0[4 * kk + 1], r0[4 * kk + 2], r0[4 * kk + 3]));
      st4(acc1 + e, make_uint4(r1[4 * kk], r1[4 * kk + 1], r1[4 * kk + 2], r1[4 * kk + 3]));
    }
    return;
  }
  // P rows: ModDown starts with an INTT; its block pass runs here on the tile
  // (inverse twist factors requested before the transforms).
  Twist4 tfi[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    tfi[kk] = twist4_load(K.T.blk_itwist(pi, blk0 + (e >> 8)), e & 255);
  }
  tw_put_perm(stwi, twwi);
  for (int c = 0; c < 2; ++c) {
    uint32_t* dst = c ? acc1 : acc0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const uint32_t* rr = c ? r1 : r0;
      lds_blk4_store(s, blk_elem(kk), make_uint4(rr[4 * kk], rr[4 * kk + 1], rr[4 * kk + 2], rr[4 * kk + 3]));
    }
    __syncthreads();
    blk_stages<true>(s, PermTw{stwi}, q, q2);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) st4(dst + blk_elem(kk), twist4(lds_blk4(s, blk_elem(kk)), tfi[kk], q));
  }
}

// Variant of K5 for contexts with at most NB digits: every digit's tile is
// staged and transformed in its own LDS slot first (all loads in flight at
// once), then the inner product runs one 16-byte quad at a time, so the
// 64-bit accumulators never hold more than four elements per component.
// NT: the key words are read with the non-temporal hint (a launch of one
// job reads its key once; batches whose jobs share a key keep it cached).
template <int LOGN1, int NB, bool NT>
__global__ __launch_bounds__(kWG) void k5s_ntt_blks_ip(KsConst K, JobArg<KsJob> JA, int part) {
  const KsJob J = JA.get(blockIdx.z);
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const KsView V = ks_view(J, K, N);
  const int r = blockIdx.y + (part == KS_PART_P ? V.L : 0);
  if (r >= V.R || (part == KS_PART_Q && r >= V.L) || J.kind == KS_HOIST) return;
  __shared__ __align__(16) uint32_t s[NB * kLds];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  const ModC m = ldc(K.T.mod + pi);
  const uint32_t q = m.q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t base = blk0 * 256;
  const size_t KR = (size_t)K.T.L_max + K.k;  // key rows

  // Every load of the staging is issued before any of them is used, in
  // straight-line code (a branch between them would make the compiler wait
  // for the earlier ones), in the order they are consumed (vmcnt counts in
  // order): the block-pass twiddles for the pads of slots 0 and 1 (so the
  // transforms issue no global load), the twist factors of the thread's
  // quads (shared by all digits: they depend on the prime and the block),
  // each digit's tile -- the digit row itself for the digit that holds r,
  // else its ModUp row; digits past beta re-read the last digit's rows,
  // unused -- and the key words of the first KPF quads, whose latency
  // overlaps the transforms.
  const uint2 tw_word = K.T.blk_tw(pi)[threadIdx.x];
  Twist4 tf[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    tf[kk] = twist4_load(K.T.blk_twist(pi, blk0 + (e >> 8)), e & 255);
  }
  uint4 raw[NB][4];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int jj = min(j, V.beta - 1);
    const int lo = jj * K.alpha, hi = min(lo + K.alpha, V.L);
    const uint32_t* src = (r >= lo && r < hi) ? (J.kind == KS_PLAIN ? J.a : V.de) + (size_t)r * N + base
                                              : V.z + ((size_t)jj * V.R + r) * N + base;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) raw[j][kk] = ld4(src + blk_elem(kk));
  }
  // The inner product loads the key words of the quads past KPF itself: a
  // third prefetched quad of three digits takes the registers past what three
  // resident work-groups per CU leave (171 VGPRs against 168).
  constexpr int KPF = NB <= 2 ? 4 : 2;
  uint4 kpre0[4][NB], kpre1[4][NB];
  auto key_quad = [&](int kk) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int jj = min(j, V.beta - 1);
      const uint32_t* k0 = J.key + ((size_t)jj * 2 * KR + pi) * N + base + blk_elem(kk);
      kpre0[kk][j] = NT ? ld4nt(k0) : ld4(k0);
      kpre1[kk][j] = NT ? ld4nt(k0 + KR * N) : ld4(k0 + KR * N);
    }
  };
#pragma unroll
  for (int kk = 0; kk < KPF; ++kk) key_quad(kk);
  stage_tw_pads_perm_word(s, tw_word);
  // stage every digit's tile: the digit row as it is, a ModUp row twisted
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j >= V.beta) break;
    const int lo = j * K.alpha, hi = min(lo + K.alpha, V.L);
    uint32_t* slot = s + j * kLds;
    if (r >= lo && r < hi) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) lds_blk4_store(slot, blk_elem(kk), raw[j][kk]);
    } else {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) lds_blk4_store(slot, blk_elem(kk), twist4(raw[j][kk], tf[kk], q));
    }
  }
  __syncthreads();
  // The block-pass transforms of all digit tiles, phase by phase: the tiles
  // share the prime, so each phase's twiddles are fetched once for all of
  // them, and there are two barrier intervals instead of two per tile.
  const PadTwP tw{s};
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int lo = j * K.alpha, hi = min(lo + K.alpha, V.L);
      if (j < V.beta && !(r >= lo && r < hi)) blk_phase<4, false>(s + j * kLds, ph ? 0 : 4, tw, q, q2);
    }
    __syncthreads();
  }

  // inner product, one quad at a time (one reduction per output, Sec. III-C2).
  // No branch on the digit count: tiles past beta (never staged) are masked
  // to zero, so the prefetched key words are consumed in straight-line code.
  // The transformed words enter uncorrected: each lies in [0, 4q) and each
  // key word below q < 2^30, so a product is below 2^62 and the sum of at
  // most four (NB <= 4) stays below 2^64 for the single exact reduction.
  static_assert(NB <= 4, "64-bit sum of lazy products");
  uint4 res0[4], res1[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    uint64_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint32_t msk = j < V.beta ? ~0u : 0u;
      uint4 v = lds_blk4(s + j * kLds, e);
      v.x &= msk;
      v.y &= msk;
      v.z &= msk;
      v.w &= msk;
      if (kk >= KPF) {
        const uint32_t* k0 = J.key + ((size_t)min(j, V.beta - 1) * 2 * KR + pi) * N + base + e;
        kpre0[kk][j] = NT ? ld4nt(k0) : ld4(k0);
        kpre1[kk][j] = NT ? ld4nt(k0 + KR * N) : ld4(k0 + KR * N);
      }
      const uint4 e0 = kpre0[kk][j], e1 = kpre1[kk][j];
      a0[0] += (uint64_t)v.x * e0.x;
      a0[1] += (uint64_t)v.y * e0.y;
      a0[2] += (uint64_t)v.z * e0.z;
      a0[3] += (uint64_t)v.w * e0.w;
      a1[0] += (uint64_t)v.x * e1.x;
      a1[1] += (uint64_t)v.y * e1.y;
      a1[2] += (uint64_t)v.z * e1.z;
      a1[3] += (uint64_t)v.w * e1.w;
    }
    res0[kk] = make_uint4(reduce64(a0[0], q, m.mu_hi, m.mu_lo), reduce64(a0[1], q, m.mu_hi, m.mu_lo),
                          reduce64(a0[2], q, m.mu_hi, m.mu_lo), reduce64(a0[3], q, m.mu_hi, m.mu_lo));
    res1[kk] = make_uint4(reduce64(a1[0], q, m.mu_hi, m.mu_lo), reduce64(a1[1], q, m.mu_hi, m.mu_lo),
                          reduce64(a1[2], q, m.mu_hi, m.mu_lo), reduce64(a1[3], q, m.mu_hi, m.mu_lo));
  }
  uint32_t* acc0 = V.acc + (size_t)r * N + base;
  uint32_t* acc1 = V.acc + ((size_t)V.R + r) * N + base;
  if (r < V.L) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int e = blk_elem(kk);
      st4(acc0 + e, res0[kk]);
      st4(acc1 + e, res1[kk]);
    }
    return;
  }
  // P rows: the INTT block pass of ModDown on both components (slots 0 and 1),
  // inverse twiddles in the same pads (the forward ones were last read before
  // the barrier that ended the transforms); the inverse twist factors are
  // requested first, so their latency overlaps the transforms
  const uint2 twi_word = K.T.blk_itw(pi)[threadIdx.x];
  Twist4 tfi[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    tfi[kk] = twist4_load(K.T.blk_itwist(pi, blk0 + (e >> 8)), e & 255);
  }
  __syncthreads();
  stage_tw_pads_perm_word(s, twi_word);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    lds_blk4_store(s, blk_elem(kk), res0[kk]);
    lds_blk4_store(s + kLds, blk_elem(kk), res1[kk]);
  }
  __syncthreads();
  blk_stages<true>(s, PadTwP{s}, q, q2);
  blk_stages<true>(s + kLds, PadTwP{s}, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    st4(acc0 + e, twist4(lds_blk4(s, e), tfi[kk], q));
    st4(acc1 + e, twist4(lds_blk4(s + kLds, e), tfi[kk], q));
  }
}

// K5 for hoisted rotations of at most NB digits.  sigma_g maps each aligned
// 4096-word tile of an evaluation-domain row onto one aligned source tile (g
// is odd, so only the low 12 bits of the bit-reversed index are permuted), so
// every digit's source tile of M is loaded whole and contiguously into its
// own LDS slot and the permutation is a read from LDS.  The key words of the
// first KPF quads are requested with the tiles; the inner product and the
// P-row INTT block pass follow as in k5s, on canonical words (M is fully
// transformed).
template <int LOGN1, int NB>
__global__ __launch_bounds__(kWG) void k5h_gather_ip(KsConst K, JobArg<KsJob> JA, int part) {
  static_assert(NB >= 2 && NB <= 4, "slots for two to four digits");
  const KsJob J = JA.get(blockIdx.z);
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const KsView V = ks_view(J, K, N);
  const int r = blockIdx.y + (part == KS_PART_P ? V.L : 0);
  if (r >= V.R || (part == KS_PART_Q && r >= V.L) || J.kind != KS_HOIST) return;
  constexpr int WORDS = NB * kTile > 2 * kLds ? NB * kTile : 2 * kLds;
  __shared__ __align__(16) uint32_t s[WORDS];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  const ModC m = ldc(K.T.mod + pi);
  const uint32_t q = m.q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t base = blk0 * 256;
  const size_t KR = (size_t)K.T.L_max + K.k;  // key rows
  const uint32_t src0 = auto_src(base, J.gal, logN) & ~(uint32_t)(kTile - 1);
  // every digit's source tile (digits past beta re-read the last one, unused)
  uint4 raw[NB][4];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int jj = min(j, V.beta - 1);
    const uint32_t* Mrow = J.b + ((size_t)jj * V.R + r) * N + src0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) raw[j][kk] = ld4(Mrow + 4 * (threadIdx.x + kk * kWG));
  }
  constexpr int KPF = NB <= 2 ? 4 : 2;
  uint4 kpre0[4][NB], kpre1[4][NB];
  auto key_quad = [&](int kk) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint32_t* k0 = J.key + ((size_t)min(j, V.beta - 1) * 2 * KR + pi) * N + base + blk_elem(kk);
      kpre0[kk][j] = ld4nt(k0);
      kpre1[kk][j] = ld4nt(k0 + KR * N);
    }
  };
#pragma unroll
  for (int kk = 0; kk < KPF; ++kk) key_quad(kk);
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      *reinterpret_cast<uint4*>(s + j * kTile + 4 * (threadIdx.x + kk * kWG)) = raw[j][kk];
  __syncthreads();

  // inner product of sigma(M) quad by quad (canonical words: products below
  // 2^60, at most four summed, one reduction per output)
  uint4 res0[4], res1[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    const uint32_t n = base + e;
    const uint32_t p0 = auto_src(n, J.gal, logN) & (kTile - 1), p1 = auto_src(n + 1, J.gal, logN) & (kTile - 1),
                   p2 = auto_src(n + 2, J.gal, logN) & (kTile - 1), p3 = auto_src(n + 3, J.gal, logN) & (kTile - 1);
    if (kk >= KPF) key_quad(kk);
    uint64_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const uint32_t msk = j < V.beta ? ~0u : 0u;
      const uint32_t* sl = s + j * kTile;
      const uint4 v = make_uint4(sl[p0] & msk, sl[p1] & msk, sl[p2] & msk, sl[p3] & msk);
      const uint4 e0 = kpre0[kk][j], e1 = kpre1[kk][j];
      a0[0] += (uint64_t)v.x * e0.x;
      a0[1] += (uint64_t)v.y * e0.y;
      a0[2] += (uint64_t)v.z * e0.z;
      a0[3] += (uint64_t)v.w * e0.w;
      a1[0] += (uint64_t)v.x * e1.x;
      a1[1] += (uint64_t)v.y * e1.y;
      a1[2] += (uint64_t)v.z * e1.z;
      a1[3] += (uint64_t)v.w * e1.w;
    }
    res0[kk] = make_uint4(reduce64(a0[0], q, m.mu_hi, m.mu_lo), reduce64(a0[1], q, m.mu_hi, m.mu_lo),
                          reduce64(a0[2], q, m.mu_hi, m.mu_lo), reduce64(a0[3], q, m.mu_hi, m.mu_lo));
    res1[kk] = make_uint4(reduce64(a1[0], q, m.mu_hi, m.mu_lo), reduce64(a1[1], q, m.mu_hi, m.mu_lo),
                          reduce64(a1[2], q, m.mu_hi, m.mu_lo), reduce64(a1[3], q, m.mu_hi, m.mu_lo));
  }
  uint32_t* acc0 = V.acc + (size_t)r * N + base;
  uint32_t* acc1 = V.acc + ((size_t)V.R + r) * N + base;
  if (r < V.L) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int e = blk_elem(kk);
      st4(acc0 + e, res0[kk]);
      st4(acc1 + e, res1[kk]);
    }
    return;
  }
  // P rows: the INTT block pass of ModDown on both components, as in k5s
  const uint32_t q2 = 2 * q;
  const uint2 twi_word = K.T.blk_itw(pi)[threadIdx.x];
  Twist4 tfi[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    tfi[kk] = twist4_load(K.T.blk_itwist(pi, blk0 + (e >> 8)), e & 255);
  }
  __syncthreads();  // the gathers have read the slots
  stage_tw_pads_perm_word(s, twi_word);
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    lds_blk4_store(s, blk_elem(kk), res0[kk]);
    lds_blk4_store(s + kLds, blk_elem(kk), res1[kk]);
  }
  __syncthreads();
  blk_stages<true>(s, PadTwP{s}, q, q2);
  blk_stages<true>(s + kLds, PadTwP{s}, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    st4(acc0 + e, twist4(lds_blk4(s, e), tfi[kk], q));
    st4(acc1 + e, twist4(lds_blk4(s + kLds, e), tfi[kk], q));
  }
}

// K5 for small grids (few tiles x rows, e.g. N = 2^12): one work-group per
// (tile, row) of BPW blocks (16: a whole 4096-word tile, 1024 threads; 4: a
// quarter tile, 256 threads, four times the work-groups for the same rows).
// Thread group d = threadIdx.x / (16 BPW) stages and transforms digit tile d,
// so the digits' transforms run side by side; then every thread forms the
// inner product of one quad over all digits.  Every barrier below is reached
// by all threads of the work-group.  The slots keep the full tile stride, so
// the twiddle table fits the pads of slots 0 and 1 for either BPW.
template <int BPW, int EPT>
constexpr int k5p_threads() { return 4 * BPW * 256 / EPT; }
template <int LOGN1, int NB, int BPW, int EPT>
__global__ __launch_bounds__((k5p_threads<BPW, EPT>())) void k5p_ntt_blks_ip(KsConst K, JobArg<KsJob> JA,
                                                                           int part) {
  static_assert(NB >= 2 && NB <= 4, "one thread group per digit tile");
  static_assert((EPT == 16 && (BPW == 4 || BPW == 16)) || (EPT == 4 && (BPW == 2 || BPW == 4)),
                "radix-16 phases on 16 elements per thread, radix-4 phases on 4");
  constexpr int GS = BPW * 256 / EPT;  // threads per digit group
  constexpr int QPG = EPT / 4;         // quads per thread in a group's tile
  constexpr int TQ = BPW * 64;         // quads of the tile: one per inner-product thread
  const KsJob J = JA.get(blockIdx.z);
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const KsView V = ks_view(J, K, N);
  const int r = blockIdx.y + (part == KS_PART_P ? V.L : 0);
  if (r >= V.R || (part == KS_PART_Q && r >= V.L) || J.kind == KS_HOIST) return;
  __shared__ __align__(16) uint32_t s[NB * kLds];
  const int pi = ks_pidx(r, V.L, K.T.L_max);
  const ModC m = ldc(K.T.mod + pi);
  const uint32_t q = m.q, q2 = 2 * q;
  const int blk0 = blockIdx.x * BPW;
  const uint32_t base = blk0 * 256;
  const size_t KR = (size_t)K.T.L_max + K.k;  // key rows
  const int grp = threadIdx.x / GS, lt = threadIdx.x % GS;
  // digit this thread group owns, and whether its tile needs the transform
  const int lo = grp * K.alpha, hi = min(lo + K.alpha, V.L);
  const bool have = grp < NB && grp < V.beta;
  const bool own = r >= lo && r < hi;
  if (have) {
    uint32_t* slot = s + grp * kLds;
    uint4 v[QPG];
    if (own) {
      const uint32_t* drow = (J.kind == KS_PLAIN ? J.a : V.de) + (size_t)r * N + base;
#pragma unroll
      for (int kk = 0; kk < QPG; ++kk) v[kk] = ld4(drow + (lt + kk * GS) * 4);
#pragma unroll
      for (int kk = 0; kk < QPG; ++kk) lds_blk4_store(slot, (lt + kk * GS) * 4, v[kk]);
    } else {
      const uint32_t* zrow = V.z + ((size_t)grp * V.R + r) * N + base;
#pragma unroll
      for (int kk = 0; kk < QPG; ++kk) v[kk] = ld4(zrow + (lt + kk * GS) * 4);
#pragma unroll
      for (int kk = 0; kk < QPG; ++kk) {
        const int e = (lt + kk * GS) * 4;
        lds_blk4_store(slot, e, twist4(v[kk], K.T.blk_twist(pi, blk0 + (e >> 8)), e & 255, q));
      }
    }
  }
  if (threadIdx.x < 256) {
    if constexpr (EPT == 16)
      stage_tw_pads_perm(s, K.T.blk_tw(pi), threadIdx.x);
    else
      stage_tw_pads(s, K.T.blk_tw(pi), threadIdx.x);
  }
  // key words of this thread's quad, requested before the transforms (the
  // first TQ threads form the inner product: all of them when EPT = 16)
  const bool ipt = EPT == 16 || (int)threadIdx.x < TQ;
  const int e = ipt ? threadIdx.x * 4 : 0;
  uint4 k0v[NB], k1v[NB];
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    const uint32_t* k0 = J.key + ((size_t)min(jj, V.beta - 1) * 2 * KR + pi) * N + base + e;
    k0v[jj] = ld4(k0);
    k1v[jj] = ld4(k0 + KR * N);
  }
  __syncthreads();
  const PadTw tw{s};
  if constexpr (EPT == 16) {
    const PadTwP twp{s};
    if (have && !own) blk_phase<4, false>(s + grp * kLds, 4, twp, q, q2, lt);
    __syncthreads();
    if (have && !own) blk_phase<4, false>(s + grp * kLds, 0, twp, q, q2, lt);
  } else {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (p) __syncthreads();
      if (have && !own) blk_phase<2, false, PadTw, 4, GS>(s + grp * kLds, 6 - 2 * p, tw, q, q2, lt);
    }
  }
  __syncthreads();

  // inner product of quad e over the digits (one reduction per output); the
  // lazy words in [0, 4q) enter uncorrected, as in k5s (NB <= 4 products of
  // at most 2^62 each)
  uint64_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    const uint32_t msk = jj < V.beta ? ~0u : 0u;
    uint4 v = lds_blk4(s + jj * kLds, e);
    v.x &= msk;
    v.y &= msk;
    v.z &= msk;
    v.w &= msk;
    a0[0] += (uint64_t)v.x * k0v[jj].x;
    a0[1] += (uint64_t)v.y * k0v[jj].y;
    a0[2] += (uint64_t)v.z * k0v[jj].z;
    a0[3] += (uint64_t)v.w * k0v[jj].w;
    a1[0] += (uint64_t)v.x * k1v[jj].x;
    a1[1] += (uint64_t)v.y * k1v[jj].y;
    a1[2] += (uint64_t)v.z * k1v[jj].z;
    a1[3] += (uint64_t)v.w * k1v[jj].w;
  }
  const uint4 res0 = make_uint4(reduce64(a0[0], q, m.mu_hi, m.mu_lo), reduce64(a0[1], q, m.mu_hi, m.mu_lo),
                                reduce64(a0[2], q, m.mu_hi, m.mu_lo), reduce64(a0[3], q, m.mu_hi, m.mu_lo));
  const uint4 res1 = make_uint4(reduce64(a1[0], q, m.mu_hi, m.mu_lo), reduce64(a1[1], q, m.mu_hi, m.mu_lo),
                                reduce64(a1[2], q, m.mu_hi, m.mu_lo), reduce64(a1[3], q, m.mu_hi, m.mu_lo));
  uint32_t* acc0 = V.acc + (size_t)r * N + base;
  uint32_t* acc1 = V.acc + ((size_t)V.R + r) * N + base;
  if (r < V.L) {  // uniform over the work-group
    if (ipt) {
      st4(acc0 + e, res0);
      st4(acc1 + e, res1);
    }
    return;
  }
  // P rows: the INTT block pass of ModDown, component c in slot c by thread
  // group c; inverse twiddles in the same pads (the forward ones were last
  // read before the previous barrier)
  __syncthreads();
  if (ipt) {
    lds_blk4_store(s, e, res0);
    lds_blk4_store(s + kLds, e, res1);
  }
  if (threadIdx.x < 256) {
    if constexpr (EPT == 16)
      stage_tw_pads_perm(s, K.T.blk_itw(pi), threadIdx.x);
    else
      stage_tw_pads(s, K.T.blk_itw(pi), threadIdx.x);
  }
  __syncthreads();
  if constexpr (EPT == 16) {
    if (grp < 2) blk_phase<4, true>(s + grp * kLds, 0, PadTwP{s}, q, q2, lt);
    __syncthreads();
    if (grp < 2) blk_phase<4, true>(s + grp * kLds, 4, PadTwP{s}, q, q2, lt);
  } else {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (p) __syncthreads();
      if (grp < 2) blk_phase<2, true, PadTw, 4, GS>(s + grp * kLds, 2 * p, PadTw{s}, q, q2, lt);
    }
  }
  __syncthreads();
  if (grp < 2) {
    uint32_t* dst = grp ? acc1 : acc0;
#pragma unroll
    for (int kk = 0; kk < QPG; ++kk) {
      const int ee = (lt + kk * GS) * 4;
      st4(dst + ee, twist4(lds_blk4(s + grp * kLds, ee), K.T.blk_itwist(pi, blk0 + (ee >> 8)), ee & 255, q));
    }
  }
}

// ============================================================================
// Stage 3: ModDown of both components
// ============================================================================

// INTT column pass of the P rows (already through the block pass) -> x [2][k].
template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void k6_intt_cols_p(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  const int c = blockIdx.y / K.k, mm = blockIdx.y % K.k;
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  constexpr int C = ColGeom<LOGN1, CW, T>::C;
  const int pi = K.T.L_max + mm;
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_itw(pi), ColGeom<LOGN1, CW, T>::N1);
  const uint32_t q = ldc(K.T.mod + pi).q, q2 = 2 * q;
  const uint2 sc = ldc(K.moddown_scale + mm);
  const int col0 = blockIdx.x * C;
  load_cols<LOGN1, CW, T>(s, V.acc + ((size_t)c * V.R + V.L + mm) * N, col0);
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, true, CW, T>(s, stw, q, q2);
  __syncthreads();
  uint32_t* row = V.x + ((size_t)c * K.k + mm) * N;
#pragma unroll
  for (int kk = 0; kk < ColGeom<LOGN1, CW, T>::QUADS; ++kk) {
    const int lin = (threadIdx.x + kk * T) * 4;
    const int pos = lin / C, cc = lin & (C - 1);
    uint4 v = *reinterpret_cast<const uint4*>(s + lidx_col(pos, cc, C));
    v.x = csub(mul_shoup(v.x, sc.x, sc.y, q), q);
    v.y = csub(mul_shoup(v.y, sc.x, sc.y, q), q);
    v.z = csub(mul_shoup(v.z, sc.x, sc.y, q), q);
    v.w = csub(mul_shoup(v.w, sc.x, sc.y, q), q);
    st4(row + pos * 256 + col0 + cc, v);
  }
}

// w[c][i] = sum_m x[c][m] (P/p_m mod q_i) mod q_i; blockIdx.y = c * groups + g.
template <int KP, int RB>
__global__ __launch_bounds__(kWG) void k7_bconv_down(KsConst K, JobArg<KsJob> JA, int groups) {
  const KsJob J = JA.get(blockIdx.z);
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  const int c = blockIdx.y / groups, g = blockIdx.y % groups;
  if (g * RB >= V.L) return;
  const size_t n = ((size_t)blockIdx.x * kWG + threadIdx.x) * 4;  // four coefficients per thread
  uint4 x[KP];
#pragma unroll
  for (int mm = 0; mm < KP; ++mm) x[mm] = ld4(V.x + ((size_t)c * KP + mm) * N + n);
  const int r1 = min(g * RB + RB, V.L);
  for (int i = g * RB; i < r1; ++i) {
    const ModC m = ldc(K.T.mod + i);
    const uint32_t* t = K.moddown_T + (size_t)i * KP;
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int mm = 0; mm < KP; ++mm) {
      const uint64_t tm = ldc(t + mm);
      a0 += x[mm].x * tm;
      a1 += x[mm].y * tm;
      a2 += x[mm].z * tm;
      a3 += x[mm].w * tm;
    }
    st4(V.w + ((size_t)c * V.L + i) * N + n,
        make_uint4(reduce64(a0, m.q, m.mu_hi, m.mu_lo), reduce64(a1, m.q, m.mu_hi, m.mu_lo),
                   reduce64(a2, m.q, m.mu_hi, m.mu_lo), reduce64(a3, m.q, m.mu_hi, m.mu_lo)));
  }
}

template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void k8_ntt_cols_w(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const size_t N = (size_t)1 << K.T.logN;
  const KsView V = ks_view(J, K, N);
  const int gr = blockIdx.y;
  if (gr >= 2 * V.L) return;
  const int i = gr % V.L;
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_tw(i), ColGeom<LOGN1, CW, T>::N1);
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  const uint32_t q = ldc(K.T.mod + i).q, q2 = 2 * q;
  const int col0 = blockIdx.x * ColGeom<LOGN1, CW, T>::C;
  uint32_t* row = V.w + (size_t)gr * N;
  load_cols<LOGN1, CW, T>(s, row, col0);
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, false, CW, T>(s, stw, q, q2);
  __syncthreads();
  store_cols<LOGN1, CW, T>(s, row, col0);
}

// out[c][i] = (acc[c][i] - NTT(w)[c][i]) P^-1 (+ the job's epilogue term).
// BPW blocks per work-group as in K1.
template <int LOGN1, int BPW>
__global__ __launch_bounds__(kWG) void k9_ntt_blks_combine(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const int logN = K.T.logN;
  const size_t N = (size_t)1 << logN;
  const KsView V = ks_view(J, K, N);
  const int gr = blockIdx.y;
  if (gr >= 2 * V.L) return;
  const int c = gr / V.L, i = gr % V.L;
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(K.T.blk_tw(i), 256);
  __shared__ __align__(16) uint32_t s[kLds];
  const ModC m = ldc(K.T.mod + i);
  const uint32_t q = m.q, q2 = 2 * q;
  constexpr int QPT = BPW / 4;  // quads per thread
  const int blk0 = blockIdx.x * BPW;
  const uint32_t base = blk0 * 256;
  const uint32_t* wrow = V.w + (size_t)gr * N + base;
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem(kk);
    lds_blk4_store(s, e, twist4(ld4(wrow + e),
                                K.T.blk_twist(i, blk0 + (e >> 8)), e & 255, q));
  }
  if constexpr (BPW == 16)
    tw_put_perm(stw, tww);
  else
    tw_put(stw, tww, 256);
  __syncthreads();
  if constexpr (BPW == 16)
    blk_stages<false>(s, PermTw{stw}, q, q2);
  else
    blk_stages_r4<false, const uint2*, kWG>(s, stw, q, q2);
  __syncthreads();
  const uint2 pv = ldc(K.pinv + i);
  const uint32_t* accr = V.acc + ((size_t)c * V.R + i) * N + base;
  uint32_t* out = J.out + ((size_t)c * V.L + i) * N + base;
  const size_t L = V.L;
  const bool hmult = J.kind == KS_HMULT;
  const bool rot = (J.kind == KS_HROT || J.kind == KS_HOIST) && c == 0;
  // Loads first (a store to out could alias a later load): the accumulator
  // quads and the term this component adds — d0 = c0 c0' or d1 = c0 c1' + c1 c0'
  // (HMULT, formed here from the inputs), sigma(c0) (rotations, c = 0), else 0.
  // The term is formed as soon as its words arrive, so at most one quad's
  // inputs are live at a time.
  uint4 av[QPT], dv[QPT];
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem(kk);
    const uint32_t n = base + e;
    av[kk] = ld4(accr + e);
    dv[kk] = make_uint4(0, 0, 0, 0);
    if (hmult) {
      const uint4 xa = ld4(J.a + i * N + n), ya = ld4(J.b + i * N + n);
      if (c == 0) {
        dv[kk] = make_uint4(mulmod(xa.x, ya.x, m), mulmod(xa.y, ya.y, m), mulmod(xa.z, ya.z, m),
                            mulmod(xa.w, ya.w, m));
      } else {
        const uint4 xb = ld4(J.a + (L + i) * N + n), yb = ld4(J.b + (L + i) * N + n);
        dv[kk] = make_uint4(
            reduce64((uint64_t)xa.x * yb.x + (uint64_t)xb.x * ya.x, q, m.mu_hi, m.mu_lo),
            reduce64((uint64_t)xa.y * yb.y + (uint64_t)xb.y * ya.y, q, m.mu_hi, m.mu_lo),
            reduce64((uint64_t)xa.z * yb.z + (uint64_t)xb.z * ya.z, q, m.mu_hi, m.mu_lo),
            reduce64((uint64_t)xa.w * yb.w + (uint64_t)xb.w * ya.w, q, m.mu_hi, m.mu_lo));
      }
    } else if (rot) {
      const uint32_t* c0 = J.a + i * N;
      dv[kk] = make_uint4(ld1(c0 + auto_src(n, J.gal, logN)), ld1(c0 + auto_src(n + 1, J.gal, logN)),
                          ld1(c0 + auto_src(n + 2, J.gal, logN)), ld1(c0 + auto_src(n + 3, J.gal, logN)));
    }
  }
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem(kk);
    // w from [0, 4q) to [0, 2q): a + 2q - w < 3q < 2^32 goes straight into
    // the Shoup product
    const uint4 w = csub4(lds_blk4(s, e), q2);
    const uint4 a = av[kk], d = dv[kk];
    const uint32_t o0 = csub(mul_shoup(a.x + q2 - w.x, pv.x, pv.y, q), q);
    const uint32_t o1 = csub(mul_shoup(a.y + q2 - w.y, pv.x, pv.y, q), q);
    const uint32_t o2 = csub(mul_shoup(a.z + q2 - w.z, pv.x, pv.y, q), q);
    const uint32_t o3 = csub(mul_shoup(a.w + q2 - w.w, pv.x, pv.y, q), q);
    st4(out + e, make_uint4(csub(o0 + d.x, q), csub(o1 + d.y, q), csub(o2 + d.z, q), csub(o3 + d.w, q)));
  }
}

// ============================================================================
// Rescale: t = INTT_{q_{L-1}}(a_{L-1}); out_i = (a_i - NTT_{q_i}(t mod q_i)) q_{L-1}^-1
// Scratch: t [2][N], u [2][L-1][N].
// ============================================================================
// BPW blocks per work-group as in K1 (4: quarter tiles in radix-4 phases).
template <int LOGN1, int BPW>
__global__ __launch_bounds__(kWG) void r1_intt_blks(KsConst K, JobArg<RsJob> JA) {
  const RsJob J = JA.get(blockIdx.z);
  const int c = blockIdx.y, L = J.L, pi = L - 1;
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(K.T.blk_itw(pi), 256);
  __shared__ __align__(16) uint32_t s[kLds];
  const size_t N = (size_t)1 << K.T.logN;
  const uint32_t q = ldc(K.T.mod + pi).q, q2 = 2 * q;
  constexpr int QPT = BPW / 4;  // quads per thread
  const int blk0 = blockIdx.x * BPW;
  const uint32_t* in = J.a + ((size_t)c * L + pi) * N + blk0 * 256;
  uint32_t* t = J.ws + (size_t)c * N + blk0 * 256;
  uint4 x[QPT];
  Twist4 tfi[QPT];  // the epilogue's twist factors, requested with the tile
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) x[kk] = ld4(in + blk_elem(kk));
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) {
    const int e = blk_elem(kk);
    tfi[kk] = twist4_load(K.T.blk_itwist(pi, blk0 + (e >> 8)), e & 255);
  }
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) lds_blk4_store(s, blk_elem(kk), x[kk]);
  if constexpr (BPW == 16)
    tw_put_perm(stw, tww);
  else
    tw_put(stw, tww, 256);
  __syncthreads();
  if constexpr (BPW == 16)
    blk_stages<true>(s, PermTw{stw}, q, q2);
  else
    blk_stages_r4<true, const uint2*, kWG>(s, stw, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < QPT; ++kk) st4(t + blk_elem(kk), twist4(lds_blk4(s, blk_elem(kk)), tfi[kk], q));
}

template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void r2_intt_cols(KsConst K, JobArg<RsJob> JA) {
  const RsJob J = JA.get(blockIdx.z);
  const int c = blockIdx.y, pi = J.L - 1;
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_itw(pi), ColGeom<LOGN1, CW, T>::N1);
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  constexpr int C = ColGeom<LOGN1, CW, T>::C;
  const size_t N = (size_t)1 << K.T.logN;
  const ModC m = ldc(K.T.mod + pi);
  const uint32_t q = m.q, q2 = 2 * q;
  const int col0 = blockIdx.x * C;
  uint32_t* row = J.ws + (size_t)c * N;
  load_cols<LOGN1, CW, T>(s, row, col0);
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, true, CW, T>(s, stw, q, q2);
  __syncthreads();
#pragma unroll
  for (int kk = 0; kk < ColGeom<LOGN1, CW, T>::QUADS; ++kk) {
    const int lin = (threadIdx.x + kk * T) * 4;
    const int pos = lin / C, cc = lin & (C - 1);
    uint4 v = *reinterpret_cast<const uint4*>(s + lidx_col(pos, cc, C));
    v.x = csub(mul_shoup(v.x, m.ninv, m.ninv_s, q), q);
    v.y = csub(mul_shoup(v.y, m.ninv, m.ninv_s, q), q);
    v.z = csub(mul_shoup(v.z, m.ninv, m.ninv_s, q), q);
    v.w = csub(mul_shoup(v.w, m.ninv, m.ninv_s, q), q);
    st4(row + pos * 256 + col0 + cc, v);
  }
}

// NTT column pass of t mod q_i for every i < L - 1 (the broadcast is the loader).
template <int LOGN1, int CW, int T>
__global__ __launch_bounds__(T) void r3_ntt_cols(KsConst K, JobArg<RsJob> JA) {
  const RsJob J = JA.get(blockIdx.z);
  const int L1 = J.L - 1;
  const int gr = blockIdx.y;
  if (gr >= 2 * L1) return;
  const int c = gr / L1, i = gr % L1;
  __shared__ uint2 stw[ColGeom<LOGN1, CW, T>::N1];
  const uint2 tww = tw_fetch(K.T.col_tw(i), ColGeom<LOGN1, CW, T>::N1);
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1, CW, T>::LDS];
  constexpr int C = ColGeom<LOGN1, CW, T>::C;
  const size_t N = (size_t)1 << K.T.logN;
  const ModC m = ldc(K.T.mod + i);
  const uint32_t q = m.q, q2 = 2 * q;
  const int col0 = blockIdx.x * C;
  const uint32_t* t = J.ws + (size_t)c * N;
#pragma unroll
  for (int kk = 0; kk < ColGeom<LOGN1, CW, T>::QUADS; ++kk) {
    const int lin = (threadIdx.x + kk * T) * 4;
    const int pos = lin / C, cc = lin & (C - 1);
    uint4 v = ld4(t + pos * 256 + col0 + cc);
    v.x = reduce32(v.x, q, m.mu32);
    v.y = reduce32(v.y, q, m.mu32);
    v.z = reduce32(v.z, q, m.mu32);
    v.w = reduce32(v.w, q, m.mu32);
    *reinterpret_cast<uint4*>(s + lidx_col(pos, cc, C)) = v;
  }
  tw_put(stw, tww, ColGeom<LOGN1, CW, T>::N1);
  __syncthreads();
  col_stages<LOGN1, false, CW, T>(s, stw, q, q2);
  __syncthreads();
  store_cols<LOGN1, CW, T>(s, J.ws + (size_t)(2 + gr) * N, col0);
}

template <int LOGN1>
__global__ __launch_bounds__(kWG) void r4_ntt_blks_combine(KsConst K, JobArg<RsJob> JA) {
  const RsJob J = JA.get(blockIdx.z);
  const int L1 = J.L - 1;
  const int gr = blockIdx.y;
  if (gr >= 2 * L1) return;
  const int c = gr / L1, i = gr % L1;
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(K.T.blk_tw(i), 256);
  __shared__ __align__(16) uint32_t s[kLds];
  const size_t N = (size_t)1 << K.T.logN;
  const uint32_t q = ldc(K.T.mod + i).q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t base = blk0 * 256;
  const uint32_t* u = J.ws + (size_t)(2 + gr) * N + base;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    lds_blk4_store(s, e, twist4(ld4(u + e),
                                K.T.blk_twist(i, blk0 + (e >> 8)), e & 255, q));
  }
  tw_put_perm(stw, tww);
  __syncthreads();
  blk_stages<false>(s, PermTw{stw}, q, q2);
  __syncthreads();
  const uint2 qi = ldc(K.rescale_inv + (size_t)J.L * K.T.L_max + i);
  const uint32_t* a = J.a + ((size_t)c * J.L + i) * N + base;
  uint32_t* out = J.out + ((size_t)c * L1 + i) * N + base;
  uint4 xs[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) xs[kk] = ld4(a + blk_elem(kk));
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int e = blk_elem(kk);
    const uint4 v = csub4(lds_blk4(s, e), q2);  // [0, 2q): x + 2q - v < 3q
    const uint4 x = xs[kk];
    st4(out + e, make_uint4(csub(mul_shoup(x.x + q2 - v.x, qi.x, qi.y, q), q), csub(mul_shoup(x.y + q2 - v.y, qi.x, qi.y, q), q),
                   csub(mul_shoup(x.z + q2 - v.z, qi.x, qi.y, q), q), csub(mul_shoup(x.w + q2 - v.w, qi.x, qi.y, q), q)));
  }
}


// ============================================================================
// Small rings (N = 2^kSrLog = 4096): a whole limb fits one work-group's LDS,
// so the two-pass NTT split -- and with it the nine-kernel pipeline -- is not
// needed.  A key-switch runs as two kernels of 1024-thread work-groups:
//   S1  per (ModUp row t, group of digits): each non-digit limb of a digit
//       transformed back whole in LDS, scaled, converted to row t (BConv),
//       the sum transformed forward, times the key rows; the products summed
//       over the group's digits -> one partial accumulator per group;
//   S2  per (Q row i, component): the partials summed; ModDown -- the P rows'
//       INTT whole in LDS, their conversion to q_i, its NTT -- combined with
//       the accumulator, plus the job's epilogue term.
// The arithmetic is that of the nine kernels (exact: the same residues).
// Scratch of a job: the partials [groups][2][L + k][N] (at most kSrGroups = 4).
// ============================================================================
constexpr int kSrN = 1 << kSrLog;
constexpr int kSrT = kSrN / 4;  // threads: one radix-4 unit / one quad each

__device__ __forceinline__ int sr_per(int beta) { return (beta + kSrGroups - 1) / kSrGroups; }  // digits per group
__device__ __forceinline__ int sr_groups(int beta) { return (beta + sr_per(beta) - 1) / sr_per(beta); }

// Forward negacyclic NTT of the limb in s (natural coefficients in,
// bit-reversed evaluations out) as six radix-4 phases; twiddle of group
// (m, g) at tw[m + g].  Unit u of the phase on stages (ls, ls + 1) covers
// a = 4 g t2 + i, a + t2, a + 2 t2, a + 3 t2 (t2 = N / (4 m), g = u / t2,
// i = u % t2).  Words in [0, 4q) throughout (Harvey butterflies).
__device__ __forceinline__ void sr_ntt(uint32_t* s, const uint2* tw, uint32_t q) {
  const uint32_t q2 = 2 * q;
  const int u = threadIdx.x;
#pragma unroll
  for (int ls = 0; ls < kSrLog; ls += 2) {
    const int lt2 = kSrLog - ls - 2;  // log2 t2
    const int m = 1 << ls;
    const int g = u >> lt2, i = u & ((1 << lt2) - 1);
    const int a = (g << (lt2 + 2)) + i, t2 = 1 << lt2;
    uint32_t x0 = s[a], x1 = s[a + t2], x2 = s[a + 2 * t2], x3 = s[a + 3 * t2];
    const uint2 w = tw[m + g], w0 = tw[2 * m + 2 * g], w1 = tw[2 * m + 2 * g + 1];
    bfly_ct(x0, x2, w.x, w.y, q, q2);
    bfly_ct(x1, x3, w.x, w.y, q, q2);
    bfly_ct(x0, x1, w0.x, w0.y, q, q2);
    bfly_ct(x2, x3, w1.x, w1.y, q, q2);
    s[a] = x0;
    s[a + t2] = x1;
    s[a + 2 * t2] = x2;
    s[a + 3 * t2] = x3;
    __syncthreads();
  }
}

// Inverse (Gentleman-Sande, bit-reversed in, natural out, no N^-1), six
// radix-4 phases: unit u of the phase on half-sizes (t, 2t) covers
// a = 4 g t + i, a + t, a + 2t, a + 3t (g = u / t, i = u % t); the stage of
// m = N / (2t) groups pairs (a, a + t) and (a + 2t, a + 3t), the next
// (a, a + 2t) and (a + t, a + 3t).  Words in [0, 2q) throughout.
__device__ __forceinline__ void sr_intt(uint32_t* s, const uint2* itw, uint32_t q) {
  const uint32_t q2 = 2 * q;
  const int u = threadIdx.x;
#pragma unroll
  for (int lt = 0; lt < kSrLog; lt += 2) {
    const int m = kSrN >> (lt + 1);
    const int g = u >> lt, i = u & ((1 << lt) - 1);
    const int a = (g << (lt + 2)) + i, t = 1 << lt;
    uint32_t x0 = s[a], x1 = s[a + t], x2 = s[a + 2 * t], x3 = s[a + 3 * t];
    const uint2 w0 = itw[m + 2 * g], w1 = itw[m + 2 * g + 1], w = itw[(m >> 1) + g];
    bfly_gs(x0, x1, w0.x, w0.y, q, q2);
    bfly_gs(x2, x3, w1.x, w1.y, q, q2);
    bfly_gs(x0, x2, w.x, w.y, q, q2);
    bfly_gs(x1, x3, w.x, w.y, q, q2);
    s[a] = x0;
    s[a + t] = x1;
    s[a + 2 * t] = x2;
    s[a + 3 * t] = x3;
    __syncthreads();
  }
}

// The quad at 4 threadIdx.x of row r of the polynomial a job key-switches
// (evaluation domain): d, c1 c1' or sigma(c1).  Loaded raw (both factors of
// the product) so that a prefetch does not wait for its data; the product is
// taken by sr_switched_finish where the quad is used.
struct SrRaw {
  uint4 x, y;
};
// Branch-free (the kind selects addresses, every load is issued): a load in
// a branch whose value merges after it makes the compiler wait for it there.
// x: row r of d, the evaluations of c1 (HMult) or sigma(c1) gathered (HRot);
// y: row r of c1' (HMult; otherwise x's row again, unused).
__device__ __forceinline__ SrRaw sr_switched_load(const KsJob& J, int r) {
  const size_t N = kSrN;
  const uint32_t n = 4 * threadIdx.x;
  const bool rot = J.kind == KS_HROT;
  const uint32_t* src = J.a + (size_t)(J.kind == KS_PLAIN ? r : J.L + r) * N;
  const uint32_t* src2 = J.kind == KS_HMULT ? J.b + (size_t)(J.L + r) * N : src;
  SrRaw o;
  o.x = make_uint4(ld1(src + (rot ? auto_src(n, J.gal, kSrLog) : n)),
                   ld1(src + (rot ? auto_src(n + 1, J.gal, kSrLog) : n + 1)),
                   ld1(src + (rot ? auto_src(n + 2, J.gal, kSrLog) : n + 2)),
                   ld1(src + (rot ? auto_src(n + 3, J.gal, kSrLog) : n + 3)));
  o.y = ld4(src2 + n);
  return o;
}
__device__ __forceinline__ uint4 sr_switched_finish(const KsJob& J, const SrRaw& v, const ModC& m) {
  if (J.kind != KS_HMULT) return v.x;
  return make_uint4(mulmod(v.x.x, v.y.x, m), mulmod(v.x.y, v.y.y, m), mulmod(v.x.z, v.y.z, m),
                    mulmod(v.x.w, v.y.w, m));
}

// A thread's four twiddle pairs of a whole-limb table (words t, t + T, t + 2T, t + 3T).
__device__ __forceinline__ void sr_load_tw(uint2 w[4], const uint2* __restrict__ src) {
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = src[threadIdx.x + k * kSrT];
}
__device__ __forceinline__ void sr_put_tw(uint2* dst, const uint2 w[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) dst[threadIdx.x + k * kSrT] = w[k];
}

// S1.  The work-group's items are its digits' limbs in order (a digit row of
// the switched polynomial is one item without transforms).  The loads of an
// item -- its quad of the switched polynomial, its prime's inverse twiddles
// and BConv constants, the digit's key words -- are issued one item ahead,
// before the current item's transforms, so only the first item waits on
// memory.
__global__ __launch_bounds__(kSrT) void s1_modup_ip(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const int L = J.L, R = L + K.k, beta = (L + K.alpha - 1) / K.alpha;
  const int t = blockIdx.x, per = sr_per(beta), gi = blockIdx.y;
  const int j0 = gi * per, j1 = min(beta, j0 + per);
  if (t >= R || j0 >= beta || J.kind > KS_HROT) return;
  __shared__ __align__(16) uint32_t sd[kSrN];
  __shared__ uint2 stw[kSrN], sitw[kSrN];
  const size_t N = kSrN;
  const size_t KR = (size_t)K.T.L_max + K.k;
  const int pt = ks_pidx(t, L, K.T.L_max);
  const ModC mt = ldc(K.T.mod + pt);
  const uint32_t n = 4 * threadIdx.x;
  // the first item of digit j: its first limb, or row t itself when t is one of the digit's rows
  auto first_limb = [&](int j) { return (t >= j * K.alpha && t < min(j * K.alpha + K.alpha, L)) ? t : j * K.alpha; };
  auto key_of = [&](int j, uint4& e0, uint4& e1) {
    const uint32_t* k0 = J.key + ((size_t)j * 2 * KR + pt) * N + n;
    e0 = ld4(k0);
    e1 = ld4(k0 + KR * N);
  };
  // BConv constants of limb i of digit j: N^-1 (D_j / q_i)^-1 and [D_j / q_i]_{q_t}
  auto consts_of = [&](int j, int i, uint2& sc, uint64_t& T) {
    sc = ldc(K.modup_scale + (size_t)L * K.T.L_max + i);
    T = ldc(K.modup_T + ldc(K.modup_T_off + (size_t)L * K.beta_max + j) + (size_t)t * K.alpha + (i - j * K.alpha));
  };
  int j = j0, i = first_limb(j0);
  SrRaw x = sr_switched_load(J, i);
  uint4 e0, e1;
  uint2 iw[4], sc, fw[4];
  uint64_t T;
  key_of(j, e0, e1);
  sr_load_tw(iw, K.T.full_itw(i));  // i < L: a Q prime's table
  consts_of(j, i, sc, T);
  sr_load_tw(fw, K.T.full_tw(pt));  // forward twiddles of q_t, issued last: their wait covers the rest
  sr_put_tw(stw, fw);               // published by the first barrier
  uint64_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
  uint64_t z0 = 0, z1 = 0, z2 = 0, z3 = 0;
  for (;;) {
    const int hi = min(j * K.alpha + K.alpha, L);
    const bool own = i == t;
    const bool last_of_digit = own || i == hi - 1;
    int jn = j, in = i + 1;  // the next item
    if (last_of_digit) {
      jn = j + 1;
      in = jn < j1 ? first_limb(jn) : -1;
    }
    // the next item's loads; the registers are written only when there is
    // one (a load left in flight at the end would hold the wave until it lands)
    SrRaw xn;
    uint4 e0n, e1n;
    uint2 iwn[4], scn;
    uint64_t Tn;
    if (in >= 0) {
      xn = sr_switched_load(J, in);
      key_of(jn, e0n, e1n);
      sr_load_tw(iwn, K.T.full_itw(in));  // a Q prime's table (in < L)
      consts_of(jn, in, scn, Tn);
    }
    uint4 v;
    bool have_v = false;
    if (own) {
      v = sr_switched_finish(J, x, mt);
      have_v = true;
    } else {
      const ModC mi = ldc(K.T.mod + i);
      const uint4 xi = sr_switched_finish(J, x, mi);
      __syncthreads();  // the previous transform has been read out of LDS
      sr_put_tw(sitw, iw);
      *reinterpret_cast<uint4*>(sd + n) = xi;
      __syncthreads();
      sr_intt(sd, sitw, mi.q);
      const uint4 y = *reinterpret_cast<const uint4*>(sd + n);
      z0 += (uint64_t)csub(mul_shoup(y.x, sc.x, sc.y, mi.q), mi.q) * T;
      z1 += (uint64_t)csub(mul_shoup(y.y, sc.x, sc.y, mi.q), mi.q) * T;
      z2 += (uint64_t)csub(mul_shoup(y.z, sc.x, sc.y, mi.q), mi.q) * T;
      z3 += (uint64_t)csub(mul_shoup(y.w, sc.x, sc.y, mi.q), mi.q) * T;
      if (last_of_digit) {  // the digit's sum, mod q_t, transformed forward
        __syncthreads();
        *reinterpret_cast<uint4*>(sd + n) =
            make_uint4(reduce64(z0, mt.q, mt.mu_hi, mt.mu_lo), reduce64(z1, mt.q, mt.mu_hi, mt.mu_lo),
                       reduce64(z2, mt.q, mt.mu_hi, mt.mu_lo), reduce64(z3, mt.q, mt.mu_hi, mt.mu_lo));
        z0 = z1 = z2 = z3 = 0;
        __syncthreads();
        sr_ntt(sd, stw, mt.q);
        v = canon4(*reinterpret_cast<const uint4*>(sd + n), mt.q, 2 * mt.q);
        have_v = true;
      }
    }
    if (have_v) {
      a0[0] += (uint64_t)v.x * e0.x;
      a0[1] += (uint64_t)v.y * e0.y;
      a0[2] += (uint64_t)v.z * e0.z;
      a0[3] += (uint64_t)v.w * e0.w;
      a1[0] += (uint64_t)v.x * e1.x;
      a1[1] += (uint64_t)v.y * e1.y;
      a1[2] += (uint64_t)v.z * e1.z;
      a1[3] += (uint64_t)v.w * e1.w;
      if (((j - j0) & 7) == 7) {  // canonical products < 2^60: fold every eighth digit
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a0[e] = reduce64(a0[e], mt.q, mt.mu_hi, mt.mu_lo);
          a1[e] = reduce64(a1[e], mt.q, mt.mu_hi, mt.mu_lo);
        }
      }
    }
    if (in < 0) break;
    j = jn;
    i = in;
    x = xn;
    e0 = e0n;
    e1 = e1n;
#pragma unroll
    for (int k = 0; k < 4; ++k) iw[k] = iwn[k];
    sc = scn;
    T = Tn;
  }
  uint32_t* p0 = J.ws + ((size_t)(2 * gi) * R + t) * N + n;
  uint32_t* p1 = p0 + (size_t)R * N;
  st4(p0, make_uint4(reduce64(a0[0], mt.q, mt.mu_hi, mt.mu_lo), reduce64(a0[1], mt.q, mt.mu_hi, mt.mu_lo),
                     reduce64(a0[2], mt.q, mt.mu_hi, mt.mu_lo), reduce64(a0[3], mt.q, mt.mu_hi, mt.mu_lo)));
  st4(p1, make_uint4(reduce64(a1[0], mt.q, mt.mu_hi, mt.mu_lo), reduce64(a1[1], mt.q, mt.mu_hi, mt.mu_lo),
                     reduce64(a1[2], mt.q, mt.mu_hi, mt.mu_lo), reduce64(a1[3], mt.q, mt.mu_hi, mt.mu_lo)));
}

// The groups' partials (at most four) at the thread's quad of row r, loaded
// raw: group indices past `groups` repeat the last group and are dropped by
// sr_partials_sum.
__device__ __forceinline__ void sr_partials_load(uint4 v[4], const uint32_t* ws, int groups, int c, int R, int r) {
  const size_t N = kSrN;
  const uint32_t n = 4 * threadIdx.x;
#pragma unroll
  for (int g = 0; g < 4; ++g) v[g] = ld4(ws + ((size_t)(2 * min(g, groups - 1) + c) * R + r) * N + n);
}
__device__ __forceinline__ uint4 sr_partials_sum(const uint4 v[4], int groups, uint32_t q) {
  uint4 s = v[0];  // canonical partials: the sum of four stays below 4q < 2^32
#pragma unroll
  for (int g = 1; g < 4; ++g) {
    const uint32_t k = g < groups ? 0xffffffffu : 0u;
    s.x += v[g].x & k;
    s.y += v[g].y & k;
    s.z += v[g].z & k;
    s.w += v[g].w & k;
  }
  return canon4(s, q, 2 * q);
}

// S2.  Every load is issued at the start (the next P row's during the
// current P row's transform): q_i's forward twiddles, the accumulator's
// partials at row i, the epilogue operands, the first P row's partials and
// inverse twiddles.
__global__ __launch_bounds__(kSrT) void s2_moddown(KsConst K, JobArg<KsJob> JA) {
  const KsJob J = JA.get(blockIdx.z);
  const int L = J.L, R = L + K.k, beta = (L + K.alpha - 1) / K.alpha;
  const int i = blockIdx.x, c = blockIdx.y, groups = sr_groups(beta);
  if (i >= L || J.kind > KS_HROT) return;
  __shared__ __align__(16) uint32_t sd[kSrN];
  __shared__ uint2 stw[kSrN], sitw[kSrN];
  const size_t N = kSrN, Lz = L;
  const uint32_t n = 4 * threadIdx.x;
  const ModC mi = ldc(K.T.mod + i);
  const uint32_t q = mi.q, q2 = 2 * q;
  uint2 fw[4], iw[4];
  sr_load_tw(fw, K.T.full_tw(i));
  uint4 pa[4], px[4];
  sr_partials_load(px, J.ws, groups, c, R, L);
  sr_load_tw(iw, K.T.full_itw(K.T.L_max));
  sr_partials_load(pa, J.ws, groups, c, R, i);
  // the epilogue operands, branch-free (as in sr_switched_load): c0, c0', c1,
  // c1' at row i (HMult: c0 c0' / c0 c1' + c1 c0'); sigma(c0) gathered (HRot, c = 0)
  const bool hm = J.kind == KS_HMULT, rot = J.kind == KS_HROT && c == 0;
  const uint32_t* ra = J.a + i * N;
  const uint32_t* rb = hm ? J.b + i * N : ra;
  const uint32_t* rc = hm ? J.a + (Lz + i) * N : ra;
  const uint32_t* rd = hm ? J.b + (Lz + i) * N : ra;
  const uint4 ea = make_uint4(ld1(ra + (rot ? auto_src(n, J.gal, kSrLog) : n)),
                              ld1(ra + (rot ? auto_src(n + 1, J.gal, kSrLog) : n + 1)),
                              ld1(ra + (rot ? auto_src(n + 2, J.gal, kSrLog) : n + 2)),
                              ld1(ra + (rot ? auto_src(n + 3, J.gal, kSrLog) : n + 3)));
  const uint4 eb = ld4(rb + n), ec = ld4(rc + n), ed = ld4(rd + n);
  sr_put_tw(stw, fw);  // published by the first barrier below
  // ModDown: w = sum_m x_m [P / p_m]_{q_i}, x_m = INTT(acc P row m) N^-1 (P / p_m)^-1
  uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
  for (int mm = 0; mm < K.k; ++mm) {
    const int pm = K.T.L_max + mm;
    const ModC mp = ldc(K.T.mod + pm);
    const uint2 sc = ldc(K.moddown_scale + mm);
    const uint64_t T = ldc(K.moddown_T + (size_t)i * K.k + mm);
    const bool more = mm + 1 < K.k;
    uint4 pxn[4];
    uint2 iwn[4];
    if (more) {  // the next P row's loads
      sr_partials_load(pxn, J.ws, groups, c, R, L + mm + 1);
      sr_load_tw(iwn, K.T.full_itw(pm + 1));
    }
    const uint4 x = sr_partials_sum(px, groups, mp.q);
    __syncthreads();  // the previous P row has been read out of LDS
    sr_put_tw(sitw, iw);
    *reinterpret_cast<uint4*>(sd + n) = x;
    __syncthreads();
    sr_intt(sd, sitw, mp.q);
    const uint4 y = *reinterpret_cast<const uint4*>(sd + n);
    w0 += (uint64_t)csub(mul_shoup(y.x, sc.x, sc.y, mp.q), mp.q) * T;
    w1 += (uint64_t)csub(mul_shoup(y.y, sc.x, sc.y, mp.q), mp.q) * T;
    w2 += (uint64_t)csub(mul_shoup(y.z, sc.x, sc.y, mp.q), mp.q) * T;
    w3 += (uint64_t)csub(mul_shoup(y.w, sc.x, sc.y, mp.q), mp.q) * T;
    if (more) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        px[k] = pxn[k];
        iw[k] = iwn[k];
      }
    }
  }
  const uint2 pv = ldc(K.pinv + i);
  __syncthreads();
  *reinterpret_cast<uint4*>(sd + n) = make_uint4(reduce64(w0, q, mi.mu_hi, mi.mu_lo), reduce64(w1, q, mi.mu_hi, mi.mu_lo),
                                                 reduce64(w2, q, mi.mu_hi, mi.mu_lo), reduce64(w3, q, mi.mu_hi, mi.mu_lo));
  __syncthreads();
  sr_ntt(sd, stw, q);
  const uint4 w = csub4(*reinterpret_cast<const uint4*>(sd + n), q2);  // [0, 2q)
  const uint4 a = sr_partials_sum(pa, groups, q);
  uint4 d = rot ? ea : make_uint4(0, 0, 0, 0);
  if (hm) {
    if (c == 0) {
      d = make_uint4(mulmod(ea.x, eb.x, mi), mulmod(ea.y, eb.y, mi), mulmod(ea.z, eb.z, mi), mulmod(ea.w, eb.w, mi));
    } else {
      d = make_uint4(reduce64((uint64_t)ea.x * ed.x + (uint64_t)ec.x * eb.x, q, mi.mu_hi, mi.mu_lo),
                     reduce64((uint64_t)ea.y * ed.y + (uint64_t)ec.y * eb.y, q, mi.mu_hi, mi.mu_lo),
                     reduce64((uint64_t)ea.z * ed.z + (uint64_t)ec.z * eb.z, q, mi.mu_hi, mi.mu_lo),
                     reduce64((uint64_t)ea.w * ed.w + (uint64_t)ec.w * eb.w, q, mi.mu_hi, mi.mu_lo));
    }
  }
  const uint32_t o0 = csub(mul_shoup(a.x + q2 - w.x, pv.x, pv.y, q), q);
  const uint32_t o1 = csub(mul_shoup(a.y + q2 - w.y, pv.x, pv.y, q), q);
  const uint32_t o2 = csub(mul_shoup(a.z + q2 - w.z, pv.x, pv.y, q), q);
  const uint32_t o3 = csub(mul_shoup(a.w + q2 - w.w, pv.x, pv.y, q), q);
  st4(J.out + ((size_t)c * Lz + i) * N + n, make_uint4(csub(o0 + d.x, q), csub(o1 + d.y, q), csub(o2 + d.z, q), csub(o3 + d.w, q)));
}
}  // namespace

size_t ks_ws_words(const Ctx& c, int L) {
  const size_t R = (size_t)L + c.k;
  return ks_hoist_ws_words(c, L) + (2 * (size_t)L + (size_t)c.beta(L) * R) * c.N;
}

size_t ks_hoist_ws_words(const Ctx& c, int L) {
  return (2 * ((size_t)L + c.k) + 2 * (size_t)c.k + 2 * (size_t)L) * c.N;
}

size_t rs_ws_words(const Ctx& c, int L) { return (2 + 2 * (size_t)L) * c.N; }

namespace {
// BConv output rows per work-group (Ctx::Sched): a group re-reads its
// inputs once, so more rows per group mean fewer re-reads but fewer groups.
template <template <int, int> class KERN, int A>
void launch_bconv(const Ctx& c, int stage, int rows, dim3 g, hipStream_t st, const KsConst& K,
                  const JobArg<KsJob>& J, int gr) {
  switch (rows) {
    case 2: klaunch(c, stage, KERN<A, 2>::fn, g, st, K, J, gr); break;
    case 4: klaunch(c, stage, KERN<A, 4>::fn, g, st, K, J, gr); break;
    case 6: klaunch(c, stage, KERN<A, 6>::fn, g, st, K, J, gr); break;
    default: klaunch(c, stage, KERN<A, 12>::fn, g, st, K, J, gr); break;
  }
}

// Launch of a pipeline kernel; when its stage is traced, the trace events
// are attached to the dispatch itself.
template <typename F, typename... A>
void klaunch_b(const Ctx& c, int stage, F kern, dim3 g, int block, hipStream_t st, A... args) {
  hipEvent_t t0, t1;
  c.trace_take(stage, &t0, &t1);
  hipExtLaunchKernelGGL(kern, g, dim3(block), 0, st, t0, t1, 0, args...);
}
template <typename F, typename... A>
void klaunch(const Ctx& c, int stage, F kern, dim3 g, hipStream_t st, A... args) {
  klaunch_b(c, stage, kern, g, kWG, st, args...);
}

// Dispatch a small compile-time count (digit size or special-prime count, 1..16).
template <int A, int RB>
struct K3fn {
  static constexpr auto fn = k3_bconv_up<A, RB>;
};
template <int A, int RB>
struct K7fn {
  static constexpr auto fn = k7_bconv_down<A, RB>;
};
template <int A>
struct K3 {
  static void run(const Ctx& c, dim3 g, hipStream_t st, const KsConst& K, const JobArg<KsJob>& J,
                  int gr, int rows) {
    launch_bconv<K3fn, A>(c, CKKS_STAGE_BCONV_UP, rows, g, st, K, J, gr);
  }
};
template <int A>
struct K7 {
  static void run(const Ctx& c, dim3 g, hipStream_t st, const KsConst& K, const JobArg<KsJob>& J,
                  int gr, int rows) {
    launch_bconv<K7fn, A>(c, CKKS_STAGE_BCONV_DOWN, rows, g, st, K, J, gr);
  }
};

template <template <int> class F, int V>
hipError_t small_dispatch(int v, const Ctx& c, dim3 g, hipStream_t st, const KsConst& K,
                          const JobArg<KsJob>& J, int gr, int rows) {
  if constexpr (V > kMaxAlpha) {
    return hipErrorInvalidValue;
  } else {
    if (v == V) {
      F<V>::run(c, g, st, K, J, gr, rows);
      return hipSuccess;
    }
    return small_dispatch<F, V + 1>(v, c, g, st, K, J, gr, rows);
  }
}

// Column passes with fewer work-groups than this (half a work-group per CU)
// use the narrowest column tiles, which double the work-groups at N = 2^16:
// for such a grid every CU that joins shortens the pass (the rescale's INTT
// of one limb: 8.4 -> 5.5 us), while at 192 or 288 work-groups the half-line
// row segments cost more than the extra CUs gain (K2: 12.1 -> 14.1 us).
constexpr int kNarrowBelow = 128;
// Threads of the column passes over whole-line tiles: 16 elements per thread
// (512 threads for the 8192-word tiles at N = 2^16).
template <int L1>
constexpr int kColThreads = ColGeom<L1>::ELEMS / 16;

template <int L1, int CW, int T>
struct K2c { static constexpr auto fn = k2_intt_cols<L1, CW, T>; };
template <int L1, int CW, int T>
struct K4c { static constexpr auto fn = k4_ntt_cols<L1, CW, T>; };
template <int L1, int CW, int T>
struct K6c { static constexpr auto fn = k6_intt_cols_p<L1, CW, T>; };
template <int L1, int CW, int T>
struct K8c { static constexpr auto fn = k8_ntt_cols_w<L1, CW, T>; };
template <int L1, int CW, int T>
struct R2c { static constexpr auto fn = r2_intt_cols<L1, CW, T>; };
template <int L1, int CW, int T>
struct R3c { static constexpr auto fn = r3_ntt_cols<L1, CW, T>; };

// Launch a column pass over `rows` rows of every job in its tile shape:
// quarter-width tiles in radix-4 phases (four elements per thread) when four
// times the work-groups still fit one per CU and the quarter is at least 32
// columns (N <= 2^13).  Otherwise a `sparse` pass (one whose launches have
// about one work-group per CU or fewer: the INTT passes K2, K6 and the
// rescale's) takes the narrowest tiles in radix-4 phases under kNarrowBelow
// work-groups; above that, whole-line tiles with eight elements per thread in
// radix-8 phases (radix8) or 16 per thread in radix-16 phases, as the
// schedule's shape bits choose (col_radix8).
template <template <int, int, int> class KF, int L1, class JA>
void col_launch(const Ctx& c, int stage, int rows, int njobs, bool sparse, hipStream_t st,
                const KsConst& K, const JA& jobs, bool radix8) {
  constexpr int TL = ColGeom<L1>::TILES;
  if constexpr (ColGeom<L1>::C / 4 >= 32) {
    if (4 * TL * rows * njobs <= 256) {
      constexpr int CW = ColGeom<L1>::C / 4;
      constexpr int T = CW * (1 << L1) / 4;
      klaunch_b(c, stage, KF<L1, CW, T>::fn, dim3(4 * TL, rows, njobs), T, st, K, jobs);
      return;
    }
  }
  if (sparse && TL * rows * njobs < kNarrowBelow) {
    // radix-4 phases, four elements per thread: four waves per SIMD
    constexpr int CW = kColNarrow<L1>;
    constexpr int T = ColGeom<L1, CW>::ELEMS / 4;
    klaunch_b(c, stage, KF<L1, CW, T>::fn, dim3(ColGeom<L1, CW>::TILES, rows, njobs), T, st, K, jobs);
    return;
  }
  if (radix8) {  // 8 elements per thread: four waves per SIMD
    constexpr int T = ColGeom<L1>::ELEMS / 8;
    klaunch_b(c, stage, KF<L1, 0, T>::fn, dim3(TL, rows, njobs), T, st, K, jobs);
    return;
  }
  klaunch_b(c, stage, KF<L1, 0, kColThreads<L1>>::fn, dim3(TL, rows, njobs), kColThreads<L1>, st, K, jobs);
}
// The whole-line radix of a column pass under schedule shape bits: sparse
// (inverse) passes default to radix-8, the others to radix-16.
inline bool col_radix8(bool sparse, int shape) {
  return sparse ? !(shape & kShapeInvRadix16) : (shape & kShapeFwdRadix8) != 0;
}

// Stage 1 (ModUp): K1-K4.
template <int L1>
hipError_t modup_stage_t(const Ctx& c, const Ctx::Sched& sc, const KsConst& K, const JobArg<KsJob>& jobs,
                         int njobs, int Lmax, hipStream_t st) {
  const int Rmax = Lmax + c.k;
  const int tiles = c.N / kTile;
  const int cols = c.N / (4 * kWG);  // BConv: four coefficients per thread
  const int bmax = c.beta(Lmax);
  const int up_rows = sc.up_rows == 2 || sc.up_rows == 4 || sc.up_rows == 6 ? sc.up_rows : 12;
  const int up_groups = (Rmax + up_rows - 1) / up_rows;
  if (4 * tiles * Lmax * njobs <= 256)  // quarter tiles still one work-group per CU
    klaunch(c, CKKS_STAGE_INTT_BLOCKS, k1_intt_blks<L1, 4>, dim3(4 * tiles, Lmax, njobs), st, K, jobs);
  else if (sc.ntt_shape & kShapeK1Radix16)
    klaunch(c, CKKS_STAGE_INTT_BLOCKS, k1_intt_blks<L1, 16, 16>, dim3(tiles, Lmax, njobs), st, K, jobs);
  else
    klaunch_b(c, CKKS_STAGE_INTT_BLOCKS, k1_intt_blks<L1, 16, 8>, dim3(tiles, Lmax, njobs), 512, st, K, jobs);
  col_launch<K2c, L1>(c, CKKS_STAGE_INTT_COLS, Lmax, njobs, true, st, K, jobs, col_radix8(true, sc.ntt_shape));
  const hipError_t e =
      small_dispatch<K3, 1>(c.alpha, c, dim3(cols, bmax * up_groups, njobs), st, K, jobs, up_groups, up_rows);
  if (e != hipSuccess) return e;
  col_launch<K4c, L1>(c, CKKS_STAGE_NTT_COLS_UP, bmax * Rmax, njobs, false, st, K, jobs,
                      col_radix8(false, sc.ntt_shape));
  return hipSuccess;
}

template <int L1>
hipError_t ks_modup_launch_t(const Ctx& c, const Ctx::Sched& sc, const KsConst& K, const JobArg<KsJob>& jobs,
                             int njobs, int Lmax, hipStream_t st) {
  const hipError_t e = modup_stage_t<L1>(c, sc, K, jobs, njobs, Lmax, st);
  if (e != hipSuccess) return e;
  klaunch(c, -1, km_ntt_blks<L1>, dim3(c.N / kTile, c.beta(Lmax) * (Lmax + c.k), njobs), st, K, jobs);
  return hipGetLastError();
}

template <int L1>
hipError_t ks_launch_t(const Ctx& c, const Ctx::Sched& sc, const KsConst& K, const JobArg<KsJob>& jobs,
                       int njobs, int Lmax, bool with_modup, bool with_hoist, hipStream_t st,
                       const KsSplit& sp) {
  const int Rmax = Lmax + c.k;
  const int tiles = c.N / kTile;
  const int cols = c.N / (4 * kWG);  // BConv: four coefficients per thread
  const int down_rows = sc.down_rows == 2 || sc.down_rows == 4 || sc.down_rows == 6 ? sc.down_rows : 12;
  const int down_groups = (Lmax + down_rows - 1) / down_rows;
  hipError_t e;
  if constexpr (L1 + kBlockLog == kSrLog) {
    // small ring: two kernels on whole limbs (plain, HMult and HRot jobs)
    if ((sc.ntt_shape & kShapeWholeLimb) && with_modup && !with_hoist && !sp.side) {
      // every job splits its own digits into sr_groups(beta) <= min(beta, kSrGroups)
      // groups, so the grid covers min(bmax, kSrGroups) (not the largest job's count)
      const int groups = std::min(c.beta(Lmax), kSrGroups);
      klaunch_b(c, CKKS_STAGE_NTT_IP, s1_modup_ip, dim3(Rmax, groups, njobs), kSrT, st, K, jobs);
      klaunch_b(c, CKKS_STAGE_NTT_COMBINE, s2_moddown, dim3(Lmax, 2, njobs), kSrT, st, K, jobs);
      return hipGetLastError();
    }
  }
  if (with_modup && (e = modup_stage_t<L1>(c, sc, K, jobs, njobs, Lmax, st)) != hipSuccess) return e;
  // Stage 2.  With a side stream, complementary pipelining (Sec. IV-B): the
  // inner product of the P rows runs on st and ModDown's P-row chain (K6..K8,
  // latency-bound) follows it there, while the Q-row inner product (key
  // streaming, HBM-heavy) runs on the side stream; K9 joins both.
  auto k5 = [&](int stage, int part, hipStream_t s5, int rows) {
    const dim3 g5(tiles, rows, njobs);
    const int nb = std::max(c.beta(Lmax), 2);  // slots for the launch's own largest digit count
    if (tiles * rows * njobs <= sc.small_grid && nb <= 4) {  // too few work-groups to fill the CUs
      // eighth tiles (radix-4 phases) while eight times the work-groups still
      // fit one per CU, else quarter tiles while four times do
      if (8 * tiles * rows * njobs <= 256) {
        const dim3 g8(8 * tiles, rows, njobs);
        constexpr int T8 = k5p_threads<2, 4>();
        switch (nb) {
          case 2: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 2, 2, 4>, g8, T8, s5, K, jobs, part); break;
          case 3: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 3, 2, 4>, g8, T8, s5, K, jobs, part); break;
          default: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 4, 2, 4>, g8, T8, s5, K, jobs, part); break;
        }
        return;
      }
      if (4 * tiles * rows * njobs <= 256) {
        const dim3 g4(4 * tiles, rows, njobs);
        constexpr int T4 = k5p_threads<4, 16>();
        switch (nb) {
          case 2: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 2, 4, 16>, g4, T4, s5, K, jobs, part); break;
          case 3: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 3, 4, 16>, g4, T4, s5, K, jobs, part); break;
          default: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 4, 4, 16>, g4, T4, s5, K, jobs, part); break;
        }
        return;
      }
      constexpr int T16 = k5p_threads<16, 16>();
      switch (nb) {
        case 2: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 2, 16, 16>, g5, T16, s5, K, jobs, part); break;
        case 3: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 3, 16, 16>, g5, T16, s5, K, jobs, part); break;
        default: klaunch_b(c, stage, k5p_ntt_blks_ip<L1, 4, 16, 16>, g5, T16, s5, K, jobs, part); break;
      }
      return;
    }
    // a single job streams its key (measured: K5 39.8 -> 35.6 us at N = 2^16,
    // L = 36, alternating keys); jobs of a batch may share one
    const bool nt = njobs == 1;
    switch (nb) {
      case 2:
        if (nt) klaunch(c, stage, k5s_ntt_blks_ip<L1, 2, true>, g5, s5, K, jobs, part);
        else klaunch(c, stage, k5s_ntt_blks_ip<L1, 2, false>, g5, s5, K, jobs, part);
        break;
      case 3:
        if (nt) klaunch(c, stage, k5s_ntt_blks_ip<L1, 3, true>, g5, s5, K, jobs, part);
        else klaunch(c, stage, k5s_ntt_blks_ip<L1, 3, false>, g5, s5, K, jobs, part);
        break;
      case 4:
        if (nt) klaunch(c, stage, k5s_ntt_blks_ip<L1, 4, true>, g5, s5, K, jobs, part);
        else klaunch(c, stage, k5s_ntt_blks_ip<L1, 4, false>, g5, s5, K, jobs, part);
        break;
      default: klaunch(c, stage, k5_ntt_blks_ip<L1, false>, g5, s5, K, jobs, part); break;
    }
  };
  auto k5h = [&](int stage, int part, hipStream_t s5, int rows) {
    const dim3 gh(tiles, rows, njobs);
    switch (std::max(c.beta(Lmax), 2)) {  // slots for the launch's own largest digit count
      case 2: klaunch(c, stage, k5h_gather_ip<L1, 2>, gh, s5, K, jobs, part); break;
      case 3: klaunch(c, stage, k5h_gather_ip<L1, 3>, gh, s5, K, jobs, part); break;
      case 4: klaunch(c, stage, k5h_gather_ip<L1, 4>, gh, s5, K, jobs, part); break;
      default: klaunch(c, stage, k5_ntt_blks_ip<L1, true>, gh, s5, K, jobs, part); break;
    }
  };
  const bool split = sp.side != nullptr;
  auto fork = [&]() -> hipError_t {
    hipError_t fe = hipEventRecord(sp.fork, st);
    return fe != hipSuccess ? fe : hipStreamWaitEvent(sp.side, sp.fork, 0);
  };
  auto part_q = [&]() {
    if (with_modup) k5(CKKS_STAGE_NTT_IP, KS_PART_Q, sp.side, Lmax);
    if (with_hoist) k5h(CKKS_STAGE_NTT_IP, KS_PART_Q, sp.side, Lmax);
  };
  if (split) {
    if (!sp.p_first) {
      if ((e = fork()) != hipSuccess) return e;
      part_q();
    }
    if (with_modup) k5(CKKS_STAGE_NTT_IP_P, KS_PART_P, st, c.k);
    if (with_hoist) k5h(CKKS_STAGE_NTT_IP_P, KS_PART_P, st, c.k);
    if (sp.p_first) {
      if ((e = fork()) != hipSuccess) return e;
      part_q();
    }
  } else {
    if (with_modup) k5(CKKS_STAGE_NTT_IP, KS_PART_ALL, st, Rmax);
    if (with_hoist) k5h(CKKS_STAGE_NTT_IP, KS_PART_ALL, st, Rmax);
  }
  if (split && (e = hipEventRecord(sp.join, sp.side)) != hipSuccess) return e;
  col_launch<K6c, L1>(c, CKKS_STAGE_INTT_COLS_P, 2 * c.k, njobs, true, st, K, jobs, col_radix8(true, sc.ntt_shape));
  e = small_dispatch<K7, 1>(c.k, c, dim3(cols, 2 * down_groups, njobs), st, K, jobs, down_groups,
                            down_rows);
  if (e != hipSuccess) return e;
  col_launch<K8c, L1>(c, CKKS_STAGE_NTT_COLS_DOWN, 2 * Lmax, njobs, false, st, K, jobs,
                      col_radix8(false, sc.ntt_shape));
  if (split && (e = hipStreamWaitEvent(st, sp.join, 0)) != hipSuccess) return e;
  if (4 * tiles * 2 * Lmax * njobs <= 256)
    klaunch(c, CKKS_STAGE_NTT_COMBINE, k9_ntt_blks_combine<L1, 4>, dim3(4 * tiles, 2 * Lmax, njobs), st, K,
            jobs);
  else
    klaunch(c, CKKS_STAGE_NTT_COMBINE, k9_ntt_blks_combine<L1, 16>, dim3(tiles, 2 * Lmax, njobs), st, K, jobs);
  return hipGetLastError();
}

template <int L1>
hipError_t rs_launch_t(const Ctx& c, const KsConst& K, const JobArg<RsJob>& jobs, int njobs,
                       int Lmax, hipStream_t st) {
  const int tiles = c.N / kTile;
  if (4 * tiles * 2 * njobs <= 256)  // quarter tiles while they fit one work-group per CU
    r1_intt_blks<L1, 4><<<dim3(4 * tiles, 2, njobs), kWG, 0, st>>>(K, jobs);
  else
    r1_intt_blks<L1, 16><<<dim3(tiles, 2, njobs), kWG, 0, st>>>(K, jobs);
  col_launch<R2c, L1>(c, -1, 2, njobs, true, st, K, jobs, col_radix8(true, c.sched.ntt_shape));
  col_launch<R3c, L1>(c, -1, 2 * (Lmax - 1), njobs, false, st, K, jobs, col_radix8(false, c.sched.ntt_shape));
  klaunch(c, CKKS_STAGE_RESCALE_NTT, r4_ntt_blks_combine<L1>, dim3(tiles, 2 * (Lmax - 1), njobs), st, K,
          jobs);
  return hipGetLastError();
}
}  // namespace

hipError_t ks_launch(const Ctx& c, const Ctx::Sched& sc, const JobArg<KsJob>& jobs, int njobs, int Lmax,
                     bool with_modup, bool with_hoist, hipStream_t st, const KsSplit& sp) {
  if (njobs <= 0) return hipSuccess;
  const KsConst K = make_const(c);
  switch (c.logN - kBlockLog) {
    case 4: return ks_launch_t<4>(c, sc, K, jobs, njobs, Lmax, with_modup, with_hoist, st, sp);
    case 5: return ks_launch_t<5>(c, sc, K, jobs, njobs, Lmax, with_modup, with_hoist, st, sp);
    case 6: return ks_launch_t<6>(c, sc, K, jobs, njobs, Lmax, with_modup, with_hoist, st, sp);
    case 7: return ks_launch_t<7>(c, sc, K, jobs, njobs, Lmax, with_modup, with_hoist, st, sp);
    case 8: return ks_launch_t<8>(c, sc, K, jobs, njobs, Lmax, with_modup, with_hoist, st, sp);
    default: return hipErrorInvalidValue;
  }
}

hipError_t ks_modup_launch(const Ctx& c, const Ctx::Sched& sc, const JobArg<KsJob>& jobs, int njobs, int Lmax,
                           hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const KsConst K = make_const(c);
  switch (c.logN - kBlockLog) {
    case 4: return ks_modup_launch_t<4>(c, sc, K, jobs, njobs, Lmax, st);
    case 5: return ks_modup_launch_t<5>(c, sc, K, jobs, njobs, Lmax, st);
    case 6: return ks_modup_launch_t<6>(c, sc, K, jobs, njobs, Lmax, st);
    case 7: return ks_modup_launch_t<7>(c, sc, K, jobs, njobs, Lmax, st);
    case 8: return ks_modup_launch_t<8>(c, sc, K, jobs, njobs, Lmax, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rs_launch(const Ctx& c, const JobArg<RsJob>& jobs, int njobs, int Lmax, hipStream_t st) {
  if (njobs <= 0 || Lmax < 2) return hipSuccess;
  const KsConst K = make_const(c);
  switch (c.logN - kBlockLog) {
    case 4: return rs_launch_t<4>(c, K, jobs, njobs, Lmax, st);
    case 5: return rs_launch_t<5>(c, K, jobs, njobs, Lmax, st);
    case 6: return rs_launch_t<6>(c, K, jobs, njobs, Lmax, st);
    case 7: return rs_launch_t<7>(c, K, jobs, njobs, Lmax, st);
    case 8: return rs_launch_t<8>(c, K, jobs, njobs, Lmax, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ckks
