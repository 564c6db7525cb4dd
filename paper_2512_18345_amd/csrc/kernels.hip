// gfx950 kernels for the stand-alone entry points: NTT / INTT (two passes,
// see ntt_tile.h), base conversion, inner product, tensor, automorphism and
// the element-wise combines.  The fused key-switching pipeline lives in
// keyswitch.hip.
#include <hip/hip_runtime.h>

#include "arith.h"
#include "ctx.h"
#include "kernels.h"
#include "ntt_tile.h"

namespace ckks {

// ============================================================================
// NTT kernels
// ============================================================================

// Forward column pass: rows r in [0, gridDim.y) except [skip_lo, skip_hi).
// Output lazy in [0, 4q).
template <int LOGN1>
__global__ __launch_bounds__(kWG) void k_ntt_cols(DevTab T, RowMap rm, const uint32_t* src,
                                                  uint32_t* dst, int skip_lo, int skip_hi) {
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1>::LDS];
  const int r = blockIdx.y;
  if (r >= skip_lo && r < skip_hi) return;
  const int pi = rm.pidx(r);
  __shared__ uint2 stw[ColGeom<LOGN1>::N1];
  const uint2 tww = tw_fetch(T.col_tw(pi), ColGeom<LOGN1>::N1);
  const size_t N = (size_t)1 << T.logN;
  const uint32_t q = ldc(T.mod + pi).q, q2 = 2 * q;
  const int col0 = blockIdx.x * ColGeom<LOGN1>::C;
  load_cols<LOGN1>(s, src + r * N, col0);
  tw_put(stw, tww, ColGeom<LOGN1>::N1);
  __syncthreads();
  col_stages<LOGN1, false>(s, stw, q, q2);
  __syncthreads();
  store_cols<LOGN1>(s, dst + r * N, col0);
}

// Forward block pass; canonical output.
template <int LOGN1>
__global__ __launch_bounds__(kWG) void k_ntt_blks(DevTab T, RowMap rm, const uint32_t* src,
                                                  uint32_t* dst, int skip_lo, int skip_hi) {
  __shared__ __align__(16) uint32_t s[kLds];
  const int r = blockIdx.y;
  if (r >= skip_lo && r < skip_hi) return;
  const int pi = rm.pidx(r);
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(T.blk_tw(pi), 256);
  const size_t N = (size_t)1 << T.logN;
  const uint32_t q = ldc(T.mod + pi).q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t* in = src + r * N + blk0 * 256;
  uint32_t* out = dst + r * N + blk0 * 256;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = blk_elem(k);
    lds_blk4_store(s, e, twist4(ld4(in + e),
                                T.blk_twist(pi, blk0 + (e >> 8)), e & 255, q));
  }
  tw_put_perm(stw, tww);
  __syncthreads();
  blk_stages<false>(s, PermTw{stw}, q, q2);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = blk_elem(k);
    st4(out + e, canon4(lds_blk4(s, e), q, q2));
  }
}

// Inverse block pass (first Gentleman-Sande stages); output in [0, 2q).
template <int LOGN1>
__global__ __launch_bounds__(kWG) void k_intt_blks(DevTab T, RowMap rm, const uint32_t* src,
                                                   uint32_t* dst, int skip_lo, int skip_hi) {
  __shared__ __align__(16) uint32_t s[kLds];
  const int r = blockIdx.y;
  if (r >= skip_lo && r < skip_hi) return;
  const int pi = rm.pidx(r);
  __shared__ uint2 stw[256];
  const uint2 tww = tw_fetch(T.blk_itw(pi), 256);
  const size_t N = (size_t)1 << T.logN;
  const uint32_t q = ldc(T.mod + pi).q, q2 = 2 * q;
  const int blk0 = blockIdx.x * 16;
  const uint32_t* in = src + r * N + blk0 * 256;
  uint32_t* out = dst + r * N + blk0 * 256;
  uint4 x[4];
  Twist4 tfi[4];  // the epilogue's twist factors, requested with the tile
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = ld4(in + blk_elem(k));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = blk_elem(k);
    tfi[k] = twist4_load(T.blk_itwist(pi, blk0 + (e >> 8)), e & 255);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) lds_blk4_store(s, blk_elem(k), x[k]);
  tw_put_perm(stw, tww);
  __syncthreads();
  blk_stages<true>(s, PermTw{stw}, q, q2);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) st4(out + blk_elem(k), twist4(lds_blk4(s, blk_elem(k)), tfi[k], q));
}

// Inverse column pass + per-row scale (N^-1 times an optional base-conversion
// pre-multiplier) -> canonical output.  scale[pidx - scale_off] = (c, Shoup(c));
// scale == nullptr means N^-1 alone.
template <int LOGN1>
__global__ __launch_bounds__(kWG) void k_intt_cols(DevTab T, RowMap rm, const uint32_t* src,
                                                   uint32_t* dst, int skip_lo, int skip_hi,
                                                   const uint2* scale, int scale_off) {
  __shared__ __align__(16) uint32_t s[ColGeom<LOGN1>::LDS];
  constexpr int C = ColGeom<LOGN1>::C;
  const int r = blockIdx.y;
  if (r >= skip_lo && r < skip_hi) return;
  const int pi = rm.pidx(r);
  __shared__ uint2 stw[ColGeom<LOGN1>::N1];
  const uint2 tww = tw_fetch(T.col_itw(pi), ColGeom<LOGN1>::N1);
  const size_t N = (size_t)1 << T.logN;
  const ModC mc = T.mod[pi];
  const uint32_t q = mc.q, q2 = 2 * q;
  const uint2 sc = scale ? scale[pi - scale_off] : make_uint2(mc.ninv, mc.ninv_s);
  const int col0 = blockIdx.x * C;
  load_cols<LOGN1>(s, src + r * N, col0);
  tw_put(stw, tww, ColGeom<LOGN1>::N1);
  __syncthreads();
  col_stages<LOGN1, true>(s, stw, q, q2);
  __syncthreads();
  uint32_t* row = dst + r * N;
#pragma unroll
  for (int k = 0; k < ColGeom<LOGN1>::QUADS; ++k) {
    const int lin = (threadIdx.x + k * kWG) * 4;
    const int pos = lin / C, c = lin & (C - 1);
    uint4 v = *reinterpret_cast<const uint4*>(s + lidx_col(pos, c, C));
    v.x = csub(mul_shoup(v.x, sc.x, sc.y, q), q);
    v.y = csub(mul_shoup(v.y, sc.x, sc.y, q), q);
    v.z = csub(mul_shoup(v.z, sc.x, sc.y, q), q);
    v.w = csub(mul_shoup(v.w, sc.x, sc.y, q), q);
    st4(row + pos * 256 + col0 + c, v);
  }
}

// ============================================================================
// Base conversion (Sec. II-B2, III-C2): z_r = sum_i y_i * T[r][i] mod prime(r),
// y canonical coefficient-domain rows (pre-multiplied already), one 64-bit
// accumulation and a single reduction per output (overflow-free by the
// bound checked at context creation).
// ============================================================================
template <int NIN>
__global__ __launch_bounds__(kWG) void k_bconv(DevTab T, RowMap rm, const uint32_t* y, int nin,
                                               uint32_t* out, int nrows, int skip_lo, int skip_hi,
                                               const uint32_t* Tt, int tstride, int rows_per_block) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = (size_t)blockIdx.x * kWG + threadIdx.x;
  uint32_t x[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) x[i] = i < nin ? y[i * N + n] : 0u;
  const int r0 = blockIdx.y * rows_per_block;
  const int r1 = min(r0 + rows_per_block, nrows);
  for (int r = r0; r < r1; ++r) {
    if (r >= skip_lo && r < skip_hi) continue;
    const ModC mc = T.mod[rm.pidx(r)];
    const uint32_t* t = Tt + (size_t)r * tstride;
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < NIN; ++i)
      if (i < nin) acc += (uint64_t)x[i] * t[i];
    out[r * N + n] = reduce64(acc, mc.q, mc.mu_hi, mc.mu_lo);
  }
}

// ============================================================================
// Element-wise kernels (Sec. II-B3)
// ============================================================================

// acc[c][r] = sum_j M[j][r] * evk[j][c][krow(r)] (Sec. IV-B stage 2).
__global__ __launch_bounds__(kWG) void k_inner_product(DevTab T, RowMap rm, const uint32_t* M,
                                                       int beta, int nrows, const uint32_t* evk,
                                                       uint32_t* acc) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = (size_t)blockIdx.x * kWG + threadIdx.x;
  const int r = blockIdx.y;
  const int pi = rm.pidx(r);
  const ModC mc = T.mod[pi];
  const size_t krows = (size_t)(T.L_max + (nrows - rm.L));
  uint64_t a0 = 0, a1 = 0;
  for (int j = 0; j < beta; ++j) {
    const uint32_t m = M[((size_t)j * nrows + r) * N + n];
    const uint32_t* e = evk + (size_t)j * 2 * krows * N + (size_t)pi * N + n;
    a0 += (uint64_t)m * e[0];
    a1 += (uint64_t)m * e[krows * N];
    if ((j & 7) == 7) {  // products below 2^60: fold before 16 of them add up
      a0 = reduce64(a0, mc.q, mc.mu_hi, mc.mu_lo);
      a1 = reduce64(a1, mc.q, mc.mu_hi, mc.mu_lo);
    }
  }
  acc[(size_t)r * N + n] = reduce64(a0, mc.q, mc.mu_hi, mc.mu_lo);
  acc[((size_t)nrows + r) * N + n] = reduce64(a1, mc.q, mc.mu_hi, mc.mu_lo);
}

// d0 = c0 c0', d1 = c0 c1' + c1 c0', d2 = c1 c1' over [L][N].
__global__ __launch_bounds__(kWG) void k_tensor(DevTab T, const uint32_t* ct1, const uint32_t* ct2,
                                                int L, uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = (size_t)blockIdx.x * kWG + threadIdx.x;
  const int r = blockIdx.y;
  const ModC mc = T.mod[r];
  const size_t e = (size_t)r * N + n, P = (size_t)L * N;
  const uint32_t a0 = ct1[e], a1 = ct1[P + e], b0 = ct2[e], b1 = ct2[P + e];
  out[e] = reduce64((uint64_t)a0 * b0, mc.q, mc.mu_hi, mc.mu_lo);
  out[P + e] = reduce64((uint64_t)a0 * b1 + (uint64_t)a1 * b0, mc.q, mc.mu_hi, mc.mu_lo);
  out[2 * P + e] = reduce64((uint64_t)a1 * b1, mc.q, mc.mu_hi, mc.mu_lo);
}

// Eval-domain automorphism: out[r][j] = in[r][j'], 2 brv(j') + 1 = g (2 brv(j) + 1) mod 2N.
__global__ __launch_bounds__(kWG) void k_automorph(int logN, const uint32_t* in, uint32_t* out,
                                                   int rows, uint32_t g, int rows_per_block) {
  const size_t N = (size_t)1 << logN;
  const uint32_t j = blockIdx.x * kWG + threadIdx.x;
  const uint32_t mask2n = (uint32_t)(2 * N - 1);
  const uint32_t bj = __builtin_bitreverse32(j) >> (32 - logN);
  const uint32_t e = (g * (2 * bj + 1)) & mask2n;
  const uint32_t src = __builtin_bitreverse32((e - 1) >> 1) >> (32 - logN);
  const int r0 = blockIdx.y * rows_per_block;
  const int r1 = min(r0 + rows_per_block, rows);
  for (int r = r0; r < r1; ++r) out[(size_t)r * N + j] = in[(size_t)r * N + src];
}

// out_i = (acc_i - z_i) * P^-1 (+ add_i) mod q_i: the ModDown combine (floor form).
__global__ __launch_bounds__(kWG) void k_moddown_combine(DevTab T, const uint32_t* acc,
                                                         const uint32_t* z, const uint2* pinv,
                                                         const uint32_t* add, uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = (size_t)blockIdx.x * kWG + threadIdx.x;
  const int i = blockIdx.y;
  const uint32_t q = T.mod[i].q;
  const size_t e = (size_t)i * N + n;
  const uint2 pv = pinv[i];
  uint32_t v = csub(mul_shoup(acc[e] + q - z[e], pv.x, pv.y, q), q);
  if (add) v = csub(v + add[e], q);
  out[e] = v;
}

// out = a + b mod q_r over [rows][N] (rows are Q rows 0..rows-1).
__global__ __launch_bounds__(kWG) void k_add(DevTab T, const uint32_t* a, const uint32_t* b,
                                             uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const size_t e = (size_t)blockIdx.y * N + (size_t)blockIdx.x * kWG + threadIdx.x;
  out[e] = csub(a[e] + b[e], T.mod[blockIdx.y].q);
}

// Rescale helpers: bc[i][n] = t[n] mod q_i (i < rows), t canonical mod q_top.
__global__ __launch_bounds__(kWG) void k_broadcast_mod(DevTab T, const uint32_t* t, uint32_t* bc) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = (size_t)blockIdx.x * kWG + threadIdx.x;
  const ModC mc = T.mod[blockIdx.y];
  bc[(size_t)blockIdx.y * N + n] = reduce32(t[n], mc.q, mc.mu32);
}

// out_i = (a_i - v_i) * qinv_i mod q_i.
__global__ __launch_bounds__(kWG) void k_sub_scale(DevTab T, const uint32_t* a, const uint32_t* v,
                                                   const uint2* qinv, uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const int i = blockIdx.y;
  const size_t e = (size_t)i * N + (size_t)blockIdx.x * kWG + threadIdx.x;
  const uint32_t q = T.mod[i].q;
  const uint2 c = qinv[i];
  out[e] = csub(mul_shoup(a[e] + q - v[e], c.x, c.y, q), q);
}

// Plaintext products summed (the baby-step inner products of a BSGS linear
// transform): out[c][i] = sum_b ct_b[c][i] * pt_b[i] mod q_i, b < nb <= 16.
// Sixteen products of canonical residues stay below 2^64: one reduction.
struct PtrList16 {
  const uint32_t* p[16];
};
__global__ __launch_bounds__(kWG) void k_pmult_sum(DevTab T, PtrList16 cts, PtrList16 pts, int nb, int L,
                                                   uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = ((size_t)blockIdx.x * kWG + threadIdx.x) * 4;  // four coefficients per thread
  const int i = blockIdx.y;
  const ModC m = ldc(T.mod + i);
  uint64_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
  for (int b = 0; b < nb; ++b) {
    const uint4 pt = ld4(pts.p[b] + (size_t)i * N + n);
    const uint4 x = ld4(cts.p[b] + (size_t)i * N + n);
    const uint4 y = ld4(cts.p[b] + ((size_t)L + i) * N + n);
    a0[0] += (uint64_t)x.x * pt.x;
    a0[1] += (uint64_t)x.y * pt.y;
    a0[2] += (uint64_t)x.z * pt.z;
    a0[3] += (uint64_t)x.w * pt.w;
    a1[0] += (uint64_t)y.x * pt.x;
    a1[1] += (uint64_t)y.y * pt.y;
    a1[2] += (uint64_t)y.z * pt.z;
    a1[3] += (uint64_t)y.w * pt.w;
  }
  st4(out + (size_t)i * N + n, make_uint4(reduce64(a0[0], m.q, m.mu_hi, m.mu_lo), reduce64(a0[1], m.q, m.mu_hi, m.mu_lo),
                                          reduce64(a0[2], m.q, m.mu_hi, m.mu_lo), reduce64(a0[3], m.q, m.mu_hi, m.mu_lo)));
  st4(out + ((size_t)L + i) * N + n,
      make_uint4(reduce64(a1[0], m.q, m.mu_hi, m.mu_lo), reduce64(a1[1], m.q, m.mu_hi, m.mu_lo),
                 reduce64(a1[2], m.q, m.mu_hi, m.mu_lo), reduce64(a1[3], m.q, m.mu_hi, m.mu_lo)));
}

// Several inner sums over the same ciphertexts (the giant steps of one BSGS
// level): out_g[c][i] = sum_b ct_b[c][i] * pt_{g,b}[i] mod q_i for g < NG.
// Each ciphertext word is read once for all NG sums.
struct PtrList128 {
  const uint32_t* p[128];
};
struct OutList8 {
  uint32_t* p[8];
};
template <int NG>
__global__ __launch_bounds__(kWG) void k_pmult_sums(DevTab T, PtrList16 cts, PtrList128 pts, OutList8 outs,
                                                    int nb, int L) {
  const size_t N = (size_t)1 << T.logN;
  const size_t n = ((size_t)blockIdx.x * kWG + threadIdx.x) * 4;  // four coefficients per thread
  const int i = blockIdx.y;
  const ModC m = ldc(T.mod + i);
  uint64_t a0[NG][4], a1[NG][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int e = 0; e < 4; ++e) a0[g][e] = a1[g][e] = 0;
  for (int b = 0; b < nb; ++b) {
    const uint4 x = ld4(cts.p[b] + (size_t)i * N + n);
    const uint4 y = ld4(cts.p[b] + ((size_t)L + i) * N + n);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const uint4 pt = ld4(pts.p[g * 16 + b] + (size_t)i * N + n);
      a0[g][0] += (uint64_t)x.x * pt.x;
      a0[g][1] += (uint64_t)x.y * pt.y;
      a0[g][2] += (uint64_t)x.z * pt.z;
      a0[g][3] += (uint64_t)x.w * pt.w;
      a1[g][0] += (uint64_t)y.x * pt.x;
      a1[g][1] += (uint64_t)y.y * pt.y;
      a1[g][2] += (uint64_t)y.z * pt.z;
      a1[g][3] += (uint64_t)y.w * pt.w;
    }
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    st4(outs.p[g] + (size_t)i * N + n,
        make_uint4(reduce64(a0[g][0], m.q, m.mu_hi, m.mu_lo), reduce64(a0[g][1], m.q, m.mu_hi, m.mu_lo),
                   reduce64(a0[g][2], m.q, m.mu_hi, m.mu_lo), reduce64(a0[g][3], m.q, m.mu_hi, m.mu_lo)));
    st4(outs.p[g] + ((size_t)L + i) * N + n,
        make_uint4(reduce64(a1[g][0], m.q, m.mu_hi, m.mu_lo), reduce64(a1[g][1], m.q, m.mu_hi, m.mu_lo),
                   reduce64(a1[g][2], m.q, m.mu_hi, m.mu_lo), reduce64(a1[g][3], m.q, m.mu_hi, m.mu_lo)));
  }
}

// Ciphertext sum: out = a + b over [2][L][N].
__global__ __launch_bounds__(kWG) void k_ct_add(DevTab T, const uint32_t* a, const uint32_t* b, int L,
                                                uint32_t* out) {
  const size_t N = (size_t)1 << T.logN;
  const int r = blockIdx.y;  // 0 .. 2L-1
  const uint32_t q = ldc(T.mod + (r % L)).q;
  const size_t e = (size_t)r * N + ((size_t)blockIdx.x * kWG + threadIdx.x) * 4;
  const uint4 x = ld4(a + e), y = ld4(b + e);
  st4(out + e, make_uint4(csub(x.x + y.x, q), csub(x.y + y.y, q), csub(x.z + y.z, q), csub(x.w + y.w, q)));
}

// ============================================================================
// Launchers
// ============================================================================
#define CKKS_DISPATCH_LOGN1(logN1, CALL) \
  switch (logN1) {                       \
    case 4: CALL(4); break;              \
    case 5: CALL(5); break;              \
    case 6: CALL(6); break;              \
    case 7: CALL(7); break;              \
    case 8: CALL(8); break;              \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_ntt(const Ctx& c, const uint32_t* src, uint32_t* dst, int rows, RowMap rm,
                      int skip_lo, int skip_hi, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int logN1 = c.logN - kBlockLog;
  const dim3 grid(c.N / kTile, rows);
#define CALL(L1)                                                                              \
  k_ntt_cols<L1><<<dim3(ColGeom<L1>::TILES, rows), kWG, 0, st>>>(c.tab(), rm, src, dst, skip_lo, skip_hi); \
  k_ntt_blks<L1><<<grid, kWG, 0, st>>>(c.tab(), rm, dst, dst, skip_lo, skip_hi);
  CKKS_DISPATCH_LOGN1(logN1, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_intt(const Ctx& c, const uint32_t* src, uint32_t* dst, int rows, RowMap rm,
                       int skip_lo, int skip_hi, const uint2* scale, int scale_off,
                       hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int logN1 = c.logN - kBlockLog;
  const dim3 grid(c.N / kTile, rows);
#define CALL(L1)                                                                              \
  k_intt_blks<L1><<<grid, kWG, 0, st>>>(c.tab(), rm, src, dst, skip_lo, skip_hi);            \
  k_intt_cols<L1><<<dim3(ColGeom<L1>::TILES, rows), kWG, 0, st>>>(c.tab(), rm, dst, dst, skip_lo, skip_hi, scale, scale_off);
  CKKS_DISPATCH_LOGN1(logN1, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_bconv(const Ctx& c, RowMap rm, const uint32_t* y, int nin, uint32_t* out,
                        int nrows, int skip_lo, int skip_hi, const uint32_t* Tt, int tstride,
                        hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  const int rpb = 4;
  const dim3 grid(c.N / kWG, (nrows + rpb - 1) / rpb);
  if (nin <= 4)
    k_bconv<4><<<grid, kWG, 0, st>>>(c.tab(), rm, y, nin, out, nrows, skip_lo, skip_hi, Tt, tstride, rpb);
  else if (nin <= 8)
    k_bconv<8><<<grid, kWG, 0, st>>>(c.tab(), rm, y, nin, out, nrows, skip_lo, skip_hi, Tt, tstride, rpb);
  else if (nin <= 12)
    k_bconv<12><<<grid, kWG, 0, st>>>(c.tab(), rm, y, nin, out, nrows, skip_lo, skip_hi, Tt, tstride, rpb);
  else if (nin <= 16)
    k_bconv<16><<<grid, kWG, 0, st>>>(c.tab(), rm, y, nin, out, nrows, skip_lo, skip_hi, Tt, tstride, rpb);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_inner_product(const Ctx& c, RowMap rm, const uint32_t* M, int beta, int nrows,
                                const uint32_t* evk, uint32_t* acc, hipStream_t st) {
  k_inner_product<<<dim3(c.N / kWG, nrows), kWG, 0, st>>>(c.tab(), rm, M, beta, nrows, evk, acc);
  return hipGetLastError();
}

hipError_t launch_tensor(const Ctx& c, const uint32_t* ct1, const uint32_t* ct2, int L,
                         uint32_t* out, hipStream_t st) {
  k_tensor<<<dim3(c.N / kWG, L), kWG, 0, st>>>(c.tab(), ct1, ct2, L, out);
  return hipGetLastError();
}

hipError_t launch_automorph(const Ctx& c, const uint32_t* in, uint32_t* out, int rows, uint32_t g,
                            hipStream_t st) {
  const int rpb = 4;
  k_automorph<<<dim3(c.N / kWG, (rows + rpb - 1) / rpb), kWG, 0, st>>>(c.logN, in, out, rows, g, rpb);
  return hipGetLastError();
}

hipError_t launch_moddown_combine(const Ctx& c, int L, const uint32_t* acc, const uint32_t* z,
                                  const uint32_t* add, uint32_t* out, hipStream_t st) {
  k_moddown_combine<<<dim3(c.N / kWG, L), kWG, 0, st>>>(c.tab(), acc, z, c.d_pinv, add, out);
  return hipGetLastError();
}

hipError_t launch_add(const Ctx& c, int rows, const uint32_t* a, const uint32_t* b, uint32_t* out,
                      hipStream_t st) {
  k_add<<<dim3(c.N / kWG, rows), kWG, 0, st>>>(c.tab(), a, b, out);
  return hipGetLastError();
}

hipError_t launch_broadcast_mod(const Ctx& c, int rows, const uint32_t* t, uint32_t* bc,
                                hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  k_broadcast_mod<<<dim3(c.N / kWG, rows), kWG, 0, st>>>(c.tab(), t, bc);
  return hipGetLastError();
}

hipError_t launch_sub_scale(const Ctx& c, int rows, const uint32_t* a, const uint32_t* v,
                            const uint2* qinv, uint32_t* out, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  k_sub_scale<<<dim3(c.N / kWG, rows), kWG, 0, st>>>(c.tab(), a, v, qinv, out);
  return hipGetLastError();
}

hipError_t launch_pmult_sum(const Ctx& c, const uint32_t* const* cts, const uint32_t* const* pts, int nb,
                            int L, uint32_t* out, hipStream_t st) {
  if (nb < 1 || nb > 16) return hipErrorInvalidValue;
  PtrList16 a{}, b{};
  for (int i = 0; i < nb; ++i) {
    a.p[i] = cts[i];
    b.p[i] = pts[i];
  }
  k_pmult_sum<<<dim3(c.N / (4 * kWG), L), kWG, 0, st>>>(c.tab(), a, b, nb, L, out);
  return hipGetLastError();
}

hipError_t launch_pmult_sums(const Ctx& c, const uint32_t* const* cts, int nb, const uint32_t* const* pts,
                             int ng, int L, uint32_t* const* outs, hipStream_t st) {
  if (nb < 1 || nb > 16 || ng < 1 || ng > 8) return hipErrorInvalidValue;
  PtrList16 a{};
  PtrList128 b{};
  OutList8 o{};
  for (int j = 0; j < nb; ++j) a.p[j] = cts[j];
  for (int g = 0; g < ng; ++g) {
    o.p[g] = outs[g];
    for (int j = 0; j < nb; ++j) b.p[g * 16 + j] = pts[g * nb + j];
  }
  const dim3 grid(c.N / (4 * kWG), L);
  switch (ng) {
    case 1: k_pmult_sums<1><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 2: k_pmult_sums<2><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 3: k_pmult_sums<3><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 4: k_pmult_sums<4><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 5: k_pmult_sums<5><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 6: k_pmult_sums<6><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    case 7: k_pmult_sums<7><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
    default: k_pmult_sums<8><<<grid, kWG, 0, st>>>(c.tab(), a, b, o, nb, L); break;
  }
  return hipGetLastError();
}

hipError_t launch_ct_add(const Ctx& c, const uint32_t* a, const uint32_t* b, int L, uint32_t* out,
                         hipStream_t st) {
  k_ct_add<<<dim3(c.N / (4 * kWG), 2 * L), kWG, 0, st>>>(c.tab(), a, b, L, out);
  return hipGetLastError();
}

}  // namespace ckks
