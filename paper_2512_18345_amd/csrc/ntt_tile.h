// Device-side building blocks of the two-pass NTT over LDS tiles (shared by
// kernels.hip and keyswitch.hip).
//
// A limb of N = N1 * 256 words is viewed as N1 rows of 256.  The column pass
// runs the first log2(N1) Cooley-Tukey stages on columns j + 256 r (r < N1);
// a work-group tile holds C adjacent columns (ColGeom).  The block pass runs
// the last 8 stages inside contiguous 256-word blocks; a tile holds 16 blocks
// (fewer for small grids).  Inside a tile the stages run as radix-16 register
// phases (16 elements per thread, four stages per LDS round trip) or, for
// small grids, radix-4 phases (4 elements per thread), with lazy Shoup
// butterflies.  The twiddle of butterfly group (m, i) is psi^brv(m + i)
// (inverse: psi^-brv(m + i)).
#pragma once
#include <hip/hip_runtime.h>

#include "arith.h"
#include "ctx.h"

namespace ckks {

constexpr int kLds = 4352;  // padded block-pass tile: 16 x (256 + 16) words

// Column-pass tile for N1 = 2^LOGN1 rows: C adjacent columns, by default at
// least 32 so that every row segment is a whole 128-byte line (narrower tiles
// fetch each line twice).  CW != 0 asks for CW columns instead (at least
// kTile / N1 for 16 elements per thread): the narrowest, kColNarrow, doubles
// the work-groups of a launch at N = 2^16.  T threads share a tile, EPT
// elements each: a multiple of 16 (radix-16 phases), or 4 (radix-4 phases:
// small grids, quarter-width tiles).
template <int LOGN1, int CW = 0, int T = kWG>
struct ColGeom {
  static_assert(CW == 0 || CW >= 16, "row segments of at least 64 bytes");
  static constexpr int N1 = 1 << LOGN1;
  static constexpr int C = CW ? CW : (kTile >> LOGN1) < 32 ? 32 : (kTile >> LOGN1);
  static constexpr int ELEMS = C * N1;             // 4096 or 8192 (fewer in quarter tiles)
  static constexpr int EPT = ELEMS / T;            // elements per thread
  static_assert(EPT % 16 == 0 || EPT == 8 || EPT == 4,
                "groups of 16 elements per thread, or 8 / 4 in radix-8 / radix-4 phases");
  static constexpr int QUADS = ELEMS / (4 * T);    // 16-byte quads per thread in load/store
  static constexpr int LDS = ELEMS + N1;           // with the 16-word pad per 16 rows
  static constexpr int TILES = 256 / C;            // column tiles per limb
};
template <int LOGN1>
constexpr int kColNarrow = kTile >> LOGN1;

__device__ __forceinline__ int lidx_col(int pos, int c, int C) { return pos * C + c + ((pos >> 4) << 4); }
__device__ __forceinline__ int lidx_blk(int line, int pos) { return line * 272 + pos + (pos >> 4); }

// The block layout leaves one unused word after every 16 data words: 256 pad
// words per tile, at line * 272 + 17 m + 16 (m < 16).  A 256-entry twiddle
// table of (w, w') pairs fits in the pads of two consecutive tiles: pad
// number u (< 512) holds word u % 2 of entry u / 2.  The data path never
// touches the pads, so a kernel whose LDS is full of tiles can still read its
// twiddles from LDS.
__device__ __forceinline__ int lidx_pad(int u) {
  return (u >> 8) * kLds + ((u >> 4) & 15) * 272 + 17 * (u & 15) + 16;
}
struct PadTw {
  const uint32_t* s;  // first of the two tiles
  __device__ __forceinline__ uint2 operator[](int i) const {
    return make_uint2(s[lidx_pad(2 * i)], s[lidx_pad(2 * i + 1)]);
  }
};
// Copy a prime's 256-entry block-pass table into the pads of tiles s, s + kLds
// (the caller's next __syncthreads() publishes it).
__device__ __forceinline__ void stage_tw_pads(uint32_t* s, const uint2* __restrict__ tw,
                                              int tid = threadIdx.x) {
  const uint2 w = tw[tid];
  s[lidx_pad(2 * tid)] = w.x;
  s[lidx_pad(2 * tid + 1)] = w.y;
}

// Bank-conflict-free order of the block-pass table for the radix-16 phases.
// In the second phase (stages on pos bits 3..0) a wave instruction reads, for
// stage bit beta, the entries 2^(7-beta) + r 2^(3-beta) + c of the 16 values
// r = line position / 16 of its lanes (c fixed by the instruction).  In
// natural order those 16 entries sit 2^(4-beta) words apart and fall on 2,
// 4 or 8 banks (up to eight-way conflicts); stored at slot 2^(7-beta) +
// 16 c + r they are 16 consecutive entries.  Entries below 16 (the first
// phase reads each of them from every lane at once) keep their place.
__device__ __forceinline__ int tw_perm_slot(int beta, int x) {
  if (beta >= 4) return (1 << (7 - beta)) | x;
  const int lo = 3 - beta;
  return (1 << (7 - beta)) + ((x & ((1 << lo) - 1)) << 4) + (x >> lo);
}
// The slot of entry i (1 <= i < 256) in that order.
__device__ __forceinline__ int tw_perm_of(int i) {
  const int beta = 7 - (31 - __clz(i));
  return tw_perm_slot(beta, i - (1 << (7 - beta)));
}
// Pad-resident table in the conflict-free order (staged by stage_tw_pads_perm).
struct PadTwP {
  const uint32_t* s;
  __device__ __forceinline__ uint2 at(int beta, int x) const {
    const int u = 2 * tw_perm_slot(beta, x);
    return make_uint2(s[lidx_pad(u)], s[lidx_pad(u + 1)]);
  }
};
// Table in its own LDS array in the conflict-free order (staged by stage_tw_perm).
struct PermTw {
  const uint2* t;
  __device__ __forceinline__ uint2 at(int beta, int x) const { return t[tw_perm_slot(beta, x)]; }
};
__device__ __forceinline__ void stage_tw_pads_perm(uint32_t* s, const uint2* __restrict__ tw,
                                                   int tid = threadIdx.x) {
  const uint2 w = tw[tid];
  const int u = 2 * (tid ? tw_perm_of(tid) : 0);
  s[lidx_pad(u)] = w.x;
  s[lidx_pad(u + 1)] = w.y;
}

// The same, from the entry of this thread already loaded (tw[tid]).
__device__ __forceinline__ void stage_tw_pads_perm_word(uint32_t* s, uint2 w, int tid = threadIdx.x) {
  const int u = 2 * (tid ? tw_perm_of(tid) : 0);
  s[lidx_pad(u)] = w.x;
  s[lidx_pad(u + 1)] = w.y;
}

// Twiddle of the block-pass pair on pos bit beta (x = pos >> (beta + 1)).
__device__ __forceinline__ uint2 blk_tw_at(const uint2* tw, int beta, int x) {
  return tw[(1 << (7 - beta)) | x];
}
__device__ __forceinline__ uint2 blk_tw_at(const PadTw& tw, int beta, int x) {
  return tw[(1 << (7 - beta)) | x];
}
__device__ __forceinline__ uint2 blk_tw_at(const PadTwP& tw, int beta, int x) { return tw.at(beta, x); }
__device__ __forceinline__ uint2 blk_tw_at(const PermTw& tw, int beta, int x) { return tw.at(beta, x); }

// ----- column-pass phases (stages on pos bits [blo, blo + LOGR)) -----------
template <int LOGR, bool INV, int ELEMS, int T = kWG>
__device__ __forceinline__ void col_phase(uint32_t* s, int logN1, int C, int blo,
                                          const uint2* __restrict__ tw, uint32_t q, uint32_t q2) {
  constexpr int R = 1 << LOGR;
  constexpr int GPT = ELEMS / R / T;
#pragma unroll
  for (int gg = 0; gg < GPT; ++gg) {
    const int g = threadIdx.x + gg * T;
    const int c = g & (C - 1);
    const int rest = g / C;
    const int base = ((rest >> blo) << (blo + LOGR)) | (rest & ((1 << blo) - 1));
    uint32_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = s[lidx_col(base | (j << blo), c, C)];
    if (!INV) {
#pragma unroll
      for (int kb = LOGR - 1; kb >= 0; --kb) {
        const int beta = blo + kb;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (j & (1 << kb)) continue;
          const int pos = base | (j << blo);
          const uint2 W = tw[(1 << (logN1 - 1 - beta)) | (pos >> (beta + 1))];
          bfly_ct(v[j], v[j | (1 << kb)], W.x, W.y, q, q2);
        }
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < LOGR; ++kb) {
        const int beta = blo + kb;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (j & (1 << kb)) continue;
          const int pos = base | (j << blo);
          const uint2 W = tw[(1 << (logN1 - 1 - beta)) | (pos >> (beta + 1))];
          bfly_gs(v[j], v[j | (1 << kb)], W.x, W.y, q, q2);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) s[lidx_col(base | (j << blo), c, C)] = v[j];
  }
}

// ----- block-pass phases (16 lines of 256; stages on pos bits [blo, blo + LOGR)) ---
// After the twist the 256-word block transform is the same for every block:
// the pair on pos bit beta uses ctw[(1 << (7 - beta)) | (pos >> (beta + 1))],
// and its stage on bit 7 (first forward / last inverse) multiplies by 1.
// TW: a twiddle table indexable as tw[i] -> uint2 (a pointer, or PadTw below).
// tid: the thread's index among the T threads that transform this tile, each
// holding EPT elements (16 by default: kWG threads on 16 blocks).
template <int LOGR, bool INV, class TW, int EPT = 16, int T = kWG>
__device__ __forceinline__ void blk_phase(uint32_t* s, int blo, const TW& tw, uint32_t q,
                                          uint32_t q2, int tid = threadIdx.x) {
  constexpr int R = 1 << LOGR;
  constexpr int GPT = EPT / R;
  static_assert(GPT >= 1, "a group of R elements per thread at least");
  constexpr int NB = 8 - LOGR;
#pragma unroll
  for (int gg = 0; gg < GPT; ++gg) {
    const int g = tid + gg * T;
    const int rest = g & ((1 << NB) - 1);
    const int line = g >> NB;
    const int base = ((rest >> blo) << (blo + LOGR)) | (rest & ((1 << blo) - 1));
    uint32_t v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = s[lidx_blk(line, base | (j << blo))];
    if (!INV) {
#pragma unroll
      for (int kb = LOGR - 1; kb >= 0; --kb) {
        const int beta = blo + kb;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (j & (1 << kb)) continue;
          if (beta == 7) {
            const uint32_t xx = csub(v[j], q2), yy = csub(v[j | (1 << kb)], q2);
            v[j] = xx + yy;
            v[j | (1 << kb)] = xx + q2 - yy;
          } else {
            const int pos = base | (j << blo);
            const uint2 W = blk_tw_at(tw, beta, pos >> (beta + 1));
            bfly_ct(v[j], v[j | (1 << kb)], W.x, W.y, q, q2);
          }
        }
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < LOGR; ++kb) {
        const int beta = blo + kb;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (j & (1 << kb)) continue;
          if (beta == 7) {
            const uint32_t x = v[j], y = v[j | (1 << kb)];
            v[j] = csub(x + y, q2);
            v[j | (1 << kb)] = csub(x + q2 - y, q2);
          } else {
            const int pos = base | (j << blo);
            const uint2 W = blk_tw_at(tw, beta, pos >> (beta + 1));
            bfly_gs(v[j], v[j | (1 << kb)], W.x, W.y, q, q2);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) s[lidx_blk(line, base | (j << blo))] = v[j];
  }
}

// All column stages of one tile, forward (high bits first) or inverse (low bits first).
template <int LOGN1, bool INV, int CW = 0, int T = kWG>
__device__ __forceinline__ void col_stages(uint32_t* s, const uint2* tw, uint32_t q, uint32_t q2) {
  using G = ColGeom<LOGN1, CW, T>;
  if constexpr (G::EPT == 8) {
    // radix-8 phases (three bits each), then the remaining one or two bits
    constexpr int P8 = LOGN1 / 3, REM = LOGN1 % 3;
    constexpr int NPH = P8 + (REM ? 1 : 0);
#pragma unroll
    for (int p = 0; p < NPH; ++p) {
      if (p) __syncthreads();
      if (!INV) {
        if (p < P8) col_phase<3, false, G::ELEMS, T>(s, LOGN1, G::C, LOGN1 - 3 - 3 * p, tw, q, q2);
        else col_phase<(REM ? REM : 1), false, G::ELEMS, T>(s, LOGN1, G::C, 0, tw, q, q2);
      } else {
        if (REM && p == 0) col_phase<(REM ? REM : 1), true, G::ELEMS, T>(s, LOGN1, G::C, 0, tw, q, q2);
        else col_phase<3, true, G::ELEMS, T>(s, LOGN1, G::C, REM + 3 * (p - (REM ? 1 : 0)), tw, q, q2);
      }
    }
    return;
  }
  if constexpr (G::EPT == 4) {
    // radix-4 phases (two bits each), a radix-2 phase for an odd log2 N1
    constexpr int P4 = LOGN1 / 2, ODD = LOGN1 & 1;
#pragma unroll
    for (int p = 0; p < P4 + ODD; ++p) {
      if (p) __syncthreads();
      if (!INV) {
        if (p < P4) col_phase<2, false, G::ELEMS, T>(s, LOGN1, G::C, LOGN1 - 2 - 2 * p, tw, q, q2);
        else col_phase<1, false, G::ELEMS, T>(s, LOGN1, G::C, 0, tw, q, q2);
      } else {
        if (p < P4) col_phase<2, true, G::ELEMS, T>(s, LOGN1, G::C, 2 * p, tw, q, q2);
        else col_phase<1, true, G::ELEMS, T>(s, LOGN1, G::C, LOGN1 - 1, tw, q, q2);
      }
    }
    return;
  }
  constexpr int REM = LOGN1 - 4;  // 0..4
  if (!INV) {
    col_phase<4, false, G::ELEMS, T>(s, LOGN1, G::C, REM, tw, q, q2);
    if constexpr (REM > 0) {
      __syncthreads();
      col_phase<(REM > 0 ? REM : 1), false, G::ELEMS, T>(s, LOGN1, G::C, 0, tw, q, q2);
    }
  } else {
    col_phase<4, true, G::ELEMS, T>(s, LOGN1, G::C, 0, tw, q, q2);
    if constexpr (REM > 0) {
      __syncthreads();
      col_phase<(REM > 0 ? REM : 1), true, G::ELEMS, T>(s, LOGN1, G::C, 4, tw, q, q2);
    }
  }
}

// The eight block stages as radix-8, radix-8 and radix-4 phases, for 16-block
// tiles of T = 512 threads with eight elements each.
template <bool INV, class TW, int T>
__device__ __forceinline__ void blk_stages_r8(uint32_t* s, const TW& tw, uint32_t q, uint32_t q2) {
  if (!INV) {
    blk_phase<3, false, TW, 8, T>(s, 5, tw, q, q2);
    __syncthreads();
    blk_phase<3, false, TW, 8, T>(s, 2, tw, q, q2);
    __syncthreads();
    blk_phase<2, false, TW, 8, T>(s, 0, tw, q, q2);
  } else {
    blk_phase<2, true, TW, 8, T>(s, 0, tw, q, q2);
    __syncthreads();
    blk_phase<3, true, TW, 8, T>(s, 2, tw, q, q2);
    __syncthreads();
    blk_phase<3, true, TW, 8, T>(s, 5, tw, q, q2);
  }
}

// The eight block stages as four radix-4 phases, for tiles of T threads with
// four elements each (small grids: a quarter as many butterflies per thread
// as the radix-16 form, on four times the work-groups).
template <bool INV, class TW, int T>
__device__ __forceinline__ void blk_stages_r4(uint32_t* s, const TW& tw, uint32_t q, uint32_t q2) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (p) __syncthreads();
    blk_phase<2, INV, TW, 4, T>(s, INV ? 2 * p : 6 - 2 * p, tw, q, q2);
  }
}

template <bool INV, class TW>
__device__ __forceinline__ void blk_stages(uint32_t* s, const TW& tw, uint32_t q, uint32_t q2,
                                           int tid = threadIdx.x) {
  if (!INV) {
    blk_phase<4, false>(s, 4, tw, q, q2, tid);
    __syncthreads();
    blk_phase<4, false>(s, 0, tw, q, q2, tid);
  } else {
    blk_phase<4, true>(s, 0, tw, q, q2, tid);
    __syncthreads();
    blk_phase<4, true>(s, 4, tw, q, q2, tid);
  }
}

// Multiply the quad at block position pos (4 | pos) by rho^pos .. rho^(pos+3),
// tb = the block's 32-entry twist table (rho^j for j < 16, rho^(16 h) at 16 + h).
// Any input below 2^32; output in [0, 2q).
__device__ __forceinline__ uint4 twist4(uint4 v, const uint2* __restrict__ tb, int pos, uint32_t q) {
  const uint2 hi = tb[16 + (pos >> 4)];
  const uint2* lo = tb + (pos & 15);
  const uint2 l0 = lo[0], l1 = lo[1], l2 = lo[2], l3 = lo[3];
  v.x = mul_shoup(mul_shoup(v.x, l0.x, l0.y, q), hi.x, hi.y, q);
  v.y = mul_shoup(mul_shoup(v.y, l1.x, l1.y, q), hi.x, hi.y, q);
  v.z = mul_shoup(mul_shoup(v.z, l2.x, l2.y, q), hi.x, hi.y, q);
  v.w = mul_shoup(mul_shoup(v.w, l3.x, l3.y, q), hi.x, hi.y, q);
  return v;
}

// The factors twist4 reads for the quad at block position pos, loaded ahead
// (they depend on the prime and the block only, so tiles of one row share them).
struct Twist4 {
  uint2 lo[4], hi;
};
__device__ __forceinline__ Twist4 twist4_load(const uint2* __restrict__ tb, int pos) {
  Twist4 t;
#pragma unroll
  for (int i = 0; i < 4; ++i) t.lo[i] = tb[(pos & 15) + i];
  t.hi = tb[16 + (pos >> 4)];
  return t;
}
__device__ __forceinline__ uint4 twist4(uint4 v, const Twist4& t, uint32_t q) {
  v.x = mul_shoup(mul_shoup(v.x, t.lo[0].x, t.lo[0].y, q), t.hi.x, t.hi.y, q);
  v.y = mul_shoup(mul_shoup(v.y, t.lo[1].x, t.lo[1].y, q), t.hi.x, t.hi.y, q);
  v.z = mul_shoup(mul_shoup(v.z, t.lo[2].x, t.lo[2].y, q), t.hi.x, t.hi.y, q);
  v.w = mul_shoup(mul_shoup(v.w, t.lo[3].x, t.lo[3].y, q), t.hi.x, t.hi.y, q);
  return v;
}

// ----- tile load / store helpers --------------------------------------------
// Thread t's k-th quad of a column tile: tile-linear word 4 (t + 256 k) = (pos, c).
template <int LOGN1, int CW = 0, int T = kWG>
__device__ __forceinline__ void col_quad(int k, int& pos, int& c) {
  using G = ColGeom<LOGN1, CW, T>;
  const int lin = (threadIdx.x + k * T) * 4;
  pos = lin / G::C;
  c = lin & (G::C - 1);
}

// Copy one prime's twiddle table of n <= kWG entries into LDS (the caller's
// next __syncthreads() publishes it).  Issued with the tile's own loads, so
// that no transform phase waits on a global load of its twiddles.
__device__ __forceinline__ void stage_tw(uint2* stw, const uint2* __restrict__ tw, int n) {
  if ((int)threadIdx.x < n) stw[threadIdx.x] = tw[threadIdx.x];
}
// The 256-entry block-pass table in the conflict-free order of PermTw.
__device__ __forceinline__ void stage_tw_perm(uint2* stw, const uint2* __restrict__ tw) {
  const int t = threadIdx.x;
  if (t < 256) stw[t ? tw_perm_of(t) : 0] = tw[t];
}

// The same staging in two halves, so that no kernel waits for its twiddles
// before it has requested its tile: tw_fetch issues the global load of the
// thread's entry (threads past n load nothing), tw_put / tw_put_perm store it
// to LDS once the tile's loads are in flight.
__device__ __forceinline__ uint2 tw_fetch(const uint2* __restrict__ tw, int n) {
  uint2 w = make_uint2(0, 0);
  if ((int)threadIdx.x < n) w = tw[threadIdx.x];
  return w;
}
__device__ __forceinline__ void tw_put(uint2* stw, uint2 w, int n) {
  if ((int)threadIdx.x < n) stw[threadIdx.x] = w;
}
__device__ __forceinline__ void tw_put_perm(uint2* stw, uint2 w) {
  const int t = threadIdx.x;
  if (t < 256) stw[t ? tw_perm_of(t) : 0] = w;
}

template <int LOGN1, int CW = 0, int T = kWG>
__device__ __forceinline__ void load_cols(uint32_t* s, const uint32_t* __restrict__ row, int col0) {
  using G = ColGeom<LOGN1, CW, T>;
#pragma unroll
  for (int k = 0; k < G::QUADS; ++k) {
    int pos, c;
    col_quad<LOGN1, CW, T>(k, pos, c);
    const uint4 v = ld4(row + pos * 256 + col0 + c);
    *reinterpret_cast<uint4*>(s + lidx_col(pos, c, G::C)) = v;
  }
}

template <int LOGN1, int CW = 0, int T = kWG>
__device__ __forceinline__ void store_cols(const uint32_t* s, uint32_t* __restrict__ row, int col0) {
  using G = ColGeom<LOGN1, CW, T>;
#pragma unroll
  for (int k = 0; k < G::QUADS; ++k) {
    int pos, c;
    col_quad<LOGN1, CW, T>(k, pos, c);
    st4(row + pos * 256 + col0 + c, *reinterpret_cast<const uint4*>(s + lidx_col(pos, c, G::C)));
  }
}

// Block tiles: element e of the tile (e < 4096) is line e >> 8, pos e & 255.
// blk_elem(k) is the first element of the k-th quad of thread t (T threads,
// tiles of a multiple of four lines) in the load/store/epilogue loops.  Quad
// number t + kT is split as (g, w, l) = (bits 8.., bits 6-7, bits 0-5): the
// 64 lanes of a wave instruction take 16 consecutive quads (256 bytes) from
// each of four lines, line 4g + l / 16, quad 16w + l % 16.  In the padded
// layout the 64 lanes then fall on 64 different banks for each word of the
// quad; 64 consecutive quads of one line would meet up to four to a bank.
template <int T = kWG>
__device__ __forceinline__ int blk_elem(int k) {
  const int qi = threadIdx.x + k * T;
  const int g = qi >> 8, w = (qi >> 6) & 3, l = qi & 63;
  return ((4 * g + (l >> 4)) << 8) | ((16 * w + (l & 15)) << 2);
}
// (The block layout's 1-in-16 padding breaks 16-byte alignment, so these
// LDS accesses stay 32-bit.)
__device__ __forceinline__ uint4 lds_blk4(const uint32_t* s, int e) {
  const uint32_t* p = s + lidx_blk(e >> 8, e & 255);  // 4 | e: no pad inside the quad
  return make_uint4(p[0], p[1], p[2], p[3]);
}
__device__ __forceinline__ void lds_blk4_store(uint32_t* s, int e, uint4 v) {
  uint32_t* p = s + lidx_blk(e >> 8, e & 255);
  p[0] = v.x; p[1] = v.y; p[2] = v.z; p[3] = v.w;
}

// [0, 2m) -> [0, m) on each word
__device__ __forceinline__ uint4 csub4(uint4 v, uint32_t m) {
  v.x = csub(v.x, m);
  v.y = csub(v.y, m);
  v.z = csub(v.z, m);
  v.w = csub(v.w, m);
  return v;
}

__device__ __forceinline__ uint4 canon4(uint4 v, uint32_t q, uint32_t q2) {
  v.x = csub(csub(v.x, q2), q);
  v.y = csub(csub(v.y, q2), q);
  v.z = csub(csub(v.z, q2), q);
  v.w = csub(csub(v.w, q2), q);
  return v;
}

}  // namespace ckks
