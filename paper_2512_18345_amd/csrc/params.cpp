// Host-side construction of a context's tables: twiddles (Sec. II-B1), the
// base-conversion tables T[i][j] = (Q^* / Q_j) mod P_i with their pre-multiply
// constants (Sec. II-B2, III-C2) for every level and digit, the ModDown and
// rescale constants.  All host arithmetic is exact (unsigned __int128 where a
// product can exceed 64 bits).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace ckks {
namespace {

using u64 = uint64_t;
using u128 = unsigned __int128;

u64 mulm(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
u64 powm(u64 b, u64 e, u64 m) {
  u64 r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulm(r, b, m);
    b = mulm(b, b, m);
    e >>= 1;
  }
  return r;
}
u64 invm(u64 a, u64 p) { return powm(a % p, p - 2, p); }  // p prime

bool is_prime(u64 n) {
  if (n < 2) return false;
  for (u64 sp : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
    if (n % sp == 0) return n == sp;
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) d >>= 1, ++s;
  for (u64 a : {2ull, 7ull, 61ull}) {  // deterministic below 4,759,123,141
    u64 x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; ++i) {
      x = mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

uint32_t brv(uint32_t x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }

uint2 shoup(u64 w, u64 q) { return make_uint2((uint32_t)w, (uint32_t)((w << 32) / q)); }

// Smallest primitive 2N-th root of unity mod q: take any element of order
// exactly 2N, then the minimum over its odd powers (all primitive 2N-th roots).
u64 min_root(u64 q, u64 N) {
  u64 c = 0;
  for (u64 x = 2;; ++x) {
    c = powm(x, (q - 1) / (2 * N), q);
    if (powm(c, N, q) == q - 1) break;
  }
  const u64 c2 = mulm(c, c, q);
  u64 best = c, w = c;
  for (u64 m = 1; m < N; ++m) {
    w = mulm(w, c2, q);
    best = std::min(best, w);
  }
  return best;
}

template <class T>
std::string upload(T** dst, const std::vector<T>& src, int* code) {
  if (src.empty()) return "";
  if (hipMalloc(dst, sizeof(T) * src.size()) != hipSuccess) {
    *code = CKKS_ENOMEM;
    return "hipMalloc failed for a context table";
  }
  if (hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess) {
    *code = CKKS_EHIP;
    return "hipMemcpy failed for a context table";
  }
  return "";
}

}  // namespace

std::string build_tables(Ctx& c, const uint32_t* q, const uint32_t* p, int* code) {
  *code = CKKS_EINVAL;
  const int nP = c.L_max + c.k;
  const u64 N = (u64)c.N;
  c.primes.assign(q, q + c.L_max);
  c.primes.insert(c.primes.end(), p, p + c.k);
  for (int i = 0; i < nP; ++i) {
    const u64 v = c.primes[i];
    if (v >= (1u << 30) || !is_prime(v) || v % (2 * N) != 1)
      return "prime " + std::to_string(i) + " (" + std::to_string(v) +
             ") is not a prime < 2^30 congruent to 1 mod 2N";
    for (int j = 0; j < i; ++j)
      if (c.primes[j] == v) return "primes are not distinct";
  }

  // per-prime constants and twiddle tables
  const u64 N1 = N >> 8;
  const int logN1 = c.logN - 8;
  std::vector<ModC> mod(nP);
  std::vector<uint2> tw((size_t)nP * N1), itw((size_t)nP * N1);
  std::vector<uint2> ctw((size_t)nP * 256), ictw((size_t)nP * 256);
  std::vector<uint2> twist((size_t)nP * N1 * 32), itwist((size_t)nP * N1 * 32);
  // whole-limb tables of small rings: all N entries of the bit-reversed table
  const bool small_ring = c.logN == kSrLog;
  std::vector<uint2> ftw(small_ring ? (size_t)nP * N : 0), fitw(small_ring ? (size_t)nP * N : 0);
  for (int i = 0; i < nP; ++i) {
    const u64 qi = c.primes[i];
    const u64 psi = min_root(qi, N), psii = invm(psi, qi);
    const u64 mu64 = ~0ull / qi;
    const u64 ninv = invm(N % qi, qi);
    const uint2 ns = shoup(ninv, qi);
    mod[i] = ModC{(uint32_t)qi, (uint32_t)((1ull << 32) / qi), (uint32_t)(mu64 >> 32),
                  (uint32_t)mu64, ns.x, ns.y};
    // column pass: the first N1 entries of the bit-reversed table
    for (u64 e = 0; e < N1; ++e) {
      const uint32_t b = brv((uint32_t)e, c.logN);
      tw[(size_t)i * N1 + e] = shoup(powm(psi, b, qi), qi);
      itw[(size_t)i * N1 + e] = shoup(powm(psii, b, qi), qi);
    }
    if (small_ring)
      for (u64 e = 0; e < N; ++e) {
        const uint32_t b = brv((uint32_t)e, c.logN);
        ftw[(size_t)i * N + e] = shoup(powm(psi, b, qi), qi);
        fitw[(size_t)i * N + e] = shoup(powm(psii, b, qi), qi);
      }
    // block pass (twisted): index 2^s + g -> psi^((N / 2^s) brv_s(g))
    ctw[(size_t)i * 256] = ictw[(size_t)i * 256] = shoup(1, qi);
    for (int s = 0; s < 8; ++s)
      for (u64 g = 0; g < (1ull << s); ++g) {
        const u64 ex = (N >> s) * (s ? brv((uint32_t)g, s) : 0);
        ctw[(size_t)i * 256 + (1u << s) + g] = shoup(powm(psi, ex, qi), qi);
        ictw[(size_t)i * 256 + (1u << s) + g] = shoup(powm(psii, ex, qi), qi);
      }
    // twist of block b: rho_b = psi^(2 brv(b) + 1)
    for (u64 b = 0; b < N1; ++b) {
      const u64 rho = powm(psi, 2 * (u64)brv((uint32_t)b, logN1) + 1, qi);
      const u64 rhoi = invm(rho, qi);
      uint2* t = &twist[((size_t)i * N1 + b) * 32];
      uint2* ti = &itwist[((size_t)i * N1 + b) * 32];
      for (u64 j = 0; j < 16; ++j) {
        t[j] = shoup(powm(rho, j, qi), qi);
        ti[j] = shoup(powm(rhoi, j, qi), qi);
        t[16 + j] = shoup(powm(rho, 16 * j, qi), qi);
        ti[16 + j] = shoup(powm(rhoi, 16 * j, qi), qi);
      }
    }
  }
  c.h_mod = mod;

  // ModUp: pre-multiply constants and BConv tables for every level and digit.
  const int bmax = c.beta_max();
  std::vector<uint2> mscale((size_t)(c.L_max + 1) * c.L_max, make_uint2(0, 0));
  std::vector<uint32_t> mT;
  c.modup_T_off.assign((size_t)(c.L_max + 1) * bmax, 0);
  for (int L = 1; L <= c.L_max; ++L) {
    const int beta = c.beta(L);
    const RowMap rm = c.rows(L);
    for (int j = 0; j < beta; ++j) {
      const int lo = j * c.alpha, hi = std::min(lo + c.alpha, L);
      c.modup_T_off[(size_t)L * bmax + j] = mT.size();
      for (int i = lo; i < hi; ++i) {
        const u64 qi = c.primes[i];
        u64 prod = 1;
        for (int t = lo; t < hi; ++t)
          if (t != i) prod = mulm(prod, c.primes[t], qi);
        const u64 s = mulm(invm(prod, qi), invm(N % qi, qi), qi);
        mscale[(size_t)L * c.L_max + i] = shoup(s, qi);
      }
      for (int r = 0; r < L + c.k; ++r) {
        const u64 pr = c.primes[rm.pidx(r)];
        u128 bound = 0;
        for (int ii = 0; ii < c.alpha; ++ii) {
          const int i = lo + ii;
          u64 v = 0;
          if (i < hi) {
            v = 1 % pr;
            for (int t = lo; t < hi; ++t)
              if (t != i) v = mulm(v, c.primes[t], pr);
            bound += (u128)v * (c.primes[i] - 1);
          }
          mT.push_back((uint32_t)v);
        }
        if (bound >> 64) {
          *code = CKKS_EUNSUPPORTED;
          return "ModUp base-conversion table violates the overflow-free bound sum T*Q < 2^64";
        }
      }
    }
  }

  // ModDown constants
  std::vector<uint2> dscale(c.k), pinv(c.L_max);
  std::vector<uint32_t> dT((size_t)c.L_max * c.k);
  for (int m = 0; m < c.k; ++m) {
    const u64 pm = c.primes[c.L_max + m];
    u64 prod = 1;
    for (int t = 0; t < c.k; ++t)
      if (t != m) prod = mulm(prod, c.primes[c.L_max + t], pm);
    dscale[m] = shoup(mulm(invm(prod, pm), invm(N % pm, pm), pm), pm);
  }
  for (int i = 0; i < c.L_max; ++i) {
    const u64 qi = c.primes[i];
    u128 bound = 0;
    u64 P = 1;
    for (int m = 0; m < c.k; ++m) {
      u64 v = 1;
      for (int t = 0; t < c.k; ++t)
        if (t != m) v = mulm(v, c.primes[c.L_max + t], qi);
      dT[(size_t)i * c.k + m] = (uint32_t)v;
      bound += (u128)v * (c.primes[c.L_max + m] - 1);
      P = mulm(P, c.primes[c.L_max + m], qi);
    }
    if (bound >> 64) {
      *code = CKKS_EUNSUPPORTED;
      return "ModDown base-conversion table violates the overflow-free bound sum T*Q < 2^64";
    }
    pinv[i] = shoup(invm(P, qi), qi);
  }

  // Rescale constants
  std::vector<uint2> rinv((size_t)(c.L_max + 1) * c.L_max, make_uint2(0, 0));
  for (int L = 2; L <= c.L_max; ++L)
    for (int i = 0; i < L - 1; ++i) {
      const u64 qi = c.primes[i];
      rinv[(size_t)L * c.L_max + i] = shoup(invm(c.primes[L - 1] % qi, qi), qi);
    }

  std::string err;
  if (!(err = upload(&c.d_mod, mod, code)).empty()) return err;
  if (!(err = upload(&c.d_tw, tw, code)).empty()) return err;
  if (!(err = upload(&c.d_itw, itw, code)).empty()) return err;
  if (!(err = upload(&c.d_ctw, ctw, code)).empty()) return err;
  if (!(err = upload(&c.d_ictw, ictw, code)).empty()) return err;
  if (!(err = upload(&c.d_twist, twist, code)).empty()) return err;
  if (!(err = upload(&c.d_itwist, itwist, code)).empty()) return err;
  if (small_ring) {
    if (!(err = upload(&c.d_ftw, ftw, code)).empty()) return err;
    if (!(err = upload(&c.d_fitw, fitw, code)).empty()) return err;
  }
  if (!(err = upload(&c.d_modup_scale, mscale, code)).empty()) return err;
  if (!(err = upload(&c.d_modup_T, mT, code)).empty()) return err;
  std::vector<uint32_t> toff(c.modup_T_off.begin(), c.modup_T_off.end());
  if (!(err = upload(&c.d_modup_T_off, toff, code)).empty()) return err;
  if (!(err = upload(&c.d_moddown_scale, dscale, code)).empty()) return err;
  if (!(err = upload(&c.d_moddown_T, dT, code)).empty()) return err;
  if (!(err = upload(&c.d_pinv, pinv, code)).empty()) return err;
  if (!(err = upload(&c.d_rescale_inv, rinv, code)).empty()) return err;
  *code = CKKS_OK;
  return "";
}

void free_tables(Ctx& c) {
  void* ptrs[] = {c.d_mod, c.d_tw, c.d_itw, c.d_ctw, c.d_ictw, c.d_twist, c.d_itwist, c.d_ftw, c.d_fitw,
                  c.d_modup_scale, c.d_modup_T, c.d_modup_T_off,
                  c.d_moddown_scale, c.d_moddown_T, c.d_pinv, c.d_rescale_inv};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

}  // namespace ckks
