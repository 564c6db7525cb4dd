/*
 * Plain CPU oracle for the RNS-CKKS key-switching path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * library: every constant it uses is derived in this directory from the
 * prime list.
 *
 * Everything here is deliberately the textbook form: modular products are
 * `(uint64_t)a * b % q`, loops are plain, there is no lazy reduction, no
 * Shoup/Barrett/Montgomery form and no tiling.  Rows (limbs) are
 * independent, so the outer loop over rows may run on several OpenMP
 * threads; that changes nothing in the arithmetic.
 *
 * Polynomials are limb-major: row r holds N residues modulo its own prime.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint32_t mulmod(uint32_t a, uint32_t b, uint32_t q) {
    return (uint32_t)(((uint64_t)a * b) % q);
}
static uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) {
    return (uint32_t)(((uint64_t)a + b) % q);
}
static uint32_t submod(uint32_t a, uint32_t b, uint32_t q) {
    return (uint32_t)(((uint64_t)a + q - b) % q);
}

static unsigned bit_reverse(unsigned x, int bits) {
    unsigned r = 0;
    for (int i = 0; i < bits; i++) {
        r = (r << 1) | (x & 1u);
        x >>= 1;
    }
    return r;
}

/* pw[e] = root^e mod q for e in [0, N) */
static void power_table(uint32_t *pw, uint32_t root, uint32_t q, int N) {
    pw[0] = 1 % q;
    for (int e = 1; e < N; e++) pw[e] = mulmod(pw[e - 1], root, q);
}

/*
 * Forward negacyclic NTT of every row, in place (Sec. II-B1).
 *
 * The transform is (N/2) log2 N butterflies BFly_NTT(x, y, w) =
 * (x + w*y, x - w*y) mod q, Cooley-Tukey order.  Stage s has m = 2^s
 * butterfly groups; group i pairs a[j] and a[j + t] (t = N / 2m) with the
 * twiddle w = psi^brv(m + i), brv over log2 N bits.  Input in natural
 * order; the output is bit-reversed:
 *     out[j] = sum_n a[n] * psi^((2 brv(j) + 1) n)  (mod q).
 */
void oracle_ntt(uint32_t *a, int rows, int logN, const uint32_t *q, const uint32_t *psi) {
    const int N = 1 << logN;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < rows; r++) {
        uint32_t *x = a + (size_t)r * N;
        uint32_t *pw = (uint32_t *)malloc(sizeof(uint32_t) * N);
        power_table(pw, psi[r], q[r], N);
        int t = N;
        for (int m = 1; m < N; m <<= 1) {
            t >>= 1;
            for (int i = 0; i < m; i++) {
                const uint32_t w = pw[bit_reverse((unsigned)(m + i), logN)];
                for (int j = 2 * i * t; j < 2 * i * t + t; j++) {
                    const uint32_t u = x[j];
                    const uint32_t v = mulmod(w, x[j + t], q[r]);
                    x[j] = addmod(u, v, q[r]);
                    x[j + t] = submod(u, v, q[r]);
                }
            }
        }
        free(pw);
    }
}

/*
 * Inverse negacyclic NTT of every row, in place (Sec. II-B1).
 *
 * Gentleman-Sande butterflies BFly_INTT(x, y, w) = (x + y, w*(x - y)) mod q
 * with w = psi^-brv(m + i), m running N/2, N/4, ..., 1, followed by the
 * scale N^-1 so that the result is the exact inverse of oracle_ntt.
 * Input bit-reversed, output natural order.
 */
void oracle_intt(uint32_t *a, int rows, int logN, const uint32_t *q, const uint32_t *psi_inv,
                 const uint32_t *n_inv) {
    const int N = 1 << logN;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < rows; r++) {
        uint32_t *x = a + (size_t)r * N;
        uint32_t *pw = (uint32_t *)malloc(sizeof(uint32_t) * N);
        power_table(pw, psi_inv[r], q[r], N);
        int t = 1;
        for (int m = N >> 1; m >= 1; m >>= 1) {
            for (int i = 0; i < m; i++) {
                const uint32_t w = pw[bit_reverse((unsigned)(m + i), logN)];
                for (int j = 2 * i * t; j < 2 * i * t + t; j++) {
                    const uint32_t u = x[j];
                    const uint32_t v = x[j + t];
                    x[j] = addmod(u, v, q[r]);
                    x[j + t] = mulmod(w, submod(u, v, q[r]), q[r]);
                }
            }
            t <<= 1;
        }
        for (int j = 0; j < N; j++) x[j] = mulmod(x[j], n_inv[r], q[r]);
        free(pw);
    }
}

/*
 * Fast base conversion (Sec. II-B2, table T of Sec. III-C2).
 *
 * Input: n_in rows x[i] modulo q_in[i] (coefficient domain), the set I of
 * input moduli with product D.  Output: n_out rows modulo p_out[t]:
 *     y_i = x_i * [(D/q_i)^-1]_{q_i}  mod q_i
 *     z_t = sum_i y_i * T[t][i]        mod p_t,   T[t][i] = (D/q_i) mod p_t.
 * The sum is reduced after every term here (the plain form); the result is
 * the same residue the deferred 64-bit reduction of the paper produces.
 */
void oracle_bconv(const uint32_t *x, int n_in, const uint32_t *q_in, const uint32_t *qhat_inv,
                  uint32_t *z, int n_out, const uint32_t *p_out, const uint32_t *T, int N) {
    uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n_in * N);
    for (int i = 0; i < n_in; i++)
        for (int n = 0; n < N; n++)
            y[(size_t)i * N + n] = mulmod(x[(size_t)i * N + n], qhat_inv[i], q_in[i]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < n_out; t++) {
        for (int n = 0; n < N; n++) {
            uint32_t acc = 0;
            for (int i = 0; i < n_in; i++) {
                const uint32_t yi = y[(size_t)i * N + n] % p_out[t];
                acc = addmod(acc, mulmod(yi, T[(size_t)t * n_in + i], p_out[t]), p_out[t]);
            }
            z[(size_t)t * N + n] = acc;
        }
    }
    free(y);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the row loops from now on (timing only; the results do not
 * depend on it). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
