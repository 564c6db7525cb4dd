/*
 * ckks.h - C-ABI of the gfx950 (MI355X) RNS-CKKS key-switching library.
 *
 * The library computes the hot path of homomorphic multiplication and
 * rotation with hybrid key-switching over RNS polynomials in exact 32-bit
 * word arithmetic: negacyclic NTT / INTT, automorphism, ModUp / ModDown base
 * conversion, the evaluation-key inner product, tensoring and rescale
 * (paper: Sec. II-A/II-B for the data and the polynomial operations, Fig.
 * keysw and Sec. IV for the three key-switching stages).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return value: 0 (CKKS_OK) or a negative CKKS_E* code.  On error nothing has
 *   been enqueued and ckks_last_error() (thread-local) describes the cause.
 *   No C++ exception crosses this boundary.
 * Pointers: every data pointer is a DEVICE pointer on the context's device,
 *   4-byte aligned (256-byte alignment is recommended), owned by the caller.
 *   The library never frees or retains them past the call.  Host pointers are
 *   named h_* and are read before the call returns.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *   stream).  Calls are asynchronous: they enqueue kernels and return.  A
 *   device fault surfaces at the caller's next synchronisation.
 * Residues: uint32, canonical in [0, q), normal (not Montgomery) form.
 *   Inputs outside [0, q) give unspecified (but in-bounds) results.
 * Layout: limb-major.  A polynomial at level L is [L][N] (row i modulo q_i),
 *   with the special-prime rows p_0..p_{k-1} appended when "with P"; a
 *   ciphertext is [2][L][N] = (c0, c1), decrypting to c0 + c1 * s.
 *   Evaluation domain = bit-reversed NTT order A[j] = a(psi^(2 brv(j) + 1)),
 *   psi the smallest primitive 2N-th root of unity modulo the row's prime.
 * Keys: a key-switching key is [beta_max][2][L_max + k][N] in the evaluation
 *   domain, beta_max = ceil(L_max / alpha), alpha = k; at level L the rows
 *   [0, L) and [L_max, L_max + k) are used.  Component 0 is b, 1 is a.
 * Digits: digit j of a level-L polynomial is Q-rows [j*alpha, min((j+1)*alpha, L)).
 * Workspace: operations that need scratch take (ws, ws_bytes), a device
 *   buffer of at least ckks_workspace_bytes(ctx, op, L) bytes owned by the
 *   caller; nothing is allocated inside an operation.  One workspace must
 *   not be used by two calls that may run concurrently.
 * Aliasing: ckks_ntt / ckks_intt are in place.  Elsewhere an output must not
 *   overlap any input unless stated.
 * Thread safety: a context is immutable after creation; calls on different
 *   streams with different workspaces may run concurrently.
 */
#ifndef CKKS_H
#define CKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CKKS_OK = 0,
    CKKS_EINVAL = -1,       /* bad argument (null pointer, level out of range, ...) */
    CKKS_ENOMEM = -2,       /* workspace too small, or device allocation failed */
    CKKS_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
    CKKS_EUNSUPPORTED = -4  /* parameters outside what the kernels support */
};

/* Operation ids for ckks_workspace_bytes. */
enum {
    CKKS_OP_NTT = 0,
    CKKS_OP_MODUP = 1,
    CKKS_OP_MODDOWN = 2,
    CKKS_OP_KEYSWITCH = 3,
    CKKS_OP_HMULT = 4,
    CKKS_OP_HROT = 5,
    CKKS_OP_RESCALE = 6,
    CKKS_OP_HROT_HOISTED = 7
};

/* Pipeline stages that can be timed with ckks_trace_begin / ckks_trace_end. */
enum {
    CKKS_STAGE_INTT_BLOCKS = 1,     /* K1: INTT block pass of the switched polynomial */
    CKKS_STAGE_INTT_COLS = 2,       /* K2: INTT column pass + BConv pre-multiply */
    CKKS_STAGE_BCONV_UP = 3,        /* K3: ModUp base conversion, all digits */
    CKKS_STAGE_NTT_COLS_UP = 4,     /* K4: NTT column pass of the ModUp rows */
    CKKS_STAGE_NTT_IP = 5,          /* K5: NTT block pass + key inner product (+ P-row INTT pass);
                                       the Q rows only when the inner product is split */
    CKKS_STAGE_INTT_COLS_P = 6,     /* K6: INTT column pass of the P rows */
    CKKS_STAGE_BCONV_DOWN = 7,      /* K7: ModDown base conversion */
    CKKS_STAGE_NTT_COLS_DOWN = 8,   /* K8: NTT column pass of the ModDown rows */
    CKKS_STAGE_NTT_COMBINE = 9,     /* K9: NTT block pass + (acc - w) P^-1 + epilogue */
    CKKS_STAGE_RESCALE_NTT = 10,    /* R4: rescale NTT block pass + combine */
    CKKS_STAGE_NTT_IP_P = 11        /* K5 on the P rows when the inner product is split */
};

typedef struct ckks_ctx ckks_ctx;

/* Thread-local description of the last error on this thread ("" if none). */
const char *ckks_last_error(void);

/*
 * Create a context for ring degree N = 2^logN (12 <= logN <= 16) over the
 * chain h_q[0..L_max) and special primes h_p[0..k) (host arrays), on HIP
 * device `device`.  Every prime must be < 2^30, prime, 1 mod 2N and
 * distinct; dnum gives the digit size alpha = ceil(L_max / dnum), which must
 * equal k (Sec. IV-A: alpha special primes per digit).  The context builds
 * its twiddle tables (Sec. II-B1), the BConv tables T[i][j] = (Q^* / Q_j)
 * mod P_i with Q^* the product of the input moduli (Sec. III-C2) for every
 * level and digit, and checks the overflow-free condition
 * sum_j T[i][j] * Q_j < 2^64 of Sec. III-C2 for every table.
 * Errors: CKKS_EINVAL (bad primes / sizes), CKKS_EUNSUPPORTED (logN or
 * L_max + k out of range, bound violated), CKKS_ENOMEM, CKKS_EHIP.
 * Owns device memory until ckks_ctx_destroy.  ckks_ctx_destroy frees device
 * memory (hipFree): it must not run while a stream capture is in progress
 * (it would invalidate the capture).  The single-operation entry points
 * launch kernels only on the given stream, so they may be captured.
 */
int ckks_ctx_create(ckks_ctx **out, int logN, const uint32_t *h_q, int L_max,
                    const uint32_t *h_p, int k, int dnum, int device);
int ckks_ctx_destroy(ckks_ctx *ctx);

/* Device bytes of workspace needed by operation `op` (CKKS_OP_*) at level L;
 * for CKKS_OP_HROT_HOISTED, per call (independent of the rotation count). */
size_t ckks_workspace_bytes(const ckks_ctx *ctx, int op, int L);

/*
 * Forward / inverse negacyclic NTT in place (Sec. II-B1: (N/2) log2 N
 * butterflies per limb, Cooley-Tukey forward, Gentleman-Sande inverse).
 * a: [L (+k if with_P)][N]; row i is modulo q_i, appended rows modulo p_m.
 * Forward maps natural coefficients to the bit-reversed evaluation domain;
 * the inverse includes the N^-1 scale.  1 <= L <= L_max.
 */
int ckks_ntt(const ckks_ctx *ctx, uint32_t *a, int L, int with_P, void *stream);
int ckks_intt(const ckks_ctx *ctx, uint32_t *a, int L, int with_P, void *stream);

/*
 * Automorphism sigma_g, g = 5^rot mod 2N, on evaluation-domain rows (Sec.
 * II-B3: a column permutation, the same for every limb):
 * out[r][j] = in[r][j'] with 2 brv(j') + 1 = g (2 brv(j) + 1) mod 2N.
 * in/out: [rows][N]; rows is any positive row count.  out must not alias in.
 */
int ckks_automorph(const ckks_ctx *ctx, const uint32_t *in, uint32_t *out, int rows, int rot,
                   void *stream);

/*
 * Tensoring (Sec. II-B3, element-wise): ct1, ct2 [2][L][N] -> out [3][L][N],
 * d0 = c0 c0', d1 = c0 c1' + c1 c0', d2 = c1 c1' (mod q_i).
 */
int ckks_tensor(const ckks_ctx *ctx, const uint32_t *ct1, const uint32_t *ct2, int L,
                uint32_t *out, void *stream);

/*
 * Plaintext products summed, the inner sums of a baby-step giant-step linear
 * transform (element-wise, Sec. II-B3): out[c][i] = sum_{b < nb} ct_b[c][i] *
 * pt_b[i] mod q_i for c = 0, 1.  h_cts: nb device pointers to [2][L][N]
 * ciphertexts; h_pts: nb device pointers to [L][N] evaluation-domain
 * plaintexts; 1 <= nb <= 16.  out: [2][L][N], must not alias an input.
 */
int ckks_pmult_sum(const ckks_ctx *ctx, const uint32_t *const *h_cts, const uint32_t *const *h_pts,
                   int nb, int L, uint32_t *out, void *stream);

/*
 * Several inner sums over the same ciphertexts in one launch (the giant steps
 * of one BSGS level, Sec. II-B3): out_g[c][i] = sum_{b < nb} ct_b[c][i] *
 * pt_{g,b}[i] mod q_i for g < ng, each ciphertext word read once for all ng
 * sums.  h_cts: nb device pointers to [2][L][N] ciphertexts; h_pts: ng * nb
 * device pointers to [L][N] evaluation-domain plaintexts, group-major
 * (pt_{g,b} at h_pts[g * nb + b]); h_outs: ng device pointers to [2][L][N]
 * outputs, none aliasing an input or each other.  1 <= nb <= 16,
 * 1 <= ng <= 8.  Each out_g equals ckks_pmult_sum of the same ciphertexts and
 * group g's plaintexts.
 */
int ckks_pmult_sums(const ckks_ctx *ctx, const uint32_t *const *h_cts, int nb, const uint32_t *const *h_pts,
                    int ng, int L, uint32_t *const *h_outs, void *stream);

/* Ciphertext sum (element-wise): out = a + b over [2][L][N]; out may alias a or b. */
int ckks_add(const ckks_ctx *ctx, const uint32_t *a, const uint32_t *b, int L, uint32_t *out,
             void *stream);

/*
 * ModUp, key-switching stage 1 (Fig. keysw, Sec. IV-A), for every digit j:
 * INTT of the digit's limbs, fast BConv (Sec. II-B2, III-C2) from D_j to the
 * other moduli of Q_L and P, NTT of the new limbs; the digit's own rows are
 * copied.  d: [L][N] evaluation domain.  out: [beta][L + k][N],
 * beta = ceil(L / alpha), rows q_0..q_{L-1}, p_0..p_{k-1}.
 */
int ckks_modup(const ckks_ctx *ctx, const uint32_t *d, int L, uint32_t *out, void *ws,
               size_t ws_bytes, void *stream);

/*
 * Evaluation-key inner product, key-switching stage 2 (Sec. IV-B):
 * acc[c][r] = sum_{j < beta} M[j][r] * evk[j][c][row(r)] for c = 0, 1,
 * row(r) = r for r < L, L_max + (r - L) otherwise.
 * M: [beta][L + k][N]; evk: key layout; acc: [2][L + k][N].
 */
int ckks_inner_product(const ckks_ctx *ctx, const uint32_t *M, int L, const uint32_t *evk,
                       uint32_t *acc, void *stream);

/*
 * ModDown, key-switching stage 3 (Fig. keysw): out = (a_Q - NTT(BConv_{P->Q}
 * (INTT(a_P)))) * P^-1 mod q_i, floor form (no rounding offset).
 * in: [L + k][N] evaluation domain; out: [L][N].
 */
int ckks_moddown(const ckks_ctx *ctx, const uint32_t *in, int L, uint32_t *out, void *ws,
                 size_t ws_bytes, void *stream);

/*
 * Key-switching (Fig. keysw): out[c] = ModDown(sum_j ModUp_j(d) * evk[j][c]).
 * d: [L][N] evaluation domain; evk: key layout; out: [2][L][N].
 */
int ckks_keyswitch(const ckks_ctx *ctx, const uint32_t *d, int L, const uint32_t *evk,
                   uint32_t *out, void *ws, size_t ws_bytes, void *stream);

/*
 * HMult with relinearisation, no rescale (Sec. II-A; key-switching of the
 * s^2 term): out = (d0 + KS_0(d2), d1 + KS_1(d2)) with (d0, d1, d2) the
 * tensor of ct1 and ct2.  ct1, ct2, out: [2][L][N]; rlk: key for s^2 -> s.
 * out may alias neither input.
 */
int ckks_hmult(const ckks_ctx *ctx, const uint32_t *ct1, const uint32_t *ct2, int L,
               const uint32_t *rlk, uint32_t *out, void *ws, size_t ws_bytes, void *stream);

/*
 * ckks_hmult without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, layouts and result as ckks_hmult
 * (bitwise); the key-switching scratch is a static 128 MiB device array that
 * the library holds on each device it runs on until the process ends (its
 * address is taken once per device by ckks_ctx_create).  Allocates nothing
 * and needs no zeroed memory: every scratch word is written before it is
 * read.  Returns CKKS_ENOMEM when ckks_workspace_bytes(ctx, CKKS_OP_HMULT, L)
 * exceeds 128 MiB (N = 2^16 with L = 36, k = 12, dnum = 3 needs 102 MiB).
 * All calls on one device share that device's scratch: calls that may
 * overlap on one device (different streams, or different host threads
 * without ordering) race and give wrong results; order them on one stream.
 */
int ckks_hmult_noalloc(const ckks_ctx *ctx, const uint32_t *ct1, const uint32_t *ct2, int L,
                       const uint32_t *rlk, uint32_t *out, void *stream);

/*
 * HRot by `rot` slots (left), g = 5^rot mod 2N: the automorphism sigma_g of
 * Sec. II-B3 (a column permutation of every limb) applied to both
 * components, then the key-switching of Fig. keysw on the permuted c1:
 * out = (sigma(c0) + KS_0(sigma(c1)), KS_1(sigma(c1))).  rotk must switch
 * sigma_g(s) -> s; the library cannot check that.  ct, out: [2][L][N].
 */
int ckks_hrot(const ckks_ctx *ctx, const uint32_t *ct, int L, int rot, const uint32_t *rotk,
              uint32_t *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Several independent rotations in one launch sequence (the giant steps of a
 * BSGS level, Sec. II-B3 and Fig. keysw): out_i = HRot(ct_i, rot_i) under key
 * rotk_i for i < n, exactly as n ckks_hrot calls, but every pipeline kernel
 * covers all n jobs (Sec. IV-A batching).  h_cts, h_rotks, h_outs: n device
 * pointers each (ciphertexts and outputs [2][L][N], keys as for ckks_hrot);
 * h_rots: n rotation amounts (host array); 1 <= n <= 16; no output may alias
 * an input or another output.  ws: n times ckks_workspace_bytes(ctx,
 * CKKS_OP_HROT, L) bytes (CKKS_ENOMEM if smaller).  Errors as ckks_hrot.
 */
int ckks_hrot_many(const ckks_ctx *ctx, const uint32_t *const *h_cts, int L, const int *h_rots,
                   const uint32_t *const *h_rotks, uint32_t *const *h_outs, int n, void *ws,
                   size_t ws_bytes, void *stream);

/*
 * Hoisted rotations (rotations reordered so that one ModUp is shared;
 * Sec. V-C): M = ModUp(c1) once; for each n: sigma_{g_n} on every row of M
 * (Q and P), inner product with h_rotks[n], ModDown, plus sigma_{g_n}(c0).
 * Not bitwise equal to n separate ckks_hrot calls (the base conversion is
 * not permutation-equivariant), but decrypts to the same rotations.
 * h_rots, h_rotks, h_outs: host arrays of n entries (keys and outputs are
 * device pointers).  n >= 1.
 */
int ckks_hrot_hoisted(const ckks_ctx *ctx, const uint32_t *ct, int L, const int *h_rots, int n,
                      const uint32_t *const *h_rotks, uint32_t *const *h_outs, void *ws,
                      size_t ws_bytes, void *stream);

/*
 * Rescale by the top prime (drop q_{L-1}), the division by the scale factor
 * that follows a multiplication (Sec. II-A: a ciphertext at level L holds L
 * limbs; Table I's Delta is the scale kept by dropping limbs).  For each
 * component, t = INTT_{q_{L-1}}(a_{L-1}); out_i = (a_i - NTT_{q_i}(t mod q_i))
 * * q_{L-1}^-1 mod q_i, floor form (no rounding offset).
 * ct: [2][L][N] -> out: [2][L-1][N]; 2 <= L <= L_max.
 */
int ckks_rescale(const ckks_ctx *ctx, const uint32_t *ct, int L, uint32_t *out, void *ws,
                 size_t ws_bytes, void *stream);

/*
 * Kernel schedule of a context's key-switching pipeline (the limb-tile and
 * work-group shapes that do not change any result):
 *   bconv_up_rows    ModUp BConv output rows per work-group: 2, 4, 6 or 12
 *                    (a work-group re-reads its digit's inputs once)
 *   bconv_down_rows  ModDown BConv output rows per work-group: 2, 4, 6 or 12
 *   small_grid       inner-product launches of at most this many
 *                    work-groups use one thread group per digit tile
 *                    (0: never)
 *   ntt_shape        NTT tile / radix choices (Sec. III-C1 NTT kernels),
 *                    a bit mask: 1 = forward column passes with 8 elements
 *                    per thread in radix-8 phases (else 16, radix-16);
 *                    2 = inverse column passes with 16 elements per thread
 *                    in radix-16 phases (else 8, radix-8); 4 = the ModUp
 *                    INTT block pass with 16 elements per thread on 256
 *                    threads (else 8 on 512); 8 = at N = 2^12, the whole
 *                    key-switch as two kernels that hold whole limbs in
 *                    LDS (ModUp + inner product per row and digit group,
 *                    ModDown + epilogue per output row) instead of the
 *                    nine-kernel pipeline (hoisted rotations and batch
 *                    plans with a split inner product keep the nine
 *                    kernels).  Small grids keep their own shapes.  0..15.
 * Default {12, 6, 128, 0}; {12, 6, 128, 8} for N = 2^12.  The schedule is read when work is enqueued (and when
 * a graph batch is captured); changing it must not overlap calls on the
 * context.  Every schedule gives bitwise the same results.
 */
typedef struct ckks_schedule {
    int bconv_up_rows;
    int bconv_down_rows;
    int small_grid;
    int ntt_shape;
} ckks_schedule;

int ckks_ctx_get_schedule(const ckks_ctx *ctx, ckks_schedule *sched);
/* Errors: CKKS_EINVAL for rows outside {2, 4, 6, 12}, small_grid outside [0, 65535]
 * or ntt_shape outside [0, 15]. */
int ckks_ctx_set_schedule(ckks_ctx *ctx, const ckks_schedule *sched);
/*
 * Schedule autotuner: times an HMult at level L on synthetic inputs (zeros;
 * the arithmetic is data-independent) under every candidate schedule
 * (rows in {2, 4, 6, 12} for both BConvs, small_grid in {0, 128, 1024},
 * ntt_shape 0..7, and 8..15 at N = 2^12: 384 or 768 candidates), one
 * warm-up and `reps` calls each between two events on `stream`, and keeps
 * the fastest.  Allocates its own device buffers (inputs, key, workspace)
 * for the duration of the call and synchronises `stream`; not for use while
 * other calls run on the context.  best / best_us (either may be NULL)
 * receive the schedule and its time per HMult in microseconds.
 */
int ckks_ctx_tune(ckks_ctx *ctx, int L, int reps, void *stream, ckks_schedule *best, float *best_us);

/*
 * Batches (Sec. IV-A batching; Sec. IV-C one submission per static graph).
 * A batch is a fixed list of independent jobs, each at its own level, run
 * together: every pipeline kernel covers all jobs of a launch group at once
 * (nine kernels for the key-switching jobs of a group, four for all rescale
 * jobs; groups as in ckks_batch_plan below), and with use_graph != 0 the
 * whole launch sequence is captured once into a hipGraph at creation, so
 * ckks_batch_launch is a single graph submission.
 * Each job's result is bitwise the result of the corresponding single call.
 */
enum {
    CKKS_JOB_KEYSWITCH = 0,  /* in0 = d [L][N]; out = KS(d) [2][L][N] */
    CKKS_JOB_HMULT = 1,      /* in0 = ct1, in1 = ct2; out = HMult [2][L][N] */
    CKKS_JOB_HROT = 2,       /* in0 = ct; out = HRot by rot [2][L][N] */
    CKKS_JOB_RESCALE = 3     /* in0 = ct; out = rescale [2][L-1][N]; key unused */
};

typedef struct ckks_job {
    int op;               /* CKKS_JOB_* */
    int L;                /* level of the job (>= 2 for RESCALE) */
    int rot;              /* rotation for CKKS_JOB_HROT */
    int reserved;
    const uint32_t *in0;  /* device pointers, as in the single-call entry points */
    const uint32_t *in1;
    const uint32_t *key;
    uint32_t *out;
} ckks_job;

typedef struct ckks_batch ckks_batch;

/*
 * Build a batch of n jobs (host array, copied).  Allocates the batch's
 * device job tables and scratch (held until ckks_batch_destroy) and, with
 * use_graph, captures the launches.  Data pointers are not read here; they
 * must be valid whenever the batch is launched, and outputs must not alias
 * each other or any input.  Errors: CKKS_EINVAL, CKKS_ENOMEM, CKKS_EHIP.
 */
int ckks_batch_create(const ckks_ctx *ctx, const ckks_job *h_jobs, int n, int use_graph,
                      ckks_batch **out);
/* Enqueue the whole batch on `stream` (asynchronous). */
int ckks_batch_launch(ckks_batch *batch, void *stream);

/*
 * Launch plan of a batch (Sec. IV-A: the batch size B trades parallelism
 * against the working set that stays in the caches).  The key-switching jobs
 * are held in non-increasing level order (jobs of one level that share a key
 * adjacent); consecutive groups of jobs_per_launch of them (0 = all) each
 * run the pipeline once, group g on branch g mod streams; branches are
 * streams forked from and joined back to the launch stream, so groups
 * overlap on the device; split != 0 runs the Q-row inner product of each
 * group on a side stream (Sec. IV-B complementary pipelining): split = 1
 * starts it beside the P-row inner product, split = 2 after it, so that it
 * overlaps only the P-row ModDown chain.
 * Rescale jobs run on the last branch.  Every plan gives bitwise the same
 * results.  Default {0, 1, 1}; {0, 1, 0} for a batch of one key-switching
 * job, and at N = 2^12 under the whole-limb schedule (ntt_shape bit 8) while
 * (L + k) * min(beta, 4) * jobs <= 800 for its largest level L (split runs
 * the nine-kernel pipeline, which pays off only past that).  A batch created with use_graph runs one
 * branch (streams = 1): a multi-branch launch sequence is not captured.
 */
typedef struct ckks_batch_plan {
    int jobs_per_launch;  /* >= 0 */
    int streams;          /* 1..4 */
    int split;            /* 0, 1 or 2 */
    int reserved;
} ckks_batch_plan;

int ckks_batch_get_plan(const ckks_batch *batch, ckks_batch_plan *plan);
/* Replace the plan (re-captures the graph of a graph batch).  Must not
 * overlap a launch of the same batch.  Errors: CKKS_EINVAL (bad plan),
 * CKKS_EUNSUPPORTED (streams > 1 on a graph batch), CKKS_EHIP.  On error the
 * batch keeps its previous plan and graph. */
int ckks_batch_set_plan(ckks_batch *batch, const ckks_batch_plan *plan);
/*
 * A batch's own kernel schedule (struct ckks_schedule above): the context's
 * at creation; set here or by ckks_batch_tune.  Setting re-captures the
 * graph of a graph batch and must not overlap a launch of the same batch.
 * Errors: CKKS_EINVAL (bad schedule, as for ckks_ctx_set_schedule), CKKS_EHIP;
 * on error the batch keeps its previous schedule and graph.
 */
int ckks_batch_get_schedule(const ckks_batch *batch, ckks_schedule *sched);
int ckks_batch_set_schedule(ckks_batch *batch, const ckks_schedule *sched);
/*
 * Autotuner: times candidate plans (jobs_per_launch in {all, 32, 16, 8, 4, 2}
 * below the job count, streams 1..4 up to the number of groups (1 for a
 * graph batch), split 0/1/2) under the batch's schedule, then, under the
 * best plan, up to four other BConv schedules ({12, 6, 128}, {6, 4, 128},
 * {4, 6, 128}, {12, 12, 128}, with the batch's ntt_shape), then the other
 * seven NTT shapes under the best of those: each candidate as one warm-up
 * launch then `reps` launches between two events on `stream`; keeps the
 * fastest plan and schedule (graph batches are re-captured and timed as graph
 * launches).  Runs the batch up to 83 x (reps + 1) times and synchronises
 * `stream`:
 * outputs are written, inputs only read.  best / best_us (either may be
 * NULL) receive the chosen plan and its time per launch in microseconds;
 * ckks_batch_get_schedule gives the chosen schedule.  On error the previous
 * plan and schedule are kept.
 */
int ckks_batch_tune(ckks_batch *batch, int reps, void *stream, ckks_batch_plan *best,
                    float *best_us);
/* The plan candidates of the last ckks_batch_tune and their microseconds
 * per launch, in the order tried: *n receives their number, the first
 * min(cap, *n) are copied to plans / us. */
int ckks_batch_tune_log(const ckks_batch *batch, ckks_batch_plan *plans, float *us, int cap,
                        int *n);
/* Device bytes the batch holds (tables + scratch). */
size_t ckks_batch_device_bytes(const ckks_batch *batch);
int ckks_batch_destroy(ckks_batch *batch);

/*
 * Serving loop: continuous batching of jobs under an HBM budget.
 *
 * A server owns a device arena of hbm_budget bytes (allocated at creation)
 * from which every admitted job's scratch is taken, a few HIP streams, and
 * one host worker thread.  ckks_server_submit queues a job for context
 * ctxs[ctx_index] (contexts of different N may be mixed; all on one device)
 * and returns a ticket at once.  The worker admits queued jobs in arrival
 * order while fewer than max_slots jobs are on the device and the job's
 * scratch fits in the arena, launches each admitted group as one batch (the
 * job-table pipeline) on the next stream, and retires batches as their
 * events complete, so requests arriving while others run are admitted as
 * slots and memory free up and their work overlaps on the device.  A job's
 * result is bitwise the same as in a single call.  Inputs, keys and outputs
 * are caller-owned device buffers that must stay valid until the ticket is
 * done.  Ordering: ckks_server_submit records an event on `stream` (the
 * stream on which the caller produced the job's inputs or last used its
 * output buffer; NULL = the null stream), and the job's kernels start only
 * after that event, so work the caller queued there before the submit is
 * complete first.  Work queued on other streams is not waited for.
 * By default the budget bounds the device memory the server itself takes:
 * the scratch of the jobs on the device (ckks_workspace_bytes of the job's
 * operation).  Inputs, keys and outputs are then not counted: the caller
 * allocated them before the submit, so admitting a job does not change their
 * footprint (keys are typically shared by many jobs).  With
 * ckks_server_set_accounting(server, 1) the budget covers each in-flight
 * job's whole footprint instead: its scratch, its inputs and output, and
 * every distinct key array (beta_max x 2 x (L_max + k) limbs) named by the
 * jobs on the device, counted once however many jobs share it.  A job whose
 * scratch (whole footprint) alone exceeds the budget is refused with
 * CKKS_ENOMEM.  Latencies are host wall-clock from submit to the worker
 * observing completion.
 */
typedef struct ckks_server ckks_server;

typedef struct ckks_stats {
    uint64_t submitted, completed, rejected, pending, in_flight, batches;
    double p50_us, p99_us, mean_us, max_us;  /* submit -> completion, completed jobs */
    double ks_per_s;                         /* completed key-switching jobs per second */
    size_t budget_bytes, peak_bytes;         /* arena size, peak scratch in use */
} ckks_stats;

int ckks_server_create(const ckks_ctx *const *ctxs, int nctx, size_t hbm_budget, int max_slots,
                       ckks_server **out);
int ckks_server_submit(ckks_server *server, int ctx_index, const ckks_job *job, void *stream,
                       uint64_t *ticket);
/* *done = 1 once the ticket's result is in its output buffer. */
int ckks_server_poll(ckks_server *server, uint64_t ticket, int *done);
/* Block until every submitted job has completed. */
int ckks_server_drain(ckks_server *server);
/* Admission accounting: 0 = job scratch only (default), 1 = whole footprint
 * (scratch + inputs + output + distinct keys).  Before the first submit,
 * else CKKS_EINVAL.  stats.peak_bytes reports the accounted peak. */
int ckks_server_set_accounting(ckks_server *server, int whole_footprint);
int ckks_server_stats(ckks_server *server, ckks_stats *stats);
/* Submit / completion times (us since server creation; completion < 0 while
 * pending) of tickets [first, first + n). */
int ckks_server_times(ckks_server *server, uint64_t first, int n, double *h_submit_us,
                      double *h_done_us);
/* Finish all queued work, stop the worker, free the arena. */
int ckks_server_destroy(ckks_server *server);

/*
 * Kernel tracing.  Between ckks_trace_begin and ckks_trace_end, every kernel
 * launch of pipeline stage `stage` (CKKS_STAGE_*) by this context carries a
 * pair of HIP events that the runtime records at the start and the end of
 * that dispatch (hipExtLaunchKernel), for the first `capacity` launches.  ckks_trace_end waits for the last recorded event,
 * writes the per-launch durations in milliseconds to h_ms (capacity floats,
 * may be NULL) and the number of recorded launches to *count, and disarms.
 * The events are created in ckks_trace_begin and destroyed in ckks_trace_end.
 * Not for concurrent use from several host threads on one context.
 */
int ckks_trace_begin(ckks_ctx *ctx, int stage, int capacity);
int ckks_trace_end(ckks_ctx *ctx, float *h_ms, int *count);

#ifdef __cplusplus
}
#endif

#endif /* CKKS_H */
