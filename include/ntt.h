/*
 * ntt.h -- C ABI of the MI355X non-negative tensor-train (nTT) library.
 *
 * The library factors a d-way non-negative tensor A (n_1 x ... x n_d) into TT cores
 * G_1..G_d, G_k of shape r_{k-1} x n_k x r_k with r_0 = r_d = 1, so that
 *     A[i_1..i_d] ~= sum_{k_1..k_{d-1}} G_1[i_1,k_1] G_2[k_1,i_2,k_2] ... G_d[k_{d-1},i_d]
 * (paper: Eq.(1) and Eq.(2), the TT format).  The factorisation is the sequential
 * sweep of Alg.2 (distnTT) run on one GPU: stage l unfolds the remaining tensor into
 * an (r_{l-1} n_l) x (n_{l+1}...n_d) matrix X_l, factors X_l ~= W H by NMF with
 * multiplicative updates (MU, the update the paper times in Sec. IV-B and IV-C),
 * keeps W as core l and reshapes H into the next unfolding; the last H is core d.
 *
 * MU, H first then W, with eps added to the denominators and a clamp at zero:
 *     H <- max(0, H .* (W^T X) ./ ((W^T W) H + eps))
 *     W <- max(0, W .* (X H^T) ./ (W (H H^T) + eps))
 * Options of ntt_config: the BCD NMF of Alg.3 instead of MU (nmf), the ranks chosen per
 * stage by the singular-value rule of Alg.2 (rank_eps), a BF16 copy of X for the
 * products (precision), and an input kept in host memory and streamed through the
 * device in column blocks (stream_cols).
 *
 * Conventions for every entry point
 *   - Arrays are row-major (C order, last index fastest) float32 unless stated.
 *   - "device" pointers point into GPU memory of the current HIP device; "host"
 *     pointers into CPU memory.  All buffers are owned by the caller; the library
 *     keeps no pointer after a call returns.
 *   - The library allocates no device memory for data itself: ntt_decompose and
 *     ntt_rel_error take a caller-provided device workspace whose size the query
 *     functions report, and the server works inside the caller's arena.  Exceptions:
 *     the rank rule (rank_eps > 0) creates one rocBLAS handle per plan on first use
 *     (the eigensolver's scratch is set to a region of the workspace, but creating a
 *     handle may allocate rocBLAS's own small device state); the streams, events and
 *     graphs a plan, batch or server creates hold HIP runtime resources; and
 *     ntt_rel_error_static uses a fixed 8 MiB device array of the library's.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued on it; every function below returns after its work has completed.
 *   - Errors come back as ntt_status codes; no C++ exception crosses the ABI.  On
 *     error the outputs are unspecified, nothing leaks and a plan stays valid.
 *     ntt_last_error() gives a thread-local detail string of the last failure.
 *   - A plan is not thread-safe: use one plan per host thread and stream.
 */
#ifndef NTT_H_
#define NTT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NTT_MAX_DIMS 16
#define NTT_MAX_RANK 32 /* largest TT rank the kernels take (padded to 16 or 32) */

typedef enum {
  NTT_OK = 0,
  NTT_ERR_INVALID_ARG = 1,         /* bad shape, rank, count, null pointer */
  NTT_ERR_RANK_INFEASIBLE = 2,     /* strict mode: r_l > min(r_{l-1} n_l, n_{l+1}..n_d) */
  NTT_ERR_NEGATIVE_INPUT = 3,      /* input holds a negative, NaN or Inf entry */
  NTT_ERR_WORKSPACE_TOO_SMALL = 4, /* workspace NULL or smaller than required */
  NTT_ERR_ZERO_NORM = 5,           /* ||A||_F = 0 where a ratio needs it */
  NTT_ERR_DEVICE = 6               /* a HIP call failed (detail in ntt_last_error) */
} ntt_status;

typedef enum {
  NTT_PREC_FP32 = 0,      /* every GEMM in FP32 (MFMA f32), norms in FP64 */
  NTT_PREC_BF16_MIXED = 1 /* W^T X and X H^T on a BF16 copy of X with FP32 accumulation;
                             r x r Grams and epilogues FP32; the last fp32_tail_iters
                             iterations of each stage FP32; norms FP64 */
} ntt_precision;

typedef enum {
  NTT_NMF_MU = 0, /* multiplicative updates (H first, then W) */
  NTT_NMF_BCD = 1 /* Alg.3: projected-gradient block steps, W then H, from extrapolated
                     points; an iteration whose pair does not lower the objective
                     1/2 ||X_l - W H||^2 is dropped and the next one starts from the kept
                     pair without extrapolation.  Step sizes 1/||H H^T||_F, 1/||W^T W||_F;
                     factors first scaled to ||W||_F = ||H||_F = sqrt(||X_l||_F) */
} ntt_nmf;

/* ntt_config.flags */
#define NTT_STRICT_RANKS 1u     /* infeasible rank -> NTT_ERR_RANK_INFEASIBLE (else clamp) */
#define NTT_VALIDATE_INPUT 2u   /* check A >= 0 and finite before the sweep */
#define NTT_RECORD_OBJECTIVE 4u /* explicit FP64 objective of every iterate into objective_trace */
#define NTT_PROFILE 8u          /* fill ntt_report.pass_ms with per-launch kernel timings */
#define NTT_NO_COOP 16u         /* every stage keeps one launch per pass and W-update (no
                                   whole-stage launch with grid barriers for m <= 256,
                                   r <= 16, k <= 32768; that launch needs its workgroups
                                   resident together and fails with NTT_ERR_DEVICE when
                                   other work keeps some of them waiting about a quarter
                                   second); the iterates are the same up to summation order */

typedef struct {
  int32_t d;            /* number of modes, 2..NTT_MAX_DIMS */
  const int64_t* dims;  /* host, d entries n_1..n_d, each >= 1 */
  const int64_t* ranks; /* host, d+1 entries r_0..r_d with r_0 = r_d = 1, inner >= 1 */
  int32_t max_iters;    /* NMF iterations per stage (>= 0) */
  double tol;           /* 0: run exactly max_iters.  > 0: stop early at t % check_every == 0
                           when sqrt(2 f_t)/||X_l|| <= tol or f_{t-K} - f_t <= tol f_{t-K},
                           f_t = 1/2 ||X_l - W_t H_t||_F^2 evaluated explicitly in FP64 */
  int32_t check_every;  /* K of the stopping test (>= 1) */
  double eps;           /* MU denominator epsilon (>= 0); 1e-12 is usual */
  uint64_t seed;        /* initial factors: SplitMix64 counter rule, W of stage l on stream
                           2l, H on stream 2l+1, uniform on [0,1) (exact in FP32) */
  int32_t precision;    /* ntt_precision */
  int32_t fp32_tail_iters; /* BF16 mode: last N iterations of each stage in FP32 */
  uint32_t flags;       /* NTT_* flags above */
  double rank_eps;      /* 0: the inner ranks are the given ranks (clamped).  > 0: the rank
                           rule of Alg.2: at each stage l, r_l is the smallest k such that
                           sqrt(s_{k+1}^2 + ... + s_N^2) / sqrt(s_1^2 + ... + s_N^2) <= rank_eps,
                           s the singular values of the current unfolding X_l (from the
                           eigenvalues of its FP64 Gram on the shorter side, which must be
                           at most 2048), capped by the given r_l as clamped; the chosen
                           ranks come back in ntt_report.eff_ranks and each core is written
                           compactly at the chosen ranks into its buffer (sized by the
                           caps).  ntt_decompose only (batched and server plans: 0). */
  int32_t nmf;          /* ntt_nmf (0: MU).  NTT_NMF_BCD runs exactly max_iters iterations
                           per stage (tol must be 0), in FP32 (precision NTT_PREC_FP32), in
                           ntt_decompose, ntt_decompose_batch and server requests; it
                           ignores eps and NTT_PROFILE, and with
                           NTT_RECORD_OBJECTIVE stores the objective of every iteration's
                           candidate pair (kept or dropped, FP64 residual).  Its workspace
                           adds two r_l x (n_{l+1}..n_d) buffers per stage; unfoldings may
                           have at most 4194240 rows. */
  double bcd_delta;     /* BCD: cap of the extrapolation weights, in [0, 1) (0.9999 is
                           usual; 0 turns extrapolation off) */
  int64_t stream_cols;  /* 0: A is device memory.  > 0: A is HOST memory (pinned for full
                           copy speed; it must stay valid until the stream has finished)
                           and stage 1 is out of core: every pass over X_1 (norm, each MU
                           iteration, final objective) copies it to the device in column
                           blocks of stream_cols columns, so only the blocks, W and H_1 are
                           resident.  The blocks' X H^T and H H^T are added in block order
                           before the W-update, so the iterates are MU's.  Later stages are
                           resident as usual.  With rank_eps > 0 the rank rule takes the
                           n_1 x n_1 Gram of X_1 as the sum of the blocks' Grams (n_1 <=
                           2048).  MU in FP32 with a fixed iteration count only (nmf 0,
                           precision FP32, tol 0, no NTT_RECORD_OBJECTIVE), ntt_decompose
                           only. */
} ntt_config;

typedef struct {
  int64_t eff_ranks[NTT_MAX_DIMS + 1]; /* ranks after clamping */
  int32_t iters[NTT_MAX_DIMS];         /* iterations run per stage */
  double objective[NTT_MAX_DIMS];      /* final 1/2||X_l - W H||^2 per stage (explicit, FP64) */
  double norm_x[NTT_MAX_DIMS];         /* ||X_l||_F per stage (FP64) */
  double stage_rel_err[NTT_MAX_DIMS];  /* sqrt(2 objective)/norm_x per stage */
  double ms[NTT_MAX_DIMS];             /* wall time per stage on the stream (hipEvents) */
  double gflop[NTT_MAX_DIMS];          /* algorithmic GFLOP per stage: T(4mkr + 4(m+k)r^2) */
  double pass_ms[NTT_MAX_DIMS];        /* NTT_PROFILE: mean duration of one MU iteration's
                                          main X pass kernel per stage */
  double total_ms;
  double total_gflop;
  double compression_ratio;            /* Eq.(4) at eff_ranks */
  int32_t corrections[NTT_MAX_DIMS];   /* BCD: dropped iterations per stage (MU: 0) */
  int32_t bf16_iters[NTT_MAX_DIMS];    /* iterations per stage whose X passes read the BF16
                                          copy of X (precision NTT_PREC_BF16_MIXED); 0 for
                                          stages that stay FP32: those the whole-stage
                                          kernels take (X stays on chip: m <= 256, r <= 16
                                          and k <= 64, or k <= 32768 for a standalone plan
                                          with tol = 0), the generic path, the
                                          one-wavefront pass at rank padding 32 (m <= 32,
                                          r > 16), BCD, streamed */
} ntt_report;

typedef struct ntt_plan_s* ntt_plan_t;

/* Build a plan for the sweep of Alg.2 (Sec. III-A), with MU (the NMF timed in Sec. IV-B)
 * or the BCD of Alg.3 (Sec. III-B) as the NMF, from a config (host only, no device work).  Validates the shape
 * (d in 2..16, n_k >= 1, r_0 = r_d = 1, product of dims at most 2^44), clamps ranks to
 * r_l <= min(r_{l-1} n_l, n_{l+1}...n_d) left to right (or fails with
 * NTT_ERR_RANK_INFEASIBLE under NTT_STRICT_RANKS), rejects an effective rank above
 * NTT_MAX_RANK, and lays out the workspace.  *out is owned by the caller and freed
 * with ntt_plan_destroy. */
ntt_status ntt_plan(const ntt_config* cfg, ntt_plan_t* out);

/* Query a plan: device workspace bytes ntt_decompose needs (bytes may be NULL),
 * effective ranks (host array of d+1 entries, may be NULL) and the Eq.(4)
 * compression ratio prod n_i / sum n_i r_{i-1} r_i at those ranks (may be NULL).
 * With rank_eps > 0 the effective ranks are the caps (the core buffer sizes). */
ntt_status ntt_plan_workspace(ntt_plan_t plan, size_t* bytes, int64_t* eff_ranks,
                              double* compression);

/* Run the sweep (Alg.2 with MU or, with nmf = NTT_NMF_BCD, Alg.3 as the NMF; ranks given,
 * or chosen by the rule of Alg.2 when rank_eps > 0).
 *   workspace : device, >= ntt_plan_workspace bytes, 256-byte aligned; contents on
 *               entry are ignored, on exit unspecified.
 *   A         : n_1*...*n_d floats, read only (never written): device memory, or host
 *               memory when the plan's stream_cols > 0 (then copied in column blocks
 *               during the call; pinned memory gives the full copy rate).
 *   cores     : host array of d device pointers; cores[k] receives G_{k+1} as
 *               r_k x n_{k+1} x r_{k+1} floats (eff ranks).  Must not alias A or the
 *               workspace.
 *   init_W, init_H : NULL, or host arrays of d-1 device pointers giving W0 (m_l x r_l)
 *               and H0 (r_l x k_l) per stage instead of the seeded rule; an entry may
 *               be NULL to use the rule for that stage.
 *   objective_trace : NULL, or device doubles, one per iteration of every stage in
 *               order (sum over stages of max_iters); with NTT_RECORD_OBJECTIVE it
 *               receives f_t = 1/2||X_l - W_t H_t||^2 after each iteration t.
 *   report    : NULL or host struct filled on success.
 * Returns after the stream has finished the sweep. */
ntt_status ntt_decompose(ntt_plan_t plan, void* stream, void* workspace, const float* A,
                         float* const* cores, const float* const* init_W,
                         const float* const* init_H, double* objective_trace,
                         ntt_report* report);

/* Device bytes ntt_rel_error needs as workspace for a TT of this shape. */
ntt_status ntt_tt_workspace(int32_t d, const int64_t* dims, const int64_t* ranks, size_t* bytes);

/* Eq.(1)/(2): expand TT cores into the full tensor.
 *   dims, ranks : host, d and d+1 entries (r_0 = r_d = 1, every r_k <= NTT_MAX_RANK).
 *   cores       : host array of d device pointers, cores[k] is r_k x n_{k+1} x r_{k+1}.
 *   A_out       : device, n_1*...*n_d floats, written. */
ntt_status ntt_reconstruct(int32_t d, const int64_t* dims, const int64_t* ranks,
                           const float* const* cores, float* A_out, void* stream);

/* Eq.(3): *rel_err (host) = ||A - Ahat||_F / ||A||_F with Ahat the TT of `cores`, never
 * materialised: the last contraction is fused with a streaming read of A and the
 * squares are summed in FP64.  workspace: device, >= ntt_tt_workspace bytes.
 * Returns NTT_ERR_ZERO_NORM when ||A||_F = 0. */
ntt_status ntt_rel_error(int32_t d, const int64_t* dims, const int64_t* ranks, const float* A,
                         const float* const* cores, void* workspace, size_t workspace_bytes,
                         double* rel_err, void* stream);

/* ntt_rel_error for callers that cannot allocate device memory or pass a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and result as ntt_rel_error without the workspace: the partial sums go
 * to a fixed device array of NTT_REL_ERROR_STATIC_BYTES inside the library (one per GPU,
 * held until the process ends; its address is looked up once per device), so the call
 * allocates nothing.  Limit: n_1*...*n_{d-1} <= 33,554,368 (the 256^4 tensor has
 * 16,777,216); larger tensors return NTT_ERR_WORKSPACE_TOO_SMALL.  Every call overwrites
 * the array before reading it.  Calls that overlap on one GPU (other threads, or other
 * streams not ordered with this one) share the array and race: serialise them. */
#define NTT_REL_ERROR_STATIC_BYTES (8u << 20)
ntt_status ntt_rel_error_static(int32_t d, const int64_t* dims, const int64_t* ranks,
                                const float* A, const float* const* cores, double* rel_err,
                                void* stream);

/* Eq.(4) for arbitrary ranks (host only). */
double ntt_compression_ratio(int32_t d, const int64_t* dims, const int64_t* ranks);

/* ---- Batched mode: many independent decompositions of uneven shape and rank.
 * Not a step of the paper: a throughput mode over the same per-problem sweep.
 * Stage levels advance together; unfoldings with m <= 256, k <= 64, r <= 16 run all their
 * iterations in grouped single-workgroup launches (one workgroup per problem), the
 * rest replay per-problem iteration graphs on a pool of streams.  Problems share no
 * reduction, so each result is bitwise the same as when the problem is decomposed alone
 * with ntt_decompose.  */
typedef struct ntt_batch_s* ntt_batch_t;

/* One config per problem (same rules as ntt_plan; the RECORD/PROFILE/VALIDATE flags are
 * not accepted).  The arrays the configs point to are read during the call only. */
ntt_status ntt_batch_plan(int32_t count, const ntt_config* cfgs, ntt_batch_t* out);

/* Device workspace bytes for the whole batch (the sum of the problems' workspaces plus
 * a work-list area). */
ntt_status ntt_batch_workspace(ntt_batch_t batch, size_t* bytes);

/* Effective ranks of problem i (0 <= i < count): d+1 entries into eff_ranks (host), the
 * same values ntt_plan_workspace gives for that problem's config; core k of problem i
 * holds eff_ranks[k] x n_k x eff_ranks[k+1] floats. */
ntt_status ntt_batch_eff_ranks(ntt_batch_t batch, int32_t i, int64_t* eff_ranks);

/* Decompose every problem of the batch.
 *   A[i]       : device input of problem i (n_1...n_d floats, read only).
 *   cores[i][k]: device core k of problem i, as in ntt_decompose.
 *   reports    : NULL or `count` host reports.
 * Returns after the stream has finished all problems. */
ntt_status ntt_decompose_batch(ntt_batch_t batch, void* stream, void* workspace,
                               const float* const* A, float* const* const* cores,
                               ntt_report* reports);

void ntt_batch_destroy(ntt_batch_t batch);

/* ---- Serving: a persistent request engine with continuous batching.
 * Not a step of the paper: a serving mode over the same per-problem sweep.
 * The caller gives the server a device arena (the HBM budget).  Requests (host input,
 * ranks, iteration count) wait in a FIFO queue.  Each ntt_server_tick (non-blocking)
 * admits queued requests while a slot is free and the request's input + cores +
 * workspace fit in the arena (first-fit), starts the input copy on a copy stream, and
 * advances every admitted request whose previous block of work has finished by
 * iters_per_tick MU iterations; small unfoldings of all such requests go in one grouped
 * launch.  Factors stay on the device; results stay in the arena until released.  A
 * request's result does not depend on which other requests share the device. */
typedef struct ntt_server_s* ntt_server_t;

typedef struct {
  void* arena;            /* device, 256-byte aligned, owned by the caller */
  size_t arena_bytes;     /* HBM budget the server may use */
  int32_t max_slots;      /* requests admitted at once, 1..64 */
  int32_t iters_per_tick; /* MU iterations a request advances per tick (>= 1) */
} ntt_server_config;

typedef struct {
  int32_t d;
  const int64_t* dims;    /* host, read during ntt_server_submit */
  const int64_t* ranks;   /* host, read during ntt_server_submit */
  int32_t max_iters;
  double eps;
  uint64_t seed;
  int32_t precision;
  int32_t fp32_tail_iters;
  const float* host_A;    /* host input (pinned for an overlapped copy); must stay valid
                             until the request is running */
  int32_t nmf;            /* ntt_nmf: NTT_NMF_MU (0) or NTT_NMF_BCD (Alg.3, FP32 only) */
  double bcd_delta;       /* BCD: cap of the extrapolation weights, in [0, 1) */
} ntt_request;

enum {
  NTT_REQ_QUEUED = 0,
  NTT_REQ_RUNNING = 1,
  NTT_REQ_DONE = 2,
  NTT_REQ_REJECTED = 3,   /* needs more than the whole arena */
  NTT_REQ_CANCELLED = 4
};

typedef struct {
  int64_t id;
  int32_t state;
  int32_t d;
  double t_submit, t_admit, t_start, t_finish; /* seconds since the server was created */
  size_t device_bytes;                         /* input + cores + workspace in the arena */
  double gflop;                                /* algorithmic GFLOP of the request */
  int64_t eff_ranks[NTT_MAX_DIMS + 1];
} ntt_request_info;

ntt_status ntt_server_create(const ntt_server_config* cfg, ntt_server_t* out);
/* Queue a request (host only); *id identifies it. */
ntt_status ntt_server_submit(ntt_server_t server, const ntt_request* req, int64_t* id);
/* One scheduler step (never waits for the device); reports running and queued counts. */
ntt_status ntt_server_tick(ntt_server_t server, int32_t* n_active, int32_t* n_queued);
ntt_status ntt_server_info(ntt_server_t server, int64_t id, ntt_request_info* info);
/* Device pointers of a finished request's d cores (valid until ntt_server_release). */
ntt_status ntt_server_cores(ntt_server_t server, int64_t id, float** core_ptrs);
/* Free a request's arena memory; cancels it if it is queued or running. */
ntt_status ntt_server_release(ntt_server_t server, int64_t id);
/* Free bytes left in the arena. */
ntt_status ntt_server_free_bytes(ntt_server_t server, size_t* bytes);
void ntt_server_destroy(ntt_server_t server);

void ntt_plan_destroy(ntt_plan_t plan);
const char* ntt_status_string(ntt_status s);
const char* ntt_last_error(void);
/* Library version string, e.g. "ntt-mi355x 0.1 gfx950". */
const char* ntt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NTT_H_ */
