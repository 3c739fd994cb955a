/*
 * s2w -- source-to-waveform map on one GPU's share of the seafloor grid.
 *
 * The map (paper Sec. II-B, eqs. 1-3) takes slip-rate histories s on Nsub
 * fault subfaults to pressure waveforms q at Nobs observation points:
 *
 *   m_n = sum_{k=0}^{n} F_{G,k} s_{n-k}     elastic response, eq. (1)
 *   v   = D_t m                             temporal difference per grid point
 *   q_n = sum_{k=0}^{n} F_{q,k} v_{n-k}     waveform response, eq. (2)
 *
 * restricted to the Ngrid seafloor points of one share I_r (opposite row /
 * column partitions, Sec. II-C): the result is one rank's term
 * F_q^(r) D_t F_G^(r) s of eq. (3); the sum over ranks is the caller's.
 * Both block lower-triangular Toeplitz products are evaluated by zero-padding
 * the time axis and diagonalising it with a real FFT (Alg. 2), the seafloor
 * field staying on the device between them (Alg. 1).
 *
 * D_t: the paper leaves the difference stencil unspecified (Sec. II-B2).
 * S2W_DIFF_BACKWARD applies v_n = (m_n - m_{n-1})/dt with m_{-1} = 0 (causal,
 * Toeplitz); S2W_DIFF_NONE makes D_t the identity.
 *
 * Conventions for every entry point:
 *  - All device pointers must be 256-byte aligned and distinct.  The caller
 *    allocates every byte of device memory (operator store, workspace, inputs,
 *    outputs); the library never allocates device memory.
 *  - Every call validates its arguments on the host before enqueuing
 *    anything; an invalid call returns an error and enqueues nothing.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *    and is asynchronous: a call returns before the GPU finishes.  Forward
 *    and adjoint allocate nothing and do not synchronise, so they may be
 *    captured into a HIP graph.  One plan is used by one stream at a time.
 *  - Failures never throw across this boundary; they return a status, and
 *    s2w_last_error() gives the message of the plan's most recent failure.
 *  - NaN or Inf in inputs or operators propagate; they are not checked.
 */
#ifndef S2W_H
#define S2W_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define S2W_ABI_VERSION 6

typedef struct s2w_plan s2w_plan;

typedef enum s2w_status {
  S2W_OK = 0,
  S2W_EINVAL = 1,        /* bad argument: null/misaligned pointer, size, batch out of range */
  S2W_ENOMEM = 2,        /* bound operator store or workspace smaller than s2w_query_sizes asks */
  S2W_ESTATE = 3,        /* call out of order: memory not bound, operators not fully set */
  S2W_EUNSUPPORTED = 4,  /* valid request the library does not implement (dtype, size limit) */
  S2W_EHIP = 5           /* a HIP runtime call or kernel launch failed; see s2w_last_error */
} s2w_status;

typedef enum s2w_dtype {
  S2W_F32 = 0,   /* complex64 spectra */
  S2W_BF16 = 1,  /* bfloat16 real/imaginary parts with one float32 power-of-two scale per (grid row, bin) */
  S2W_F16 = 2    /* float16 real/imaginary parts with one float32 power-of-two scale per (grid row, bin) */
} s2w_dtype;

typedef enum s2w_diff { S2W_DIFF_NONE = 0, S2W_DIFF_BACKWARD = 1 } s2w_diff;

/* Matrix-core products of the bfloat16 stores (float16 stores always take float16 products;
 * products accumulate in float32 always).
 *  AUTO  as F16.
 *  BF16  bfloat16 products; each float32 activation value enters as a high and a low
 *        bfloat16 term (two products, about 16 significant bits).
 *  F16   float16 products: bfloat16 operator words are converted to float16 in registers,
 *        exactly for every word within 2^31 of its row's largest (the power-of-two row scales
 *        keep that largest in [2^14, 2^15]); each activation value enters as one float16 term
 *        (11 significant bits) under a power-of-two scale per (bin, rupture).  Half the
 *        products and activation bytes of BF16. */
typedef enum s2w_products {
  S2W_PRODUCTS_AUTO = 0,
  S2W_PRODUCTS_BF16 = 1,
  S2W_PRODUCTS_F16 = 2
} s2w_products;

/* Storage of the spectra and the kernels that go with it.
 *  SINGLE   float32 only: each (grid row, column) spectrum contiguous over the bins; forward
 *           runs one fused streaming kernel per rupture (the seafloor field stays on chip),
 *           B ruptures as B such passes.  Best for B = 1.
 *  BATCHED  per-bin operator matrices (grid row, bin, column) for matrix-core GEMMs over all
 *           B ruptures of a call; the seafloor field of the batch goes through the workspace.
 *           The only layout of the half-precision stores.
 *  DIRECT   float32 only, no FFT: the time-domain blocks are stored as given (each series
 *           padded with zero lags to a multiple of 16) and forward/adjoint evaluate the
 *           defining sums of eqs. (1)-(2) in the channel form of eq. (4), the paper's direct
 *           reference evaluation (Sec. II-C2), on the float32 matrix cores: Nt(Nt+1)/2 lag
 *           products per (row, column) pair instead of one complex product per bin, so about
 *           2*Nt/(log2 L) times the FFT path's arithmetic.  The seafloor field is differenced
 *           in the time domain between the two products; B ruptures run as B passes.
 *           Operator store: (Nsub + Nobs) * Ngrid * ntp * 4 bytes, ntp = Nt rounded up to 16.
 *  AUTO     BATCHED for half-precision stores or max_batch >= 8, else SINGLE. */
typedef enum s2w_layout {
  S2W_LAYOUT_AUTO = 0,
  S2W_LAYOUT_SINGLE = 1,
  S2W_LAYOUT_BATCHED = 2,
  S2W_LAYOUT_DIRECT = 3
} s2w_layout;

/* Problem description.  Limits of the library: 1 <= nt <= 512, 1 <= nsub <= 1024,
 * 1 <= nobs <= 256, 1 <= ngrid, 0 <= max_batch <= 1024. */
typedef struct s2w_desc {
  int32_t nsub;       /* Nf: fault subfaults (columns of F_{G,k}) */
  int32_t ngrid;      /* N_m^(r): seafloor points of this share (rows of F_{G,k}, columns of F_{q,k}) */
  int32_t nobs;       /* N_q: observation points (rows of F_{q,k}) */
  int32_t nt;         /* N_t: time steps */
  int32_t max_batch;  /* largest number of ruptures per forward/adjoint call */
  int32_t diff;       /* s2w_diff */
  int32_t g_dtype;    /* s2w_dtype of the stored elastic spectra */
  int32_t f_dtype;    /* s2w_dtype of the stored acoustic-gravity spectra */
  double dt;          /* time step in seconds (> 0); enters only through D_t */
  int32_t layout;     /* s2w_layout */
  int32_t products;   /* s2w_products; must be 0 for float32 stores */
} s2w_desc;

/* Create a plan for `desc` on HIP device `device`.  Host-side only: no device
 * memory is allocated.  *out receives the plan (NULL on failure). */
s2w_status s2w_plan_create(const s2w_desc* desc, int32_t device, s2w_plan** out);

/* Destroy a plan.  The caller must have synchronised the streams that used it.
 * The bound memory is the caller's and is not freed.  NULL is a no-op. */
s2w_status s2w_plan_destroy(s2w_plan* plan);

/* Bytes of device memory the plan needs: the persistent operator store (the
 * frequency-domain blocks of Alg. 2, resident between calls) and the scratch
 * workspace used by set_operators, forward and adjoint at up to max_batch. */
s2w_status s2w_query_sizes(const s2w_plan* plan, uint64_t* operator_bytes, uint64_t* workspace_bytes);

/* Give the plan its memory.  Both regions stay owned by the caller and must
 * outlive every call that uses the plan.  Sizes below s2w_query_sizes give
 * S2W_ENOMEM.  Re-binding discards all operators set so far. */
s2w_status s2w_bind_memory(s2w_plan* plan, void* operator_store, uint64_t operator_bytes, void* workspace,
                           uint64_t workspace_bytes);

/* One-time setup (excluded from the paper's timings, Sec. III-C): transform
 * the time-domain blocks of grid rows [row0, row0+nrows) and keep their
 * spectra in the operator store.  Device inputs, row-major float32:
 *   G_chunk[r][j][k] = [F_{G,k}]_{row0+r, j}   shape [nrows][nsub][nt]   (eq. 1)
 *   F_chunk[r][o][k] = [F_{q,k}]_{o, row0+r}   shape [nrows][nobs][nt]   (eq. 2)
 * Chunks may arrive in any order and may overlap (later wins); the inputs may
 * be freed once `stream` has passed this call.  Forward and adjoint require
 * every row to have been set since the last bind. */
s2w_status s2w_set_operators(s2w_plan* plan, const float* G_chunk, const float* F_chunk, int64_t row0, int64_t nrows,
                             void* stream);

/* Forward map for B ruptures (0 <= B <= max_batch; B = 0 enqueues nothing):
 *   s[b][j][n]  slip rate, float32 [B][nsub][nt] (device)
 *   y[b][o][n]  this share's partial waveforms F_q^(r) D_t F_G^(r) s, float32 [B][nobs][nt] (device, overwritten)
 * Deterministic: identical inputs give bit-identical outputs. */
s2w_status s2w_forward(s2w_plan* plan, const float* s, int32_t B, float* y, void* stream);

/* Forward map that also returns the share's seafloor displacement, the intermediate field of
 * eq. (1) (Sec. III-C shows it beside the waveforms), from the same pass: the displacement is
 * written where the mid-chain forms it (the first product's inverse transform truncated to
 * n < nt, before D_t; on the direct layout the time-domain sum), so the elastic store is read
 * once for both outputs.
 *   s[b][j][n]   as s2w_forward;  y[b][o][n] as s2w_forward
 *   m[b][g][i]   float32 [B][ngrid][ntimes] (device, 256-byte aligned, distinct from s and y):
 *                m_n at grid row g of the share, n = times[i]:
 *                m_n = sum_j sum_{k<=n} [F_{G,k}]_{g,j} s_{j,n-k}
 *   times        host array of ntimes steps, strictly increasing, each in [0, nt); or NULL with
 *                ntimes = nt for every step.  Read during the call only.
 * Every layout and store precision has it; the displacement carries the precision of the
 * path's elastic store (float32, or the bf16/f16 rounding of a half store).  y is identical,
 * bit for bit, to s2w_forward's.  Invalid time lists give S2W_EINVAL before any enqueue. */
s2w_status s2w_forward_displacement(s2w_plan* plan, const float* s, int32_t B, float* y, float* m,
                                    const int32_t* times, int32_t ntimes, void* stream);

/* Adjoint (transpose) of the forward map as a real linear operator, including
 * the transpose of D_t: gs = A^T r, so that for L = 0.5 ||A s - y_obs||^2 the
 * gradient is dL/ds = adjoint(A s - y_obs).
 *   r[b][o][n]   float32 [B][nobs][nt] (device)
 *   gs[b][j][n]  float32 [B][nsub][nt] (device, overwritten)
 * Every layout and store precision has it.  With half-precision stores the residual and the
 * mid-chain output enter the matrix cores as half terms the same way the slip spectra do in
 * the forward map (a high and a low bfloat16 term, or one scaled float16 term), so the
 * adjoint's error is of the forward map's order. */
s2w_status s2w_adjoint(s2w_plan* plan, const float* r, int32_t B, float* gs, void* stream);

/* Forward map without the bound workspace, for callers that cannot allocate device memory
 * or call into an allocator at all (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and validation as s2w_forward,
 * bit for bit; the operator store must still be bound and set.  Its scratch (the source
 * spectrum, the per-workgroup partial spectra of the fused kernel and their sum) lives in a
 * fixed device array of S2W_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends; no call allocates or frees anything.
 * Limits: single-layout (float32) plans whose fused kernel fits the array, i.e.
 * (M*nsp + nwg*M*nop + nop*M) * 8 bytes, each term rounded up to 256, is at most
 * S2W_NOALLOC_SCRATCH_BYTES, with M = L/2 slots, nsp / nop = nsub / nobs rounded up to even,
 * nwg = compute units x fused_wg_per_cu (the Cascadia-sized share, 963 x 37,760 x 64 x 256
 * at one workgroup per CU, needs 35.6 MB); larger plans, batched or half-precision plans and
 * plans whose observers need the unfused kernel get S2W_EUNSUPPORTED with the byte count in
 * s2w_last_error, before anything is enqueued.
 * Concurrency: every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (two streams, or two plans, at once) race and corrupt each other's results; serialize
 * them.  Nothing in the array needs clearing between calls: each call writes every byte it
 * reads before reading it. */
#define S2W_NOALLOC_SCRATCH_BYTES (64u << 20)
s2w_status s2w_forward_noalloc(s2w_plan* plan, const float* s, int32_t B, float* y, void* stream);

/* Kernel-shape controls for the tuner.  Zero fields keep the library default. */
typedef struct s2w_tuning {
  int32_t fused_wg_per_cu;   /* single-rupture fused kernel: workgroups per compute unit (1..4) */
  int32_t fused_rows;        /* single-rupture fused kernel: grid rows per tile (4 or 8) */
  int32_t adj_cols;          /* grid-row contractions (adjoint elastic stage): columns per thread (8 or 16) */
  int32_t adj_splits;        /* single-rupture adjoint: grid splits of the transposed elastic stage */
  int32_t batch_path_min_b;  /* reserved: ignored (the layout, fixed at plan creation, picks the path) */
  int32_t gemm_cfg;          /* batched elastic GEMM tile, 256 grid rows tall, persistent workgroups:
                                -1 automatic (12 for B <= 64, else 18; with float16 products on
                                bfloat16 words 16 and 24); 4 = 16 columns (four waves,
                                register operands); 10 = 256 columns (eight waves, three-stage LDS copy
                                pipeline); 12 = 128 columns (eight waves, four stages); 16 = 128 columns
                                (four waves, two stages, two workgroups per compute unit); 17, 18 = 256
                                columns on real-column activation fragments (eight waves, four and three
                                stages); 24 = 256 columns (eight waves of 64 x 128, three stages).
                                A rupture takes two columns (real and imaginary part).  All tiles
                                give the same results bit for bit. */
  int32_t fgemm_splits;      /* batched acoustic GEMM: grid-row splits (1..16) */
  int32_t fgemm_lds;         /* batched acoustic GEMM: 1 automatic (LDS-staged kernel for bfloat16 products
                                with B <= 64 where its tile fits, else the eight-wave kernel on
                                real-column activation fragments), 2 eight-wave kernel on full
                                fragments, 3 eight-wave kernel on real-column fragments (2 and 3 give the
                                same results bit for bit), 4 LDS-staged kernel on packed bfloat16
                                activations where its tile fits (else, and for float16 products, as 3) */
  int32_t gemm32_cfg;        /* batched float32 GEMMs over grid rows (forward elastic, adjoint acoustic): tile,
                                -1 automatic, 1..4 = rows x ruptures 64 x 128, 128 x 32, 256 x 8, 64 x 64 */
  int32_t gemm32_cfg_k;      /* batched float32 forward acoustic GEMM (reduces over grid rows): tile, same
                                values (automatic: 256 x 8 for B <= 8, 64 x 64 up to B = 64, 64 x 128
                                beyond) */
  int32_t gemm32_splits;     /* batched float32 acoustic GEMM: grid-row splits (1..16) */
  int32_t adj32_splits;      /* batched adjoint (float32 and half stores), transposed elastic GEMM: grid-row
                                splits (1..8; half stores may clamp to what the partial region holds) */
  int32_t hadj_tile_f;       /* half-precision adjoint, transposed acoustic GEMM tile (eight waves, both
                                operands through LDS): -1 automatic, 3 = 256 x 64 rows x columns, 4 =
                                256 x 128, then 6..8 = 256 x 64, 256 x 128, 256 x 256 holding only
                                real-column activation fragments in LDS (same results bit for bit) */
  int32_t hadj_tile_g;       /* half-precision adjoint, transposed elastic GEMM tile: same values */
  int32_t mid_rupts;         /* batched mid-chain (Nt = 256): ruptures per work unit, 16 or 32 */
  int32_t adj32_cfg;         /* batched float32 adjoint, transposed elastic GEMM (reduces over grid rows):
                                tile, values as gemm32_cfg (automatic: 256 x 8 for B <= 8, 128 x 32 up
                                to B = 64, 64 x 128 beyond) */
} s2w_tuning;

s2w_status s2w_set_tuning(s2w_plan* plan, const s2w_tuning* t);
s2w_status s2w_get_tuning(const s2w_plan* plan, s2w_tuning* t);

/* Measurement hook: when both events are non-NULL (hipEvent_t), the next
 * forward/adjoint calls record `begin` immediately before and `end` immediately
 * after their dominant kernel (the one streaming the elastic spectra), on the
 * call's stream.  Pass NULLs to stop.  Events are created and owned by the caller. */
s2w_status s2w_set_profile_events(s2w_plan* plan, void* begin, void* end);

/* Padded transform length L (a power of two >= 2*nt - 1, at least 32) and the
 * number of stored complex values per spectrum, L/2 (bins 0 and L/2 are real
 * and share one slot). */
s2w_status s2w_transform_length(const s2w_plan* plan, int32_t* L);

/* ---------------------------------------------------------------------------------------
 * One block lower-triangular Toeplitz operator on its own (Alg. 2, Sec. II-C1):
 *   y_n = sum_{k=0}^{n} F_k x_{n-k},  F_k in R^{nrow x ncol},  n < nt,
 * evaluated by zero-padding to L, a real FFT, one complex product per bin and the inverse
 * FFT truncated to nt.  With F_k = F_{G,k} restricted to a share's rows this gives the
 * seafloor displacement of eq. (1) (x = slip rate, y = displacement per grid row); with
 * F_k = F_{q,k} restricted to a share's columns, eq. (2) (x = seafloor motion, y = the
 * share's partial waveforms).  Float32 spectra in a per-bin GEMM layout; products on the
 * matrix cores for every batch size.  The conventions of the map's entry points apply
 * (caller-owned 256-byte aligned device memory, host-side validation before any enqueue,
 * asynchronous on `stream`, no allocation, deterministic, no exceptions).
 * Limits: 1 <= nt <= 512, 1 <= nrow, ncol <= 2^24, 0 <= max_batch <= 1024. */
typedef struct s2w_bltt s2w_bltt;

typedef struct s2w_bltt_desc {
  int32_t nrow;       /* rows of each block F_k (output channels) */
  int32_t ncol;       /* columns of each block F_k (input channels) */
  int32_t nt;         /* time steps */
  int32_t max_batch;  /* largest number of input histories per call */
} s2w_bltt_desc;

s2w_status s2w_bltt_create(const s2w_bltt_desc* desc, int32_t device, s2w_bltt** out);
s2w_status s2w_bltt_destroy(s2w_bltt* op);
s2w_status s2w_bltt_query_sizes(const s2w_bltt* op, uint64_t* operator_bytes, uint64_t* workspace_bytes);
/* Same contract as s2w_bind_memory; re-binding discards the blocks set so far. */
s2w_status s2w_bltt_bind_memory(s2w_bltt* op, void* operator_store, uint64_t operator_bytes, void* workspace,
                                uint64_t workspace_bytes);
/* Spectra of rows [row0, row0+nrows): F_chunk[r][c][k] = [F_k]_{row0+r, c}, float32
 * [nrows][ncol][nt] (device, row-major).  Chunks in any order; apply and adjoint require
 * every row to have been set since the last bind. */
s2w_status s2w_bltt_set_blocks(s2w_bltt* op, const float* F_chunk, int64_t row0, int64_t nrows, void* stream);
/* y[b][r][n] = sum_c sum_{k<=n} [F_k]_{r,c} x[b][c][n-k]: x float32 [B][ncol][nt], y float32 [B][nrow][nt]. */
s2w_status s2w_bltt_apply(s2w_bltt* op, const float* x, int32_t B, float* y, void* stream);
/* Transpose: x[b][c][n] = sum_r sum_{k<nt-n} [F_k]_{r,c} y[b][r][n+k]. */
s2w_status s2w_bltt_adjoint(s2w_bltt* op, const float* y, int32_t B, float* x, void* stream);
const char* s2w_bltt_last_error(const s2w_bltt* op);

/* The layout of the plan: S2W_LAYOUT_SINGLE, S2W_LAYOUT_BATCHED (AUTO resolves to one of these)
 * or S2W_LAYOUT_DIRECT. */
s2w_status s2w_plan_layout(const s2w_plan* plan, int32_t* layout);

const char* s2w_status_string(s2w_status st);
const char* s2w_last_error(const s2w_plan* plan);
int32_t s2w_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* S2W_H */
