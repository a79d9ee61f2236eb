/*
 * camelot.h - C ABI of libcamelot, an MI355X (gfx950) runtime for pipelines of GPU
 * microservices co-located on one GPU under spatial CU partitioning.
 *
 * What the library implements (Zhang et al., "Towards QoS-Aware and
 * Resource-Efficient GPU Microservices Based on Spatial Multitasking GPUs In
 * Datacenters", arXiv 2005.02088):
 *   - global-memory communication between pipeline stages on one GPU (Section VI-B):
 *     here a device-global ring buffer with doorbell flags between persistent stage
 *     workers, one copy of the data, no host round trip; the host-staged
 *     (device->host->device) path of Section VI-A is kept as the baseline;
 *   - the allocation problems of Section VII: maximise the supported peak load under
 *     the QoS target (Eq. 1) and minimise the computational resources at low load
 *     (Eq. 3), solved exactly over a measured integer profile table;
 *   - the query flow of Section V-B: a wait queue, batch formation, per-stage
 *     processing on the stage's CU share.
 *
 * Conventions (every entry point):
 *   - Return value: CAMELOT_OK (0) or a negative camelot_status. No entry point
 *     aborts or throws; camelot_last_error() returns a thread-local message
 *     describing the last failure on the calling thread.
 *   - Pointers are host pointers unless the parameter says "device". Device
 *     pointers are plain HIP device allocations (hipMalloc or a PyTorch tensor's
 *     data pointer) on the current device.
 *   - The caller owns every buffer it passes; the library never frees them.
 *     Objects the library creates (pipelines, streams, rings) are released by the
 *     matching destroy call.
 *   - Streams are hipStream_t passed as void*; NULL means the library's own stream.
 *   - Allocation entry points are pure host computations: deterministic, the same
 *     inputs give the same bytes out, no GPU needed.
 */
#ifndef CAMELOT_H
#define CAMELOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef enum {
  CAMELOT_OK = 0,
  CAMELOT_EINVAL = -1,       /* bad argument (message says which)                    */
  CAMELOT_ENOMEM = -2,       /* device/host allocation failed or footprint > budget  */
  CAMELOT_EAGAIN = -3,       /* ingest queue full: back-pressure, retry later        */
  CAMELOT_ETIMEDOUT = -4,    /* a wait ran past its limit (host or device side)      */
  CAMELOT_EINFEASIBLE = -5,  /* no allocation satisfies the constraints              */
  CAMELOT_EDEVICE = -6,      /* a HIP call failed or a device worker reported error  */
  CAMELOT_ESTOPPED = -7      /* pipeline already stopped / workers exited            */
} camelot_status;

/* Thread-local description of the last error on this thread ("" if none). */
const char* camelot_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t camelot_version(void);

/* ------------------------------------------------------------------ device info */
typedef struct {
  int32_t n_cus;             /* compute units (256 on MI355X)                        */
  int32_t n_xcds;            /* XCDs (8); CU-mask bit i lands on XCD i % n_xcds      */
  int64_t wall_clock_hz;     /* rate of the device's constant wall clock             */
  int64_t hbm_bytes;         /* device memory capacity                               */
  char arch[32];             /* e.g. "gfx950"                                        */
} camelot_device_info;

/* Fills *out for the current device. */
int32_t camelot_device_query(camelot_device_info* out);

/* ------------------------------------------------------------------ allocation
 * Section VII, Eq. 1 and Eq. 3 over an integer profile table.
 *
 * Decision variables per stage i: instance count N_i (1..max_inst_per_stage, or
 * 1..inst_max[i] when inst_max is given) and
 * CU share p_i = (k_i + 1) * cu_step (k_i = 0 .. cu_total/cu_step - 1); one batch
 * size b = batches[j] for the whole pipeline.
 * Throughput T = min_i N_i * b * 1e9 / lat_ns[i][k_i][j]   (queries/s, exact rational)
 * Constraints (Eq. 1 / Eq. 3):
 *   sum N_i p_i <= cu_total; sum N_i <= max_instances;
 *   sum N_i bw_bps[i][k_i][j] <= hbm_bw_budget; sum N_i mem_bytes[i][j] <= hbm_bytes_budget;
 *   batch_wait_ns[j] + sum lat_ns[i][k_i][j] <= qos_ns.
 * A table entry lat_ns <= 0 marks an unmeasured point, never chosen.
 * Ties: peak -> larger T, fewer CUs, lower latency, then the lexicographically
 * smallest (j, N_1, k_1, N_2, k_2, ...); min -> fewer CUs, larger T, lower latency,
 * lexicographic.  Results are exact: integer tables, 128-bit cross-multiplied
 * rational comparisons.
 * Table layouts: lat_ns and bw_bps are [n_stages][cu_total/cu_step][n_batches]
 * row-major int64; mem_bytes is [n_stages][n_batches]; batch_wait_ns is
 * [n_batches] or NULL (all zero); inst_max is [n_stages] or NULL (every stage
 * bounded by max_inst_per_stage alone). All owned by the caller, read only.
 */
#define CAMELOT_MAX_STAGES 8
#define CAMELOT_MAX_INSTANCES 6     /* instances of one pipeline stage              */
#define CAMELOT_MAX_WORKERS 16      /* stage instances of one pipeline in total     */

typedef struct {
  int32_t n_stages;            /* 1..CAMELOT_MAX_STAGES                              */
  int32_t cu_total;            /* R: CUs available (<= 256)                          */
  int32_t cu_step;             /* share granularity; cu_total % cu_step == 0         */
  int32_t max_instances;       /* I: cap on sum of N_i (Eq. 1 constraint 2)          */
  int32_t max_inst_per_stage;  /* search bound on each N_i (<= max_instances)       */
  int32_t n_batches;           /* >= 1                                               */
  const int32_t* batches;      /* [n_batches], each >= 1                             */
  int64_t qos_ns;              /* latency target                                     */
  int64_t hbm_bytes_budget;    /* F                                                  */
  int64_t hbm_bw_budget;       /* BW, bytes/s                                        */
  const int64_t* lat_ns;
  const int64_t* bw_bps;
  const int64_t* mem_bytes;
  const int64_t* batch_wait_ns;
  const int32_t* inst_max;     /* per-stage bound on N_i, each >= 1, or NULL         */
} camelot_problem;

typedef struct {
  int32_t n_stages;
  int32_t batch;               /* chosen b                                           */
  int32_t batch_index;         /* its index in problem.batches                       */
  int32_t n[CAMELOT_MAX_STAGES];   /* instances per stage                            */
  int32_t cu[CAMELOT_MAX_STAGES];  /* CUs per instance                               */
  int64_t thr_num, thr_den;    /* T = thr_num / thr_den queries/s, gcd-reduced       */
  int64_t lat_ns;              /* batch_wait + sum of stage latencies                */
  int64_t cu_used;             /* sum N_i * cu_i                                     */
} camelot_alloc;

/* Eq. 1: maximise T. CAMELOT_EINFEASIBLE when no point satisfies the constraints. */
int32_t camelot_alloc_peak(const camelot_problem* problem, camelot_alloc* out);

/* Eq. 3 with the load constraint T >= load_num / load_den (queries/s):
 * minimise sum N_i p_i. CAMELOT_EINFEASIBLE when no point reaches the load. */
int32_t camelot_alloc_min(const camelot_problem* problem, int64_t load_num,
                          int64_t load_den, camelot_alloc* out);

/* Evaluate one given point (instances/shares in *inout, batch_index set): fills
 * thr/lat/cu_used and returns CAMELOT_OK if it satisfies every constraint,
 * CAMELOT_EINFEASIBLE otherwise (fields still filled when the table has the point). */
int32_t camelot_alloc_eval(const camelot_problem* problem, camelot_alloc* inout);

/* Section VII-C's solver for both problems: simulated annealing over V = (batch
 * index, N_1..N_S, share index k_1..k_S), for search spaces too large to enumerate
 * (many stages and instances). Each of `iters` iterations moves one coordinate of
 * V by +-1 (coordinate and direction uniform, a move off the grid is no move); a
 * candidate that breaks a constraint is rejected (while the current state itself is
 * invalid every move is taken); a better or equal valid one is taken, a worse one
 * with probability exp(-d / temp), d the relative loss (CAMELOT_OBJ_PEAK: relative
 * throughput drop; CAMELOT_OBJ_MIN: relative growth of the CUs in use, with
 * throughput >= load_num / load_den as a constraint), temp = 0.3 * 0.95^(t / 100)
 * (integer division). Start: the largest batch, N_i = 1, k_i = K / S - 1. The best
 * valid state seen is returned, compared with camelot_alloc_peak's /
 * camelot_alloc_min's tie rules. Randomness: one SplitMix64 stream seeded with
 * `seed` (a draw for the coordinate, mod 2S + 1, one for the direction, its low
 * bit, and one for u = (draw >> 11) / 2^53 only when a worse valid candidate is
 * tested), so the result is a deterministic function of (problem, objective, load,
 * iters, seed). It may miss the optimum camelot_alloc_peak/min finds; it never
 * returns an invalid allocation. EINFEASIBLE if no valid state was visited. */
enum { CAMELOT_OBJ_PEAK = 0, CAMELOT_OBJ_MIN = 1 };
int32_t camelot_alloc_sa(const camelot_problem* problem, int32_t objective, int64_t load_num,
                         int64_t load_den, int32_t iters, uint64_t seed, camelot_alloc* out);

/* ------------------------------------------------------------------ stages
 * The synthetic microservice stages. Row = one query. All activations are
 * row-major [rows][dim].
 *   GEMM_RELU    in f32[in_dim], out f32[out_dim] = max(0, x W); weights[0] = W f32
 *                [in_dim][out_dim] row-major ([in, out]).
 *   GEMM_ARGMAX  in f32[in_dim]; s = x W with W f32 [in_dim][out_dim]; output is a
 *                result of k = 1: (argmax, max score), lowest index on ties.
 *   LOGMEL       in f32[2000] (16 kHz); 11 frames of 400 (hop 160), Hamming window,
 *                512-point FFT power, 40 HTK mel bands over 0..8 kHz,
 *                ln(max(E, 1e-10)); out f32[440] frame-major. No weights.
 *   MLP_BF16     in f32[dims[0]] rounded to BF16 (nearest-even); layers l = 1..L with
 *                weights[l-1] BF16 [dims[l]][dims[l-1]] ([out, in]);
 *                hidden h_l = bf16(max(0, h_{l-1} W_l^T)), FP32 accumulation;
 *                out f32[dims[L]] = h_{L-1} W_L^T (no rounding). dims[l] % 16 == 0
 *                for l >= 1 and dims[l] % 8 == 0 for all l.
 *   TOPK         in f32[in_dim]; output is a result of k entries (index, value) in
 *                descending value, equal values by ascending index.
 *   GATHER       in int32[dims[0]] row ids; weights[0] = FP16 table [k][dims[1]] (k rows,
 *                dims[1] <= 1024, a multiple of 64); out f32[dims[1]] = mean over the
 *                ids of table[id] (FP32 sums in id order). Ids outside [0, k) add zero.
 *   CONV_POOL    in BF16 feature map [dims[0]=H][dims[1]=W][dims[2]=C] (NHWC, C = 64);
 *                weights[0] = BF16 [dims[3]=Cout=64][3][3][C] ([out][ky][kx][in]);
 *                out f32[Cout] = mean over the H*W pixels of max(0, 3x3 convolution,
 *                stride 1, zero padding 1), FP32 accumulation on MFMA.
 *   GATHER_SCORE in f32[dims[0] = heads * dims[1]] query vectors; the row's side bytes
 *                (camelot_pipeline_config.side_bytes, or the input row's tail in
 *                camelot_stage_run) hold int32 ids[dims[2]]; weights[0] = FP16 table
 *                [k][dims[1]]; out f32[heads * dims[2]], score[h * dims[2] + j] =
 *                sum_d q[h * dims[1] + d] * table[id_j][d]; ids outside [0, k) score 0.
 *   ARTIFACT_P / ARTIFACT_M  the artifact suite's PCIe- and memory-intensive stages
 *                (Section III-B, Section VIII-E): in and out u32[D], D = dims[0] (a
 *                multiple of 1024, <= 16384); weights[0] = a table of k u32 words:
 *                pinned host memory read over the host link (P; a device-accessible
 *                host pointer) or device memory (M); dims[1] = words read per row (the
 *                intensity; a multiple of D, <= k). Block b = in[0] mod (k / dims[1])
 *                of the table (words b dims[1] .. + dims[1]) is folded into D words by
 *                XOR (fold[j] = XOR over t of block[t D + j]); P outputs in[j] ^
 *                fold[j]; M outputs f32: ((in[j] ^ fold[j]) >> 8) * 2^-24.
 *   ARTIFACT_C   the compute-intensive stage: in and out u32[D], D = dims[0] (a
 *                multiple of 1024, <= 16384); word w -> x = f32 with bits
 *                (w >> 9) | 0x3F800000 (a value in [1, 2)), then dims[1] times (the
 *                intensity, 0..2^20) x = (x * (1 - 2^-11)) + 2^-10, the product and
 *                the sum each rounded to FP32 (no fused multiply-add); out = the bits of
 *                x. No weights.
 * GEMM_ARGMAX and TOPK produce results and must be the last stage of a pipeline.
 */
typedef enum {
  CAMELOT_STAGE_GEMM_RELU = 1,
  CAMELOT_STAGE_GEMM_ARGMAX = 2,
  CAMELOT_STAGE_LOGMEL = 3,
  CAMELOT_STAGE_MLP_BF16 = 4,
  CAMELOT_STAGE_TOPK = 5,
  CAMELOT_STAGE_GATHER = 6,
  CAMELOT_STAGE_CONV_POOL = 7,
  CAMELOT_STAGE_GATHER_SCORE = 8,
  CAMELOT_STAGE_ARTIFACT_P = 9,
  CAMELOT_STAGE_ARTIFACT_C = 10,
  CAMELOT_STAGE_ARTIFACT_M = 11
} camelot_stage_kind;

#define CAMELOT_MAX_LAYERS 8
#define CAMELOT_MAX_K 128
#define CAMELOT_MAX_BATCH 128

typedef struct {
  int32_t kind;                          /* camelot_stage_kind                       */
  int32_t n_layers;                      /* MLP_BF16: L; GEMM_*: 1; others 0          */
  int32_t dims[CAMELOT_MAX_LAYERS + 1];  /* dims[0] = in_dim, dims[n_layers] = out   */
  int32_t k;                             /* TOPK: k (1..CAMELOT_MAX_K); GATHER: table rows */
  const void* weights[CAMELOT_MAX_LAYERS]; /* device pointers, borrowed for the
                                              lifetime of any object using them      */
} camelot_stage_desc;

/* Bytes of one input row / one output row of a stage (result stages: k entries of
 * int32 index + f32 value = 8 * k bytes). Returns < 0 on a bad descriptor. */
int64_t camelot_stage_row_bytes_in(const camelot_stage_desc* stage);
int64_t camelot_stage_row_bytes_out(const camelot_stage_desc* stage);

/* GATHER_SCORE reads its ids from the side bytes: in camelot_stage_run each input row
 * is row_bytes_in + 4 * dims[2] bytes (the ids follow the query vectors). */
/* Run one stage over `rows` rows (0..CAMELOT_MAX_BATCH) on `n_cus` CUs starting
 * at CU-mask bit `cu_offset` (n_cus and cu_offset multiples of 8; 0 n_cus = all
 * CUs), `reps` times back to back (the same input each time), with the compute
 * code and compute grid of the persistent worker (one workgroup per CU; one
 * kernel launch, grid barriers between reps; a pipeline's worker adds one control
 * workgroup that forms and publishes the batches).
 *   in   device, rows * row_bytes_in
 *   out  device, rows * row_bytes_out (result stages: [rows][k] int32 indices
 *        followed by [rows][k] f32 values, i.e. 2 planes)
 *   ns_per_rep (may be NULL) receives the launch's duration measured with HIP
 *        events on the stream it ran on, divided by reps, in ns.
 *   device_ns_per_rep (may be NULL) receives the device-clock time of the reps
 *        alone (after the grid has started, excluding the launch), divided by reps.
 * Synchronous: returns after the work completed. */
int32_t camelot_stage_run(const camelot_stage_desc* stage, const void* in, void* out,
                          int32_t rows, int32_t n_cus, int32_t cu_offset, int32_t reps,
                          double* ns_per_rep, double* device_ns_per_rep);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): camelot_stage_run's
 * computation with no allocation of any kind on the device. The control block, the
 * log-mel tables and the stage's scratch live in one static device array per GPU of
 * at most CAMELOT_NOALLOC_SCRATCH_BYTES of stage scratch (held until the process
 * ends). Stage scratch needed: MLP_BF16 512 * round_up(max dims[l], 32) bytes
 * (so every MLP the library accepts, widths <= 16384), CONV_POOL 32768 * ceil(H * W / 64) bytes (maps up to
 * 16384 pixels), other kinds none; a stage needing more is refused with
 * CAMELOT_EINVAL before anything runs.
 *   stage, in, out, rows, reps   as camelot_stage_run (same layouts, same results,
 *        bit for bit: the same kernel and grid)
 *   n_cus  compute workgroups, one per CU of the caller's share: a multiple of 8 in
 *        8..256, at most the device's CUs; the stream must give the kernel room for
 *        all of them at once (an unmasked stream, or one masked to >= n_cus / 2 CUs)
 *   stream the caller's HIP stream (NULL: the null stream); the run is enqueued on
 *        it and the call returns without waiting (except once per device, the first
 *        LOGMEL call outside capture, which writes the tables and waits for them).
 * Writes to the device only through kernels (no memset or copy nodes), so it may be
 * captured into a HIP graph. Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents; calls whose work overlaps on one GPU race and give
 * undefined results. In-kernel waits are bounded (2 s); a run that times out
 * leaves `out` undefined. Returns CAMELOT_EINVAL on a bad argument, CAMELOT_EDEVICE
 * on a HIP error. */
#define CAMELOT_NOALLOC_SCRATCH_BYTES (8 << 20)
int32_t camelot_stage_run_noalloc(const camelot_stage_desc* stage, const void* in, void* out,
                                  int32_t rows, int32_t n_cus, int32_t reps, void* stream);

/* ------------------------------------------------------------------ pipelines
 * The query flow of Section V-B (queries wait in a queue, are batched, and pass
 * through the microservice stages in order, each stage on its own share of the
 * GPU) with the communication of Section VI: a pipeline is a chain of stages, each
 * run by one persistent worker kernel on its own CU-masked stream (stage i on
 * cu[i] CUs). Stage i hands its batch to stage i+1 through a device-global ring of
 * ring_depth slots with doorbells, one copy of the data in device memory
 * (CAMELOT_HANDOFF_DEVICE, Section VI-B) or, for the baseline, by a device->pinned
 * host->device copy per batch driven by a host thread (CAMELOT_HANDOFF_HOST, the
 * main-memory communication of Section VI-A). The CU shares, instance counts and
 * batch size come from an allocation (camelot_alloc: cu[], n[], batch), copied into
 * cu[], n_inst[] and max_batch / batch_target here.
 *
 * Queries arrive as requests of 1..max_rows_per_request rows. Stage 0 forms a
 * batch from whole waiting requests in arrival order, at most max_batch rows,
 * and starts it when at least batch_target rows wait or the oldest waiting request
 * has waited batch_timeout_ns (batch_target 1 = start as soon as anything waits:
 * continuous batching). Results come out in submit order, one per row.
 *
 * Ingest modes:
 *   CAMELOT_INGEST_HOST    camelot_pipeline_submit copies each request into a
 *                          pinned ingest ring; arrival time = submit time.
 *   CAMELOT_INGEST_REPLAY  the requests (ids, rows, arrival times, payload rows)
 *                          are resident in device memory before the run starts
 *                          (camelot_pipeline_replay); stage 0 admits request r
 *                          once the device clock passes its arrival time.
 *   CAMELOT_INGEST_IPC     stage 0 reads the batches another process's pipeline
 *                          exports (out_ipc there), from the ring behind
 *                          ipc_handle (see "Pipelines across processes" below).
 */
typedef enum { CAMELOT_HANDOFF_DEVICE = 0, CAMELOT_HANDOFF_HOST = 1 } camelot_handoff;
typedef enum { CAMELOT_INGEST_HOST = 0, CAMELOT_INGEST_REPLAY = 1, CAMELOT_INGEST_IPC = 2 } camelot_ingest;
#define CAMELOT_IPC_HANDLE_BYTES 64

typedef struct {
  int32_t n_stages;
  camelot_stage_desc stages[CAMELOT_MAX_STAGES];
  int32_t cu[CAMELOT_MAX_STAGES];  /* CUs per stage instance, multiples of 8           */
  int32_t n_inst[CAMELOT_MAX_STAGES]; /* instances per stage (N_i of Eq. 1; 0 means 1).
                                  Only stages between the first and the last may have
                                  more than one (up to CAMELOT_MAX_INSTANCES): instance j
                                  of stage i takes batches j, j + N_i, j + 2 N_i, ... on
                                  its own cu[i] CUs, and the next stage still consumes
                                  batches in order. Stages are laid out from cu_offset,
                                  instance after instance: sum_i N_i cu[i] <= 256 -
                                  cu_offset. ring_depth must be >= 2 max_i N_i.       */
  int32_t cu_offset;           /* first CU-mask bit of this pipeline (multiple of 8) */
  int32_t max_batch;           /* rows per batch, 1..CAMELOT_MAX_BATCH               */
  int32_t batch_target;        /* start a batch once this many rows wait (>= 1)     */
  int64_t batch_timeout_ns;    /* ... or once the oldest waited this long           */
  int32_t ring_depth;          /* slots per device ring, >= 2                        */
  int32_t handoff;             /* camelot_handoff                                    */
  int32_t ingest;              /* camelot_ingest                                     */
  int32_t max_rows_per_request;/* 1..max_batch                                       */
  int32_t ingest_capacity;     /* requests the ingest queue holds (host mode)        */
  int32_t egress_capacity;     /* result rows buffered for drain                     */
  int64_t idle_timeout_ns;     /* workers exit after this long with nothing to do;
                                  with host ingest the next submit starts them again
                                  where they left off                               */
  int64_t hbm_budget_bytes;    /* admission: ENOMEM if the footprint exceeds it (0 = no limit) */
  int32_t side_bytes;          /* per-row bytes carried unchanged from the end of each
                                  payload row through every stage (0..4096, multiple of
                                  16): e.g. a query's item ids for a GATHER_SCORE stage.
                                  Payload rows are row_bytes_in(stage 0) + side_bytes. */
  int32_t out_ipc;             /* 1: the last stage is not a result stage; its batches go
                                  to a ring exported to another process (no results,
                                  no drain here)                                      */
  uint8_t ipc_handle[CAMELOT_IPC_HANDLE_BYTES]; /* ingest == CAMELOT_INGEST_IPC: the
                                  exporting pipeline's handle (camelot_pipeline_ipc_info) */
} camelot_pipeline_config;

typedef struct camelot_pipeline camelot_pipeline;

/* Builds rings, streams and workers and launches the workers (HOST ingest) or
 * prepares them (REPLAY ingest; workers start in camelot_pipeline_replay).
 * *out receives the handle. ENOMEM when the footprint exceeds hbm_budget_bytes. */
int32_t camelot_pipeline_create(const camelot_pipeline_config* cfg, camelot_pipeline** out);

/* Pipelines across processes (Section VI-B: microservices in separate processes
 * exchange batches through GPU global memory, not through the host). A pipeline
 * created with out_ipc = 1 allocates its last stage's output ring (header with the
 * ring's geometry, slot state words, ring_depth slots; under 2 GiB, else EINVAL) in
 * one device allocation and exports it; a pipeline in another process, created with
 * ingest = CAMELOT_INGEST_IPC and that handle, opens it and its stage 0 consumes the
 * batches with the same slot protocol as between two stages of one pipeline (the
 * batch, its requests' ids and arrival times and the stage times travel in the
 * slot). The importer checks the geometry (EINVAL if its stage 0 consumes another
 * row size, another side_bytes, or a smaller max_batch than the exporter's); its
 * stages follow the exporter's in the result timestamps, which are then absolute
 * device-clock ns (epoch 0). Both pipelines must run on the same GPU. The importer
 * launches its workers at create; destroy the importer before the exporter's memory
 * is needed back (the exporter frees its allocation at destroy, the importer closes
 * its mapping at destroy).
 * camelot_pipeline_ipc_info: the exported handle (zeros for an importer that does not
 * export) and the host time the export and/or the open took (allocation, clearing,
 * header, handle; open, header read and checks). EINVAL for a pipeline that neither
 * exports nor imports. */
int32_t camelot_pipeline_ipc_info(const camelot_pipeline* p, uint8_t* handle, int64_t* setup_ns);

/* HBM bytes the pipeline holds (rings, scratch, control; weights are borrowed and
 * not counted). */
int64_t camelot_pipeline_footprint(const camelot_pipeline* p);

/* The device-clock time (ns) of the pipeline's epoch, the zero of its result
 * timestamps: the create call (host ingest) or the workers' start (replay ingest;
 * EAGAIN until the replay has started). Pipelines on one device share the clock, so
 * epoch + t_ns puts the results of several pipelines on one time line. */
int32_t camelot_pipeline_epoch_ns(const camelot_pipeline* p, int64_t* epoch_ns);

/* Host ingest. Copies `rows` rows of payload (host pointer, rows * row_bytes_in of
 * stage 0) before returning. query_id must exceed every id submitted before on this
 * pipeline. EAGAIN when the ingest queue is full; ESTOPPED after destroy/stop. */
int32_t camelot_pipeline_submit(camelot_pipeline* p, uint64_t query_id,
                                const void* payload, int32_t rows);

/* Host ingest paced by a library thread, the host-submit counterpart of
 * camelot_pipeline_replay (Section V-B: queries enter the pipeline's wait queue from
 * the host as they arrive): request r (ids[r], rows[r] rows of host payload starting
 * at payload row payload_row[r], rows of row_bytes_in of stage 0 plus side_bytes)
 * goes through camelot_pipeline_submit once arrival_ns[r] ns have passed since this
 * call, waiting while the ingest queue is full; its arrival time (the zero of its
 * latency) is the scheduled one, so a submitter that falls behind adds to the
 * latencies instead of hiding. Returns at once; the arrays are
 * copied, the payload (host memory, payload_rows rows) is borrowed until the last
 * request is submitted. One paced submission per pipeline, and no other submit
 * calls meanwhile; destroy stops it. EINVAL on bad arguments (as replay). */
int32_t camelot_pipeline_submit_replay(camelot_pipeline* p, int32_t n_req, const uint64_t* ids,
                                       const int32_t* rows, const int64_t* arrival_ns,
                                       const int64_t* payload_row, const void* payload,
                                       int64_t payload_rows);
/* Requests the paced submission has submitted so far; returns its error, if it
 * stopped on one (a worker failure or ESTOPPED), else CAMELOT_OK. */
int32_t camelot_pipeline_submit_status(camelot_pipeline* p, int64_t* submitted);

/* One result row. t_ns: [0] arrival, then per stage (start, end) of the batch,
 * then done; all in ns of the device clock since the pipeline's epoch. */
typedef struct {
  uint64_t query_id;
  int32_t row;                          /* row index within the request            */
  int32_t n_out;                        /* k                                       */
  int32_t idx[CAMELOT_MAX_K];
  float val[CAMELOT_MAX_K];
  uint64_t t_ns[2 * CAMELOT_MAX_STAGES + 2];
} camelot_result;

/* Copies up to max finished rows into out[] in submit order; *n_out receives the
 * count. Waits up to timeout_ns for at least one (0 = poll). ETIMEDOUT when none
 * arrived in time; EDEVICE if a worker reported a failure. */
int32_t camelot_pipeline_drain(camelot_pipeline* p, camelot_result* out, int32_t max,
                               int32_t* n_out, int64_t timeout_ns);

/* Bulk drain for load tests: for up to max finished rows, in the same order as
 * camelot_pipeline_drain, the request id and the latency done - arrival in ns.
 * ids and lat_ns are host arrays of max entries. Same waiting and errors as
 * camelot_pipeline_drain. */
int32_t camelot_pipeline_drain_latency(camelot_pipeline* p, uint64_t* ids, int64_t* lat_ns,
                                       int32_t max, int32_t* n_out, int64_t timeout_ns);

/* Device replay ingest: n_req requests with ids[] (strictly increasing), rows[],
 * arrival_ns[] (ns after the start, non-decreasing) and payload_row[] (index of
 * the request's first row in `payload`, a device buffer of payload_rows rows of
 * row_bytes_in). Host arrays are copied. Starts the workers and returns at once;
 * results are drained as in host mode. */
int32_t camelot_pipeline_replay(camelot_pipeline* p, int32_t n_req, const uint64_t* ids,
                                const int32_t* rows, const int64_t* arrival_ns,
                                const int64_t* payload_row, const void* payload,
                                int64_t payload_rows);

/* Counters of the run so far. */
typedef struct {
  uint64_t submitted_requests, submitted_rows;
  uint64_t delivered_rows;
  uint64_t batches[CAMELOT_MAX_STAGES];          /* batches finished per stage (all
                                                    its instances; so are the sums
                                                    below)                          */
  uint64_t id_sum[CAMELOT_MAX_STAGES];           /* sum of splitmix64(id) per row
                                                    leaving stage i (mod 2^64)      */
  uint64_t id_xor[CAMELOT_MAX_STAGES];           /* xor of the same                 */
  int32_t worker_status[CAMELOT_MAX_STAGES];     /* 0 running/ok, else the first
                                                    instance's error code           */
  uint64_t rows[CAMELOT_MAX_STAGES];             /* rows finished per stage         */
  int64_t busy_ns[CAMELOT_MAX_STAGES];           /* sum over batches of the time from
                                                    batch start (input and output
                                                    slots held) to publish          */
  int64_t wait_ns[CAMELOT_MAX_STAGES];           /* sum of the waits for input and
                                                    output space before each batch  */
} camelot_pipeline_stats;

int32_t camelot_pipeline_stats_get(camelot_pipeline* p, camelot_pipeline_stats* out);

/* Stops the workers (they finish the batch in hand and exit), waits for them and
 * frees everything. *undelivered (may be NULL) receives the number of submitted
 * rows never delivered. */
int32_t camelot_pipeline_destroy(camelot_pipeline* p, uint64_t* undelivered);

/* ------------------------------------------------------------------ serving: admission
 * A server is a set of pipelines co-located on one GPU under one HBM budget (F of
 * Eq. 1 / Eq. 3; global memory capacity is the binding resource for co-location,
 * Section IV-C). A pipeline is admitted only if its footprint - the library's
 * rings, scratch and control (camelot_pipeline_footprint) plus every weight buffer
 * not already held by an admitted pipeline - fits what is left. Weight buffers are
 * identified by pointer, so instances sharing a model count it once (Section VII-D).
 * Admission does not place CUs: the configs' cu_offset/cu ranges must not overlap
 * those of admitted pipelines (EINVAL otherwise). */
typedef struct camelot_server camelot_server;

int32_t camelot_server_create(int64_t hbm_budget_bytes, camelot_server** out);
/* ENOMEM (and nothing created) when the pipeline does not fit the budget. */
int32_t camelot_server_admit(camelot_server* s, const camelot_pipeline_config* cfg,
                             camelot_pipeline** out);
/* Destroys an admitted pipeline (as camelot_pipeline_destroy) and returns its bytes. */
int32_t camelot_server_release(camelot_server* s, camelot_pipeline* p, uint64_t* undelivered);
/* HBM bytes held by admitted pipelines (shared weights once). */
int64_t camelot_server_used_bytes(const camelot_server* s);
/* Releases every admitted pipeline and frees the server. */
int32_t camelot_server_destroy(camelot_server* s);

/* Bytes of the weight buffers a stage reads (0 for stages without weights). */
int64_t camelot_stage_weight_bytes(const camelot_stage_desc* stage);

/* Resources of the kernel that runs a stage kind: one_shot != 0 for the kernel of
 * camelot_stage_run, else the pipeline worker. *regs: registers per lane;
 * *lds_bytes: static LDS per workgroup; *fits: 1 when two workgroups fit on a CU
 * and the kernel needs no scratch (what launching a worker requires), else 0.
 * EINVAL for an unknown kind. */
int32_t camelot_stage_kernel_info(int32_t kind, int32_t one_shot, int32_t* regs, int64_t* lds_bytes,
                                  int32_t* fits);

/* ------------------------------------------------------------------ share bandwidth
 * The attainable HBM bandwidth of a CU share, the bandwidth roofline of a stage
 * confined to it (the paper's stages get SM shares; only compute units are
 * partitioned, memory bandwidth is shared, Section IV). Plain streaming kernels,
 * two workgroups per CU, 8 independent 16-byte accesses in flight per thread,
 * non-temporal, over `bytes` (a multiple of 16; >= 1 GiB exceeds the 256 MB MALL so
 * the traffic reaches HBM), `reps` passes, timed on the device clock:
 *   CAMELOT_STREAM_READ   a reduction of one buffer on n_cus CUs at cu_offset
 *   CAMELOT_STREAM_WRITE  a fill of one buffer
 *   CAMELOT_STREAM_COPY   dst = src (bytes read + bytes written)
 *   CAMELOT_STREAM_SPLIT  a fill on [cu_offset, +n_cus) while a reduction of
 *                         another buffer runs on the next n_cus CUs: the ceiling of
 *                         the device-global handoff at that producer/consumer split
 * out[0] = seconds, out[1] = bytes moved, out[2] = GB/s. The library allocates the
 * buffers; synchronous. EINVAL on bad sizes or shares (multiples of 8 CUs). */
enum { CAMELOT_STREAM_READ = 0, CAMELOT_STREAM_WRITE = 1, CAMELOT_STREAM_COPY = 2, CAMELOT_STREAM_SPLIT = 3 };
int32_t camelot_stream_bench(int32_t mode, int64_t bytes, int32_t n_cus, int32_t cu_offset, int32_t reps,
                             double* out);

/* ------------------------------------------------------------------ handoff benchmark
 * Section VI-B's claim, measured: a producer worker on cu_producer CUs writes
 * n_slots_total slots of slot_bytes (a multiple of 16, at most 2^30) into a device
 * ring of depth slots; a consumer
 * worker on the next cu_consumer CUs waits on each slot's doorbell, reads every
 * word into a checksum and frees the slot. Both run concurrently.
 * out: [0] seconds of the run (device clock), [1] bytes moved (written + read),
 *      [2] checksum sum, [3] checksum xor (compare with
 *      camelot_handoff_expected), [4] handoff GB/s.
 * mode CAMELOT_HANDOFF_HOST measures the host-staged path instead: per slot a
 * device->pinned and a pinned->device copy (out[1] counts the bytes of both). */
int32_t camelot_handoff_bench(int32_t mode, int64_t slot_bytes, int32_t depth,
                              int64_t n_slots_total, int32_t cu_producer,
                              int32_t cu_consumer, double* out);

/* Expected (sum, xor) checksum of the handoff pattern (host computation). */
int32_t camelot_handoff_expected(int64_t slot_bytes, int64_t n_slots_total,
                                 uint64_t* sum, uint64_t* xr);

/* The same handoff between two processes on one GPU (Section VI-B: the microservices
 * of a pipeline are separate processes; the slot goes through global memory the two
 * share, not through the host). One process creates a region (its ring of depth slots
 * of slot_bytes, the per-(slot, channel) doorbells and the results; under 2 GiB, else
 * EINVAL) and exports it (*handle: CAMELOT_IPC_HANDLE_BYTES); the other opens it.
 * Every channel is a producer/consumer workgroup pair owning a chunk of each slot:
 * min(channels, slot_bytes / 16) of them, at least 16 bytes each.
 * camelot_ipc_handoff_run runs one side in the calling process on the CUs from
 * cu_offset (as many as the region's channels, rounded up to a multiple of 8) and
 * returns when it has finished: role CAMELOT_IPC_PRODUCER writes n_slots slots (the
 * pattern of camelot_handoff_expected), CAMELOT_IPC_CONSUMER reads them; each region
 * carries one producer run and one consumer run, started in either order (each waits
 * at most timeout_ms for the other, ETIMEDOUT after). The side that ends last (the
 * consumer) returns out as camelot_handoff_bench does: [0] seconds from the
 * producer's first store to the consumer's last read, [1] bytes written + read,
 * [2], [3] the checksum bits, [4] GB/s.
 * camelot_ipc_region_info: host time the create (allocation, clearing, handle) or
 * the open (mapping, header read) took, and the channel count.
 * camelot_ipc_region_destroy: the creator frees the region, an opener unmaps it. */
typedef struct camelot_ipc_region camelot_ipc_region;
enum { CAMELOT_IPC_PRODUCER = 0, CAMELOT_IPC_CONSUMER = 1 };
int32_t camelot_ipc_region_create(int64_t slot_bytes, int32_t depth, int32_t channels, uint8_t* handle,
                                  camelot_ipc_region** out);
int32_t camelot_ipc_region_open(const uint8_t* handle, camelot_ipc_region** out);
int32_t camelot_ipc_region_info(const camelot_ipc_region* r, int64_t* setup_ns, int32_t* channels);
int32_t camelot_ipc_handoff_run(camelot_ipc_region* r, int32_t role, int64_t n_slots, int32_t cu_offset,
                                int32_t timeout_ms, double* out);
int32_t camelot_ipc_region_destroy(camelot_ipc_region* r);

/* ------------------------------------------------------------------ predictor
 * Learned contention predictor (replaces Section VII-A's per-microservice model):
 * MLP 16 -> 64 (ReLU) -> 64 (ReLU) -> 1, FP32, predicting ln(latency ns).
 * Parameters live in one device buffer of CAMELOT_PRED_NPARAMS floats in the order
 * W1[16][64], b1[64], W2[64][64], b2[64], W3[64][1], b3[1] (weights [in, out]).
 * Loss L = mean over the minibatch of (yhat - y)^2.
 */
#define CAMELOT_PRED_NIN 16
#define CAMELOT_PRED_NHID 64
#define CAMELOT_PRED_NPARAMS (16 * 64 + 64 + 64 * 64 + 64 + 64 + 1)

/* yhat[m] (device f32) for x (device f32 [m][16]). */
int32_t camelot_predictor_forward(const float* params, const float* x, int32_t m,
                                  float* yhat, void* stream);

/* grad (device f32 [NPARAMS]) = dL/dparams over the minibatch x [m][16], y [m];
 * *loss_out (host, may be NULL) receives L. */
int32_t camelot_predictor_grad(const float* params, const float* x, const float* y,
                               int32_t m, float* grad, float* loss_out, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at step t >= 1 on device buffers
 * params, grad, m1, m2 (each NPARAMS floats; m1 and m2 start at zero). */
int32_t camelot_predictor_adam(float* params, const float* grad, float* m1, float* m2,
                               int32_t t, float lr, void* stream);

/* Trains for `epochs` over x [n][16], y [n] (device) with minibatches of `batch`
 * rows in a fixed order (row permutation `perm` [epochs][n] int32 device, or NULL
 * for sequential); params/m1/m2 device as above; step counter continues from *t.
 * Per-epoch mean loss written to epoch_loss (host [epochs], may be NULL). */
int32_t camelot_predictor_train(float* params, float* m1, float* m2, int32_t* t,
                                const float* x, const float* y, int32_t n, int32_t batch,
                                int32_t epochs, const int32_t* perm, float lr,
                                float* epoch_loss, void* stream);

/* ------------------------------------------------------------------ contention profiles
 * The paper profiles each microservice alone and observes that co-located stages
 * run slower than their solo profiles (Section IV-A, the balanced deployment
 * policy). These calls measure that contention.
 *
 * camelot_stage_corun: runs n stages at once, stage j on n_cus[j] CUs from mask bit
 * cu_offset[j] (shares disjoint, multiples of 8), each repeating batches of rows[j]
 * rows of in[j] into out[j] (as camelot_stage_run) for duration_ns of device time,
 * and writes each stage's mean time per batch while the others ran. */
int32_t camelot_stage_corun(int32_t n, const camelot_stage_desc* stages, const void* const* in,
                            void* const* out, const int32_t* rows, const int32_t* n_cus,
                            const int32_t* cu_offset, int64_t duration_ns, double* ns_per_batch);

#define CAMELOT_MAX_CORUN 8     /* kernels of one co-location profile or candidate */

typedef struct {
  int32_t m;                            /* kernels in this run, 1..CAMELOT_MAX_CORUN     */
  int32_t kinds[CAMELOT_MAX_CORUN];     /* which of the n_kinds stages (repeats allowed) */
  int32_t cu[CAMELOT_MAX_CORUN];        /* CUs of each                                   */
  int32_t bi[CAMELOT_MAX_CORUN];        /* batch index of each                           */
  double ns[CAMELOT_MAX_CORUN];         /* measured time per batch of each               */
} camelot_corun_record;

/* Random co-location profiles: n_runs runs of a random walk over co-locations.
 * Every 16th run (the first included) is a fresh draw: m kernels, m uniform in
 * 1..min(CAMELOT_MAX_CORUN, cu_total / cu_step); with probability 1/2 (when m >=
 * n_kinds) the first n_kinds kernels are one of each stage (a deployment's shape),
 * and every other kernel's kind is uniform over the n_kinds stages (independently,
 * so a kind can run as several instances, as in an allocation with N_i > 1);
 * shares drawn uniformly in cu_step steps with total <= cu_total and placed side by
 * side from bit 0, batch indices equal for all kernels with probability 1/2 and
 * independent otherwise. Each other run makes one move from the previous one: a
 * kernel's kind and batch re-drawn, its share re-drawn within the free CUs after it,
 * a kernel added in a free range, or one removed (batches of changed kernels equal
 * to another kernel's with probability 1/2). Kernels that keep their CUs keep their
 * masked streams, which makes a run cost its ~1 ms of work rather than the ~5 ms a
 * masked stream takes to create. The draws come from a SplitMix64 stream seeded
 * with `seed`. in[k]/out[k] are kind k's device buffers for max(batches) rows
 * (instances of one kind share them). */
int32_t camelot_profile_coruns(int32_t n_kinds, const camelot_stage_desc* stages, const void* const* in,
                               void* const* out, int32_t cu_total, int32_t cu_step, int32_t n_batches,
                               const int32_t* batches, int32_t n_runs, uint64_t seed,
                               int64_t duration_ns, camelot_corun_record* records);

/* ------------------------------------------------------------------ learned predictor features
 * Solo summaries the features use, per stage kind, CU share index k ((k + 1) * cu_step
 * CUs) and batch index: hbm = solo algorithmic HBM bytes/s / HBM peak, mfma = solo
 * flop rate / MFMA peak of the whole GPU; both [n_kinds][n_shares][n_batches] host
 * float arrays. */
typedef struct {
  int32_t n_kinds, cu_step, n_shares, n_batches;
  const int32_t* batches;
  const float* hbm;
  const float* mfma;
} camelot_solo_tables;

#define CAMELOT_PRED_FEATURES 16

/* Features of one co-location of m <= CAMELOT_MAX_CORUN kernels: kernel j has kind
 * kinds[j] (< 3), share cu[j] and batch index bi[j]. Row j (16 floats) of feat (host)
 * is: own share / 256, log2(own batch) / 7, own solo hbm, own solo mfma, one-hot kind
 * (3); then two aggregate co-runner slots, the other kernels of the same kind (its
 * sibling instances) and the kernels of other kinds, each holding the sum of their
 * shares / 256, the mean of their log2(batch) / 7, the sum of their solo hbm and the
 * sum of their solo mfma (zeros when empty); last, the CUs of all m kernels / 256. */
int32_t camelot_predictor_features(const camelot_solo_tables* t, int32_t m, const int32_t* kinds,
                                   const int32_t* cu, const int32_t* bi, float* feat);

/* Standardisation fitted on n rows of host features x [n][16]: mean and std (host
 * [16], std floored at 1e-6); camelot_predictor_standardize applies it in place. */
int32_t camelot_predictor_fit_norm(const float* x, int32_t n, float* mean, float* std);
int32_t camelot_predictor_standardize(float* x, int32_t n, const float* mean, const float* std);

/* Contention-aware Eq. 1: camelot_alloc_peak's problem (N_i up to max_inst_per_stage
 * and inst_max, at most CAMELOT_MAX_CORUN instances in all; n_stages <= 3, stage i of
 * kind i), but every stage's latency is its solo latency (lat_ns) times exp(y), y =
 * the learned predictor's output for one of its instances in the co-location the
 * candidate forms (all instances of every stage; the network predicts the log
 * slowdown over the solo profile) clamped to [0, 10] (co-runners never make a stage
 * faster than alone), rounded up to ns. Candidates are taken in the lexicographic
 * order (batch index, N_1, share_1, N_2, share_2, ...) and the objective, constraints
 * and tie rules are those of camelot_alloc_peak. The clamp makes the solo table an
 * upper bound of every candidate's throughput: the search predicts candidates in
 * decreasing order of that bound and stops once no candidate left can win, with the
 * same result as predicting them all (the overhead budget of Section VIII-G). params:
 * device [CAMELOT_PRED_NPARAMS]; mean/std: host [16]. lat_pred_ns (host [n_stages],
 * may be NULL) receives the predicted latencies of the chosen point. */
int32_t camelot_alloc_peak_learned(const camelot_problem* problem, const camelot_solo_tables* t,
                                   const float* params, const float* mean, const float* std,
                                   camelot_alloc* out, int64_t* lat_pred_ns);

/* ---------------------------------------------------------------- decision tree */
/* Decision-tree regressor, the kind of latency predictor the paper fits to its
 * co-location profiles (Section VII-A). CART regression with the squared error: a node
 * splits on the feature and threshold (midpoint between consecutive distinct values;
 * x <= thr goes left) that maximise sum_L^2/n_L + sum_R^2/n_R, both children keeping
 * at least min_leaf samples, if that lowers the error; otherwise, or at max_depth,
 * it is a leaf predicting the mean of its y. Deterministic: features in index order,
 * samples in (value, index) order, sums in double in that order, the first best
 * split kept. Host code, host memory throughout.
 *   x    [n][n_feat] f32, y [n] f32 (all finite); 1 <= n, 1 <= n_feat,
 *        0 <= max_depth <= 64, min_leaf >= 1.
 *   *out receives the tree (caller frees it with camelot_dt_destroy).
 * EINVAL on bad arguments or a non-finite value, ENOMEM. */
typedef struct camelot_dt camelot_dt;
int32_t camelot_dt_fit(const float* x, const float* y, int32_t n, int32_t n_feat, int32_t max_depth,
                       int32_t min_leaf, camelot_dt** out);
/* Predictions for n host rows x [n][n_feat] into host out [n]. */
int32_t camelot_dt_predict(const camelot_dt* t, const float* x, int32_t n, float* out);
/* The nodes in creation (depth-first, left first) order: *n_nodes always; with
 * cap >= *n_nodes also feat (-1: leaf), thr, value, left, right (host arrays [cap];
 * -1 children for a leaf). cap 0 asks for the count only. */
int32_t camelot_dt_export(const camelot_dt* t, int32_t cap, int32_t* n_nodes, int32_t* feat, double* thr,
                          double* value, int32_t* left, int32_t* right);
void camelot_dt_destroy(camelot_dt* t);

/* Contention-aware Eq. 1 with the tree as the predictor: the candidates, features,
 * objective, constraints and tie rules of camelot_alloc_peak_learned, each stage's
 * latency its solo latency times exp(the tree's prediction for one of its
 * instances in the candidate's co-location), rounded up to ns; the tree is applied
 * to the raw (not standardised) 16 features. Host code. */
int32_t camelot_alloc_peak_dt(const camelot_problem* problem, const camelot_solo_tables* t, const camelot_dt* dt,
                              camelot_alloc* out, int64_t* lat_pred_ns);

#ifdef __cplusplus
}
#endif
#endif /* CAMELOT_H */
