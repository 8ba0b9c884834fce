/*
 * stab.h -- C ABI of the MI355X stabilizer-tableau library (libstab.so).
 *
 * The library simulates Clifford circuits with single-qubit Z measurements on the
 * Aaronson-Gottesman (CHP) tableau that the STABSim paper builds on (Sec. 2.3-2.4): 2n rows
 * (n destabilizers, n stabilizers) of x|z bits plus a sign bit, Clifford gates as per-row bit
 * rules (Table 1), and measurements that either run rowsum from the first anticommuting
 * stabilizer (random outcome) or reduce a product of stabilizers into a scratch row
 * (deterministic outcome; rowsum of Appendix A.2, Alg. 2).  Every kernel is HIP for gfx950.
 *
 * Conventions for every call:
 *   - Return 0 on success or a negative STAB_E* code; stab_last_error() then gives a message
 *     (thread-local).  Arguments are validated before anything is enqueued, so a call that
 *     fails validation has no side effect.
 *   - Device pointers are HIP device memory the caller owns (typically a torch uint8 tensor);
 *     the library never frees them.  Host pointers are ordinary host memory, written only on
 *     success.  hip_stream is a hipStream_t (NULL = default stream); every call is synchronous
 *     with respect to the host unless it says otherwise.
 *   - A context is not thread-safe.  Distinct contexts are independent.
 *   - A device error leaves the context unusable (every later call returns STAB_EDEVICE).
 *
 * Op-stream format (the input of stab_run / stab_sample):
 *   An array of stab_instr plus one flat int32 target array.  Instruction k consumes the next
 *   instr[k].ntargets targets.  Two-qubit kinds (CX, DEP2) consume (a, b) pairs.  Targets of
 *   one instruction act in order, as if each were its own instruction.
 *   Randomness: Philox4x64-10 (Salmon et al., SC'11), key = (seed, shot), counter =
 *   (instruction index, target position, 0, 0), outputs u0..u3.  The instruction index counts
 *   every instruction a context has executed, TICK included.
 *     DEP1:   error iff u0 < t0; Pauli 1 + mulhi64(u1, 3) (1=X, 2=Y, 3=Z)
 *     DEP2:   error iff u0 < t0; k = 1 + mulhi64(u1, 15); Pauli on a = k >> 2, on b = k & 3
 *     PAULI1: X iff u0 < t0, else Y iff u0 < t1, else Z iff u0 < t2 (cumulative thresholds)
 *     M/MR/R: a random outcome is u0 >> 63; MR and R then apply X if the outcome is 1 and R
 *             records nothing.  Records hold 1 bit per M/MR target (1 = eigenvalue -1).
 *     T1T2:   exact relaxation (T1) then dephasing (T2) for T1 >= T2 (Sec. 4.2), as a mixture
 *             of stochastic Clifford+reset operations: reset iff u0 < t0 (a Z measurement
 *             whose random outcome is u1 >> 63, then X if it is 1; nothing recorded), else Z
 *             iff u0 < t1, else nothing.  It changes x|z shot by shot, so only the batch calls
 *             (one tableau per circuit) accept it; stab_compile/stab_run reject it.
 */
#ifndef LIBSTAB_ABI_H_
#define LIBSTAB_ABI_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define STAB_OK         0
#define STAB_EINVAL    -1   /* bad argument or malformed op stream */
#define STAB_ENOMEM    -2   /* buffer too small or device allocation failed */
#define STAB_EDEVICE   -3   /* HIP runtime error (context poisoned) */
#define STAB_ERANGE    -4   /* size outside what the library supports */
#define STAB_EINTERNAL -5   /* an internal consistency check failed on the device */

/* instruction kinds */
enum {
    STAB_TICK = 0, STAB_H = 1, STAB_S = 2, STAB_X = 3, STAB_Y = 4, STAB_Z = 5, STAB_CX = 6,
    STAB_M = 7, STAB_MR = 8, STAB_R = 9, STAB_DEP1 = 10, STAB_DEP2 = 11, STAB_PAULI1 = 12,
    STAB_T1T2 = 13
};

/* One instruction (32 bytes, no implicit padding). */
typedef struct stab_instr {
    uint32_t kind;      /* STAB_* kind */
    uint32_t ntargets;  /* int32 targets consumed (even for CX and DEP2) */
    uint64_t t0, t1, t2;/* noise thresholds (see the format above); 0 otherwise */
} stab_instr;

/* Storage modes.  SHARED keeps one x|z tableau and one sign vector per shot: exact because
 * x|z never depends on signs, outcomes or Pauli noise (only signs do).  FULL keeps one
 * complete tableau per shot. */
#define STAB_MODE_SHARED 0
#define STAB_MODE_FULL   1

typedef struct stab_ctx stab_ctx;

/* Largest qubit count the library supports: 10240 (160 64-bit words of x or z per row; the
 * random-measurement kernel keeps a target's column, 2 * 160 band words, in the registers of
 * one wave, and half a band of the tableau must fit in the 160 KB of LDS of one compute
 * unit). */
int32_t stab_max_qubits(void);

/* Bytes of device memory a context needs in dev_buf for n qubits and `shots` shots in the
 * given mode: the 2n-row x|z tableau plus signs of Sec. 2.3 (4n^2 + 2n bits per copy, rows
 * padded to 64-bit words), one copy per shot in STAB_MODE_FULL.  Writes *bytes_out.  Errors: STAB_EINVAL (n < 1, shots < 1, bad mode),
 * STAB_ERANGE (n > stab_max_qubits()). */
int stab_tableau_bytes(int32_t n, int32_t shots, int32_t mode, uint64_t *bytes_out);

/* Create a context holding `shots` tableaux of n qubits in |0...0> (destabilizer i = +X_i,
 * stabilizer i = +Z_i; the initial state the paper leaves implicit), stored in dev_buf
 * (>= stab_tableau_bytes bytes, 256-byte aligned, owned by the caller, which must keep it
 * alive until stab_destroy).  The RNG key is (seed, first_shot + b) for shot b.
 * Errors: STAB_EINVAL, STAB_ERANGE, STAB_ENOMEM (buffer too small), STAB_EDEVICE. */
int stab_create(int32_t n, int32_t shots, int32_t mode, uint64_t seed, uint64_t first_shot,
                void *dev_buf, uint64_t buf_bytes, void *hip_stream, stab_ctx **out);

/* Release the context's own scratch memory (the column, pivot-log and record buffers the
 * measurement steps of Sec. 2.4 use).  Never frees dev_buf.  NULL is ignored. */
void stab_destroy(stab_ctx *ctx);

/* Run an op stream on every shot of the context (the paper's sim(circuit), Sec. 3.1.4, and
 * the race-safe gate/measurement ordering of Fig. 2).  Measurement outcomes are written to
 * out_bits (host, may be NULL when the stream records nothing): shot b's bits start at byte
 * b * ceil(nrec / 8), LSB first, where nrec = number of M/MR targets in the stream.  The
 * instruction counter advances by ninstr.  Errors: STAB_EINVAL (malformed stream, target out
 * of range, CX with equal qubits), STAB_ENOMEM, STAB_EDEVICE, STAB_EINTERNAL. */
int stab_run(stab_ctx *ctx, const stab_instr *instrs, int32_t ninstr, const int32_t *targets,
             int64_t ntargets, uint8_t *out_bits);

/* Apply gate and noise instructions only (no measurement kinds): a layer, or several, of
 * Clifford gates (Table 1) and Pauli channels.  Same as stab_run otherwise. */
int stab_apply_layer(stab_ctx *ctx, const stab_instr *instrs, int32_t ninstr,
                     const int32_t *targets, int64_t ntargets);

/* Measure qubits[0..k-1] in Z, in order (one M instruction; MR/R via `kind`), writing
 * ceil(k/8) bytes per shot to out_bits (host; NULL allowed for R).  Pivot search, rowsum
 * and the deterministic reduction follow Sec. 2.4 and Alg. 2 of the paper. */
int stab_measure(stab_ctx *ctx, uint32_t kind, const int32_t *qubits, int32_t k,
                 uint8_t *out_bits);

/* Copy one shot's tableau to the host in row-major bytes, in the layout of Sec. 2.3 (the
 * tableau of Fig. 2's state): x[2n][n], z[2n][n] (0/1 per byte), r[2n]; rows 0..n-1
 * destabilizers, n..2n-1 stabilizers.  Any pointer may be NULL.  Errors: STAB_EINVAL (NULL
 * context, shot out of range), STAB_EDEVICE. */
int stab_get_tableau(stab_ctx *ctx, int32_t shot, uint8_t *x, uint8_t *z, uint8_t *r);

/* A compiled op stream: validated, split into gate/noise segments and measurement layers,
 * and uploaded to the device once, so it can be executed many times.  The RNG instruction
 * index is taken relative to the context's counter at execution time. */
typedef struct stab_program stab_program;

/* Compile a stream for the context's geometry (n, shots).  Errors: STAB_EINVAL (malformed
 * stream, target out of range, CX with equal qubits, target count mismatch), STAB_ENOMEM,
 * STAB_EDEVICE. */
int stab_compile(stab_ctx *ctx, const stab_instr *instrs, int32_t ninstr,
                 const int32_t *targets, int64_t ntargets, stab_program **out);

/* Execute a compiled stream (same semantics and out_bits layout as stab_run).  If elapsed_ms
 * is not NULL it receives the device time from the first kernel to the record on the host.
 * The first execution of prog that starts from |0...0> (instruction counter 0) records which
 * measurement layers had a random target; since x|z never depends on outcomes or Pauli noise
 * this holds for every such execution, and later ones skip the random-measurement kernels of
 * the other layers (same results, fewer launches).  prog is updated by this, so one program
 * is not executed by two threads at once. */
int stab_execute(stab_ctx *ctx, stab_program *prog, uint8_t *out_bits, float *elapsed_ms);

/* Number of M/MR targets a compiled stream records per shot. */
int64_t stab_program_records(const stab_program *prog);

void stab_program_destroy(stab_program *prog);

/* Put every shot back in |0...0>, set the RNG key to (seed, first_shot + b) and the
 * instruction counter to 0. */
int stab_reset(stab_ctx *ctx, uint64_t seed, uint64_t first_shot);

/* Set the RNG key of later draws to (seed, first_shot + b) for shot b, leaving the tableaux and
 * the instruction counter as they are (a draw's counter is its instruction's index in
 * everything the context ran since stab_create or stab_reset, so a stream run after this call
 * draws as the same stream would at that position under the new key).  The random outcomes of
 * Sec. 2.4 and the noise draws come from this key.  Host only.  Errors: STAB_EINVAL (NULL),
 * STAB_EDEVICE (poisoned context). */
int stab_set_rng(stab_ctx *ctx, uint64_t seed, uint64_t first_shot);

/* Host-only: validate an op stream and describe how it would be executed for n qubits and
 * `shots` shots, without touching a device.  out[0..nout) receives, in order: segments (runs of
 * gate/noise layers between measurement layers), measurement layers, gate layers, gates, noise
 * instructions, noise units, recorded measurements per shot, largest measurement layer.
 * Errors: as stab_compile, STAB_EINVAL for nout outside [0, 8]. */
#define STAB_PLAN_FIELDS 8
int stab_plan_describe(int32_t n, int32_t shots, int32_t mode, const stab_instr *instrs,
                       int32_t ninstr, const int32_t *targets, int64_t ntargets, int64_t *out,
                       int32_t nout);

/* One-call sampler: the paper's sim(circuit) of Sec. 3.1 run for `shots` shots (parallel
 * sampling, named as future work in Sec. 6): create a context on dev_buf, run the stream,
 * write the packed record (shots * ceil(nrec/8) bytes, the stab_run layout) to out_bits,
 * destroy the context.  elapsed_ms (may be NULL) receives the device time from the first
 * kernel to the record on the host.  Errors: as stab_create and stab_run. */
int stab_sample(const stab_instr *instrs, int32_t ninstr, const int32_t *targets,
                int64_t ntargets, int32_t n, int32_t shots, int32_t mode, uint64_t seed,
                void *dev_buf, uint64_t buf_bytes, void *hip_stream, uint8_t *out_bits,
                float *elapsed_ms);

/* stab_sample without device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, semantics and out_bits layout as stab_sample (no elapsed time).  The
 * caller still provides the tableaux (dev_buf, stab_tableau_bytes bytes) and the host output;
 * every buffer stab_sample would allocate (error flag, counters, the uploaded program, target
 * columns, noise events, pivot log, records) is carved instead from one static device array of
 * STAB_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the process ends.
 * Nothing is allocated or freed on the device: no hipMalloc, hipFree, event or stream creation
 * (host-side the stream is compiled in ordinary heap memory, as by stab_sample).  Noise is drawn
 * segment by segment unless the whole program's draws also fit.  Every call on one GPU uses
 * that GPU's array and leaves its last contents there (each call clears what it needs), so
 * calls that overlap on one GPU race: serialise them.  Errors: as stab_sample, and STAB_ERANGE,
 * before the device is touched, when the workload needs more scratch than the array holds
 * (a d=25 surface-code memory experiment with 100 shots needs about 9 MB; d=71 does not fit). */
#define STAB_NOALLOC_SCRATCH_BYTES (64ull << 20)
int stab_sample_noalloc(const stab_instr *instrs, int32_t ninstr, const int32_t *targets,
                        int64_t ntargets, int32_t n, int32_t shots, int32_t mode, uint64_t seed,
                        void *dev_buf, uint64_t buf_bytes, void *hip_stream, uint8_t *out_bits);

/* Work counters accumulated by a context since creation (for accounting and bandwidth
 * figures): [0] rounds of the random-measurement chain, [1] chain rounds run by a whole block
 * (targets touching many rows), [2] measurements deterministic at layer start, [3] stabilizer
 * rows multiplied by deterministic reductions, [4] random measurements, [5] stabilizer rows
 * updated by rowsum, [6] measurements found deterministic inside the chain, [7] noise events,
 * [8] destabilizer rows updated by rowsum (replay), [9] destabilizer rows the replay walked,
 * [10] of those, rows it replayed by testing each run target (a pending list overflowed or
 * the lists did not fit), [11] rowsums and replacements in those rows.
 * ncounters <= 12.  Synchronizes the stream. */
int stab_get_counters(stab_ctx *ctx, uint64_t *counters, int32_t ncounters);

/* Per-kernel device timing with HIP events recorded on the context's stream around every
 * launch of the selected kernels.  stab_set_timing(ctx, mask) clears the totals and times the
 * kernel ids whose bit is set in mask (0 stops timing; (1 << STAB_NUM_KERNELS) - 1 times all;
 * each timed launch costs two event records on the stream).
 * stab_get_kernel_times writes, for each kernel id, the summed milliseconds and the number of
 * launches since timing started.  Kernel ids: 0 init, 1 noise draw, 2 segment (gates + noise
 * + column extraction), 3 classes and deterministic outcomes at layer start, 4 outcomes of
 * targets the random chain left deterministic, 5 random chain (stabilizer rows),
 * 6 reset/record, 7 record packing, 8 destabilizer replay, 9 column extraction after a layer
 * with random outcomes.  nkernels <= 10. */
#define STAB_NUM_KERNELS 10
int stab_set_timing(stab_ctx *ctx, int32_t kernel_mask);

/* Graph replay of stab_execute.  With enable != 0 (and no per-kernel timing selected),
 * stab_execute captures the device work of a program (every kernel launch up to the record
 * packing) into a hipGraph the first time it runs it, and replays the graph while the program,
 * the RNG seed and first shot, the instruction counter and the context's buffers are the same
 * as at capture (a program executed right after stab_reset, again and again, replays); any
 * other execution captures anew.  Results are those of the eager launches.  The record copy
 * to the host and the consistency check stay outside the graph.  Errors: STAB_EINVAL (null
 * context). */
int stab_set_graph(stab_ctx *ctx, int32_t enable);
int stab_get_kernel_times(stab_ctx *ctx, double *ms, uint64_t *launches, int32_t nkernels);

/* ---------------------------------------------------------------------------------------
 * Uneven multi-circuit batching.  A batch holds C independent circuits, circuit c on n[c]
 * qubits with its own tableau and its own op stream, and runs all of them in one persistent
 * launch (one workgroup per circuit, largest first).  This is the batched form of the
 * paper's wide random-circuit benchmark (Sec. 4.1, random Clifford layers with interleaved
 * measurements) and of the parallel sampling it names as future work (Sec. 6).
 * Semantics per circuit are exactly those of a one-shot context with first_shot = c: RNG key
 * (seed, c), counter (instruction index, target position), the index counting every
 * instruction circuit c has executed since the batch was created or reset.
 * ------------------------------------------------------------------------------------- */
typedef struct stab_batch stab_batch;
typedef struct stab_batch_program stab_batch_program;

/* Device bytes for the tableaux of `ncirc` circuits of n[0..ncirc-1] qubits (each n[c] in
 * [1, 8192]).  Errors: STAB_EINVAL (ncirc < 1, n NULL, n[c] < 1, bytes_out NULL),
 * STAB_ERANGE (n[c] > 8192). */
int stab_batch_bytes(int32_t ncirc, const int32_t *n, uint64_t *bytes_out);

/* Create a batch of circuits in |0...0> on dev_buf (>= stab_batch_bytes bytes, 256-byte
 * aligned, owned by the caller and kept alive until stab_batch_destroy).  Errors: as
 * stab_batch_bytes, STAB_ENOMEM (buffer too small), STAB_EDEVICE. */
int stab_batch_create(int32_t ncirc, const int32_t *n, uint64_t seed, void *dev_buf,
                      uint64_t buf_bytes, void *hip_stream, stab_batch **out);

/* Release the batch's own memory (never dev_buf).  NULL is ignored. */
void stab_batch_destroy(stab_batch *batch);

/* Put every circuit back in |0...0>, set the RNG seed and the instruction counters to 0. */
int stab_batch_reset(stab_batch *batch, uint64_t seed);

/* Compile the circuits' op streams (the stab_instr format above).  Circuit c's instructions
 * are instrs[instr_off[c] .. instr_off[c+1]) and its targets targets[target_off[c] ..
 * target_off[c+1]) (both offset arrays have ncirc + 1 entries, start at 0 and do not
 * decrease).  Errors: STAB_EINVAL (malformed stream, naming the circuit and instruction),
 * STAB_ERANGE, STAB_ENOMEM, STAB_EDEVICE. */
int stab_batch_compile(stab_batch *batch, const stab_instr *instrs, const int64_t *instr_off,
                       const int32_t *targets, const int64_t *target_off,
                       stab_batch_program **out);

/* Records (M/MR targets) circuit c writes, or -1 for a bad argument. */
int64_t stab_batch_program_records(const stab_batch_program *prog, int32_t circuit);

void stab_batch_program_destroy(stab_batch_program *prog);

/* Run every circuit's program once from the batch's current state.  out_bits (host, may be
 * NULL) receives the records: circuit c's bits LSB-first from byte sum_{c' < c}
 * ceil(records(c') / 8).  elapsed_ms (may be NULL) receives the device time of the launch.
 * Errors: STAB_EINVAL (program of another batch), STAB_ERANGE, STAB_ENOMEM, STAB_EDEVICE,
 * STAB_EINTERNAL (device consistency check; the batch is then unusable). */
int stab_batch_execute(stab_batch *batch, const stab_batch_program *prog, uint8_t *out_bits,
                       float *elapsed_ms);

/* Launch configuration of a batch program: the row tile of its rowsum updates.  Bits 0-7:
 * rows each lane group keeps in flight (2, 4 or 8); bit 8 (STAB_TILE_WHOLE_WAVE): every row
 * takes a whole 64-lane wave, else a row takes the smallest power of two of lanes that holds
 * its x words, so one wave updates several rows of a small circuit per load.  With two x
 * words per lane (a circuit above 4096 qubits in the batch) 8 rows in flight run as 4.  Bit 9
 * (STAB_TILE_ONE_BLOCK): the kernel variant whose registers are sized for one block per compute
 * unit (no spills), else capped so two blocks share one.  0 = the default (8 rows in flight with
 * one x word per lane, 2 with two; lanes sized to the row; two blocks per compute unit).
 * The configuration changes speed only: every configuration writes the same records and
 * leaves the same tableaux. */
#define STAB_TILE_WHOLE_WAVE 0x100
#define STAB_TILE_ONE_BLOCK  0x200
#define STAB_TUNE_FORCE 1

/* Autotuner: time every launch configuration on this program from the batch's current
 * state and keep the fastest in prog (used by later stab_batch_execute calls).  Each
 * candidate runs the first meas_quota measurement instructions of every circuit (0: the
 * whole program) from the same saved state; the records of all candidates must agree, and
 * the batch's tableaux, instruction counters and work counters are restored afterwards, so
 * tuning leaves no trace in what the batch computes.  A device copy of the batch
 * (stab_batch_bytes) is allocated for the duration of the call.  The choice is cached per
 * process under a fingerprint of the program's shape (circuit sizes, step, gate and measured
 * target counts) and the device's compute-unit count; when the environment variable
 * STAB_TUNE_CACHE names a file, choices are also read from and appended to it ("<key hex>
 * <tile>" lines); when STAB_TUNE_LOG is set, each candidate's time is printed to stderr.  A
 * cached choice is used without timing unless flags has STAB_TUNE_FORCE.
 * tile_out (may be NULL) receives the configuration.  Errors: as stab_batch_execute;
 * STAB_EINTERNAL also when two configurations disagree (the batch is then restored). */
int stab_batch_autotune(stab_batch *batch, stab_batch_program *prog, int32_t meas_quota,
                        int32_t flags, int32_t *tile_out);

/* Set prog's launch configuration by hand (0 or a configuration as above).  Errors:
 * STAB_EINVAL (NULL program, unknown configuration). */
int stab_batch_program_set_tile(stab_batch_program *prog, int32_t tile);

/* prog's launch configuration, or -1 for NULL. */
int32_t stab_batch_program_tile(const stab_batch_program *prog);

/* Circuit c's tableau in the stab_get_tableau layout (x[2n][n], z[2n][n], r[2n]). */
int stab_batch_get_tableau(stab_batch *batch, int32_t circuit, uint8_t *x, uint8_t *z, uint8_t *r);

/* Work counters of the batch since creation: [2] deterministic measurements, [4] random
 * measurements, [5] rows updated by rowsum or multiplied by deterministic reductions,
 * [6] bytes the measurements must move (target columns at one 8-byte word per row, pivot
 * row, rowsum rows read and written, row moves; multiplied rows read), [7] bytes of the
 * band passes (every row read, and written when a gate changed x|z); the others stay 0.
 * ncounters <= 12. */
int stab_batch_get_counters(stab_batch *batch, uint64_t *counters, int32_t ncounters);

/* Pairwise commutation of Pauli strings, the grouping check of Sec. 3.2: strings A_i
 * (i < na) and B_j (j < nb) on n qubits, each stored like a tableau row (ceil(n/64) uint64
 * x-words, then as many z-words; bit q%64 of word q/64 is qubit q), device memory.  Writes,
 * packed 64 columns per uint64 word, out[i][j / 64] bit j % 64:
 *   gc  (group-wise): 1 iff A_i and B_j anticommute, i.e. the parity of
 *       sum_q (xA_q zB_q + zA_q xB_q) is odd;
 *   qwc (qubit-wise): 1 iff some qubit's single-qubit factors anticommute.
 * gc and qwc are device arrays [na][ceil(nb/64)] (either may be NULL, not both); padding bits
 * of a row's last word are 0.  Asynchronous on hip_stream; nothing is allocated.  Errors:
 * STAB_EINVAL (NULL or misaligned arrays, n < 1, negative counts), STAB_ERANGE
 * (na > 65535 * 64), STAB_EDEVICE (launch failure). */
int stab_commute(const uint64_t *A, int32_t na, const uint64_t *B, int32_t nb, int32_t n,
                 uint64_t *gc, uint64_t *qwc, void *hip_stream);

/* ---------------------------------------------------------------------------------------
 * Continuous batching of sampling requests (the parallel sampling of Sec. 6 of the paper, run
 * as a service).  A server owns a caller-provided device arena; a request (a registered op
 * stream, a shot count, a seed) is admitted in arrival order once its bytes
 * (stab_server_request_bytes) fit in the free arena.  Shot s of a request with seed k draws with
 * RNG key (k, s) and counts its own instructions from 0, so its records equal those of
 * stab_sample(stream, shots, seed = k) run alone, whatever else is resident.  Two lanes:
 *   STAB_LANE_BATCH  every shot has its own tableau; each stab_server_step() runs ONE launch
 *                    that advances every resident batch-lane shot by one measurement step (a
 *                    round of a memory experiment; four while no request waits for admission):
 *                    rounds of all resident requests share the launch, new requests join at
 *                    the next step, finished ones leave.
 *   STAB_LANE_SHARED the request's shots share one x|z tableau (STAB_MODE_SHARED; Pauli noise
 *                    only).  Admission enqueues the request's whole stream on one of the
 *                    server's device streams; requests on different streams overlap on the
 *                    device, and a step retires those that completed.
 *   STAB_LANE_AUTO   (default) SHARED for streams without T1T2 noise, else BATCH.
 * A server is not thread-safe.  Per request it allocates nothing on the device: the shared lane
 * compiles and uploads a stream once per power-of-two shot bucket (at its first request), and
 * stages records in 64 MiB of pinned host memory allocated at the first shared-lane request.
 * ------------------------------------------------------------------------------------- */
typedef struct stab_server stab_server;

#define STAB_LANE_AUTO   0
#define STAB_LANE_BATCH  1
#define STAB_LANE_SHARED 2

/* Create a server on dev_buf (buf_bytes, 256-byte aligned, owned by the caller until
 * stab_server_destroy; its size is the admission cap).  hip_stream carries the batch lane; the
 * shared lane runs on streams of the server's own. */
int stab_server_create(void *dev_buf, uint64_t buf_bytes, void *hip_stream, stab_server **out);
void stab_server_destroy(stab_server *server);

/* Validate, compile and upload an op stream for n qubits (<= 8192); *prog_out receives its
 * id.  Errors as stab_batch_compile. */
int stab_server_program(stab_server *server, const stab_instr *instrs, int32_t ninstr,
                        const int32_t *targets, int64_t ntargets, int32_t n, int32_t *prog_out);

/* Lane of the program's later requests (STAB_LANE_*).  Errors: STAB_EINVAL (unknown program or
 * lane; SHARED for a stream with T1T2 noise). */
int stab_server_set_lane(stab_server *server, int32_t prog, int32_t lane);

/* Records per shot of a registered program, or -1. */
int64_t stab_server_program_records(const stab_server *server, int32_t prog);

/* Arena bytes a request of `shots` shots of a registered program occupies in its lane (batch:
 * per shot its tableau, signs and the columns of its largest measurement instruction, then the
 * records; shared: one tableau with the signs of the shot bucket and the execution scratch). */
int stab_server_request_bytes(const stab_server *server, int32_t prog, int32_t shots,
                              uint64_t *bytes_out);

/* Queue a request (host only; nothing runs until stab_server_step).  *id_out receives its id.
 * Errors: STAB_EINVAL (unknown program, shots < 1), STAB_ERANGE (larger than the arena, or its
 * records larger than the pinned staging), STAB_ENOMEM (the pinned staging). */
int stab_server_submit(stab_server *server, int32_t prog, int32_t shots, uint64_t seed,
                       int64_t *id_out);

/* Retire shared-lane requests that completed, admit what fits (shared-lane requests start at
 * once), run one batch-lane launch over every resident batch-lane shot and retire the batch-lane
 * requests that finished (their records are copied to host memory and their bytes freed).  Waits
 * for the batch launch only.  *finished_out (may be NULL) receives the number of requests that
 * finished. */
int stab_server_step(stab_server *server, int32_t *finished_out);

/* Drop a request: queued, resident (a shared-lane request's launches finish; its bytes are freed
 * when they have) or finished and not taken.  It never appears in stab_server_poll afterwards.
 * Errors: STAB_EINVAL (unknown id, or already cancelled or taken). */
int stab_server_cancel(stab_server *server, int64_t id);

/* Ids of finished requests not returned before, oldest first; returns how many it wrote. */
int stab_server_poll(stab_server *server, int64_t *ids, int32_t max_ids);

/* Records per shot of a finished request (-1 if unknown or already taken). */
int64_t stab_server_records(const stab_server *server, int64_t id);

/* Copy a finished request's records (shot s's bits LSB-first from byte s * ceil(M/8)) and
 * forget the request. */
int stab_server_result(stab_server *server, int64_t id, uint8_t *out_bits);

/* [0] queued requests, [1] resident requests, [2] resident unfinished shots, [3] arena bytes
 * in use, [4] arena bytes, [5] batch launches run, [6] requests finished, [7] shared-lane
 * requests in flight, [8] requests cancelled.  nout <= 9. */
int stab_server_stats(const stab_server *server, int64_t *out, int32_t nout);

/* Message of the last error on this thread ("" if none).  The paper defines no error
 * reporting; this is the library's own convention for every call above. */
const char *stab_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LIBSTAB_ABI_H_ */
