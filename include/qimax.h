/* qimax.h -- C ABI of the MI355X (gfx950) generator-propagation library.
 *
 * The library propagates the n stabilizer generators of |0^n> through a circuit in
 * the Heisenberg picture (paper, Sec. II-A, eq. (1)): every generator starts as
 * Z_j (qubit j holds Z, the others I) and each operator U replaces a generator G by
 * U G U^dagger. A generator is a real linear combination of Pauli strings (the
 * paper's "simple form", Sec. II-A and III-B), stored on the device as a sorted
 * list of (key, weight) terms per generator.
 *
 * Keys are the paper's base-4 Pauli index (Sec. III-B): digit d_j of qubit j in
 * {I=0, X=1, Y=2, Z=3}, key = sum_j d_j 4^(n-1-j), qubit 0 the most significant digit.
 * For n <= 32 a key is one uint64 word; for 32 < n <= 64 it is two words, word 0 the
 * low 64 bits. On the device keys are 32-, 64- or 128-bit integers (n <= 16, 32, 64).
 *
 * Threading: a context is not thread-safe; distinct contexts are independent.
 * Errors: every call returns a qimax_status; no exception crosses this boundary.
 * qimax_last_error() describes the last failure of a context.
 */
#ifndef QIMAX_H
#define QIMAX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qimax_ctx qimax_ctx;

typedef enum {
  QIMAX_OK = 0,
  QIMAX_EINVAL = -1,    /* bad argument: qubit out of range, bad PTM, bad gate code  */
  QIMAX_ENOMEM = -2,    /* device memory (or opts.mem_cap_bytes) exhausted           */
  QIMAX_EDEVICE = -3,   /* a HIP call failed, or a kernel reported an inconsistency  */
  QIMAX_ETOOLARGE = -4, /* request outside the implemented range (n, fan-out, ...)   */
  QIMAX_ESTATE = -5     /* the context is unusable after an earlier device error     */
} qimax_status;

/* Gate codes of the instruction form {gate, wire, theta} (Sec. III-A). Rotations are
 * R_s(theta) = exp(-i theta s / 2); T = R_z(pi/4) and SX = R_x(pi/2) up to a phase. The
 * two-qubit gates (codes 12-17) form the V_k runs; consecutive two-qubit gates of a run on
 * the same pair of wires (no gate of the run touching either wire between them) are fused
 * into one 16x16 operator. ISWAP is Clifford; RXX / RYY / RZZ expand a term that
 * anticommutes with the rotation's Pauli pair into two images (Sec. II-C). */
enum {
  QIMAX_GATE_H = 0, QIMAX_GATE_S = 1, QIMAX_GATE_SDG = 2, QIMAX_GATE_T = 3, QIMAX_GATE_TDG = 4,
  QIMAX_GATE_SX = 5, QIMAX_GATE_X = 6, QIMAX_GATE_Y = 7, QIMAX_GATE_Z = 8,
  QIMAX_GATE_RX = 9, QIMAX_GATE_RY = 10, QIMAX_GATE_RZ = 11,
  QIMAX_GATE_CX = 12, /* q0 = control, q1 = target */
  QIMAX_GATE_CZ = 13,
  QIMAX_GATE_ISWAP = 14, /* exp(i pi/4 (XX + YY)) on (q0, q1) */
  QIMAX_GATE_RXX = 15,   /* exp(-i theta XX / 2) on (q0, q1); RYY, RZZ likewise */
  QIMAX_GATE_RYY = 16,
  QIMAX_GATE_RZZ = 17
};

typedef struct {
  int precision;        /* 64: FP64 weights; 32: FP32 weights                                */
  int fp32_merge;       /* precision 32 only: 0 = compensated FP32 sums (TwoSum), 1 = sums
                           accumulated in FP64 and rounded once                               */
  double prune_eps;     /* at the end of each apply call, drop terms with |w| <= prune_eps;
                           internal passes drop exact zeros only (Sec. III-B)                 */
  size_t mem_cap_bytes; /* 0 = limited by the device only; otherwise a cap on the bytes the
                           context may hold on the device                                     */
  void* hip_stream;     /* hipStream_t to run on, or NULL for the context's own stream        */
  int validate;         /* 1 (default): every PTM must be unital, trace-preserving and
                           orthogonal within 1e-12; 0 admits any real matrix                  */
  int device;           /* HIP device ordinal; -1 = the current device                        */
} qimax_opts;

/* Fills *o with the defaults: precision 64, fp32_merge 0, prune_eps 0, no memory cap,
 * own stream, validate 1, current device. */
void qimax_default_opts(qimax_opts* o);

/* One grouped operator as its real Pauli transfer matrix (PTM), Sec. III-C:
 * R[a][b] = (1/2^k) Tr(P_a U P_b U^dagger) over the Pauli basis (I, X, Y, Z), row-major
 * R[out][in], 4x4 for arity 1 and 16x16 for arity 2. The two-qubit basis index is
 * 4*p(q[0]) + p(q[1]). The image of a term whose local Pauli is b is
 * sum_a R[a][b] * (the term with that local Pauli replaced by a). */
typedef struct {
  uint32_t arity;    /* 1 or 2                                                           */
  uint32_t q[2];     /* wires; q[1] ignored for arity 1; q[0] != q[1] for arity 2         */
  const double* ptm; /* host pointer, 16 or 256 doubles; copied before the call returns   */
} qimax_op;

/* Creates a context on the device holding the n generators Z_0 .. Z_{n-1} of |0^n>
 * (Sec. II-A; the initial simple form of Sec. IV: weights all 1, every digit string a
 * single Z). 1 <= n <= 64 (QIMAX_ETOOLARGE beyond). opts may be NULL
 * for the defaults. On success *out owns all device memory of the context. */
qimax_status qimax_create(uint32_t n, const qimax_opts* opts, qimax_ctx** out);

/* Resets the generators to Z_0 .. Z_{n-1} (the state qimax_create leaves), keeping the
 * context's device buffers and options. Counters (qimax_get_stats) keep accumulating. */
qimax_status qimax_reset(qimax_ctx* ctx);

/* Applies the operators in array order: each generator G becomes U G U^dagger with
 * U = U_{n_ops-1} ... U_0. Every term expands into its nonzero images (the flatten of
 * Sec. IV, eq. (3)); images with equal keys are summed and exact zeros dropped; at the
 * end of the call terms with |w| <= prune_eps are dropped. Operators on disjoint wires
 * may be fused into one pass; overlapping ones keep their order (Alg. 2).
 * Inputs are host memory and are copied. On failure the generators are unchanged. */
qimax_status qimax_apply_layer(qimax_ctx* ctx, const qimax_op* ops, size_t n_ops);

/* Applies m instructions {gate[i], (q0[i], q1[i]), theta[i]} (host arrays, Sec. III-A)
 * as one layer: the library splits them into the paper's alternating runs U_k (one-qubit
 * gates only) and V_k (two-qubit gates only) (Sec. III-A, Alg. 2), composes the gates of
 * every U_{k,j} into one transfer matrix on the device (Alg. 1), and applies the result as
 * qimax_apply_layer does. theta is ignored for gates without a parameter.
 * On failure the generators are unchanged. */
qimax_status qimax_apply_circuit(qimax_ctx* ctx, const uint8_t* gate, const uint32_t* q0,
                                 const uint32_t* q1, const double* theta, size_t m);

/* The grouping of qimax_apply_circuit without applying it: writes up to `cap` grouped
 * operators (ops[i].ptm points into ptm_buf, 16 or 256 doubles each, packed in order;
 * ptm_buf must hold 256*cap doubles) and sets *n_ops to the total count; *n_u / *n_v
 * receive K and K', the numbers of U and V runs. cap = 0 only counts. */
qimax_status qimax_group_circuit(qimax_ctx* ctx, const uint8_t* gate, const uint32_t* q0,
                                 const uint32_t* q1, const double* theta, size_t m,
                                 qimax_op* ops, double* ptm_buf, size_t cap, size_t* n_ops,
                                 size_t* n_u, size_t* n_v);

/* Applies the operators a call kept back: a call whose operators are all Clifford (signed
 * permutations of the terms, Sec. III-C-2) only records them; they join the next call's
 * first pass, or readout applies them first. (A call with an expanding operator applies its
 * Clifford operators within its own passes.) After qimax_flush the device holds the
 * generators of every operator applied so far (the end of the paper's timing window, Sec. V).
 * On failure the generators are unchanged. */
qimax_status qimax_flush(qimax_ctx* ctx);

/* A recorded step, replayed as one HIP graph (multi-circuit execution and fixed circuits are
 * the paper's stated next step, Sec. VI): qimax_graph_record runs reset, every layer of the
 * circuit (layer_end[0..n_layers), NULL for one layer) and qimax_flush once, capturing the
 * launches between the host's synchronisations; qimax_graph_launch then replays them on the
 * context's stream with no host work in between, leaving the same generators (bit for bit)
 * and counting the same statistics. The replay is asynchronous (qimax_sync waits).
 * The record call runs the step uncaptured until three runs in a row grew no buffer (a step
 * moves the term buffers through up to three roles), then once captured (recording itself
 * never allocates; a step that still needs a larger buffer fails with QIMAX_ESTATE and the
 * context is reset). The autotuner does not explore during these runs. A graph
 * refers to its context's buffers: a replay is refused (QIMAX_ESTATE) once any of them has
 * been reallocated or freed since the recording. Destroy graphs before their context. */
typedef struct qimax_graph qimax_graph;
qimax_status qimax_graph_record(qimax_ctx* ctx, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                                const double* theta, size_t m, const uint64_t* layer_end, size_t n_layers,
                                qimax_graph** out);
qimax_status qimax_graph_launch(qimax_graph* g);
void qimax_graph_destroy(qimax_graph* g);

/* Total number of terms held (all generators). Cheap; synchronises the stream. Operators
 * kept back by the last call (see qimax_flush) do not change the count. */
qimax_status qimax_num_terms(qimax_ctx* ctx, uint64_t* T);

/* Copies the generators to host memory (the paper's Lambda and index tensor, Alg. 2):
 * gen_off[0..n] (n+1 words, generator j owns terms gen_off[j] .. gen_off[j+1]-1),
 * keys (T*W words, W = 1 for n <= 32, 2 for n <= 64) and weights as FP64. Terms come out ascending by
 * key within each generator. Two-call size query: with cap < T only *T is written
 * (gen_off, keys and w may then be NULL) and QIMAX_OK is returned. */
qimax_status qimax_get_generators(qimax_ctx* ctx, uint64_t* gen_off, uint64_t* keys, double* w,
                                  size_t cap, size_t* T);

/* The generators in the paper's x/z form (Sec. II-A; the index tensor of Alg. 2 as bit
 * vectors): gen_off[0..n] as for qimax_get_generators; for term i, bit q of x[i] is set when
 * qubit q holds X or Y, bit q of z[i] when it holds Y or Z (one word each: n <= 64); weights
 * as FP64. Terms come out in the same order as qimax_get_generators (ascending base-4 index
 * within each generator). The conversion runs on the device. Two-call size query as above
 * (gen_off is written in both calls when not NULL). */
qimax_status qimax_get_generators_xz(qimax_ctx* ctx, uint64_t* gen_off, uint64_t* x, uint64_t* z,
                                     double* w, size_t cap, size_t* T);

/* <psi|P|psi> = Tr(rho P) for rho = 2^-n prod_j (I + G_j) (eq. (2)), P given as n letters
 * of "IXYZ", qubit 0 first. This is the coefficient of P in prod_j (I + G_j), not the sum
 * of P's weights over the generators (that reading of the probability formula of Sec. II-B
 * fails as soon as two generators share a string). Two methods, both exact up to rounding:
 *  - every generator a single term of weight +-1 (a stabilizer state): GF(2) elimination of
 *    the generators' x/z vectors on the host, O(n^3);
 *  - otherwise, for n <= 30: a statevector on the device (2^n complex doubles, twice, plus
 *    the terms; allocated for the call and freed): a seeded random vector is projected by
 *    (I + G_j)/2 for every j, normalised, and <v|P|v> is reduced on the device. Cost: the
 *    sum of all generators' term counts times 2^n. QIMAX_ETOOLARGE for n > 30 or a cost
 *    above 4e13; QIMAX_ENOMEM when the statevector does not fit.
 * Not part of propagation; the generators stay as they are. */
qimax_status qimax_expect(qimax_ctx* ctx, const char* pauli, double* out);

/* qimax_expect for k strings at once (paulis: k*n letters, string i at paulis + i*n; no
 * terminators needed): one elimination or one projected statevector for all of them. */
qimax_status qimax_expect_many(qimax_ctx* ctx, const char* paulis, size_t k, double* out);

/* The paper's single-qubit outcome probabilities p_{k,0} = (1 + <Z_k>)/2 (Sec. II-B) for
 * every qubit k in one call (p0: n doubles), by the methods of qimax_expect. */
qimax_status qimax_prob_zero_all(qimax_ctx* ctx, double* p0);

/* Compares the generators of two contexts of the same n on the same device, term lists
 * matched by key, a missing key counting as weight 0: per generator j, diff_norm[j] =
 * ||w_a - w_b||_2 over the union of keys, ref_norm[j] = ||w_b||_2, and n_tau_diff[j] = the
 * number of keys with |w| > tau on exactly one side. Used to state the error of an FP32
 * result (a) against an FP64 one (b): per generator diff_norm / ref_norm. Runs on the
 * device, on a's stream (both streams are synchronised first). */
qimax_status qimax_compare(qimax_ctx* a, qimax_ctx* b, double tau, double* diff_norm, double* ref_norm,
                           uint64_t* n_tau_diff);

/* qimax_compare for callers that cannot allocate device memory (code under stream capture,
 * serving loops that must not call hipMalloc): same arguments, same results. Instead of
 * allocating, the tile arrays, sums and counters of the comparison live in a fixed 4 MiB
 * device array that every GPU the library runs on holds until the process ends; that bounds
 * the two contexts' tiles (4096 terms each, per generator) to roughly 200,000 together, about
 * 8e8 terms: beyond, QIMAX_ETOOLARGE. Deferred operators are refused, not applied (applying
 * them allocates): QIMAX_ESTATE until qimax_flush has run on both contexts. Every call on a
 * GPU uses that GPU's one array: calls that overlap on the same GPU (from several threads)
 * race and must be serialised by the caller. Device memory is never allocated or freed. */
qimax_status qimax_compare_noalloc(qimax_ctx* a, qimax_ctx* b, double tau, double* diff_norm, double* ref_norm,
                                   uint64_t* n_tau_diff);

/* Counters since qimax_create (host-side bookkeeping, no device work). */
typedef struct {
  uint64_t terms;          /* current number of terms                                     */
  uint64_t passes;         /* expanding passes executed                                   */
  uint64_t term_updates;   /* term updates: one per output image of every grouped operator
                              (U_k / V_k run) of the circuit, each group counted once: an
                              expanding group counts its images, sum over terms of the
                              product of the nonzero counts of its wires' PTM columns; a
                              Clifford group counts the terms it acts on                  */
  uint64_t images;         /* images materialised by the expand kernel                    */
  uint64_t sort_elems;     /* elements sorted                                             */
  uint64_t peak_bytes;     /* peak device bytes held by the context                       */
  uint64_t alloc_bytes;    /* device bytes currently held                                 */
  double host_wait_ms;     /* host time blocked in stream synchronisations of passes      */
  double host_busy_ms;     /* host time spent inside apply calls outside those waits      */
  uint64_t syncs;          /* stream synchronisations of passes                           */
  uint64_t sort_redos;     /* rounds sorted again with global passes only (a bucket of
                              equal top digits did not fit a chunk-local sort)            */
  uint64_t tuned_classes;  /* round size classes whose sort variant the autotuner fixed   */
  uint64_t rounds;         /* propagation rounds run (one set of launches per pass)        */
  double alg_bytes;        /* algorithmic bytes of those rounds: (T_in + T_out) * (key bytes
                              + weight bytes) per round, the terms a pass must read and write */
} qimax_stats;

qimax_status qimax_get_stats(const qimax_ctx* ctx, qimax_stats* out);

/* The autotuner's state (multi-circuit execution, Sec. VI: tile and bucket choices made per
 * size class of rounds). A size class is the key size, the weight precision, floor(log2) of
 * the round's image capacity and whether dense accumulation applies. The candidates are the
 * same sort with: 0 the heuristic number of top-digit passes, 1 one pass more, 2 sort tiles
 * claimed in one global order instead of per XCD, 3 and 4 as 0 and 1 with multi-launch
 * global passes (histogram, scan, scatter) instead of single-sweep ones, 5 dense
 * accumulation (classes where it applies). Writes min(cap, classes) entries to out (out may
 * be NULL when cap is 0) and the number of classes to *n. Host bookkeeping, no device work. */
typedef struct {
  uint32_t key_bytes;        /* 4, 8 or 16                                                 */
  uint32_t weight_bits;      /* 32 or 64                                                   */
  uint32_t log2_images;      /* floor(log2) of the round's image capacity                  */
  uint32_t dense_candidate;  /* 1 when dense accumulation is a candidate                   */
  int32_t best;              /* the chosen candidate, -1 while candidates are still timed  */
  uint32_t tried;            /* rounds timed so far (each candidate twice, in turns)       */
  float ms[6];               /* each candidate's least round time on the device (ms; 1e30
                                for a candidate whose buckets overflowed a chunk)           */
} qimax_tune_entry;
qimax_status qimax_get_tuning(const qimax_ctx* ctx, qimax_tune_entry* out, size_t cap, size_t* n);

/* The term_updates counter split by generator: out[j] for j < n (host bookkeeping). */
qimax_status qimax_get_generator_updates(const qimax_ctx* ctx, uint64_t* out, size_t n);

/* Per-kernel timing with HIP events on the context's stream. qimax_profile(ctx, 1) clears
 * the totals and starts recording every kernel launch; qimax_profile(ctx, 0) stops.
 * qimax_profile_read synchronises, then writes up to `cap` entries (one per kernel kind that
 * ran) and sets *n to the number of kinds. alg_bytes is the algorithmic traffic of those
 * launches: the bytes the kernel's job has to read and write, not the bytes it moved.
 * `name` points to a static string. */
typedef struct {
  const char* name;
  uint64_t launches;
  double total_ms;
  double alg_bytes;
} qimax_kernel_time;

qimax_status qimax_profile(qimax_ctx* ctx, int enable);
/* Restrict the timing to one kernel kind (its name as qimax_profile_read reports it, e.g.
 * "sort_scatter"); NULL or "" times every kind again. Fewer timed kinds, fewer event records
 * on the host. QIMAX_EINVAL for an unknown name. */
qimax_status qimax_profile_only(qimax_ctx* ctx, const char* kernel);
qimax_status qimax_profile_read(qimax_ctx* ctx, qimax_kernel_time* out, size_t cap, size_t* n);

/* ------------------------------------------------------------------ batches of circuits
 * A batch holds the generators of many circuits (each with its own n <= max_n, layers and
 * prune threshold) in one device term array. Every qimax_batch_step advances each active
 * circuit by one propagation pass, all circuits together in one set of kernel launches, so
 * small circuits share launches instead of paying them one by one (multi-circuit execution
 * is the paper's stated next step, Sec. VI). Circuits may be submitted at any time; they
 * join the array at the next step (continuous batching). A finished circuit's generators
 * are copied to host memory at the end of its last step and are identical to what a
 * single-circuit context computes for the same instructions: each generator is its own
 * segment and is never mixed with other segments. */
typedef struct qimax_batch qimax_batch;

typedef struct {
  uint32_t n;               /* qubits, 1..max_n of the batch                              */
  const uint8_t* gate;      /* instruction arrays as for qimax_apply_circuit (host memory) */
  const uint32_t* q0;
  const uint32_t* q1;
  const double* theta;      /* may be NULL when no gate has a parameter                    */
  size_t m;
  const uint64_t* layer_end; /* optional: ends of the layers (prune points); NULL = one layer */
  size_t n_layers;
  double prune_eps;         /* as qimax_opts.prune_eps, for this circuit                   */
} qimax_circuit;

typedef struct {
  uint64_t queued, active, finished, rounds, terms, term_updates, alloc_bytes, peak_bytes;
} qimax_batch_info_t;

/* opts: precision, fp32_merge, mem_cap_bytes, hip_stream, device apply to the whole batch
 * (prune_eps is per circuit). max_n: the largest n the batch accepts; it picks the key
 * class (<= 16: 32-bit, <= 32: 64-bit, <= 64: 128-bit keys), so group circuits by class. */
qimax_status qimax_batch_create(const qimax_opts* opts, uint32_t max_n, qimax_batch** out);
/* Groups and plans the circuit (inputs are copied) and queues it; *id names it. */
qimax_status qimax_batch_submit(qimax_batch* b, const qimax_circuit* c, uint64_t* id);
/* Admits queued circuits, then runs one pass of every active circuit. *n_active (may be
 * NULL) receives the number of circuits still queued or active afterwards. */
qimax_status qimax_batch_step(qimax_batch* b, size_t* n_active);
/* Steps until no circuit is queued or active. */
qimax_status qimax_batch_run(qimax_batch* b);
/* Ids of circuits finished since the last poll. With cap < count only *n is written. */
qimax_status qimax_batch_poll(qimax_batch* b, uint64_t* ids, size_t cap, size_t* n);
/* A finished circuit's generators in the qimax_get_generators format (two-call size query;
 * a successful full copy releases the circuit). */
qimax_status qimax_batch_fetch(qimax_batch* b, uint64_t id, uint64_t* gen_off, uint64_t* keys, double* w,
                               size_t cap, size_t* T);
qimax_status qimax_batch_info(const qimax_batch* b, qimax_batch_info_t* out);
/* Term updates attributed to one circuit so far (same definition as qimax_stats). */
qimax_status qimax_batch_circuit_updates(const qimax_batch* b, uint64_t id, uint64_t* updates);
/* The batch's internal context, for qimax_profile / qimax_profile_read / qimax_get_stats /
 * qimax_sync only. */
qimax_ctx* qimax_batch_context(qimax_batch* b);
const char* qimax_batch_last_error(const qimax_batch* b);
void qimax_batch_destroy(qimax_batch* b);

/* Measurement aid, not part of propagation: copies `bytes` (rounded down to 8-byte words)
 * between two fresh device buffers `reps` times with a plain copy kernel on the null stream
 * and returns the average milliseconds per copy. Read traffic counters of this run give
 * the scale between counter units and bytes moved. */
qimax_status qimax_copy_probe(size_t bytes, int reps, double* ms);

/* Blocks until all work of the context has finished. */
qimax_status qimax_sync(qimax_ctx* ctx);

/* Text of the last error of ctx (owned by ctx, valid until its next call); ctx may be
 * NULL for errors of qimax_create. */
const char* qimax_last_error(const qimax_ctx* ctx);

/* Releases all device memory of the context. NULL is ignored. */
void qimax_destroy(qimax_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* QIMAX_H */
