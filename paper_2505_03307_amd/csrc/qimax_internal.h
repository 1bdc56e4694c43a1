// Internal declarations shared by the host runtime (qimax_ctx.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace qimax {

// ---------------------------------------------------------------------------------
// Operator descriptors as the kernels read them (device memory, uniform per launch).
//
// Digits: a key is the base-4 Pauli index; the digit of qubit q sits at bit position
// pos(q) = 2*(n-1-q). Local index of a two-qubit op = 4*d(q0) + d(q1).

// A signed permutation of the local Pauli basis (a Clifford operator: every column of
// its PTM holds a single +-1). table byte e for local input index i (i < 16):
// bits 0..3 output index, bit 4 sign flip. Entries 0..7 in lo, 8..15 in hi.
struct PermDesc {
  uint32_t arity;
  uint32_t pa;  // bit position of q[0]
  uint32_t pb;  // bit position of q[1] (arity 2)
  uint32_t pad;
  uint64_t lo, hi;
};

// An expanding one-qubit operator: for local digit d, cnt[d] nonzero images with output
// digit out[d][k] and PTM value val[d][k] (FP64) / valf[d][k] (rounded to FP32).
struct Exp1Desc {
  uint32_t pos;
  uint8_t cnt[4];
  uint8_t out[4][4];
  uint32_t rcp[4];  // ceil(2^32 / cnt) for cnt >= 2 (division by the count without a divide)
  double val[4][4];
  float valf[4][4];
};

// An expanding two-qubit operator (same layout over 16 local indices).
struct Exp2Desc {
  uint32_t pa, pb;
  uint8_t cnt[16];
  uint8_t out[16][16];
  uint32_t rcp[16];
  double val[16][16];
  float valf[16][16];
};

// One pass: terms -> [A perms] -> [E expanding ops] -> [B perms] -> images.
// A Clifford chain compiled into per-byte tables: byte k of a key holds the digits of four
// qubits; tab_key[k*256 + b] is the image key of that 4-qubit Pauli string under the chain
// and tab_neg[k*256 + b] its sign bit (bit 0) and number of Y digits mod 4 (bits 1-2).
// Conjugation is multiplicative, so the image of a whole key is the product of its bytes'
// images (they commute) with the product's phase.
struct ChainTable {
  const void* tab_key;     // K[nbytes * 256]
  const uint8_t* tab_neg;  // [nbytes * 256]
};

struct PassArgs {
  const PermDesc* A;
  const Exp1Desc* E1;
  const Exp2Desc* E2;
  const PermDesc* B;
  uint32_t nA, nE1, nE2, nB;
  ChainTable tA, tB;       // used instead of the op lists when useA / useB is set
  uint32_t useA, useB;
  uint32_t drop;           // the entry's terms leave the array (f = 0)
  uint32_t pad;
  double thr;              // merge keeps |w| > thr
};

// A chain of permutation ops to compile into a ChainTable.
struct TableJob {
  const PermDesc* ops;
  uint32_t n_ops;
  uint32_t pad;
  void* tab_key;
  uint8_t* tab_neg;
};

constexpr int kChainTableMin = 12;  // chains at least this long are compiled into tables

// Segment-aligned tiling of an array of segments (generators): block b covers
// [blk_begin[b], blk_end[b]) inside segment blk_seg[b]; segment s owns blocks
// seg_blk[s] .. seg_blk[s+1]-1.
struct Tiling {
  const uint64_t* blk_begin;
  const uint64_t* blk_end;
  const uint32_t* blk_seg;
  const uint32_t* seg_blk;
  uint32_t n_blocks;  // tiles launched (an upper bound when n_dev is set)
  uint32_t n_segs;
  const uint32_t* n_dev;  // if set: the actual number of tiles, known only on the device;
                          // tiles beyond it are empty and their blocks return at once
  const uint32_t* xrange; // if set (9 entries): tiles [xrange[x], xrange[x+1]) form whole
                          // segments and are claimed first by the blocks running on XCD x
};
constexpr int kXcds = 8;  // accelerator complex dies of the chip; each has its own L2

constexpr int kSortBlock = 256;            // threads per sort / merge block
constexpr int kSortItems = 16;             // items per thread
constexpr int kSortTile = kSortBlock * kSortItems;  // elements per tile (4096)
constexpr int kRadixBits = 8;
constexpr uint32_t kSmallMaxSegs = 8192;  // segments of a small round (one block each)
constexpr int kChunkCap = 4096;  // elements a chunk-local sort holds in LDS
// largest nominal chunk of a fused round (other rounds: the expansion tiles, kExpandTile); a
// chunk extends to whole buckets at both ends, so the slack below kChunkCap takes the
// straddling buckets
constexpr int kChunkTile = 3584;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kExpandBlock = 256;
constexpr int kExpandItems = 8;
constexpr int kExpandTile = kExpandBlock * kExpandItems;
// the expansion's LDS before its tables: a window of kExpandTile + 1 32-bit relative offsets
// and an image -> parent map of 16-bit entries, rounded up to 16 bytes
constexpr size_t kExpandLdsHead = ((size_t)(kExpandTile + 1) * 4 + (size_t)kExpandTile * 2 + 15) / 16 * 16;
constexpr uint32_t kExpandHistPasses = 2;  // digit histograms the expansion may count itself
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Error bits a kernel may raise in the context's device flag word.
enum : uint32_t {
  kErrIndex = 1u,      // an index left its buffer (kernel refused to write)
  kErrFanout = 2u,     // fan-out of a term exceeded the 32-bit range
  kErrOrder = 4u,      // sorted order violated (debug checks)
  kErrSpin = 8u,       // a look-back wait gave up (bounded spin)
  kErrExpand = 16u,    // set with kErrIndex by the expand kernel
  kErrSort = 32u,      // set with kErrIndex by the sort kernels
  kErrMerge = 64u,     // set with kErrIndex by the merge kernel
  kErrRedo = 128u,     // not an error: a chunk-local sort met a bucket larger than a chunk
};

// ------------------------------------------------------------------------ kernel timing
// Optional per-kernel timing with HIP events recorded on the launch stream, plus the
// algorithmic bytes each launch must move (what the roofline is measured against).
enum KernelKind : int {
  kKInit, kKCount, kKScan, kKExpand, kKSortHist, kKSortScatter, kKMergeCount, kKMergeWrite, kKCompose, kKChunkSort,
  kKCountExpand, kKDense, kKChunkFinish, kKSmallPasses, kKNum
};
const char* kernel_kind_name(int k);

struct Prof {
  bool on = false;
  uint32_t mask = ~0u;  // kernel kinds timed while on (bit k: kind k)
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
    uint32_t count;  // back-to-back launches of `kind` between the two events
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  uint64_t launches[kKNum] = {};
  double ms[kKNum] = {};
  double bytes[kKNum] = {};
};
hipEvent_t prof_begin(Prof* p, hipStream_t s, int kind);  // nullptr when `kind` is not timed
void prof_end(Prof* p, hipStream_t s, hipEvent_t a, int kind, double bytes, uint32_t count = 1);
void prof_resolve(Prof* p);  // after the stream has been synchronised
void prof_reset(Prof* p);
void prof_destroy(Prof* p);

// ----------------------------------------------------------------------------- launchers
// KC: key class (0: uint32 keys, n <= 16; 1: uint64 keys, n <= 32).
// WP: weight precision (64 or 32).

hipError_t launch_init(int KC, int WP, void* keys, void* w, uint64_t* seg_off, uint32_t n,
                       hipStream_t s, Prof* prof = nullptr);

// T terms converted for the host: keys to n_words (1 or 2) uint64 words each, weights to FP64.
hipError_t launch_export(int KC, int WP, const void* keys, const void* w, uint64_t T, uint32_t n_words,
                         uint64_t* words, double* wd, hipStream_t s);

// Fan-out count fused with its scan (single sweep with decoupled look-back over the tiles of
// tl, claimed through *ctr): off[i] = first image of input term i, off[T] = image count;
// akeys[i] / asign[i] = the term's image under its pass's A chain and that image's sign (the
// expand kernel starts from them). status: tl.n_blocks words whose epoch field differs from
// `epoch`.
hipError_t launch_count_scan(int KC, const void* keys, uint64_t T, const Tiling& tl, const PassArgs* pas,
                             const uint32_t* seg_entry, uint64_t* off, uint64_t* status, uint32_t* ctr, uint64_t epoch,
                             uint32_t* err, void* akeys, uint8_t* asign, hipStream_t s, Prof* prof = nullptr,
                             bool wide = false);  // wide: 64-bit in-tile offsets always (tests)

// out[i] = exclusive prefix sum of in[0..i-1] for i in [0, N]; out has N+1 entries.
// tmp must hold scan_tmp_words(N) uint64 words.
size_t scan_tmp_words(uint64_t N);
hipError_t launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t N, uint64_t* tmp,
                           hipStream_t s, Prof* prof = nullptr);
hipError_t launch_scan_u64(const uint64_t* in, uint64_t* out, uint64_t N, uint64_t* tmp,
                           hipStream_t s, Prof* prof = nullptr);

// dst[s] = src_off[idx[s]] for s in [0, S]
hipError_t launch_gather_u64(const uint64_t* src_off, const uint64_t* idx, uint64_t* dst,
                             uint32_t S1, hipStream_t s, Prof* prof = nullptr);

// Images of each tile of tl (segment-aligned, at most kExpandTile each).
// keys/asign: the input terms' images under the A chain and their signs (from the count);
// any_tables: some entry has a B-chain table (sizes the dynamic LDS). With ghist set, the
// images' digits of the sort passes hp_begin .. n_pass-1 (at most kExpandHistPasses) are
// added to the segments' digit histograms ghist[(s*n_pass + p)*256 + d] (cleared before).
hipError_t launch_expand(int KC, int WP, const void* keys, const uint8_t* asign, const void* w, uint64_t T_in,
                         const uint64_t* off,
                         uint64_t T_img, const Tiling& tl, const PassArgs* pas, const uint32_t* seg_entry,
                         const uint64_t* seg_in, bool any_tables, size_t e_bytes, void* keys_out, void* w_out,
                         uint32_t* ghist, uint32_t n_pass, uint32_t hp_begin, uint32_t* err, hipStream_t s,
                         Prof* prof = nullptr, bool wide = false);  // wide: parents found in global memory (tests)

// One LSD radix pass over digit `shift` of every segment, stable, segment-local.
// hist must hold kRadix * n_blocks uint64 words; tmp scan_tmp_words(kRadix * n_blocks).
hipError_t launch_sort_pass(int KC, int WP, const void* keys_in, const void* w_in, void* keys_out,
                            void* w_out, uint64_t T, uint32_t shift, const Tiling& tl,
                            uint64_t* hist, uint64_t* hist_off, uint64_t* tmp, uint32_t* err,
                            hipStream_t s, Prof* prof = nullptr);

// The whole segment-local LSD sort in single-sweep form: one upfront histogram of every
// digit position, then one decoupled-look-back scatter per digit. keys/w are ping-pong
// pairs with the input in slot 0; *cur receives the slot holding the sorted result.
// ghist: n_segs*n_pass*256 u32, zero on entry; seg_off: the segment offsets (n_segs + 1);
// status: n_blocks*256 u64 (zeroed when allocated); tile_ctr: n_pass*kXcds u32, zero on
// entry; *epoch is advanced per digit pass.
// p_begin: first digit pass (the passes p_begin .. n_pass-1 run; p_begin > 0 groups the
// segments by their top digits only); upsweep: compute ghist for those passes first (else
// it is current).
hipError_t launch_sort_sweep(int KC, int WP, void* const keys[2], void* const w[2], uint64_t T, uint32_t key_bits,
                             uint32_t p_begin, bool upsweep, const Tiling& tl, const uint64_t* seg_off,
                             uint32_t* ghist, uint64_t* status, uint32_t* tile_ctr, uint64_t* epoch, uint32_t* err,
                             int* cur, hipStream_t s, Prof* prof = nullptr);


hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);

// Segmented sum of equal adjacent keys; keeps sums with |w| > thr (thr < 0 keeps
// everything non-zero); compacts. seg_off_out[s] for s in [0, n_segs].
// blk_cnt / blk_off must hold n_blocks (+1) words.
// status != nullptr: single-sweep merge (status: n_blocks u64 words with a fresh epoch,
// tile_ctr: one u32); otherwise count, scan, write.
// fin: seg_off_out and the packed readback area are written by one small kernel after the
// merge; in a single sweep *tile_ctr must then be zero on entry.
struct MergeFin {
  const uint64_t* img_seg;  // image offsets of the segments (S + 1)
  uint64_t* result;         // [0..S] output offsets, [S+1..2S+1] img_seg, [2S+2] error word,
                            // [2S+3] seq, written after every other word has reached memory
  uint64_t seq;
};
hipError_t launch_merge(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in, uint64_t T,
                        const Tiling& tl, const PassArgs* pas, const uint32_t* seg_entry, void* keys_out, void* w_out,
                        uint64_t out_cap, uint64_t* seg_off_out, uint32_t* blk_cnt, uint64_t* blk_off, uint64_t* tmp,
                        uint64_t* status, uint32_t* tile_ctr, uint64_t epoch, uint32_t* err, const MergeFin* fin,
                        hipStream_t s, Prof* prof = nullptr);

// Chunk-local sort and merge after the top m digit passes (see k_chunk_sort): nominal chunks
// are the tiles of tc (at most kChunkCap/2 images, segment-aligned). Each chunk is sorted in
// LDS and its runs of equal keys summed and pruned (|sum| > its pass's thr); chunks are claimed
// in order (co.ticket) and each writes its kept runs straight to its output offset, found by
// a decoupled look-back over the earlier chunks' kept counts (co.status, tagged co.epoch); a
// chunk whose earlier chunks are slow to publish is deferred instead: it leaves its runs at
// the front of its own range of co.tmp_keys / co.tmp_w. A one-block launch then scans the
// counts into co.chunk_off and writes seg_off_out and the packed readback area (co.fin), and a
// last launch moves the deferred chunks' runs. Sets kErrRedo when a bucket does
// not fit a chunk (the outputs are then not valid). With m = 0 every chunk must be a whole
// segment (at most kChunkCap elements). co.img_cnt (S words, or null): the image counts of
// the segments, scanned into the readback area instead of fin.img_seg. co.ticket must be zero
// at launch.
struct ChunkOut {
  uint32_t* ticket;
  uint64_t* status;
  uint64_t epoch;
  uint32_t* chunk_cnt;     // kept terms per chunk
  uint64_t* chunk_start;   // where a deferred chunk left its runs in tmp (~0: written in place)
  uint64_t* chunk_off;     // output offset per chunk (tc.n_blocks + 1)
  void* tmp_keys;          // scratch arrays of the image length
  void* tmp_w;
  uint64_t* seg_off_out;
  MergeFin fin;
  const uint32_t* img_cnt;
  uint32_t defer_spins;    // look-back polls before a chunk is deferred
  uint64_t in_len;         // elements of the image arrays (keys_in / w_in) that may be read
};
hipError_t launch_chunk_sort_merge(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in, void* keys_out,
                                   void* w_out, uint64_t T, const Tiling& tc, uint32_t n_pass, uint32_t m,
                                   const PassArgs* pas, const uint32_t* seg_entry, const ChunkOut& co, uint32_t* err,
                                   hipStream_t s, Prof* prof = nullptr);

// Dense accumulation instead of the sort and merge (see k_dense_scatter): the T_img images
// (32-bit keys, every key < per_seg) of segments tiled by tl are added into acc (S * per_seg
// 64-bit fixed-point slots, cleared here), the slots are compacted in key order into
// keys_out / w_out (|sum| > thr, nonzero), tiles claimed through *ticket (zero at launch) with
// look-back on status (tagged epoch; dense_tile() slots per tile, S * ceil(per_seg /
// dense_tile()) tiles, tile_off one word more), and one block writes seg_off_out and fin.
size_t dense_tile();
hipError_t launch_dense_merge(int KC, int WP, const void* keys_in, const void* w_in, uint64_t T_img, const Tiling& tl,
                              uint64_t per_seg, uint32_t S, void* acc, double thr, uint32_t* ticket, uint64_t* status,
                              uint64_t epoch, uint64_t* tile_off, void* keys_out, void* w_out, uint64_t out_cap,
                              uint64_t* seg_off_out, const MergeFin& fin, uint32_t* err, hipStream_t s,
                              Prof* prof = nullptr);

// Compile chains of permutation ops into ChainTables, one job per chain (jobs in device memory).
hipError_t launch_build_tables(int KC, const TableJob* jobs, uint32_t n_jobs, hipStream_t s, Prof* prof = nullptr);

// Z_j of n_circ new circuits: circuit c's nq[c] terms are written from position dst[c].
hipError_t launch_init_many(int KC, int WP, void* keys, void* w, const uint32_t* nq, const uint64_t* dst,
                            uint32_t n_circ, hipStream_t s);

// One segment-aligned tiling built on the device: at most `tile` elements per tile, cap tiles
// written (the ones past the actual count are empty), the actual count in *n_dev and the
// per-XCD ranges of whole segments in xrange[0..8].
struct TileJob2 {
  uint64_t tile;
  uint32_t cap, pad;
  uint64_t* blk_begin;
  uint64_t* blk_end;
  uint32_t* blk_seg;
  uint32_t* seg_blk;  // S + 1 entries
  uint32_t* n_dev;
  uint32_t* xrange;   // kXcds + 1 entries
};
// The two image tilings (expand, sort/merge) of a round from the image offsets of the
// segments, so[s] = off[seg_in[s]], which also go to img_seg[0..S]. Tile ranges are clamped
// to [0, limit) (elements of the buffers they index); a tile count above cap or so[S] above
// limit sets an error bit.
hipError_t launch_make_tiles2(const uint64_t* off, const uint64_t* seg_in, uint32_t S, uint64_t* img_seg,
                              const TileJob2& j0, const TileJob2& j1, uint64_t limit, uint32_t* err, hipStream_t s);

// Count and expansion fused (see k_count_expand), for rounds whose fan-out bound is at most
// kFuseMaxFanout: tl is the tiling of the input terms into tiles of fuse_tile() terms, claimed
// in order through *ctr (zero at launch); status / epoch as for the count. img_seg (S + 1
// words) receives the segments' first images and the image count; images go to keys_out /
// w_out (out_cap elements), digit counts of passes hp_begin .. n_pass-1 to ghist.
constexpr int kFuseMaxFanout = 16;
size_t fuse_tile();

// Several consecutive passes of one circuit in one launch (k_small_passes), for passes whose
// segments stay within kChunkCap terms and images (the caller's fan-out bound): pas holds
// n_grp PassArgs (pass p of the group), kslot / wslot two slot buffers and wimg one scratch
// of S * kChunkCap elements each; cnt (n_grp * S * 3 words) receives every pass's input,
// image and kept counts per segment; the last pass's terms go to keys_out / w_out with the
// segment offsets in seg_off_out (S + 1). Keys of 4 or 8 bytes.
hipError_t launch_small_passes(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in,
                               const uint64_t* seg_in, uint32_t S, const PassArgs* pas, uint32_t n_grp,
                               void* const kslot[2], void* const wslot[2], void* wimg, uint32_t* cnt,
                               void* keys_out, void* w_out, uint64_t* seg_off_out, uint32_t* err, hipStream_t s,
                               Prof* prof = nullptr);
hipError_t launch_count_expand(int KC, int WP, const void* keys, const void* w, uint64_t T_in, const Tiling& tl,
                               const PassArgs* pas, const uint32_t* seg_entry, uint64_t* status, uint32_t* ctr,
                               uint64_t epoch, uint64_t* img_seg, void* keys_out, void* w_out, uint64_t out_cap,
                               uint32_t* ghist, uint32_t n_pass, uint32_t hp_begin, uint32_t* err, hipStream_t s,
                               Prof* prof = nullptr);

// A round whose segments each hold at most kChunkCap terms and images, one block per
// segment: A chain, fan-out, scan and images of segment s, written to its chunk
// [s*kChunkCap, s*kChunkCap + n_img(s)) of keys_out / w_out (S*kChunkCap elements); the
// chunk tiling goes to tiles.blk_begin / blk_end / blk_seg (S entries) and seg_blk (S + 1),
// n_img(s) to img_cnt[s]. Segments whose counts exceed the bound raise kErrFanout.
hipError_t launch_expand_small(int KC, int WP, const void* keys, const void* w, const uint64_t* seg_in, uint32_t S,
                               uint64_t T_in, const PassArgs* pas, const uint32_t* seg_entry, void* keys_out,
                               void* w_out, uint32_t* img_cnt, const TileJob2& tiles, uint32_t* err, hipStream_t s,
                               Prof* prof = nullptr);
// The first launch of a round: clears *err, ctr[0..n_ctr) and ghist[0..nh), copies blob_bytes
// (a multiple of 16, both addresses 16-byte aligned) from blob_host (mapped host memory, its
// device address) to blob_dev, and builds one tiling of the terms themselves (segments at
// seg_in[0..S] on the device, T terms in all; no image offsets stored).
// bytes (a multiple of 16, both addresses 16-byte aligned) from src (mapped host memory, its
// device address) to dst (device memory), in stream order: an upload with no copy call.
hipError_t launch_pull(const void* src, void* dst, size_t bytes, hipStream_t s);

hipError_t launch_round_start(const void* blob_host, void* blob_dev, size_t blob_bytes, uint32_t* err, uint32_t* ctr,
                              uint32_t n_ctr, uint32_t* ghist, uint64_t nh, const uint64_t* seg_in, uint32_t S,
                              const TileJob2& job, uint64_t T, hipStream_t s);

// Zero the error word, n_ctr tile counters and nh digit-histogram words (one launch).
hipError_t launch_round_prep(uint32_t* err, uint32_t* ctr, uint32_t n_ctr, uint32_t* ghist, uint64_t nh,
                             hipStream_t s);

// Plain copy of n words (calibration of hardware traffic counters).
hipError_t launch_copy_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s);

// Weights to FP64 (readout).
hipError_t launch_weights_to_f64(int WP, const void* w, double* out, uint64_t T, hipStream_t s, Prof* prof = nullptr);

// Grouping pass: compose chains of one-qubit gates into 4x4 PTMs (R[out][in], FP64).
// chain c covers gate indices idx[chain_off[c] .. chain_off[c+1]-1] in application order.
hipError_t launch_compose_ptm(const uint8_t* gate, const double* theta, const uint32_t* idx,
                              const uint32_t* chain_off, uint32_t n_chains, double* ptm_out,
                              hipStream_t s, Prof* prof = nullptr);

// ------------------------------------------------------------- readout (readout.hip)
// Keys as x / z bit words (bit q: qubit q), one word each (n <= 64).
hipError_t launch_keys_to_xz(int KC, const void* keys, uint64_t T, uint32_t n, uint64_t* x, uint64_t* z,
                             hipStream_t s);
// Per-generator comparison of side a with side b (see k_compare); tiles of at most
// compare_tile() elements of side a, each inside one segment; acc[2s] / acc[2s+1] and cnt[s]
// accumulate (zeroed by the caller).
size_t compare_tile();
// The fixed device array of qimax_compare_noalloc on `device` (which must be current): its
// address on that device (looked up once per device) and its size in bytes.
hipError_t compare_scratch(int device, void** ptr, size_t* bytes);
hipError_t launch_compare(int KC, int WPa, int WPb, const void* ka, const void* wa, const void* kb, const void* wb,
                          const uint64_t* b_off, const uint64_t* t_begin, const uint64_t* t_end, const uint32_t* t_seg,
                          uint32_t n_tiles, int count_ref, double tau, double* acc, unsigned long long* cnt,
                          hipStream_t s);
// Statevector readout: 2^n complex amplitudes (double2).
hipError_t launch_sv_terms(int KC, int WP, const void* keys, const void* w, uint64_t T, uint32_t n, uint64_t* xm,
                           uint64_t* zm, void* cf, hipStream_t s);
hipError_t launch_sv_random(void* v, uint64_t D, uint64_t seed, hipStream_t s);
// v <- (v + G v) / 2 for the generator given by T terms (masks and coefficients); tmp: D amplitudes.
hipError_t launch_sv_project(void* v, void* tmp, uint64_t D, const uint64_t* xm, const uint64_t* zm, const void* cf,
                             uint64_t T, hipStream_t s);
// acc[0] += |v|^2; zall = 0: acc[1] + i acc[2] += <v|c P|v> for the string (xm, zm, c);
// zall = 1: acc[1 + q] += sum_i |v_i|^2 (1 - 2 bit_q(i)) for every qubit q < n (n <= 32).
hipError_t launch_sv_reduce(const void* v, uint64_t D, uint32_t n, uint64_t xm, uint64_t zm, double c_re,
                            double c_im, int zall, double* acc, hipStream_t s);

}  // namespace qimax
