// Host runtime behind the C ABI: context and device memory, operator validation and
// classification, the pass planner, the grouping of instructions into the paper's U_k /
// V_k operators, readout and expectation values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <random>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qimax.h"
#include "qimax_internal.h"

using namespace qimax;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A transfer matrix R[out][in], immutable once made and shared by every copy of an
// operator (all CX and all CZ gates share one each), with its permutation table: per input
// index, the last nonzero row and its sign (out | 16 * negative), eight per word.
struct PtmData {
  std::vector<double> v;
  uint64_t lo = 0, hi = 0;
};
struct Ptm {
  std::shared_ptr<const PtmData> p;
  void assign(const double* a, const double* b) {
    auto d = std::make_shared<PtmData>();
    d->v.assign(a, b);
    const int dim = (int)std::lround(std::sqrt((double)d->v.size()));
    for (int in = 0; in < dim; ++in) {
      int out = 0;
      bool neg = false;
      for (int r = 0; r < dim; ++r) {
        const double x = d->v[r * dim + in];
        if (x != 0.0) {
          out = r;
          neg = x < 0;
        }
      }
      const uint64_t e = (uint64_t)(out | (neg ? 16 : 0));
      if (in < 8) d->lo |= e << (8 * in);
      else d->hi |= e << (8 * (in - 8));
    }
    p = std::move(d);
  }
  const std::vector<double>& vec() const {
    static const std::vector<double> none;
    return p ? p->v : none;
  }
  operator const std::vector<double>&() const { return vec(); }
  double operator[](size_t i) const { return p->v[i]; }
  size_t size() const { return vec().size(); }
  std::vector<double>::const_iterator begin() const { return vec().begin(); }
  std::vector<double>::const_iterator end() const { return vec().end(); }
};

// One operator on the host: PTM R[out][in] (dim 4 or 16), its wires and its operator
// group (the index of the U_k / V_k run it belongs to).
struct HostOp {
  int arity = 1;
  int q0 = 0, q1 = 0;
  int dim = 4;
  int64_t group = 0;  // operator group (U_k / V_k run); ids increase in circuit order
  bool perm = false;
  bool conj = false;  // a signed permutation that is a conjugation by a unitary (multiplicative)
  uint64_t mask = 0;  // wires touched
  Ptm R;              // dim*dim
};

// Autotuner state of one size class of rounds: the rounds timed so far, each candidate's
// least device time, and the winner once every candidate has been timed kTuneSamples times.
// Candidates: 0 the heuristic number of top-digit passes, 1 one more, 2 one global tile
// order instead of per-XCD ranges, 3 / 4 as 0 / 1 with multi-launch global passes, 5 dense
// accumulation (classes where it applies and is enabled).
constexpr int kTuneSamples = 2;

struct TuneState {
  static constexpr int kCand = 6;
  int tried = 0;
  int best = -1;
  float ms[kCand] = {};
};

inline int ilog2_u64(uint64_t x) { return x ? 63 - __builtin_clzll(x) : 0; }

struct Pass {
  std::vector<const HostOp*> A, E, B;
  uint64_t emask = 0, bmask = 0;
  int64_t egroup = -1;
  double fanout_bound = 1.0;
  ChainTable pre[2] = {};  // A / B chain tables compiled ahead of the rounds (tab_key set)
  // Term updates of the pass's Clifford operator groups (each group counted once, whichever
  // of A and B holds its operators): ng_in groups precede the expanding group in circuit
  // order and see the pass's input terms, ng_out follow it and see the merged output.
  // Operators of an expanding group that sit in A or B are counted by that group's images.
  uint64_t ng_in = 0, ng_out = 0;
};

// The paper's CX look-up tables (Sec. III-C-2), indexed [p_c][p_t] with I=0, X=1, Y=2, Z=3:
// new control digit, new target digit and sign.
const int kLutC[4][4] = {{0, 0, 3, 3}, {1, 1, 2, 2}, {2, 2, 1, 1}, {3, 3, 0, 0}};
const int kLutT[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {1, 0, 3, 2}, {0, 1, 2, 3}};
const int kLutSign[4][4] = {{1, 1, 1, 1}, {1, 1, 1, -1}, {1, 1, -1, 1}, {1, 1, 1, 1}};

void cx_ptm(double* R) {
  std::fill(R, R + 256, 0.0);
  for (int pc = 0; pc < 4; ++pc)
    for (int pt = 0; pt < 4; ++pt) {
      const int in = 4 * pc + pt, out = 4 * kLutC[pc][pt] + kLutT[pc][pt];
      R[out * 16 + in] = (double)kLutSign[pc][pt];
    }
}

// Hadamard's PTM on one digit: X <-> Z, Y -> -Y.
void h_ptm(double* R) {
  std::fill(R, R + 16, 0.0);
  R[0 * 4 + 0] = 1;
  R[3 * 4 + 1] = 1;
  R[2 * 4 + 2] = -1;
  R[1 * 4 + 3] = 1;
}

// CZ = (I x H) CX (I x H) on (q0, q1); the transfer matrices compose the same way.
void cz_ptm(double* R) {
  double cx[256], h[16], ih[256], tmp[256];
  cx_ptm(cx);
  h_ptm(h);
  std::fill(ih, ih + 256, 0.0);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c) ih[(4 * a + b) * 16 + (4 * a + c)] = h[b * 4 + c];
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double s = 0;
      for (int k = 0; k < 16; ++k) s += cx[i * 16 + k] * ih[k * 16 + j];
      tmp[i * 16 + j] = s;
    }
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double s = 0;
      for (int k = 0; k < 16; ++k) s += ih[i * 16 + k] * tmp[k * 16 + j];
      R[i * 16 + j] = s;
    }
}

bool is_signed_perm(const std::vector<double>& R, int dim) {
  for (int c = 0; c < dim; ++c) {
    int nz = 0;
    for (int r = 0; r < dim; ++r) {
      const double v = R[r * dim + c];
      if (v == 0.0) continue;
      if (v != 1.0 && v != -1.0) return false;
      ++nz;
    }
    if (nz != 1) return false;
  }
  return true;
}

int max_col_nnz(const std::vector<double>& R, int dim) {
  int m = 0;
  for (int c = 0; c < dim; ++c) {
    int nz = 0;
    for (int r = 0; r < dim; ++r) nz += R[r * dim + c] != 0.0;
    m = std::max(m, nz);
  }
  return m;
}

// Unital, trace preserving and orthogonal (R^T R = I) within tol.
bool is_valid_ptm(const std::vector<double>& R, int dim, double tol) {
  if (std::fabs(R[0] - 1.0) > tol) return false;
  for (int a = 1; a < dim; ++a)
    if (std::fabs(R[a * dim]) > tol || std::fabs(R[a]) > tol) return false;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) {
      double s = 0;
      for (int k = 0; k < dim; ++k) s += R[k * dim + i] * R[k * dim + j];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > tol) return false;
    }
  for (double v : R)
    if (!std::isfinite(v)) return false;
  return true;
}

// single-qubit Pauli products: sigma_a sigma_b = i^kPh[a][b] sigma_{kMul[a][b]}
const int kMul[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
const int kPh[4][4] = {{0, 0, 0, 0}, {0, 0, 1, 3}, {0, 3, 0, 1}, {0, 1, 3, 0}};

// Product of two local Pauli strings of `nq` digits (index 4*d0 + d1 for two digits).
void local_product(int a, int b, int nq, int* r, int* ph) {
  *r = 0;
  *ph = 0;
  for (int k = nq - 1; k >= 0; --k) {
    const int da = (a >> (2 * k)) & 3, db = (b >> (2 * k)) & 3;
    *r |= kMul[da][db] << (2 * k);
    *ph += kPh[da][db];
  }
  *ph &= 3;
}

// A signed permutation PTM that maps products to products (with phases) is a conjugation
// by a unitary, so its action on a whole Pauli string is the product of its actions on
// any split of the string; only such operators may be compiled into chain tables.
bool is_conjugation(const std::vector<double>& R, int dim) {
  const int nq = dim == 4 ? 1 : 2;
  std::vector<int> out(dim), neg(dim);
  for (int i = 0; i < dim; ++i) {
    out[i] = -1;
    for (int r = 0; r < dim; ++r)
      if (R[r * dim + i] != 0.0) {
        out[i] = r;
        neg[i] = R[r * dim + i] < 0;
      }
    if (out[i] < 0) return false;
  }
  if (out[0] != 0 || neg[0]) return false;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) {
      int r, ph, r2, ph2;
      local_product(a, b, nq, &r, &ph);
      local_product(out[a], out[b], nq, &r2, &ph2);
      if (out[r] != r2) return false;
      const int lhs = (neg[r] ? 2 : 0) + ph;
      const int rhs = ((neg[a] ^ neg[b]) ? 2 : 0) + ph2;
      if ((lhs - rhs) & 3) return false;
    }
  return true;
}

constexpr int kMaxE1 = 64;
constexpr int kBoundPathMaxFanout = 16;  // rounds with a larger fan-out bound read back their image count
// tile counters of a round (after the per-pass, per-XCD sort counters)
constexpr int kCtrCount = 252, kCtrMerge = 253, kCtrChunk = 254;
constexpr uint32_t kDenseMaxN = 12;           // dense accumulation: at most 4^12 slots per generator
constexpr double kDenseMaxBytes = 4.0e9;      // and at most this many bytes of slots in all
constexpr double kDenseRatio = 8.0;           // tuned only where slots <= 8 x images
constexpr int kMaxE2 = 8;
constexpr double kMaxFanout = 2147483647.0;

}  // namespace

struct qimax_ctx {
  uint32_t n = 0;
  int KC = 1;
  int WP = 64;
  int fp64_acc = 0;
  double eps = 0.0;
  size_t cap = 0;
  int validate = 1;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t kb = 8, wb = 8;  // bytes per key / weight

  // committed state
  DevBuf keys, w, seg;
  uint64_t T = 0;
  std::vector<uint64_t> h_seg;
  std::vector<HostOp> pending;  // deferred Clifford operators (not yet applied)
  int64_t group_base = 0;       // operator-group ids of the next call start here

  // pass outputs (ping-pong) and their segment offsets
  DevBuf pk[2], pw[2], pseg[2];
  // images and sort ping-pong
  DevBuf ik[2], iw[2];
  DevBuf cnt, off, scan_tmp, hist, hist_off, blk_begin, blk_end, blk_seg, seg_blk, blk_cnt, blk_off, img_seg;
  DevBuf desc, desc2, err, f64tmp;
  DevBuf ptab;  // chain tables of a whole call, compiled in one launch
  DevBuf akeys, asign;  // input terms after their pass's A chain, and the signs (count -> expand)
  DevBuf chunk_off, chunk_cnt, chunk_start;  // chunk-local merge: offset, kept terms, deferred runs per chunk
  DevBuf grp_cnt;  // persistent small passes: counts per pass and segment
  DevBuf img_cnt;                            // small rounds: image count per segment
  DevBuf ghist, sbase, sstatus, tile_ctr;  // single-sweep sort state
  uint64_t epoch = 0;
  DevBuf mstatus;  // single-sweep count and merge state (one word per tile)
  DevBuf dtile[3];  // device-built tilings: images (expand, sort/merge; bound path), input terms
  uint64_t mepoch = 0;
  bool classic_sort = false;
  bool host_tiling = false;
  bool xcd_ranges = true;
  bool local_sort = true;     // top-digit passes + chunk-local sorts instead of all global passes
  bool small_rounds = true;   // rounds of small segments: one block per segment (see run_round)
  bool fused_expand = true;   // bound-path rounds: count and expansion in one launch
  uint32_t defer_spins = 0;   // chunk-local merge: look-back polls before a chunk is deferred (0: one look)
  uint32_t chunk_tile = 0;    // nominal chunk of a fused round (0: from the expected bucket size)
  bool wide_offsets = false;  // count and expansion take their paths for 2^32 / 2^31 images (tests)
  bool classic_passes = false;  // multi-launch global sort passes in every round (tests)
  bool small_groups = true;  // consecutive small passes in one launch (k_small_passes)
  int dense_mode = 0;         // dense accumulation: 0 off, 1 wherever it applies, 2 a tuner candidate
  DevBuf dense_acc;           // its fixed-point slots
  int local_sort_m = -1;      // >= 0: force the number of top-digit passes
  uint32_t redo_cooldown = 0; // rounds left with global passes only after a chunk overflow
  bool autotune = true;       // choose among sort variants by measured time per size class
  bool tune_frozen = false;   // no exploration: settled variants, else the heuristic (recording)
  std::map<uint32_t, TuneState> tune;
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  DevBuf gr_in, gr_out;  // grouping pass inputs; batch admission lists
  uint64_t* pinned = nullptr;  // small pinned host scratch
  size_t pinned_words = 0;

  size_t alloc_bytes = 0, peak_bytes = 0;
  std::string last_error;
  bool broken = false;
  qimax_stats st{};
  Prof prof;
  std::vector<uint64_t> gen_updates;
  // pinned, device-mapped host staging: [0] a round's descriptors (read by its first launch),
  // [1] the image tilings of the unbound path; each is rewritten only after the stream
  // synchronisation that follows its use
  void* stage[2] = {nullptr, nullptr};
  void* stage_dev[2] = {nullptr, nullptr};  // device addresses of the same memory
  size_t stage_bytes[2] = {0, 0};
  // pinned, device-mapped words the last launch of a round writes its results into
  uint64_t* zres = nullptr;
  uint64_t* zres_dev = nullptr;
  size_t zres_words = 0;
  uint64_t zseq = 0;  // sequence word of the last results asked for
  // step recording (qimax_graph_record): the work of a step is captured between the host's
  // synchronisations and replayed later as one graph
  struct qimax_graph* rec = nullptr;
  bool rec_capturing = false;
  uint64_t buf_gen = 0;  // counts every (re)allocation or release of the context's memory
};

namespace {


thread_local std::string g_create_error;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

qimax_status fail(qimax_ctx* c, qimax_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

qimax_status hip_fail(qimax_ctx* c, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return fail(c, QIMAX_ENOMEM, msg);
  }
  c->broken = true;
  return fail(c, QIMAX_EDEVICE, msg);
}

#define HIPCHK(c, expr, what)                          \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail((c), _e, (what)); \
  } while (0)

void dev_free(qimax_ctx* c, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    c->alloc_bytes -= b.bytes;
    c->buf_gen += 1;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// Grow-only device buffer with the context's memory cap.
qimax_status ensure(qimax_ctx* c, DevBuf& b, size_t bytes, bool headroom = true) {
  if (bytes <= b.bytes && b.p) return QIMAX_OK;
  if (c->rec) return fail(c, QIMAX_ESTATE, "a device buffer must grow while recording: run the step once first");
  c->buf_gen += 1;
  size_t want = bytes == 0 ? 256 : bytes;
  if (headroom) want = want + want / 4;
  want = (want + 255) & ~(size_t)255;
  const size_t after = c->alloc_bytes - b.bytes + want;
  if (c->cap && after > c->cap) {
    if (bytes > 0 && c->alloc_bytes - b.bytes + bytes <= c->cap)
      want = (bytes + 255) & ~(size_t)255;
    if (c->alloc_bytes - b.bytes + want > c->cap)
      return fail(c, QIMAX_ENOMEM, "memory cap exceeded (requested " + std::to_string(bytes) + " bytes)");
  }
  if (b.p) {
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    dev_free(c, b);
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, QIMAX_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  b.p = p;
  b.bytes = want;
  c->alloc_bytes += want;
  c->peak_bytes = std::max(c->peak_bytes, c->alloc_bytes);
  return QIMAX_OK;
}

// Grow a buffer keeping its first `keep` bytes.
qimax_status ensure_keep(qimax_ctx* c, DevBuf& b, size_t bytes, size_t keep) {
  if (bytes <= b.bytes && b.p) return QIMAX_OK;
  if (c->rec) return fail(c, QIMAX_ESTATE, "a device buffer must grow while recording: run the step once first");
  c->buf_gen += 1;
  DevBuf nb;
  size_t want = align256(bytes + bytes / 4 + 256);
  if (c->cap && c->alloc_bytes + want > c->cap) {
    want = align256(bytes);
    if (c->alloc_bytes + want > c->cap)
      return fail(c, QIMAX_ENOMEM, "memory cap exceeded (requested " + std::to_string(bytes) + " bytes)");
  }
  hipError_t e = hipMalloc(&nb.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, QIMAX_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  nb.bytes = want;
  c->alloc_bytes += want;
  c->peak_bytes = std::max(c->peak_bytes, c->alloc_bytes);
  if (b.p && keep) {
    e = hipMemcpyAsync(nb.p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      (void)hipFree(nb.p);
      c->alloc_bytes -= want;
      return hip_fail(c, e, "grow copy");
    }
  }
  if (b.p) {
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, b);
  }
  b = nb;
  return QIMAX_OK;
}

#define QCHK(expr)                         \
  do {                                     \
    qimax_status _s = (expr);              \
    if (_s != QIMAX_OK) return _s;         \
  } while (0)


uint32_t bitpos(uint32_t n, int q) { return 2u * (n - 1u - (uint32_t)q); }

PermDesc make_perm(uint32_t n, const HostOp& op) {
  PermDesc d{};
  d.arity = (uint32_t)op.arity;
  d.pa = bitpos(n, op.q0);
  d.pb = op.arity == 2 ? bitpos(n, op.q1) : 0u;
  d.lo = op.R.p->lo;  // made with the matrix
  d.hi = op.R.p->hi;
  return d;
}

// ceil(2^32 / k) for an image count k >= 2 (0 otherwise): see the expansion's division.
uint32_t count_reciprocal(int k) {
  return k >= 2 ? (uint32_t)(((1ull << 32) + (uint64_t)k - 1) / (uint64_t)k) : 0u;
}

Exp1Desc make_exp1(uint32_t n, const HostOp& op) {
  Exp1Desc d{};
  d.pos = bitpos(n, op.q0);
  for (int in = 0; in < 4; ++in) {
    int k = 0;
    for (int r = 0; r < 4; ++r) {
      const double v = op.R[r * 4 + in];
      if (v == 0.0) continue;
      d.out[in][k] = (uint8_t)r;
      d.val[in][k] = v;
      d.valf[in][k] = (float)v;
      ++k;
    }
    d.cnt[in] = (uint8_t)k;
    d.rcp[in] = count_reciprocal(k);
  }
  return d;
}

Exp2Desc make_exp2(uint32_t n, const HostOp& op) {
  Exp2Desc d{};
  d.pa = bitpos(n, op.q0);
  d.pb = bitpos(n, op.q1);
  for (int in = 0; in < 16; ++in) {
    int k = 0;
    for (int r = 0; r < 16; ++r) {
      const double v = op.R[r * 16 + in];
      if (v == 0.0) continue;
      d.out[in][k] = (uint8_t)r;
      d.val[in][k] = v;
      d.valf[in][k] = (float)v;
      ++k;
    }
    d.cnt[in] = (uint8_t)k;
    d.rcp[in] = count_reciprocal(k);
  }
  return d;
}

// Segment-aligned tiles of at most `tile` elements over segment offsets so[0..S].
struct HostTiling {
  std::vector<uint64_t> begin, end;
  std::vector<uint32_t> seg, seg_blk;
  uint32_t xr[kXcds + 1] = {};  // per-XCD ranges of whole segments (see Tiling::xrange)
};

void make_tiling(const std::vector<uint64_t>& so, uint64_t tile, HostTiling& t) {
  const size_t S = so.size() - 1;
  t.begin.clear(); t.end.clear(); t.seg.clear(); t.seg_blk.assign(S + 1, 0);
  for (size_t s = 0; s < S; ++s) {
    t.seg_blk[s] = (uint32_t)t.begin.size();
    for (uint64_t b = so[s]; b < so[s + 1]; b += tile) {
      t.begin.push_back(b);
      t.end.push_back(std::min(b + tile, so[s + 1]));
      t.seg.push_back((uint32_t)s);
    }
  }
  t.seg_blk[S] = (uint32_t)t.begin.size();
  const uint32_t total = t.seg_blk[S];
  for (int x = 0; x < kXcds; ++x) {
    const uint32_t target = (uint32_t)(((uint64_t)x * total + kXcds - 1) / kXcds);
    t.xr[x] = *std::lower_bound(t.seg_blk.begin(), t.seg_blk.end(), target);
  }
  t.xr[kXcds] = total;
}

// Bytes a tiling occupies in a staging area (four arrays, each 256-aligned).
size_t tiling_bytes(const HostTiling& t) {
  const size_t nb = std::max<size_t>(t.begin.size(), 1);
  return align256(nb * 8) * 2 + align256(nb * 4) + align256(t.seg_blk.size() * 4) + 256;
}

// Copy a tiling into host staging at `off` and describe it by its device addresses.
size_t put_tiling(const HostTiling& t, uint8_t* host, uint8_t* dev, size_t off, Tiling& tl) {
  const size_t nb = t.begin.size(), nbm = std::max<size_t>(nb, 1);
  const size_t o1 = off, o2 = o1 + align256(nbm * 8), o3 = o2 + align256(nbm * 8), o4 = o3 + align256(nbm * 4);
  if (nb) {
    std::memcpy(host + o1, t.begin.data(), nb * 8);
    std::memcpy(host + o2, t.end.data(), nb * 8);
    std::memcpy(host + o3, t.seg.data(), nb * 4);
  }
  std::memcpy(host + o4, t.seg_blk.data(), t.seg_blk.size() * 4);
  const size_t o5 = o4 + align256(t.seg_blk.size() * 4);
  std::memcpy(host + o5, t.xr, sizeof(t.xr));
  tl.xrange = (const uint32_t*)(dev + o5);
  tl.blk_begin = (const uint64_t*)(dev + o1);
  tl.blk_end = (const uint64_t*)(dev + o2);
  tl.blk_seg = (const uint32_t*)(dev + o3);
  tl.seg_blk = (const uint32_t*)(dev + o4);
  tl.n_blocks = (uint32_t)nb;
  tl.n_segs = (uint32_t)(t.seg_blk.size() - 1);
  return o5 + 256;
}

qimax_status ensure_stage(qimax_ctx* c, int i, size_t bytes) {
  if (bytes <= c->stage_bytes[i] && c->stage[i]) return QIMAX_OK;
  if (c->rec) return fail(c, QIMAX_ESTATE, "a staging buffer must grow while recording: run the step once first");
  c->buf_gen += 1;
  if (c->stage[i]) {
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    (void)hipHostFree(c->stage[i]);
    c->stage[i] = nullptr;
    c->stage_bytes[i] = 0;
  }
  const size_t want = align256(bytes + bytes / 4 + 4096);
  HIPCHK(c, hipHostMalloc(&c->stage[i], want, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc staging");
  c->stage_bytes[i] = want;
  HIPCHK(c, hipHostGetDevicePointer(&c->stage_dev[i], c->stage[i], 0), "hipHostGetDevicePointer");
  return QIMAX_OK;
}

// Result words written by the device into mapped host memory (read after a synchronisation).
qimax_status ensure_zres(qimax_ctx* c, size_t words) {
  if (words <= c->zres_words && c->zres) return QIMAX_OK;
  if (c->rec) return fail(c, QIMAX_ESTATE, "a result buffer must grow while recording: run the step once first");
  c->buf_gen += 1;
  if (c->zres) {
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    (void)hipHostFree(c->zres);
    c->zres = c->zres_dev = nullptr;
    c->zres_words = 0;
  }
  const size_t want = std::max<size_t>(words + words / 4, 512);
  HIPCHK(c, hipHostMalloc((void**)&c->zres, want * 8, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc");
  c->zres_words = want;
  void* d = nullptr;
  HIPCHK(c, hipHostGetDevicePointer(&d, c->zres, 0), "hipHostGetDevicePointer");
  c->zres_dev = (uint64_t*)d;
  return QIMAX_OK;
}

// ------------------------------------------------------------------ step recording
// While a step is recorded, the stream is captured between the host's synchronisations: at
// each one the captured part becomes a graph, which is launched at once (so the recording run
// computes the step as usual) and kept; the replay launches the parts in order with no host
// work in between. Data the host stages for a launch (descriptors in mapped memory, rewritten
// every round) is copied into memory owned by the recording.
}  // namespace

struct qimax_graph {
  qimax_ctx* ctx = nullptr;
  std::vector<hipGraph_t> parts;
  hipGraph_t whole = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> snaps;  // pinned copies of staged data, read by the parts
  std::vector<hipGraphExec_t> runs;  // the parts as launched while recording
  uint64_t gen = 0;          // ctx->buf_gen when recorded
  uint64_t epoch_end = 0, mepoch_end = 0;  // the last look-back epochs the parts use
  bool failed = false;
  // the context's state after the step
  DevBuf keys, w, seg, pk[2], pw[2], pseg[2];
  std::vector<uint64_t> h_seg;
  uint64_t T = 0;
  qimax_stats st_delta{};
  std::vector<uint64_t> upd_delta;
};

namespace {

qimax_status rec_cut(qimax_ctx* c) {
  if (!c->rec || !c->rec_capturing) return QIMAX_OK;
  c->rec_capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess || !g) {
    c->rec->failed = true;
    return hip_fail(c, e == hipSuccess ? hipErrorUnknown : e, "hipStreamEndCapture");
  }
  c->rec->parts.push_back(g);
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (x) c->rec->runs.push_back(x);  // destroyed once the recording run has finished
  if (e == hipSuccess) e = hipGraphLaunch(x, c->stream);
  if (e != hipSuccess) {
    c->rec->failed = true;
    return hip_fail(c, e, "recorded part");
  }
  return QIMAX_OK;
}

qimax_status rec_resume(qimax_ctx* c) {
  if (!c->rec || c->rec_capturing || c->rec->failed) return QIMAX_OK;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  c->rec_capturing = true;
  return QIMAX_OK;
}

// The device address a launch should read `bytes` of staged host data from: the staging
// area itself, or while recording a pinned copy of it that lives as long as the recording.
qimax_status rec_src(qimax_ctx* c, const void* host, const void* dev, size_t bytes, const void** out) {
  *out = dev;
  if (!c->rec || bytes == 0) return QIMAX_OK;
  void* h = nullptr;
  HIPCHK(c, hipHostMalloc(&h, bytes, hipHostMallocMapped | hipHostMallocCoherent), "hipHostMalloc (recording)");
  c->rec->snaps.push_back(h);
  std::memcpy(h, host, bytes);
  void* d = nullptr;
  HIPCHK(c, hipHostGetDevicePointer(&d, h, 0), "hipHostGetDevicePointer");
  *out = d;
  return QIMAX_OK;
}

// Wait for the words the device writes into zres (words - 2: the error word, words - 1: the
// sequence word, stored last). The host polls the sequence word rather than waiting for the
// stream: launches queued after the publishing one (a compaction) keep running meanwhile.
// Once a millisecond of polling the stream is queried (a query is not free: it is kept rare),
// so that a failed or finished stream ends the wait.
qimax_status wait_zres(qimax_ctx* c, size_t words, uint32_t* err_out) {
  QCHK(rec_cut(c));
  const auto t0 = std::chrono::steady_clock::now();
  auto t_query = t0;
  volatile const uint64_t* seq = c->zres + words - 1;
  for (uint32_t it = 1; *seq != c->zseq; ++it) {
    if ((it & 63u) == 0 && std::chrono::steady_clock::now() - t_query > std::chrono::milliseconds(1)) {
      t_query = std::chrono::steady_clock::now();
      const hipError_t q = hipStreamQuery(c->stream);
      if (q == hipSuccess) {
        if (*seq != c->zseq) return fail(c, QIMAX_EDEVICE, "round results missing after the stream finished");
        break;
      }
      if (q != hipErrorNotReady) return hip_fail(c, q, "hipStreamQuery");
    }
    __builtin_ia32_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  c->st.host_wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->st.syncs += 1;
  prof_resolve(&c->prof);
  *err_out = (uint32_t)(c->zres[words - 2] & 0xFFFFFFFFu);
  return rec_resume(c);
}

// Copy `words` uint64 from device to the pinned scratch (plus the error word) and wait.
// `words` uint64 from the device to the pinned scratch, then the error word: the context's
// (one more copy) or, with err_packed, the last of the words.
qimax_status readback(qimax_ctx* c, const void* dev, size_t words, uint32_t* err_out, bool err_packed = false) {
  QCHK(rec_cut(c));
  if (words + 1 > c->pinned_words) {
    if (c->rec) return fail(c, QIMAX_ESTATE, "a readback buffer must grow while recording: run the step once first");
    c->buf_gen += 1;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    size_t want = std::max<size_t>(words + 1, 4096);
    HIPCHK(c, hipHostMalloc((void**)&c->pinned, want * 8, hipHostMallocDefault), "hipHostMalloc");
    c->pinned_words = want;
  }
  if (words)
    HIPCHK(c, hipMemcpyAsync(c->pinned, dev, words * 8, hipMemcpyDeviceToHost, c->stream), "readback");
  if (!err_packed)
    HIPCHK(c, hipMemcpyAsync(c->pinned + words, c->err.p, 4, hipMemcpyDeviceToHost, c->stream), "readback err");
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->st.host_wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  c->st.syncs += 1;
  prof_resolve(&c->prof);
  *err_out = (uint32_t)(c->pinned[err_packed ? words - 1 : words] & 0xFFFFFFFFu);
  return rec_resume(c);
}

std::string err_text(uint32_t e) {
  std::string s;
  if (e & kErrIndex) s += " index-out-of-range";
  if (e & kErrFanout) s += " fanout-overflow";
  if (e & kErrOrder) s += " order";
  if (e & kErrSpin) s += " look-back-timeout";
  if (e & kErrExpand) s += " (expand)";
  if (e & kErrSort) s += " (sort)";
  if (e & kErrMerge) s += " (merge)";
  return s;
}

// One circuit's share of a round: its next pass (or a drop of all its terms), the digit
// positions of its n qubits and the merge threshold of that pass.
struct RoundEntry {
  const Pass* pass = nullptr;
  uint32_t n = 0;
  double thr = 0.0;
  bool drop = false;
};

// Term updates of segment s in a pass: one per output image of every operator group (an
// expanding group counts its images, a Clifford group the terms it sees), each group once.
inline uint64_t pass_updates(const Pass& p, uint64_t t_in, uint64_t t_img, uint64_t t_out) {
  return p.ng_in * t_in + (p.E.empty() ? 0 : t_img) + p.ng_out * t_out;
}

// A round's descriptors staged for upload (in c->stage[0]; their device copy, c->desc, is
// pulled by the round's first launch): the entries' permutations and expanding-operator
// descriptors, one PassArgs per entry, the segments' entry numbers and the chain-table jobs.
struct RoundDesc {
  const PassArgs* pas = nullptr;   // device addresses
  const uint32_t* sent = nullptr;
  const TableJob* jobs = nullptr;
  size_t n_jobs = 0;
  size_t host_bytes = 0;
  size_t e_bytes = 0;              // largest expanding-operator descriptor set of an entry
  bool any_b_tables = false;
  uint32_t max_n = 1;
};

qimax_status build_round_desc(qimax_ctx* c, const std::vector<RoundEntry>& entries,
                              const std::vector<uint32_t>& seg_entry, RoundDesc& rd) {
  const uint32_t S = (uint32_t)seg_entry.size();
  const size_t E = entries.size();
  std::vector<PermDesc> perms;
  std::vector<Exp1Desc> e1;
  std::vector<Exp2Desc> e2;
  struct Lay { size_t a, b, x1, x2; uint32_t nA, nB, nE1, nE2; bool useA, useB; };
  std::vector<Lay> lay(E);
  size_t n_jobs = 0;
  size_t e_bytes = 0;  // largest expanding-operator descriptor set of an entry (staged in LDS)
  bool any_tables = false;
  bool any_b_tables = false;
  uint32_t max_n = 1;
  auto tableable = [c](const std::vector<const HostOp*>& v) {
    if (c->kb > 8 || (int)v.size() < kChainTableMin) return false;  // no tables for 16-byte keys
    for (auto* op : v)
      if (!op->conj) return false;
    return true;
  };
  for (size_t e = 0; e < E; ++e) {
    Lay& L = lay[e];
    L = Lay{perms.size(), 0, e1.size(), e2.size(), 0, 0, 0, 0, false, false};
    max_n = std::max(max_n, entries[e].n);
    const Pass* p = entries[e].pass;
    if (!p || entries[e].drop) continue;
    for (auto* op : p->A) perms.push_back(make_perm(entries[e].n, *op));
    L.nA = (uint32_t)p->A.size();
    L.b = perms.size();
    for (auto* op : p->B) perms.push_back(make_perm(entries[e].n, *op));
    L.nB = (uint32_t)p->B.size();
    for (auto* op : p->E) {
      if (op->arity == 1) { e1.push_back(make_exp1(entries[e].n, *op)); ++L.nE1; }
      else { e2.push_back(make_exp2(entries[e].n, *op)); ++L.nE2; }
    }
    e_bytes = std::max(e_bytes, L.nE1 * sizeof(Exp1Desc) + L.nE2 * sizeof(Exp2Desc));
    L.useA = tableable(p->A);
    L.useB = tableable(p->B);
    n_jobs += (L.useA && !p->pre[0].tab_key) + (L.useB && !p->pre[1].tab_key);
    any_tables |= L.useA || L.useB;
    any_b_tables |= L.useB;
  }
  const size_t entries_tab = c->kb * 256;
  const size_t tab_bytes = align256(entries_tab * c->kb) + align256(entries_tab);
  const size_t oP = 0;
  const size_t o1 = align256(oP + perms.size() * sizeof(PermDesc));
  const size_t o2 = align256(o1 + e1.size() * sizeof(Exp1Desc));
  const size_t oA = align256(o2 + e2.size() * sizeof(Exp2Desc));
  const size_t oS = align256(oA + E * sizeof(PassArgs));
  const size_t oJ = align256(oS + S * 4);
  const size_t host_bytes = align256(oJ + n_jobs * sizeof(TableJob));
  const size_t oTab = align256(host_bytes);
  const size_t total = oTab + n_jobs * tab_bytes + 256;
  QCHK(ensure(c, c->desc, total));
  QCHK(ensure_stage(c, 0, host_bytes));
  uint8_t* hs = (uint8_t*)c->stage[0];
  uint8_t* ds = (uint8_t*)c->desc.p;
  std::memset(hs, 0, host_bytes);
  if (!perms.empty()) std::memcpy(hs + oP, perms.data(), perms.size() * sizeof(PermDesc));
  if (!e1.empty()) std::memcpy(hs + o1, e1.data(), e1.size() * sizeof(Exp1Desc));
  if (!e2.empty()) std::memcpy(hs + o2, e2.data(), e2.size() * sizeof(Exp2Desc));
  PassArgs* pas_h = (PassArgs*)(hs + oA);
  TableJob* jobs_h = (TableJob*)(hs + oJ);
  size_t job = 0;
  for (size_t e = 0; e < E; ++e) {
    const Lay& L = lay[e];
    PassArgs pa{};
    pa.A = (const PermDesc*)(ds + oP + L.a * sizeof(PermDesc));
    pa.B = (const PermDesc*)(ds + oP + L.b * sizeof(PermDesc));
    pa.E1 = (const Exp1Desc*)(ds + o1 + L.x1 * sizeof(Exp1Desc));
    pa.E2 = (const Exp2Desc*)(ds + o2 + L.x2 * sizeof(Exp2Desc));
    pa.nA = L.nA; pa.nB = L.nB; pa.nE1 = L.nE1; pa.nE2 = L.nE2;
    pa.drop = entries[e].drop ? 1u : 0u;
    pa.thr = entries[e].thr;
    auto table_for = [&](const PermDesc* ops, uint32_t nops, ChainTable& t) {
      uint8_t* tk = ds + oTab + job * tab_bytes;
      uint8_t* tn = tk + align256(entries_tab * c->kb);
      jobs_h[job] = TableJob{ops, nops, 0, tk, tn};
      t = ChainTable{tk, tn};
      ++job;
    };
    const Pass* pp = entries[e].pass;
    if (L.useA) {
      pa.useA = 1;
      if (pp->pre[0].tab_key) pa.tA = pp->pre[0]; else table_for(pa.A, pa.nA, pa.tA);
    }
    if (L.useB) {
      pa.useB = 1;
      if (pp->pre[1].tab_key) pa.tB = pp->pre[1]; else table_for(pa.B, pa.nB, pa.tB);
    }
    pas_h[e] = pa;
  }
  std::memcpy(hs + oS, seg_entry.data(), S * 4);
  rd.pas = (const PassArgs*)(ds + oA);
  rd.sent = (const uint32_t*)(ds + oS);
  rd.jobs = (const TableJob*)(ds + oJ);
  rd.n_jobs = n_jobs;
  rd.host_bytes = host_bytes;
  rd.e_bytes = e_bytes;
  rd.any_b_tables = any_b_tables;
  rd.max_n = max_n;
  return QIMAX_OK;
}

// Runs one round: every segment s of the input (k_in, w_in; device offsets seg_in, host
// offsets so_in) is processed with the pass of entries[seg_entry[s]], in one set of
// launches for all segments. The merged result goes to pass slot `slot`; so_out / so_img
// receive the output and image segment offsets. upd[e] receives entry e's term updates.
qimax_status run_round(qimax_ctx* c, const std::vector<RoundEntry>& entries, const std::vector<uint32_t>& seg_entry,
                       const void* k_in, const void* w_in, const uint64_t* seg_in, const std::vector<uint64_t>& so_in,
                       int slot, std::vector<uint64_t>& so_out, std::vector<uint64_t>& so_img,
                       std::vector<uint64_t>* upd) {
  const uint32_t S = (uint32_t)seg_entry.size();
  const uint64_t T_in = so_in[S];
  const size_t E = entries.size();
  RoundDesc rd;
  QCHK(build_round_desc(c, entries, seg_entry, rd));
  uint8_t* ds = (uint8_t*)c->desc.p;
  const PassArgs* pas = rd.pas;
  const uint32_t* sent = rd.sent;
  const size_t host_bytes = rd.host_bytes, n_jobs = rd.n_jobs, e_bytes = rd.e_bytes;
  const bool any_b_tables = rd.any_b_tables;
  const uint32_t max_n = rd.max_n;
  const bool sweep = !c->classic_sort;
  const uint32_t key_bits = 2u * max_n;
  const uint32_t n_pass = (key_bits + kRadixBits - 1) / kRadixBits;
  // ---- round prep: error word, tile counters, digit histograms (one launch)
  // tile_ctr: [0, n_pass*kXcds) sort passes, [kCtrCount] count tiles, [kCtrMerge] merge tiles,
  // [kCtrChunk] chunk tickets
  const uint64_t nh = sweep ? (uint64_t)S * n_pass * kRadix : 0;
  if (sweep) QCHK(ensure(c, c->ghist, std::max<uint64_t>(nh, 1) * 4));
  QCHK(ensure(c, c->tile_ctr, 256 * 4));
  uint32_t* const ctr = (uint32_t*)c->tile_ctr.p;
  // Bound path: with a small fan-out bound f, T_img <= f * T_in, so the image tilings are
  // built on the device and every launch is sized by the bound (tiles past the real count
  // are empty), and the image offsets come back with the merge's. Otherwise the image
  // offsets are read back after the count and the tilings are built on the host.
  double f_round = 0.0;
  for (const RoundEntry& en : entries)
    if (en.pass && !en.drop) f_round = std::max(f_round, en.pass->fanout_bound);
  const bool bound_path = sweep && !c->host_tiling && f_round <= (double)kBoundPathMaxFanout && T_in > 0;
  // Small round: every segment's terms and bounded images fit one chunk. One block per
  // segment counts and expands it, then the chunk-local sort (whole segments) and merge run:
  // four launches in all, where the fixed costs of the general path's launches would
  // dominate rounds this small.
  bool small = false;
  if (bound_path && c->small_rounds && S <= kSmallMaxSegs) {
    uint64_t len_max = 0;
    for (uint32_t s = 0; s < S; ++s) len_max = std::max<uint64_t>(len_max, so_in[s + 1] - so_in[s]);
    small = std::max(1.0, f_round) * (double)len_max <= (double)kChunkCap;
  }
  // input tiling: segment-aligned tiles of at most kSortTile terms, built on the device from
  // the segment offsets (the tile count is known here exactly) by the round's first launch,
  // which also clears the error word, counters and histograms and pulls the descriptors
  // Fused round: the count and the expansion in one launch (a small fan-out bound keeps every
  // tile's images in reach of one block); its input tiles are smaller.
  const bool fused = bound_path && !small && c->fused_expand && (double)f_round <= (double)kFuseMaxFanout;
  const uint64_t in_tile = fused ? (uint64_t)fuse_tile() : (uint64_t)kSortTile;
  Tiling tl_in{};
  {
    uint32_t n_tin = 0;
    for (uint32_t s = 0; s < S; ++s) n_tin += (uint32_t)((so_in[s + 1] - so_in[s] + in_tile - 1) / in_tile);
    const size_t o1 = 0, o2 = align256((size_t)n_tin * 8), o3 = o2 + align256((size_t)n_tin * 8);
    const size_t o4 = o3 + align256((size_t)n_tin * 4), o5 = o4 + align256((size_t)(S + 1) * 4);
    const size_t o6 = o5 + 256;
    QCHK(ensure(c, c->dtile[2], o6 + 256));
    uint8_t* d = (uint8_t*)c->dtile[2].p;
    const TileJob2 job{in_tile, n_tin, 0, (uint64_t*)(d + o1), (uint64_t*)(d + o2), (uint32_t*)(d + o3),
                       (uint32_t*)(d + o4), (uint32_t*)(d + o5), (uint32_t*)(d + o6)};
    tl_in = Tiling{(const uint64_t*)(d + o1), (const uint64_t*)(d + o2), (const uint32_t*)(d + o3),
                   (const uint32_t*)(d + o4), n_tin, S, nullptr, nullptr};
    const void* blob = nullptr;
    QCHK(rec_src(c, c->stage[0], c->stage_dev[0], host_bytes, &blob));
    HIPCHK(c, launch_round_start(blob, ds, host_bytes, (uint32_t*)c->err.p, ctr, 256,
                                 (uint32_t*)c->ghist.p, nh, seg_in, S, job, T_in, c->stream), "round start");
  }
  HIPCHK(c, launch_build_tables(c->KC, rd.jobs, (uint32_t)n_jobs, c->stream, &c->prof), "chain tables");
  // ---- fan-out count fused with its scan -> image offsets of every input term
  // mstatus: one word per tile, shared by the count and merge sweeps (distinct epochs)
  auto status_words = [&](uint64_t tiles) -> qimax_status {
    const size_t old_m = c->mstatus.bytes;
    QCHK(ensure(c, c->mstatus, (size_t)(tiles + 1) * 8));
    if (c->mstatus.bytes != old_m || c->mepoch + 2 >= 0xFFFFull) {
      // fresh memory or epoch wrap: clear every word so that no stale epoch can match
      HIPCHK(c, launch_fill_u64((uint64_t*)c->mstatus.p, c->mstatus.bytes / 8, 0ull, c->stream), "clear status");
      c->mepoch = 0;
    }
    return QIMAX_OK;
  };
  if (!small && !fused) {
    QCHK(ensure(c, c->off, (T_in + 1) * 8));
    QCHK(ensure(c, c->akeys, std::max<uint64_t>(T_in, 1) * c->kb));
    QCHK(ensure(c, c->asign, std::max<uint64_t>(T_in, 1)));
    QCHK(status_words(tl_in.n_blocks));
    c->mepoch += 1;
    HIPCHK(c, launch_count_scan(c->KC, k_in, T_in, tl_in, pas, sent, (uint64_t*)c->off.p, (uint64_t*)c->mstatus.p,
                                ctr + kCtrCount, c->mepoch, (uint32_t*)c->err.p, c->akeys.p, (uint8_t*)c->asign.p,
                                c->stream, &c->prof, c->wide_offsets), "count");
  }
  QCHK(ensure(c, c->img_seg, (S + 1) * 8));
  uint32_t e = 0;
  uint64_t T_img = 0;
  Tiling tl_exp{}, tl{};
  TileJob2 img_jobs[2];
  if (bound_path) {
    T_img = (uint64_t)f_round * T_in;  // capacity: an upper bound of the image count
    const uint32_t caps[2] = {(uint32_t)((T_img + kExpandTile - 1) / kExpandTile + S),
                              (uint32_t)((T_img + kSortTile - 1) / kSortTile + S)};
    const uint64_t tiles[2] = {(uint64_t)kExpandTile, (uint64_t)kSortTile};
    Tiling* tls[2] = {&tl_exp, &tl};
    TileJob2* jobs = img_jobs;
    for (int i = 0; i < 2; ++i) {
      const size_t o1 = 0, o2 = align256((size_t)caps[i] * 8), o3 = o2 + align256((size_t)caps[i] * 8);
      const size_t o4 = o3 + align256((size_t)caps[i] * 4), o5 = o4 + align256((size_t)(S + 1) * 4);
      const size_t o6 = o5 + 256;
      QCHK(ensure(c, c->dtile[i], o6 + 256));
      uint8_t* d = (uint8_t*)c->dtile[i].p;
      jobs[i] = TileJob2{tiles[i], caps[i], 0, (uint64_t*)(d + o1), (uint64_t*)(d + o2), (uint32_t*)(d + o3),
                         (uint32_t*)(d + o4), (uint32_t*)(d + o5), (uint32_t*)(d + o6)};
      *tls[i] = Tiling{(const uint64_t*)(d + o1), (const uint64_t*)(d + o2), (const uint32_t*)(d + o3),
                       (const uint32_t*)(d + o4), caps[i], S, (const uint32_t*)(d + o5), (const uint32_t*)(d + o6)};
    }
    if (!small && !fused)  // (a fused round builds them after its launch, from the image offsets it wrote)
      HIPCHK(c, launch_make_tiles2((const uint64_t*)c->off.p, seg_in, S, (uint64_t*)c->img_seg.p, jobs[0], jobs[1],
                                   T_img, (uint32_t*)c->err.p, c->stream), "tiles");
  } else {
    HIPCHK(c, launch_gather_u64((const uint64_t*)c->off.p, seg_in, (uint64_t*)c->img_seg.p, S + 1, c->stream,
                                &c->prof), "gather");
    QCHK(readback(c, c->img_seg.p, S + 1, &e));
    if (e) return fail(c, (e & kErrFanout) ? QIMAX_ETOOLARGE : QIMAX_EDEVICE, "count pass:" + err_text(e));
    so_img.assign(c->pinned, c->pinned + S + 1);
    T_img = so_img[S];
    // ---- image tilings (expand tiles, sort/merge tiles) in one upload
    HostTiling t_exp, t_sort;
    make_tiling(so_img, kExpandTile, t_exp);
    make_tiling(so_img, kSortTile, t_sort);
    const size_t img_bytes = tiling_bytes(t_exp) + tiling_bytes(t_sort);
    QCHK(ensure(c, c->desc2, img_bytes + 256));
    QCHK(ensure_stage(c, 1, img_bytes));
    const size_t mid = put_tiling(t_exp, (uint8_t*)c->stage[1], (uint8_t*)c->desc2.p, 0, tl_exp);
    put_tiling(t_sort, (uint8_t*)c->stage[1], (uint8_t*)c->desc2.p, mid, tl);
    if (c->rec) {  // the recording's own copy, pulled by a kernel
      const void* src = nullptr;
      QCHK(rec_src(c, c->stage[1], c->stage_dev[1], img_bytes, &src));
      HIPCHK(c, launch_pull(src, c->desc2.p, img_bytes, c->stream), "upload tiling");
    } else {
      HIPCHK(c, hipMemcpyAsync(c->desc2.p, c->stage[1], img_bytes, hipMemcpyHostToDevice, c->stream), "upload tiling");
    }
  }
  // ---- sort plan (single-sweep sort): global passes over every digit, or over the top m
  // digits only, followed by chunk-local sorts in LDS. m is the fewest top digits that split
  // the largest segment (its image count or a bound of it) into buckets of about 512 on
  // average; the autotuner may add one, and may turn the per-XCD tile ranges off, by what it
  // measured for rounds of this size (the expansion, sort and merge, timed together). The
  // expansion counts the digits of up to kExpandHistPasses global passes itself.
  uint32_t m_top = n_pass;  // digits sorted by global passes (the rest chunk-locally)
  uint32_t tune_key = 0;    // autotuner: size class of this round's sort, candidate, timed?
  int tune_cand = 0;
  bool tune_timed = false;
  bool xr = c->xcd_ranges;
  // the global passes as multi-launch passes (histogram, scan, scatter per digit) instead of
  // single-sweep ones: no look-back chain over a segment's tiles, at one more read per pass
  bool classic_passes = c->classic_passes;
  // Dense accumulation instead of the sort: one circuit, 32-bit keys, a dense space of 4^n
  // slots per generator that stays small next to the images, bounded weights (orthogonal
  // transfer matrices). Forced (QIMAX_DENSE=1) or a tuner candidate (QIMAX_DENSE=auto).
  const uint64_t per_seg = (c->KC == 0 && max_n <= kDenseMaxN) ? (1ull << (2 * max_n)) : 0;
  const bool dense_ok = c->dense_mode && sweep && !small && E == 1 && per_seg && c->validate &&
                        !entries[0].drop && (double)S * (double)per_seg * 8.0 <= kDenseMaxBytes &&
                        (c->dense_mode == 1 || (double)S * (double)per_seg <= kDenseRatio * (double)T_img);
  bool dense = dense_ok && c->dense_mode == 1;
  if (small) m_top = 0;  // whole segments sorted in LDS
  uint64_t seg_max = 0;     // the largest segment's image count (or its bound)
  if (sweep && !small) {
    if (c->local_sort && c->redo_cooldown == 0) {
      for (uint32_t s = 0; s < S; ++s)
        seg_max = std::max<uint64_t>(seg_max, bound_path ? (uint64_t)(f_round * (double)(so_in[s + 1] - so_in[s]))
                                                         : so_img[s + 1] - so_img[s]);
      uint32_t mm = 0;
      for (double cap_b = 512.0; mm < n_pass && (double)seg_max > cap_b; cap_b *= 256.0) ++mm;
      m_top = c->local_sort_m >= 0 ? std::min<uint32_t>((uint32_t)c->local_sort_m, n_pass) : mm;
      if (c->autotune && c->local_sort_m < 0 && (m_top < n_pass || dense_ok)) {
        // size class: key class << 8 | FP64 weights << 6 | log2 of the image capacity (| 2^20 with dense)
        tune_key = ((uint32_t)c->KC << 8) + (c->WP == 64 ? 64u : 0u) + (uint32_t)std::min(63, ilog2_u64(T_img)) +
                   (dense_ok ? (1u << 20) : 0u);
        TuneState& ts = c->tune[tune_key];
        // (a recording never explores: its rounds are not timed)
        // (each candidate is timed kTuneSamples times, in turns; its time is the least)
        const int n_cand = dense_ok ? TuneState::kCand : TuneState::kCand - 1;
        tune_cand = ts.best >= 0 ? ts.best : (c->tune_frozen ? 0 : ts.tried % n_cand);
        if (tune_cand == 1 || tune_cand == 4) m_top = std::min(m_top + 1, n_pass);
        if (tune_cand == 2) xr = false;
        if (tune_cand == 3 || tune_cand == 4) classic_passes = true;
        if (tune_cand == 5) dense = true;
        if (ts.best < 0 && !c->tune_frozen) {  // exploring: time this round
          HIPCHK(c, hipEventRecord(c->tune_ev[0], c->stream), "tune event");
          tune_timed = true;
        }
      }
    }
    if (c->redo_cooldown > 0) --c->redo_cooldown;
  }
  const bool hist_in_expand = sweep && !dense && !classic_passes && m_top <= kExpandHistPasses;
  // ---- expand into images
  const size_t eb = c->kb, wbt = c->wb;
  // image buffers: the capacity, or for a small round S chunks of kChunkCap
  const uint64_t n_work = std::max<uint64_t>(small ? std::max<uint64_t>(T_img, (uint64_t)S * kChunkCap) : T_img, 1);
  QCHK(ensure(c, c->ik[0], n_work * eb));
  QCHK(ensure(c, c->iw[0], n_work * wbt));
  QCHK(ensure(c, c->ik[1], n_work * eb));
  QCHK(ensure(c, c->iw[1], n_work * wbt));
  Tiling tc_small{};
  if (small) {
    const size_t o1 = 0, o2 = align256((size_t)S * 8), o3 = o2 + align256((size_t)S * 8);
    const size_t o4 = o3 + align256((size_t)S * 4), o5 = o4 + align256((size_t)(S + 1) * 4);
    QCHK(ensure(c, c->dtile[0], o5 + 256));
    QCHK(ensure(c, c->img_cnt, (size_t)std::max<uint32_t>(S, 1) * 4));
    uint8_t* d = (uint8_t*)c->dtile[0].p;
    const TileJob2 job{(uint64_t)kChunkCap, S, 0, (uint64_t*)(d + o1), (uint64_t*)(d + o2), (uint32_t*)(d + o3),
                       (uint32_t*)(d + o4), nullptr, nullptr};
    tc_small = Tiling{(const uint64_t*)(d + o1), (const uint64_t*)(d + o2), (const uint32_t*)(d + o3),
                      (const uint32_t*)(d + o4), S, S, nullptr, nullptr};
    HIPCHK(c, launch_expand_small(c->KC, c->WP, k_in, w_in, seg_in, S, T_in, pas, sent, c->ik[0].p, c->iw[0].p,
                                  (uint32_t*)c->img_cnt.p, job, (uint32_t*)c->err.p, c->stream, &c->prof),
           "expand");
  } else if (fused) {
    QCHK(status_words(tl_in.n_blocks));
    c->mepoch += 1;
    HIPCHK(c, launch_count_expand(c->KC, c->WP, k_in, w_in, T_in, tl_in, pas, sent, (uint64_t*)c->mstatus.p,
                                  ctr + kCtrCount, c->mepoch, (uint64_t*)c->img_seg.p, c->ik[0].p, c->iw[0].p, T_img,
                                  hist_in_expand ? (uint32_t*)c->ghist.p : nullptr, n_pass, n_pass - m_top,
                                  (uint32_t*)c->err.p, c->stream, &c->prof), "count and expand");
    // A fused round has no separate expansion: its first tiling only sets the chunk-local
    // sort's nominal chunks, as large as the buckets straddling their ends leave room for in
    // a chunk (kChunkCap): 4096 less four times the largest segment's average bucket, within
    // [kExpandTile, kChunkTile] (the capacity was sized for kExpandTile).
    if (c->chunk_tile) {
      img_jobs[0].tile = c->chunk_tile;
    } else if (m_top < n_pass) {
      const double bucket = (double)seg_max / std::ldexp(1.0, 8 * (int)m_top);
      const double t = std::min((double)kChunkTile, std::max((double)kExpandTile, (double)kChunkCap - 4.0 * bucket));
      img_jobs[0].tile = (uint64_t)t / 256 * 256;
    }
    HIPCHK(c, launch_make_tiles2(nullptr, (const uint64_t*)c->img_seg.p, S, nullptr, img_jobs[0], img_jobs[1], T_img,
                                 (uint32_t*)c->err.p, c->stream), "tiles");
  } else
  HIPCHK(c, launch_expand(c->KC, c->WP, c->akeys.p, (const uint8_t*)c->asign.p, w_in, T_in,
                          (const uint64_t*)c->off.p, T_img, tl_exp, pas, sent, seg_in, any_b_tables, e_bytes,
                          c->ik[0].p, c->iw[0].p, hist_in_expand ? (uint32_t*)c->ghist.p : nullptr, n_pass,
                          n_pass - m_top, (uint32_t*)c->err.p, c->stream, &c->prof, c->wide_offsets), "expand");
  // ---- segment-local LSD radix sort of the images
  const uint64_t hsize = (uint64_t)kRadix * std::max<uint32_t>(tl.n_blocks, 1);
  int cur = 0;
  int pre_chunk = -1;       // slot holding the images before the chunk-local sort
  if (small) {
    pre_chunk = 0;
  } else if (dense) {
    // no sort: the images are added into the dense slots by the merge below
  } else if (!sweep) {
    QCHK(ensure(c, c->scan_tmp, scan_tmp_words(std::max<uint64_t>(hsize, T_in)) * 8));
    QCHK(ensure(c, c->hist, hsize * 8));
    QCHK(ensure(c, c->hist_off, (hsize + 1) * 8));
    for (uint32_t shift = 0; shift < key_bits; shift += kRadixBits) {
      HIPCHK(c, launch_sort_pass(c->KC, c->WP, c->ik[cur].p, c->iw[cur].p, c->ik[cur ^ 1].p, c->iw[cur ^ 1].p, T_img,
                                 shift, tl, (uint64_t*)c->hist.p, (uint64_t*)c->hist_off.p, (uint64_t*)c->scan_tmp.p,
                                 (uint32_t*)c->err.p, c->stream, &c->prof), "sort");
      cur ^= 1;
    }
  } else {
    // a grown buffer may come back at the same address with stale contents: detect the
    // reallocation by its size, never by its pointer
    const size_t old_bytes = c->sstatus.bytes;
    QCHK(ensure(c, c->sstatus, hsize * 8));
    if (c->sstatus.bytes != old_bytes || c->epoch + n_pass >= 0xFFFFull) {
      // fresh memory or epoch wrap: clear every word so that no stale epoch can match
      HIPCHK(c, launch_fill_u64((uint64_t*)c->sstatus.p, c->sstatus.bytes / 8, 0ull, c->stream), "clear status");
      c->epoch = 0;
    }
    void* const kk[2] = {c->ik[0].p, c->ik[1].p};
    void* const ww[2] = {c->iw[0].p, c->iw[1].p};
    if (!xr) tl.xrange = nullptr;
    if (classic_passes) {
      QCHK(ensure(c, c->scan_tmp, scan_tmp_words(hsize) * 8));
      QCHK(ensure(c, c->hist, hsize * 8));
      QCHK(ensure(c, c->hist_off, (hsize + 1) * 8));
      cur = 0;
      for (uint32_t p = n_pass - m_top; p < n_pass; ++p) {
        HIPCHK(c, launch_sort_pass(c->KC, c->WP, kk[cur], ww[cur], kk[cur ^ 1], ww[cur ^ 1], T_img, p * kRadixBits,
                                   tl, (uint64_t*)c->hist.p, (uint64_t*)c->hist_off.p, (uint64_t*)c->scan_tmp.p,
                                   (uint32_t*)c->err.p, c->stream, &c->prof), "sort");
        cur ^= 1;
      }
    } else {
      HIPCHK(c, launch_sort_sweep(c->KC, c->WP, kk, ww, T_img, key_bits, n_pass - m_top, !hist_in_expand, tl,
                                  (const uint64_t*)c->img_seg.p, (uint32_t*)c->ghist.p, (uint64_t*)c->sstatus.p, ctr,
                                  &c->epoch, (uint32_t*)c->err.p, &cur, c->stream, &c->prof), "sort");
    }
    if (m_top < n_pass) pre_chunk = cur;  // the chunk-local sort runs with the merge
  }
  // ---- segmented reduce + prune + compaction into the pass output slot
  QCHK(ensure(c, c->pk[slot], std::max<uint64_t>(T_img, 1) * eb));
  QCHK(ensure(c, c->pw[slot], std::max<uint64_t>(T_img, 1) * wbt));
  QCHK(ensure(c, c->pseg[slot], (S + 1) * 8));
  QCHK(ensure(c, c->blk_cnt, (size_t)(tl.n_blocks + 1) * 4));
  QCHK(ensure(c, c->blk_off, (size_t)(tl.n_blocks + 1) * 8));
  QCHK(ensure_zres(c, 2 * (size_t)S + 4));
  MergeFin fin{(const uint64_t*)c->img_seg.p, c->zres_dev, 0};
  bool chunk_path = pre_chunk >= 0;  // chunk-local sort fused with the merge
  const Tiling& tc_chunk = small ? tc_small : tl_exp;  // the chunks' nominal tiles (see the tilings)
  auto merge_and_read = [&]() -> qimax_status {
    if (sweep) {  // a fresh sequence word for these results
      fin.seq = ++c->zseq;
      c->zres[2 * (size_t)S + 3] = 0;
    }
    if (dense) {
      const uint64_t tps = (per_seg + dense_tile() - 1) / dense_tile();
      const uint64_t n_tiles = tps * S;
      QCHK(ensure(c, c->dense_acc, (size_t)(S * per_seg) * 8));
      QCHK(ensure(c, c->chunk_off, (size_t)(n_tiles + 1) * 8));
      QCHK(status_words(n_tiles));
      c->mepoch += 1;
      HIPCHK(c, launch_dense_merge(c->KC, c->WP, c->ik[0].p, c->iw[0].p, T_img, tl, per_seg, S, c->dense_acc.p,
                                   entries[0].thr, ctr + kCtrChunk, (uint64_t*)c->mstatus.p, c->mepoch,
                                   (uint64_t*)c->chunk_off.p, c->pk[slot].p, c->pw[slot].p, T_img,
                                   (uint64_t*)c->pseg[slot].p, fin, (uint32_t*)c->err.p, c->stream, &c->prof),
             "dense merge");
    } else if (chunk_path) {
      const size_t nc = std::max<uint32_t>(tc_chunk.n_blocks, 1);
      QCHK(ensure(c, c->chunk_off, (nc + 1) * 8));
      QCHK(ensure(c, c->chunk_cnt, nc * 4));
      QCHK(ensure(c, c->chunk_start, nc * 8));
      QCHK(status_words(nc));
      c->mepoch += 1;
      const ChunkOut co{ctr + kCtrChunk, (uint64_t*)c->mstatus.p, c->mepoch, (uint32_t*)c->chunk_cnt.p,
                        (uint64_t*)c->chunk_start.p, (uint64_t*)c->chunk_off.p, c->ik[cur ^ 1].p, c->iw[cur ^ 1].p,
                        (uint64_t*)c->pseg[slot].p, fin, small ? (const uint32_t*)c->img_cnt.p : nullptr,
                        c->defer_spins, n_work};
      HIPCHK(c, launch_chunk_sort_merge(c->KC, c->WP, c->fp64_acc, c->ik[cur].p, c->iw[cur].p, c->pk[slot].p,
                                        c->pw[slot].p, T_img, tc_chunk, n_pass, m_top, pas, sent, co,
                                        (uint32_t*)c->err.p, c->stream, &c->prof), "chunk sort");
    } else {
      uint64_t* mstatus = nullptr;
      if (sweep) {
        QCHK(status_words(tl.n_blocks));
        c->mepoch += 1;
        mstatus = (uint64_t*)c->mstatus.p;
      }
      HIPCHK(c, launch_merge(c->KC, c->WP, c->fp64_acc, c->ik[cur].p, c->iw[cur].p, T_img, tl, pas, sent,
                             c->pk[slot].p, c->pw[slot].p, T_img, (uint64_t*)c->pseg[slot].p, (uint32_t*)c->blk_cnt.p,
                             (uint64_t*)c->blk_off.p, (uint64_t*)c->scan_tmp.p, mstatus, ctr + kCtrMerge, c->mepoch,
                             (uint32_t*)c->err.p, sweep ? &fin : nullptr, c->stream, &c->prof), "merge");
    }
    if (tune_timed) HIPCHK(c, hipEventRecord(c->tune_ev[1], c->stream), "tune event");
    // ---- one readback: output offsets, image offsets, error word
    if (sweep) {
      QCHK(wait_zres(c, 2 * (size_t)S + 4, &e));
      if (tune_timed) HIPCHK(c, hipEventSynchronize(c->tune_ev[1]), "tune event");
      return QIMAX_OK;
    }
    return readback(c, c->pseg[slot].p, S + 1, &e);
  };
  QCHK(merge_and_read());
  bool sorted_again = false;
  if (e == kErrRedo && chunk_path && !small) {  // (whole-segment chunks never overflow)
    sorted_again = true;
    // a bucket did not fit a chunk: sort the round again with global passes over every digit
    // (stable passes on the top-digit grouping give the same order as on the images) and merge
    // again; the next rounds use global passes only for a while
    c->redo_cooldown = 8;
    c->st.sort_redos += 1;
    HIPCHK(c, launch_round_prep((uint32_t*)c->err.p, ctr, 256, (uint32_t*)c->ghist.p, nh, c->stream), "prep");
    void* const kk2[2] = {c->ik[pre_chunk].p, c->ik[pre_chunk ^ 1].p};
    void* const ww2[2] = {c->iw[pre_chunk].p, c->iw[pre_chunk ^ 1].p};
    int cur2 = 0;
    if (c->epoch + n_pass >= 0xFFFFull) {
      HIPCHK(c, launch_fill_u64((uint64_t*)c->sstatus.p, c->sstatus.bytes / 8, 0ull, c->stream), "clear status");
      c->epoch = 0;
    }
    HIPCHK(c, launch_sort_sweep(c->KC, c->WP, kk2, ww2, T_img, key_bits, 0, true, tl, (const uint64_t*)c->img_seg.p,
                                (uint32_t*)c->ghist.p, (uint64_t*)c->sstatus.p, ctr, &c->epoch, (uint32_t*)c->err.p,
                                &cur2, c->stream, &c->prof), "sort");
    cur = pre_chunk ^ cur2;
    chunk_path = false;
    tune_timed = false;
    QCHK(merge_and_read());
  }
  if (tune_timed) {  // the round has synchronised: both events are complete
    TuneState& ts = c->tune[tune_key];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->tune_ev[0], c->tune_ev[1]) != hipSuccess) ms = 1e30f;
    if (sorted_again) ms = 1e30f;  // a candidate that overflows chunks is never chosen
    const int n_cand = (tune_key >> 20) & 1u ? TuneState::kCand : TuneState::kCand - 1;  // dense: the last
    ts.ms[tune_cand] = ts.tried < n_cand ? ms : std::min(ts.ms[tune_cand], ms);
    if (++ts.tried >= kTuneSamples * n_cand) {
      ts.best = 0;
      for (int i = 1; i < n_cand; ++i)
        if (ts.ms[i] < ts.ms[ts.best]) ts.best = i;
      c->st.tuned_classes += 1;
    }
  }
  if (e) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), " [segments %u, T_in %llu, T_img %llu, tiles %u, key bits %u, entries %zu]", S,
                  (unsigned long long)T_in, (unsigned long long)T_img, tl.n_blocks, key_bits, E);
    return fail(c, (e & kErrFanout) ? QIMAX_ETOOLARGE : QIMAX_EDEVICE, "propagation round:" + err_text(e) + buf);
  }
  const uint64_t* rb = sweep ? c->zres : c->pinned;  // where the round's results came back
  so_out.assign(rb, rb + S + 1);
  const uint64_t T_out = so_out[S];
  if (bound_path) {
    so_img.assign(rb + S + 1, rb + 2 * (S + 1));
    // the launches were recorded with the capacity; count the real images
    const uint64_t cap = T_img;
    T_img = so_img[S];
    if (c->prof.on) {
      const double d = (double)(cap - T_img);
      auto fix = [&](int kind, double bytes) {
        if ((c->prof.mask >> kind) & 1u) c->prof.bytes[kind] -= bytes;
      };
      if (small) {  // the images' bytes, known now
        if ((c->prof.mask >> kKExpand) & 1u) c->prof.bytes[kKExpand] += (double)(eb + wbt) * (double)T_img;
      } else if (fused) {
        if ((c->prof.mask >> kKCountExpand) & 1u) c->prof.bytes[kKCountExpand] += (double)(eb + wbt) * (double)T_img;
      } else {
        fix(kKExpand, (double)(eb + wbt) * d);
      }
      if (dense) {
        fix(kKDense, (4.0 + (double)wbt) * d);
      } else {
        if (!small) fix(kKSortHist, (double)eb * d * ((hist_in_expand ? 0 : 1) + (sorted_again ? 1 : 0)));  // upsweeps run
        if (!small) fix(kKSortScatter, 2.0 * (double)(eb + wbt) * (sorted_again ? n_pass + m_top : m_top) * d);
        if (m_top < n_pass) fix(kKChunkSort, (double)(eb + wbt) * d);
        if (!chunk_path) fix(kKMergeWrite, (double)(eb + wbt) * d);
      }
    }
  }
  if (c->prof.on) {  // the kept terms' bytes, known now
    const double kept = (double)T_out * (double)(eb + wbt);
    if (dense) {
      if ((c->prof.mask >> kKDense) & 1u) c->prof.bytes[kKDense] += kept;
    } else if (!chunk_path && ((c->prof.mask >> kKMergeWrite) & 1u)) {
      c->prof.bytes[kKMergeWrite] += kept;
    }
    if (chunk_path && ((c->prof.mask >> kKChunkSort) & 1u)) c->prof.bytes[kKChunkSort] += kept;
  }
  // ---- bookkeeping: one update per output image of every operator (a Clifford operator
  // counts its terms, the expanding operator its images), attributed per entry
  if (upd) upd->assign(E, 0);
  uint64_t total_upd = 0;
  for (uint32_t s = 0; s < S; ++s) {
    const RoundEntry& en = entries[seg_entry[s]];
    if (en.drop || !en.pass) continue;
    const uint64_t u = pass_updates(*en.pass, so_in[s + 1] - so_in[s], so_img[s + 1] - so_img[s],
                                    so_out[s + 1] - so_out[s]);
    total_upd += u;
    if (upd) (*upd)[seg_entry[s]] += u;
  }
  c->st.term_updates += total_upd;
  // algorithmic bytes of the round: every live input term read once, every merged output
  // term written once (a leaving circuit's terms move nowhere)
  double alg = 0.0;
  for (uint32_t s = 0; s < S; ++s) {
    const RoundEntry& en = entries[seg_entry[s]];
    if (en.drop || !en.pass) continue;
    alg += (double)((so_in[s + 1] - so_in[s]) + (so_out[s + 1] - so_out[s]));
  }
  c->st.alg_bytes += alg * (double)(eb + wbt);
  c->st.rounds += 1;
  c->st.images += T_img;
  c->st.sort_elems += T_img * ((key_bits + kRadixBits - 1) / kRadixBits);
  return QIMAX_OK;
}

// Sets p.ng_in / p.ng_out: the distinct operator groups of p's A and B chains that hold no
// expanding operator (exp_groups, sorted), split by their place before or after p's
// expanding group in circuit order (group ids increase in circuit order). A pass without an
// expanding operator counts all of them on its input.
void count_clifford_groups(Pass& p, const std::vector<int64_t>& exp_groups) {
  std::vector<int64_t> g;
  for (const auto* v : {&p.A, &p.B})
    for (const HostOp* op : *v)
      if (!std::binary_search(exp_groups.begin(), exp_groups.end(), op->group)) g.push_back(op->group);
  std::sort(g.begin(), g.end());
  g.erase(std::unique(g.begin(), g.end()), g.end());
  p.ng_in = p.ng_out = 0;
  for (int64_t x : g) {
    if (p.E.empty() || x < p.egroup) ++p.ng_in;
    else ++p.ng_out;
  }
}

// The pass planner: operators in order become passes [A perms] -> [E expanding ops of one
// operator group on disjoint wires] -> [B perms]. A perm after E that touches none of E's
// wires commutes past E into A. Trailing perms with no expanding operator after them are
// returned in `pending` (deferred). thr: merge threshold of the last pass, 0 for the others.
void plan_passes(const std::vector<const HostOp*>& all, std::vector<Pass>& passes,
                 std::vector<const HostOp*>& pending) {
  Pass cur;
  for (const HostOp* opp : all) {
    const HostOp& op = *opp;
    if (op.perm) {
      if (cur.E.empty() || (cur.B.empty() && !(op.mask & cur.emask))) {
        cur.A.push_back(&op);
      } else {
        cur.B.push_back(&op);
        cur.bmask |= op.mask;
      }
      continue;
    }
    const double f = (double)max_col_nnz(op.R, op.dim);
    int n1 = 0, n2 = 0;
    for (auto* e : cur.E) (e->arity == 1 ? n1 : n2)++;
    const bool fits = (op.arity == 1 ? n1 + 1 <= kMaxE1 : n2 + 1 <= kMaxE2) && cur.fanout_bound * f <= kMaxFanout;
    // one-qubit expanding operators of one U_k on disjoint wires share a pass; a two-qubit
    // expanding operator has a pass of its own (its images are counted operator by operator)
    const bool join = !cur.E.empty() && op.arity == 1 && op.group == cur.egroup && !(op.mask & cur.emask) &&
                      !(op.mask & cur.bmask) && fits;
    if (!cur.E.empty() && !join) {
      passes.push_back(cur);
      cur = Pass();
    }
    cur.E.push_back(&op);
    cur.emask |= op.mask;
    cur.egroup = op.group;
    cur.fanout_bound *= f;
  }
  pending.clear();
  if (cur.E.empty()) {
    pending = cur.A;
  } else {
    passes.push_back(cur);
  }
  // update counts: a group with an expanding operator is counted by its images only; every
  // other group once, before or after the pass's expanding group in circuit order
  std::vector<int64_t> exp_groups;
  for (const HostOp* op : all)
    if (!op->perm) exp_groups.push_back(op->group);
  std::sort(exp_groups.begin(), exp_groups.end());
  for (Pass& p : passes) count_clifford_groups(p, exp_groups);
}

// Single-circuit contexts: plan the operators (after the deferred ones of earlier calls) and
// run the passes as one-entry rounds; commit only when every pass succeeded.
// Host time of a call minus the time it spent blocked in pass synchronisations.
struct BusyTimer {
  qimax_ctx* c;
  std::chrono::steady_clock::time_point t0;
  double wait0;
  explicit BusyTimer(qimax_ctx* cc) : c(cc), t0(std::chrono::steady_clock::now()), wait0(cc->st.host_wait_ms) {}
  ~BusyTimer() {
    const double all = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->st.host_busy_ms += all - (c->st.host_wait_ms - wait0);
  }
};

// Compile every chain table of a call's passes in one launch ahead of the rounds (a chain
// table depends on the operators only), so that rounds need no table launch of their own.
qimax_status prebuild_tables(qimax_ctx* c, std::vector<Pass>& passes) {
  if (c->kb > 8) return QIMAX_OK;  // no tables for 16-byte keys
  auto tableable = [](const std::vector<const HostOp*>& v) {
    if ((int)v.size() < kChainTableMin) return false;
    for (auto* op : v)
      if (!op->conj) return false;
    return true;
  };
  std::vector<std::pair<Pass*, int>> chains;
  size_t n_perm = 0;
  for (auto& p : passes)
    for (int ab = 0; ab < 2; ++ab) {
      const auto& v = ab ? p.B : p.A;
      if (tableable(v)) {
        chains.push_back({&p, ab});
        n_perm += v.size();
      }
    }
  if (chains.empty()) return QIMAX_OK;
  const size_t entries_tab = c->kb * 256;
  const size_t tab_bytes = align256(entries_tab * c->kb) + align256(entries_tab);
  const size_t oJ = 0, oP = align256(chains.size() * sizeof(TableJob));
  const size_t host_bytes = oP + align256(n_perm * sizeof(PermDesc));
  const size_t oT = align256(host_bytes);
  QCHK(ensure(c, c->ptab, oT + chains.size() * tab_bytes + 256));
  QCHK(ensure_stage(c, 1, host_bytes));
  uint8_t* hs = (uint8_t*)c->stage[1];
  uint8_t* ds = (uint8_t*)c->ptab.p;
  TableJob* jobs = (TableJob*)(hs + oJ);
  PermDesc* perms = (PermDesc*)(hs + oP);
  size_t np = 0;
  for (size_t j = 0; j < chains.size(); ++j) {
    Pass& p = *chains[j].first;
    const int ab = chains[j].second;
    const auto& v = ab ? p.B : p.A;
    const size_t first = np;
    for (auto* op : v) perms[np++] = make_perm(c->n, *op);
    uint8_t* tk = ds + oT + j * tab_bytes;
    uint8_t* tn = tk + align256(entries_tab * c->kb);
    jobs[j] = TableJob{(const PermDesc*)(ds + oP) + first, (uint32_t)v.size(), 0, tk, tn};
    p.pre[ab] = ChainTable{tk, tn};
  }
  const void* src = nullptr;  // (a recording reads its own copy: the staging area is rewritten later)
  QCHK(rec_src(c, c->stage[1], c->stage_dev[1], host_bytes, &src));
  HIPCHK(c, launch_pull(src, ds, host_bytes, c->stream), "upload chains");
  HIPCHK(c, launch_build_tables(c->KC, (const TableJob*)(ds + oJ), (uint32_t)chains.size(), c->stream, &c->prof),
         "chain tables");
  return QIMAX_OK;
}

// How many passes from i0 on (at most kMaxGroupPasses) one launch of k_small_passes can run:
// every segment's terms, multiplied by each pass's fan-out bound in turn, stay within a chunk
// (so do its images). 0 or 1: run the passes as rounds.
constexpr size_t kMaxGroupPasses = 64;
size_t small_group_len(const qimax_ctx* c, const std::vector<Pass>& passes, size_t i0,
                       const std::vector<uint64_t>& so_in) {
  if (!c->small_groups || !c->small_rounds || c->classic_sort || c->host_tiling || c->KC > 1 || c->n > kSmallMaxSegs)
    return 0;
  std::vector<double> len(c->n);
  for (uint32_t s = 0; s < c->n; ++s) len[s] = (double)(so_in[s + 1] - so_in[s]);
  size_t k = 0;
  while (i0 + k < passes.size() && k < kMaxGroupPasses) {
    const double f = std::max(1.0, passes[i0 + k].fanout_bound);
    bool fits = true;
    for (uint32_t s = 0; s < c->n && fits; ++s) fits = f * len[s] <= (double)kChunkCap;
    if (!fits) break;
    for (uint32_t s = 0; s < c->n; ++s) len[s] *= f;
    ++k;
  }
  return k;
}

// Passes i0 .. i0+k-1 of the context's circuit in one launch of k_small_passes (one block per
// generator, the terms in LDS-sized slots between the passes); so_ins / so_imgs / so_outs
// receive each pass's segment offsets of its input terms, images and kept terms, and the
// last pass's terms go to pass slot `slot`. Counters as for k rounds.
qimax_status run_small_group(qimax_ctx* c, std::vector<Pass>& passes, size_t i0, size_t k, const void* k_in,
                             const void* w_in, const uint64_t* s_in, const std::vector<uint64_t>& so_in, int slot,
                             std::vector<std::vector<uint64_t>>& so_ins, std::vector<std::vector<uint64_t>>& so_imgs,
                             std::vector<std::vector<uint64_t>>& so_outs) {
  const uint32_t S = c->n;
  std::vector<RoundEntry> en(k);
  for (size_t p = 0; p < k; ++p) {
    en[p].pass = &passes[i0 + p];
    en[p].n = c->n;
    en[p].thr = (i0 + p + 1 == passes.size()) ? c->eps : 0.0;
  }
  const std::vector<uint32_t> seg_entry(S, 0);
  RoundDesc rd;
  QCHK(build_round_desc(c, en, seg_entry, rd));
  const uint64_t T_in = so_in[S];
  QCHK(ensure(c, c->tile_ctr, 256 * 4));
  {
    // the round's first launch clears the error word and counters and pulls the descriptors
    // (the input tiling it also builds is not used by the group)
    uint32_t n_tin = 0;
    for (uint32_t s = 0; s < S; ++s) n_tin += (uint32_t)((so_in[s + 1] - so_in[s] + kSortTile - 1) / kSortTile);
    const size_t o1 = 0, o2 = align256((size_t)n_tin * 8), o3 = o2 + align256((size_t)n_tin * 8);
    const size_t o4 = o3 + align256((size_t)n_tin * 4), o5 = o4 + align256((size_t)(S + 1) * 4);
    const size_t o6 = o5 + 256;
    QCHK(ensure(c, c->dtile[2], o6 + 256));
    uint8_t* d = (uint8_t*)c->dtile[2].p;
    const TileJob2 job{(uint64_t)kSortTile, n_tin, 0, (uint64_t*)(d + o1), (uint64_t*)(d + o2), (uint32_t*)(d + o3),
                       (uint32_t*)(d + o4), (uint32_t*)(d + o5), (uint32_t*)(d + o6)};
    const void* blob = nullptr;
    QCHK(rec_src(c, c->stage[0], c->stage_dev[0], rd.host_bytes, &blob));
    HIPCHK(c, launch_round_start(blob, c->desc.p, rd.host_bytes, (uint32_t*)c->err.p, (uint32_t*)c->tile_ctr.p, 256,
                                 (uint32_t*)c->ghist.p, 0, s_in, S, job, T_in, c->stream), "round start");
  }
  HIPCHK(c, launch_build_tables(c->KC, rd.jobs, (uint32_t)rd.n_jobs, c->stream, &c->prof), "chain tables");
  const size_t eb = c->kb, wbt = c->wb;
  const uint64_t n_work = (uint64_t)S * kChunkCap;
  for (int i = 0; i < 2; ++i) {
    QCHK(ensure(c, c->ik[i], n_work * eb));
    QCHK(ensure(c, c->iw[i], n_work * wbt));
  }
  QCHK(ensure(c, c->pk[slot], n_work * eb));
  QCHK(ensure(c, c->pw[slot], n_work * wbt));  // (also the images' weights during the passes)
  QCHK(ensure(c, c->pseg[slot], (S + 1) * 8));
  const size_t cnt_words = (k * S * 3 + 1) / 2;
  QCHK(ensure(c, c->grp_cnt, cnt_words * 8));
  void* const ks[2] = {c->ik[0].p, c->ik[1].p};
  void* const ws[2] = {c->iw[0].p, c->iw[1].p};
  HIPCHK(c, launch_small_passes(c->KC, c->WP, c->fp64_acc, k_in, w_in, s_in, S, rd.pas, (uint32_t)k, ks, ws,
                                c->pw[slot].p, (uint32_t*)c->grp_cnt.p, c->pk[slot].p, c->pw[slot].p,
                                (uint64_t*)c->pseg[slot].p, (uint32_t*)c->err.p, c->stream, &c->prof),
         "small passes");
  uint32_t e = 0;
  QCHK(readback(c, c->grp_cnt.p, cnt_words, &e));
  if (e) return fail(c, (e & kErrFanout) ? QIMAX_ETOOLARGE : QIMAX_EDEVICE, "small passes:" + err_text(e));
  const uint32_t* h = (const uint32_t*)c->pinned;
  so_ins.assign(k, {});
  so_imgs.assign(k, {});
  so_outs.assign(k, {});
  const uint32_t n_digits = (2u * c->n + kRadixBits - 1) / kRadixBits;
  double prof_bytes = 0.0;
  for (size_t p = 0; p < k; ++p) {
    auto& si = so_ins[p];
    auto& sg = so_imgs[p];
    auto& so = so_outs[p];
    si.assign(S + 1, 0);
    sg.assign(S + 1, 0);
    so.assign(S + 1, 0);
    for (uint32_t s = 0; s < S; ++s) {
      const uint32_t* q = h + (p * S + s) * 3;
      si[s + 1] = si[s] + q[0];
      sg[s + 1] = sg[s] + q[1];
      so[s + 1] = so[s] + q[2];
    }
    if (si != (p ? so_outs[p - 1] : so_in))
      return fail(c, QIMAX_EDEVICE, "small passes: a pass's input counts do not match the previous output");
    uint64_t upd = 0;
    for (uint32_t s = 0; s < S; ++s)
      upd += pass_updates(*en[p].pass, si[s + 1] - si[s], sg[s + 1] - sg[s], so[s + 1] - so[s]);
    c->st.term_updates += upd;
    c->st.alg_bytes += (double)(si[S] + so[S]) * (double)(eb + wbt);
    c->st.rounds += 1;
    c->st.images += sg[S];
    c->st.sort_elems += sg[S] * n_digits;
    prof_bytes += (double)(si[S] + sg[S] + so[S]) * (double)(eb + wbt);
  }
  if (c->prof.on && ((c->prof.mask >> kKSmallPasses) & 1u)) c->prof.bytes[kKSmallPasses] += prof_bytes;
  return QIMAX_OK;
}

qimax_status apply_ops(qimax_ctx* c, std::vector<HostOp>& ops) {
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  BusyTimer bt(c);
  // group ids continue from earlier calls, so that deferred operators precede this call's
  int64_t next_base = c->group_base;
  for (auto& op : ops) {
    op.group += c->group_base;
    next_base = std::max(next_base, op.group + 1);
  }
  c->group_base = next_base;
  std::vector<const HostOp*> ptrs;  // the deferred operators, then these (both outlive the passes)
  ptrs.reserve(c->pending.size() + ops.size());
  for (auto& op : c->pending) ptrs.push_back(&op);
  for (auto& op : ops) ptrs.push_back(&op);
  std::vector<Pass> passes;
  std::vector<const HostOp*> pend;
  plan_passes(ptrs, passes, pend);
  std::vector<HostOp> new_pending;
  for (auto* op : pend) new_pending.push_back(*op);
  if (passes.empty()) {
    c->pending.swap(new_pending);
    return QIMAX_OK;
  }
  QCHK(prebuild_tables(c, passes));
  const void* k_in = c->keys.p;
  const void* w_in = c->w.p;
  const uint64_t* s_in = (const uint64_t*)c->seg.p;
  std::vector<uint64_t> so_in = c->h_seg, so_out, so_img, upd;
  std::vector<uint32_t> seg_entry(c->n, 0);
  int slot = 0;
  for (size_t i = 0; i < passes.size(); ++i) {
    const size_t kg = small_group_len(c, passes, i, so_in);
    if (kg >= 2) {  // consecutive small passes: one launch
      std::vector<std::vector<uint64_t>> gi, gg, go;
      qimax_status s = run_small_group(c, passes, i, kg, k_in, w_in, s_in, so_in, slot, gi, gg, go);
      if (s != QIMAX_OK) return s;  // committed state untouched
      if (c->gen_updates.size() != c->n) c->gen_updates.assign(c->n, 0);
      for (size_t p = 0; p < kg; ++p) {
        for (uint32_t j = 0; j < c->n; ++j)
          c->gen_updates[j] += pass_updates(passes[i + p], gi[p][j + 1] - gi[p][j], gg[p][j + 1] - gg[p][j],
                                            go[p][j + 1] - go[p][j]);
        if (!passes[i + p].E.empty()) c->st.passes += 1;
      }
      k_in = c->pk[slot].p;
      w_in = c->pw[slot].p;
      s_in = (const uint64_t*)c->pseg[slot].p;
      so_in = go.back();
      slot ^= 1;
      i += kg - 1;
      continue;
    }
    RoundEntry en;
    en.pass = &passes[i];
    en.n = c->n;
    en.thr = (i + 1 == passes.size()) ? c->eps : 0.0;
    qimax_status s = run_round(c, {en}, seg_entry, k_in, w_in, s_in, so_in, slot, so_out, so_img, nullptr);
    if (s != QIMAX_OK) return s;  // committed state untouched
    if (c->gen_updates.size() != c->n) c->gen_updates.assign(c->n, 0);
    for (uint32_t j = 0; j < c->n; ++j)
      c->gen_updates[j] += pass_updates(*en.pass, so_in[j + 1] - so_in[j], so_img[j + 1] - so_img[j],
                                        so_out[j + 1] - so_out[j]);
    if (!en.pass->E.empty()) c->st.passes += 1;
    k_in = c->pk[slot].p;
    w_in = c->pw[slot].p;
    s_in = (const uint64_t*)c->pseg[slot].p;
    so_in = so_out;
    slot ^= 1;
  }
  const int last = slot ^ 1;
  std::swap(c->keys, c->pk[last]);
  std::swap(c->w, c->pw[last]);
  std::swap(c->seg, c->pseg[last]);
  c->h_seg = so_in;
  c->T = so_in[c->n];
  c->pending.swap(new_pending);
  c->st.terms = c->T;
  return QIMAX_OK;
}

qimax_status flush_pending(qimax_ctx* c) {
  if (c->pending.empty()) return QIMAX_OK;
  // a pass with only Clifford operators: images are the permuted terms, then sorted
  Pass p;
  for (auto& op : c->pending) p.A.push_back(&op);
  count_clifford_groups(p, {});
  RoundEntry en;
  en.pass = &p;
  en.n = c->n;
  std::vector<uint64_t> so_out, so_img;
  std::vector<uint32_t> seg_entry(c->n, 0);
  qimax_status s = run_round(c, {en}, seg_entry, c->keys.p, c->w.p, (const uint64_t*)c->seg.p, c->h_seg, 0, so_out,
                             so_img, nullptr);
  if (s != QIMAX_OK) return s;
  if (c->gen_updates.size() != c->n) c->gen_updates.assign(c->n, 0);
  for (uint32_t j = 0; j < c->n; ++j)
    c->gen_updates[j] += pass_updates(p, c->h_seg[j + 1] - c->h_seg[j], 0, 0);
  std::swap(c->keys, c->pk[0]);
  std::swap(c->w, c->pw[0]);
  std::swap(c->seg, c->pseg[0]);
  c->h_seg = so_out;
  c->T = so_out[c->n];
  c->pending.clear();
  return QIMAX_OK;
}

qimax_status check_op_input(qimax_ctx* c, const qimax_op& in, int64_t group, HostOp& op) {
  if (in.arity != 1 && in.arity != 2) return fail(c, QIMAX_EINVAL, "op arity must be 1 or 2");
  if (!in.ptm) return fail(c, QIMAX_EINVAL, "op ptm is NULL");
  if (in.q[0] >= c->n || (in.arity == 2 && (in.q[1] >= c->n || in.q[1] == in.q[0])))
    return fail(c, QIMAX_EINVAL, "op qubit out of range or repeated");
  op.arity = (int)in.arity;
  op.q0 = (int)in.q[0];
  op.q1 = in.arity == 2 ? (int)in.q[1] : op.q0;
  op.dim = in.arity == 1 ? 4 : 16;
  op.group = group;
  op.R.assign(in.ptm, in.ptm + op.dim * op.dim);
  op.mask = (1ull << op.q0) | (in.arity == 2 ? (1ull << op.q1) : 0ull);
  for (double v : op.R)
    if (!std::isfinite(v)) return fail(c, QIMAX_EINVAL, "op ptm has a non-finite entry");
  if (c->validate && !is_valid_ptm(op.R, op.dim, 1e-12))
    return fail(c, QIMAX_EINVAL, "op ptm is not unital/orthogonal (set validate = 0 to allow)");
  op.perm = is_signed_perm(op.R, op.dim);
  op.conj = op.perm && is_conjugation(op.R, op.dim);
  return QIMAX_OK;
}

bool is_2q_code(uint8_t g) { return g >= QIMAX_GATE_CX && g <= QIMAX_GATE_RZZ; }

// One-qubit Pauli products sigma_a sigma_b = i^kMulPhase[a][b] sigma_kMulOut[a][b], Pauli
// order I, X, Y, Z (X Y = i Z and cyclic; the reverse order gives -i).
constexpr int kMulOut[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
constexpr int kMulPhase[4][4] = {{0, 0, 0, 0}, {0, 0, 1, 3}, {0, 3, 0, 1}, {0, 1, 3, 0}};

// Transfer matrix of exp(-i t A / 2), A = sigma_P (x) sigma_P (P in 1..3), from c = cos t and
// s = sin t: a Pauli pair Q commuting with A is kept; one anticommuting with A goes to
// c Q + s (-i A Q), -i A Q being a Pauli pair with a real sign.
void pair_rotation_ptm(int P, double c, double s, double* R) {
  std::fill(R, R + 256, 0.0);
  auto anti = [P](int a) { return a != 0 && a != P; };  // a one-qubit Pauli anticommuting with sigma_P
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int in = 4 * a + b;
      if (anti(a) == anti(b)) {
        R[in * 16 + in] = 1.0;
        continue;
      }
      R[in * 16 + in] = c;
      const int out = 4 * kMulOut[P][a] + kMulOut[P][b];
      const int k = (kMulPhase[P][a] + kMulPhase[P][b] + 3) & 3;  // -i = i^3
      R[out * 16 + in] += (k == 0 ? s : -s);                      // k is 0 or 2 here
    }
}

// ISWAP = exp(i pi/4 XX) exp(i pi/4 YY) (the factors commute), each a pair rotation at
// t = -pi/2 taken with its exact cosine 0 and sine -1: a signed permutation.
void iswap_ptm(double* R) {
  double xx[256], yy[256];
  pair_rotation_ptm(1, 0.0, -1.0, xx);
  pair_rotation_ptm(2, 0.0, -1.0, yy);
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 16; ++k) acc += yy[i * 16 + k] * xx[k * 16 + j];
      R[i * 16 + j] = acc;
    }
}

// The 16x16 R of a 16x16 operator on (q0, q1) written for the wires in the other order.
void swap_wires_ptm(const double* R, double* out) {
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      const int i2 = 4 * (i & 3) + (i >> 2), j2 = 4 * (j & 3) + (j >> 2);
      out[i2 * 16 + j2] = R[i * 16 + j];
    }
}

// A 4x4 matrix with one entry of +-1 per column and zeros elsewhere, as a code: per column c,
// (row | 4 * negative) << 3c; -1 for any other matrix.
int signed_perm_code4(const double* R) {
  int code = 0;
  for (int col = 0; col < 4; ++col) {
    int row = -1, neg = 0;
    for (int r = 0; r < 4; ++r) {
      const double v = R[r * 4 + col];
      if (v == 0.0) continue;
      if ((v != 1.0 && v != -1.0) || row >= 0) return -1;
      row = r;
      neg = v < 0;
    }
    if (row < 0) return -1;
    code |= (row | (neg << 2)) << (3 * col);
  }
  return code;
}
constexpr int kIdentityCode4 = 0 | (1 << 3) | (2 << 6) | (3 << 9);

// The paper's grouping (Sec. III-A, Alg. 2): maximal runs of one-qubit gates (U_k) and
// of two-qubit gates (V_k) in instruction order; inside U_k the gates of each wire form
// U_{k,j}, composed into one transfer matrix on the device (Alg. 1).
qimax_status group_circuit(qimax_ctx* c, uint32_t n, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                           const double* theta, size_t m, std::vector<HostOp>& ops, size_t* n_u, size_t* n_v) {
  for (size_t i = 0; i < m; ++i) {
    if (gate[i] > QIMAX_GATE_RZZ) return fail(c, QIMAX_EINVAL, "unknown gate code at instruction " + std::to_string(i));
    if (q0[i] >= n) return fail(c, QIMAX_EINVAL, "qubit out of range at instruction " + std::to_string(i));
    if (is_2q_code(gate[i]) && (q1[i] >= n || q1[i] == q0[i]))
      return fail(c, QIMAX_EINVAL, "bad second qubit at instruction " + std::to_string(i));
    if (theta && !std::isfinite(theta[i])) return fail(c, QIMAX_EINVAL, "non-finite angle");
  }
  // runs
  struct Run { bool two; size_t a, b; };
  std::vector<Run> runs;
  for (size_t i = 0; i < m;) {
    const bool two = is_2q_code(gate[i]);
    size_t j = i;
    while (j < m && is_2q_code(gate[j]) == two) ++j;
    runs.push_back({two, i, j});
    i = j;
  }
  size_t nu = 0, nv = 0;
  // one-qubit chains: per U run, per wire in increasing order
  std::vector<uint32_t> idx, chain_off{0};
  struct ChainRef { int run; int wire; };
  std::vector<ChainRef> chains;
  std::vector<std::vector<uint32_t>> per_wire(n);
  for (size_t r = 0; r < runs.size(); ++r) {
    if (runs[r].two) { ++nv; continue; }
    ++nu;
    for (auto& v : per_wire) v.clear();
    for (size_t i = runs[r].a; i < runs[r].b; ++i) per_wire[q0[i]].push_back((uint32_t)i);
    for (uint32_t j = 0; j < n; ++j) {
      if (per_wire[j].empty()) continue;
      for (uint32_t gi : per_wire[j]) idx.push_back(gi);
      chain_off.push_back((uint32_t)idx.size());
      chains.push_back({(int)r, (int)j});
    }
  }
  const double* ptm = nullptr;
  if (!chains.empty()) {
    // inputs through mapped staging, pulled to the device by a kernel; the composed PTMs
    // written by the kernel straight into mapped staging. (No launch still reads or writes
    // the staging areas here: a round's first launch reads them, and every round's results
    // have been waited for; a call's grouping result has been read.)
    const size_t oG = 0, oT = align256(m), oI = oT + align256(m * 8), oO = oI + align256(idx.size() * 4);
    const size_t up = oO + align256(chain_off.size() * 4), down = chains.size() * 16 * 8;
    QCHK(ensure(c, c->gr_in, up));
    QCHK(ensure_stage(c, 0, up));
    QCHK(ensure_stage(c, 1, down));
    uint8_t* hs = (uint8_t*)c->stage[0];
    std::memcpy(hs + oG, gate, m);
    if (theta) std::memcpy(hs + oT, theta, m * 8);
    else std::memset(hs + oT, 0, m * 8);
    std::memcpy(hs + oI, idx.data(), idx.size() * 4);
    std::memcpy(hs + oO, chain_off.data(), chain_off.size() * 4);
    const uint8_t* dg = (const uint8_t*)c->gr_in.p;
    const void* gsrc = nullptr;
    QCHK(rec_src(c, c->stage[0], c->stage_dev[0], up, &gsrc));
    HIPCHK(c, launch_pull(gsrc, c->gr_in.p, up, c->stream), "group upload");
    HIPCHK(c, launch_compose_ptm(dg + oG, (const double*)(dg + oT), (const uint32_t*)(dg + oI),
                                 (const uint32_t*)(dg + oO), (uint32_t)chains.size(), (double*)c->stage_dev[1],
                                 c->stream, &c->prof), "compose_ptm");
    QCHK(rec_cut(c));
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    QCHK(rec_resume(c));
    ptm = (const double*)c->stage[1];
  }
  // assemble the operator list in run order
  static const Ptm kCx = [] {
    double R[256];
    cx_ptm(R);
    Ptm t;
    t.assign(R, R + 256);
    return t;
  }();
  static const Ptm kCz = [] {
    double R[256];
    cz_ptm(R);
    Ptm t;
    t.assign(R, R + 256);
    return t;
  }();
  static const Ptm kIswap = [] {
    double R[256];
    iswap_ptm(R);
    Ptm t;
    t.assign(R, R + 256);
    return t;
  }();
  size_t ci = 0;
  ops.clear();
  ops.reserve(m);
  // the one-qubit Clifford chains give few distinct signed permutations: one shared matrix
  // and one classification each
  struct Cls { Ptm R; bool conj = false; };
  std::unordered_map<int, Cls> perm_cache;
  for (size_t r = 0; r < runs.size(); ++r) {
    if (runs[r].two) {
      // last operator of this run on each wire (index into ops), for fusing same-pair gates
      std::unordered_map<uint32_t, size_t> last;
      for (size_t i = runs[r].a; i < runs[r].b; ++i) {
        Ptm R;
        double buf[256];
        bool perm = true, conj = true;  // CX, CZ and ISWAP are Clifford
        switch (gate[i]) {
          case QIMAX_GATE_CX: R = kCx; break;
          case QIMAX_GATE_CZ: R = kCz; break;
          case QIMAX_GATE_ISWAP: R = kIswap; break;
          default: {  // RXX, RYY, RZZ
            const double th = theta ? theta[i] : 0.0;
            pair_rotation_ptm(gate[i] - QIMAX_GATE_RXX + 1, std::cos(th), std::sin(th), buf);
            R.assign(buf, buf + 256);
            perm = is_signed_perm(R, 16);
            conj = perm && is_conjugation(R, 16);
          }
        }
        auto ia = last.find(q0[i]), ib = last.find(q1[i]);
        if (ia != last.end() && ib != last.end() && ia->second == ib->second) {
          // the run's previous operator on both wires acts on exactly this pair, and nothing
          // in between touched them: fuse (this gate acts on that operator's images)
          HostOp& prev = ops[ia->second];
          double g[256], f[256];
          if (prev.q0 == (int)q0[i]) std::copy(R.begin(), R.end(), g);
          else swap_wires_ptm(R.vec().data(), g);
          for (int a = 0; a < 16; ++a)
            for (int b = 0; b < 16; ++b) {
              double acc = 0.0;
              for (int k = 0; k < 16; ++k) acc += g[a * 16 + k] * prev.R[k * 16 + b];
              f[a * 16 + b] = acc;
            }
          prev.R.assign(f, f + 256);
          prev.perm = is_signed_perm(prev.R, 16);
          prev.conj = prev.perm && is_conjugation(prev.R, 16);
          continue;
        }
        HostOp op;
        op.arity = 2; op.dim = 16; op.q0 = (int)q0[i]; op.q1 = (int)q1[i]; op.group = (int)r;
        op.R = R;
        op.mask = (1ull << op.q0) | (1ull << op.q1);
        op.perm = perm;
        op.conj = conj;
        last[q0[i]] = last[q1[i]] = ops.size();
        ops.push_back(std::move(op));
      }
    } else {
      while (ci < chains.size() && chains[ci].run == (int)r) {
        const double* R = ptm + ci * 16;
        HostOp op;
        op.arity = 1; op.dim = 4; op.q0 = op.q1 = chains[ci].wire; op.group = (int)r;
        op.mask = 1ull << op.q0;
        const int code = signed_perm_code4(R);
        if (code < 0) {  // not a signed permutation (a rotation chain)
          op.R.assign(R, R + 16);
          op.perm = op.conj = false;
          ops.push_back(std::move(op));
        } else if (code != kIdentityCode4) {
          auto it = perm_cache.find(code);
          if (it == perm_cache.end()) {
            Cls k;
            k.R.assign(R, R + 16);
            k.conj = is_conjugation(k.R, 4);
            it = perm_cache.emplace(code, std::move(k)).first;
          }
          op.R = it->second.R;
          op.perm = true;
          op.conj = it->second.conj;
          ops.push_back(std::move(op));
        }
        ++ci;
      }
    }
  }
  if (n_u) *n_u = nu;
  if (n_v) *n_v = nv;
  return QIMAX_OK;
}

// ------------------------------------------------------------------ host readout helpers
using u128 = unsigned __int128;

struct HostGens {
  std::vector<uint64_t> off;
  std::vector<u128> key;
  std::vector<double> w;
};

// Copy T keys of class KC from device memory into host u128 values.
hipError_t keys_to_host(const qimax_ctx* c, const void* dev, uint64_t T, std::vector<u128>& out) {
  out.resize(T);
  if (T == 0) return hipSuccess;
  if (c->KC == 2) return hipMemcpy(out.data(), dev, T * 16, hipMemcpyDeviceToHost);
  if (c->KC == 1) {
    std::vector<uint64_t> k(T);
    hipError_t e = hipMemcpy(k.data(), dev, T * 8, hipMemcpyDeviceToHost);
    for (uint64_t i = 0; i < T; ++i) out[i] = k[i];
    return e;
  }
  std::vector<uint32_t> k(T);
  hipError_t e = hipMemcpy(k.data(), dev, T * 4, hipMemcpyDeviceToHost);
  for (uint64_t i = 0; i < T; ++i) out[i] = k[i];
  return e;
}

// Keys as W little-endian uint64 words each (W = 1 for n <= 32, else 2).
void keys_to_words(const std::vector<u128>& k, uint32_t n, uint64_t* out) {
  const int W = n <= 32 ? 1 : 2;
  for (size_t i = 0; i < k.size(); ++i) {
    out[i * W] = (uint64_t)k[i];
    if (W == 2) out[i * W + 1] = (uint64_t)(k[i] >> 64);
  }
}

qimax_status fetch(qimax_ctx* c, HostGens& g) {
  QCHK(flush_pending(c));
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  g.off = c->h_seg;
  const uint64_t T = c->T;
  g.w.resize(T);
  HIPCHK(c, keys_to_host(c, c->keys.p, T, g.key), "keys D2H");
  if (T == 0) return QIMAX_OK;
  if (c->WP == 64) {
    HIPCHK(c, hipMemcpy(g.w.data(), c->w.p, T * 8, hipMemcpyDeviceToHost), "weights D2H");
  } else {
    std::vector<float> w32(T);
    HIPCHK(c, hipMemcpy(w32.data(), c->w.p, T * 4, hipMemcpyDeviceToHost), "weights D2H");
    for (uint64_t i = 0; i < T; ++i) g.w[i] = w32[i];
  }
  return QIMAX_OK;
}

// Terms [a, a + T) of the committed term arrays to host memory as the C-ABI returns them
// (n_words uint64 words per key, FP64 weights): converted on the device and copied in chunks
// through the image buffers, which are idle between calls and between rounds. *done stays
// false (nothing written) where those buffers cannot hold a chunk of 64 Ki terms or a graph
// is being recorded; the caller then converts on the host.
qimax_status export_terms(qimax_ctx* c, uint64_t a, uint64_t T, uint32_t n_words, uint64_t* words, double* w,
                          bool* done) {
  *done = false;
  if (c->rec) return QIMAX_OK;
  if (T == 0) {
    *done = true;
    return QIMAX_OK;
  }
  if (!c->ik[0].p || !c->iw[0].p) return QIMAX_OK;
  const uint64_t cap = std::min<uint64_t>(c->ik[0].bytes / (8ull * n_words), c->iw[0].bytes / 8);
  if (cap < (1ull << 16)) return QIMAX_OK;
  const uint8_t* kb = (const uint8_t*)c->keys.p + a * c->kb;
  const uint8_t* wb = (const uint8_t*)c->w.p + a * c->wb;
  for (uint64_t i = 0; i < T; i += cap) {
    const uint64_t m = std::min(cap, T - i);
    HIPCHK(c, launch_export(c->KC, c->WP, kb + i * c->kb, wb + i * c->wb, m, n_words, (uint64_t*)c->ik[0].p,
                            (double*)c->iw[0].p, c->stream), "export");
    HIPCHK(c, hipMemcpyAsync(words + i * n_words, c->ik[0].p, m * n_words * 8, hipMemcpyDeviceToHost, c->stream),
           "export D2H");
    HIPCHK(c, hipMemcpyAsync(w + i, c->iw[0].p, m * 8, hipMemcpyDeviceToHost, c->stream), "export D2H");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  *done = true;
  return QIMAX_OK;
}

int digit_of(u128 key, uint32_t n, uint32_t q) { return (int)((key >> (2 * (n - 1 - q))) & 3u); }


// <P> when every generator is one signed Pauli string (the Clifford case): P is +-(a
// product of generators) or anticommutes with one of them (then <P> = 0). The generators'
// GF(2) vectors (x|z bits) are reduced once; every string is then reduced against the pivots.
struct CliffordReducer {
  uint32_t n = 0;
  std::vector<std::vector<int>> dig;           // digits of generator j's string
  std::vector<double> sign;                    // its weight's sign
  std::vector<std::vector<uint8_t>> rows, combo;  // reduced rows and the generators they combine
  std::vector<int> piv_col;                    // pivot column of row r (-1: zero row)

  std::vector<uint8_t> vec(const std::vector<int>& d) const {
    std::vector<uint8_t> v(2 * n, 0);
    for (uint32_t q = 0; q < n; ++q) {
      v[q] = (d[q] == 1 || d[q] == 2);
      v[n + q] = (d[q] == 2 || d[q] == 3);
    }
    return v;
  }
  void init(uint32_t nq, const HostGens& g) {
    n = nq;
    const uint32_t N2 = 2 * n;
    dig.assign(n, std::vector<int>(n));
    sign.assign(n, 1.0);
    rows.assign(n, {});
    combo.assign(n, std::vector<uint8_t>(n, 0));
    piv_col.assign(n, -1);
    for (uint32_t j = 0; j < n; ++j) {
      for (uint32_t q = 0; q < n; ++q) dig[j][q] = digit_of(g.key[g.off[j]], n, q);
      sign[j] = g.w[g.off[j]] < 0 ? -1.0 : 1.0;
      rows[j] = vec(dig[j]);
      combo[j][j] = 1;
    }
    std::vector<uint8_t> used(n, 0);
    for (uint32_t col = 0; col < N2; ++col) {
      int piv = -1;
      for (uint32_t r = 0; r < n; ++r)
        if (!used[r] && rows[r][col]) { piv = (int)r; break; }
      if (piv < 0) continue;
      used[piv] = 1;
      piv_col[piv] = (int)col;
      for (uint32_t r = 0; r < n; ++r)
        if (r != (uint32_t)piv && rows[r][col]) {
          for (uint32_t k = 0; k < N2; ++k) rows[r][k] ^= rows[piv][k];
          for (uint32_t k = 0; k < n; ++k) combo[r][k] ^= combo[piv][k];
        }
    }
  }
  // returns false on inconsistent phases
  bool expect(const std::vector<int>& P, double* out) const {
    for (uint32_t j = 0; j < n; ++j) {  // anticommutes with a generator: <P> = 0
      int anti = 0;
      for (uint32_t q = 0; q < n; ++q) {
        const int a = dig[j][q], b = P[q];
        if (a && b && a != b) anti ^= 1;
      }
      if (anti) { *out = 0.0; return true; }
    }
    const uint32_t N2 = 2 * n;
    std::vector<uint8_t> target = vec(P), sel(n, 0);
    for (uint32_t r = 0; r < n; ++r) {
      if (piv_col[r] < 0 || !target[piv_col[r]]) continue;
      for (uint32_t k = 0; k < N2; ++k) target[k] ^= rows[r][k];
      for (uint32_t k = 0; k < n; ++k) sel[k] ^= combo[r][k];
    }
    for (uint32_t k = 0; k < N2; ++k)
      if (target[k]) { *out = 0.0; return true; }
    // product of the selected generators with its phase
    std::vector<int> acc(n, 0);
    int ph = 0;
    double sg = 1.0;
    for (uint32_t j = 0; j < n; ++j) {
      if (!sel[j]) continue;
      sg *= sign[j];
      for (uint32_t q = 0; q < n; ++q) {
        ph += kPh[acc[q]][dig[j][q]];
        acc[q] = kMul[acc[q]][dig[j][q]];
      }
    }
    ph &= 3;
    if (ph == 1 || ph == 3) return false;
    *out = sg * (ph == 2 ? -1.0 : 1.0);
    return true;
  }
};

constexpr uint32_t kSvMaxN = 30;     // device statevector readout: at most 2^30 amplitudes
constexpr double kSvMaxWork = 4e13;  // sum over generators of terms x 2^n

// Every generator a single term of weight +-1 (the state is a stabilizer state)?
qimax_status clifford_reducer(qimax_ctx* c, bool* is_cliff, CliffordReducer& red) {
  *is_cliff = false;
  for (uint32_t j = 0; j < c->n; ++j)
    if (c->h_seg[j + 1] - c->h_seg[j] != 1) return QIMAX_OK;
  HostGens g;
  QCHK(fetch(c, g));
  for (uint32_t j = 0; j < c->n; ++j)
    if (std::fabs(std::fabs(g.w[g.off[j]]) - 1.0) >= 1e-6) return QIMAX_OK;
  red.init(c->n, g);
  *is_cliff = true;
  return QIMAX_OK;
}

// Strings of n letters "IXYZ" as digits.
qimax_status parse_paulis(qimax_ctx* c, const char* s, size_t k, std::vector<std::vector<int>>& out) {
  out.assign(k, std::vector<int>(c->n));
  for (size_t i = 0; i < k; ++i)
    for (uint32_t q = 0; q < c->n; ++q) {
      const char ch = s[i * c->n + q];
      const char* pos = ch ? std::strchr("IXYZ", ch) : nullptr;
      if (!pos) return fail(c, QIMAX_EINVAL, "pauli strings must be n letters of IXYZ");
      out[i][q] = (int)(pos - "IXYZ");
    }
  return QIMAX_OK;
}

// <P> for every string of Ps (zall: <Z_q> for every qubit instead) from a statevector on the
// device: a seeded random vector projected by (I + G_j)/2 for every generator j is, once
// normalised, the state rho = 2^-n prod_j (I + G_j) projects onto (eq. (2)).
qimax_status expect_device(qimax_ctx* c, const std::vector<std::vector<int>>& Ps, bool zall, double* out) {
  const uint32_t n = c->n;
  if (n > kSvMaxN) return fail(c, QIMAX_ETOOLARGE, "expect: a state with non-Clifford generators and n > 30");
  const uint64_t D = 1ull << n, T = c->T;
  if ((double)T * (double)D > kSvMaxWork) return fail(c, QIMAX_ETOOLARGE, "expect: too many terms for the projection");
  const size_t sv_bytes = (size_t)D * 16, t_bytes = (size_t)std::max<uint64_t>(T, 1) * 32;
  const size_t need = 2 * sv_bytes + t_bytes + 512;
  if (c->cap && c->alloc_bytes + need > c->cap) return fail(c, QIMAX_ENOMEM, "expect: memory cap exceeded");
  void* mem = nullptr;
  if (hipMalloc(&mem, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, QIMAX_ENOMEM, "expect: hipMalloc of the statevector failed");
  }
  c->peak_bytes = std::max(c->peak_bytes, (uint64_t)(c->alloc_bytes + need));
  uint8_t* m = (uint8_t*)mem;
  void* v = m;
  void* tmp = m + sv_bytes;
  uint64_t* xm = (uint64_t*)(m + 2 * sv_bytes);
  uint64_t* zm = xm + std::max<uint64_t>(T, 1);
  void* cf = zm + std::max<uint64_t>(T, 1);
  double* acc = (double*)(m + 2 * sv_bytes + t_bytes);
  auto done = [&](qimax_status st) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(mem);
    return st;
  };
  hipError_t e = launch_sv_terms(c->KC, c->WP, c->keys.p, c->w.p, T, n, xm, zm, cf, c->stream);
  if (e == hipSuccess) e = launch_sv_random(v, D, 0x5eed5eedull + n, c->stream);
  for (uint32_t j = 0; j < n && e == hipSuccess; ++j) {
    const uint64_t a = c->h_seg[j], b = c->h_seg[j + 1];
    e = launch_sv_project(v, tmp, D, xm + a, zm + a, (uint8_t*)cf + a * 16, b - a, c->stream);
  }
  auto reduce = [&](uint64_t x, uint64_t z, double cre, double cim, int za, double* h) -> hipError_t {
    hipError_t r = hipMemsetAsync(acc, 0, 64 * 8, c->stream);
    if (r == hipSuccess) r = launch_sv_reduce(v, D, n, x, z, cre, cim, za, acc, c->stream);
    if (r == hipSuccess) r = hipMemcpyAsync(h, acc, 64 * 8, hipMemcpyDeviceToHost, c->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(c->stream);
    return r;
  };
  double h[64];
  if (e == hipSuccess && zall) {
    e = reduce(0, 0, 0.0, 0.0, 1, h);
    if (e == hipSuccess) {
      if (!(h[0] > 1e-280)) return done(fail(c, QIMAX_EDEVICE, "expect: projection vanished"));
      for (uint32_t q = 0; q < n; ++q) out[q] = h[1 + q] / h[0];
    }
  }
  for (size_t i = 0; i < Ps.size() && e == hipSuccess && !zall; ++i) {
    uint64_t x = 0, z = 0;
    int ny = 0;
    for (uint32_t q = 0; q < n; ++q) {
      const int d = Ps[i][q];
      const uint64_t bit = 1ull << (n - 1 - q);
      if (d == 1 || d == 2) x |= bit;
      if (d == 2 || d == 3) z |= bit;
      ny += d == 2;
    }
    static const double ph[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    e = reduce(x, z, ph[ny & 3][0], ph[ny & 3][1], 0, h);
    if (e == hipSuccess) {
      if (!(h[0] > 1e-280)) return done(fail(c, QIMAX_EDEVICE, "expect: projection vanished"));
      out[i] = h[1] / h[0];
    }
  }
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(c, e, "expect (device statevector)");
  }
  return done(QIMAX_OK);
}

// <P> for k strings: the GF(2) path for a stabilizer state, else the device statevector.
qimax_status expect_strings(qimax_ctx* c, const std::vector<std::vector<int>>& Ps, double* out) {
  QCHK(flush_pending(c));
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  bool cliff = false;
  CliffordReducer red;
  QCHK(clifford_reducer(c, &cliff, red));
  if (cliff) {
    for (size_t i = 0; i < Ps.size(); ++i)
      if (!red.expect(Ps[i], &out[i])) return fail(c, QIMAX_EDEVICE, "inconsistent generator phases");
    return QIMAX_OK;
  }
  return expect_device(c, Ps, false, out);
}

}  // namespace

// ================================================================================ C ABI

extern "C" {

void qimax_default_opts(qimax_opts* o) {
  if (!o) return;
  o->precision = 64;
  o->fp32_merge = 0;
  o->prune_eps = 0.0;
  o->mem_cap_bytes = 0;
  o->hip_stream = nullptr;
  o->validate = 1;
  o->device = -1;
}

qimax_status qimax_create(uint32_t n, const qimax_opts* opts, qimax_ctx** out) {
  if (!out) return QIMAX_EINVAL;
  *out = nullptr;
  qimax_opts o;
  qimax_default_opts(&o);
  if (opts) o = *opts;
  if (n < 1) { g_create_error = "n must be >= 1"; return QIMAX_EINVAL; }
  if (n > 64) { g_create_error = "n must be <= 64"; return QIMAX_ETOOLARGE; }
  if (o.precision != 64 && o.precision != 32) { g_create_error = "precision must be 32 or 64"; return QIMAX_EINVAL; }
  if (!(o.prune_eps >= 0.0) || !std::isfinite(o.prune_eps)) { g_create_error = "prune_eps must be >= 0"; return QIMAX_EINVAL; }
  qimax_ctx* c = new (std::nothrow) qimax_ctx;
  if (!c) return QIMAX_ENOMEM;
  c->n = n;
  c->KC = n <= 16 ? 0 : (n <= 32 ? 1 : 2);
  c->kb = (size_t)4 << c->KC;
  c->WP = o.precision;
  c->wb = o.precision == 64 ? 8 : 4;
  c->fp64_acc = o.fp32_merge ? 1 : 0;
  c->eps = o.prune_eps;
  c->cap = o.mem_cap_bytes;
  c->validate = o.validate;
  {
    const char* env = std::getenv("QIMAX_SORT_CLASSIC");
    c->classic_sort = env && env[0] == '1';
    env = std::getenv("QIMAX_HOST_TILING");  // always read the image count back before expanding
    c->host_tiling = env && env[0] == '1';
    env = std::getenv("QIMAX_XCD_RANGES");  // 0: sort tiles claimed in one global order
    c->xcd_ranges = !(env && env[0] == '0');
    env = std::getenv("QIMAX_SMALL_ROUNDS");  // 0: small rounds take the general path too
    c->small_rounds = !(env && env[0] == '0');
    env = std::getenv("QIMAX_FUSED_EXPAND");  // 0: separate count and expansion launches
    c->fused_expand = !(env && env[0] == '0');
    env = std::getenv("QIMAX_DENSE");  // 1: dense accumulation wherever it applies; auto: tuned
    c->dense_mode = (env && env[0] == '1') ? 1 : (env && std::strcmp(env, "auto") == 0) ? 2 : 0;
    env = std::getenv("QIMAX_LOCAL_SORT");  // 0: every digit by global passes
    c->local_sort = !(env && env[0] == '0');
    env = std::getenv("QIMAX_LOCAL_SORT_M");  // force the number of top-digit passes (tests)
    if (env && env[0]) c->local_sort_m = std::atoi(env);
    env = std::getenv("QIMAX_DEFER_SPINS");  // chunk-local merge: polls before deferring a chunk
    if (env && env[0]) c->defer_spins = (uint32_t)std::strtoul(env, nullptr, 10);
    env = std::getenv("QIMAX_CHUNK_TILE");  // fixed nominal chunk of a fused round (2048 .. 4096)
    if (env && env[0])
      c->chunk_tile = std::min<uint32_t>(std::max<uint32_t>((uint32_t)std::strtoul(env, nullptr, 10), kExpandTile),
                                         (uint32_t)kChunkCap);
    env = std::getenv("QIMAX_SMALL_GROUPS");  // 0: every small pass as a round of its own
    c->small_groups = !(env && env[0] == '0');
    env = std::getenv("QIMAX_CLASSIC_PASSES");  // 1: multi-launch global passes in the single-sweep rounds
    c->classic_passes = env && env[0] == '1';
    env = std::getenv("QIMAX_WIDE_OFFSETS");  // 1: the count's and expansion's paths for huge rounds
    c->wide_offsets = env && env[0] == '1';
    env = std::getenv("QIMAX_AUTOTUNE");  // 0: always the heuristic's sort variant
    c->autotune = !(env && env[0] == '0');
  }
  hipError_t e;
  if (o.device >= 0) {
    e = hipSetDevice(o.device);
    if (e != hipSuccess) { g_create_error = hipGetErrorString(e); delete c; return QIMAX_EDEVICE; }
  }
  e = hipGetDevice(&c->device);
  if (e != hipSuccess) { g_create_error = hipGetErrorString(e); delete c; return QIMAX_EDEVICE; }
  if (o.hip_stream) {
    c->stream = (hipStream_t)o.hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) { g_create_error = hipGetErrorString(e); delete c; return QIMAX_EDEVICE; }
    c->own_stream = true;
  }
  for (hipEvent_t& ev : c->tune_ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      ev = nullptr;
      c->autotune = false;
    }
  qimax_status s;
  if ((s = ensure(c, c->keys, n * c->kb, false)) != QIMAX_OK || (s = ensure(c, c->w, n * c->wb, false)) != QIMAX_OK ||
      (s = ensure(c, c->seg, (n + 1) * 8, false)) != QIMAX_OK || (s = ensure(c, c->err, 256, false)) != QIMAX_OK) {
    g_create_error = c->last_error;
    qimax_destroy(c);
    return s;
  }
  e = launch_init(c->KC, c->WP, c->keys.p, c->w.p, (uint64_t*)c->seg.p, n, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_create_error = hipGetErrorString(e);
    qimax_destroy(c);
    return QIMAX_EDEVICE;
  }
  c->h_seg.resize(n + 1);
  for (uint32_t j = 0; j <= n; ++j) c->h_seg[j] = j;
  c->T = n;
  c->st.terms = n;
  *out = c;
  return QIMAX_OK;
}

qimax_status qimax_reset(qimax_ctx* c) {
  if (!c) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  HIPCHK(c, launch_init(c->KC, c->WP, c->keys.p, c->w.p, (uint64_t*)c->seg.p, c->n, c->stream, &c->prof), "init");
  for (uint32_t j = 0; j <= c->n; ++j) c->h_seg[j] = j;
  c->T = c->n;
  c->st.terms = c->n;
  c->pending.clear();
  return QIMAX_OK;
}

qimax_status qimax_flush(qimax_ctx* c) {
  if (!c) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  return flush_pending(c);
}

qimax_status qimax_apply_layer(qimax_ctx* c, const qimax_op* ops, size_t n_ops) {
  if (!c) return QIMAX_EINVAL;
  if (n_ops && !ops) return fail(c, QIMAX_EINVAL, "ops is NULL");
  std::vector<HostOp> hops(n_ops);
  // the paper's partition of the operator list: maximal runs of equal arity
  int group = 0;
  for (size_t i = 0; i < n_ops; ++i) {
    if (i && ops[i].arity != ops[i - 1].arity) ++group;
    QCHK(check_op_input(c, ops[i], group, hops[i]));
  }
  return apply_ops(c, hops);
}

qimax_status qimax_apply_circuit(qimax_ctx* c, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                                 const double* theta, size_t m) {
  if (!c) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (m && (!gate || !q0 || !q1)) return fail(c, QIMAX_EINVAL, "instruction arrays are NULL");
  std::vector<HostOp> ops;
  {
    BusyTimer bt(c);
    QCHK(group_circuit(c, c->n, gate, q0, q1, theta, m, ops, nullptr, nullptr));
  }
  return apply_ops(c, ops);
}

// ------------------------------------------------------------------------ step graphs

void qimax_graph_destroy(qimax_graph* g) {
  if (!g) return;
  if (g->ctx && g->ctx->stream) (void)hipStreamSynchronize(g->ctx->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  for (hipGraphExec_t x : g->runs) (void)hipGraphExecDestroy(x);
  if (g->whole) (void)hipGraphDestroy(g->whole);
  for (hipGraph_t p : g->parts) (void)hipGraphDestroy(p);
  for (void* h : g->snaps) (void)hipHostFree(h);
  delete g;
}

qimax_status qimax_graph_record(qimax_ctx* c, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                                const double* theta, size_t m, const uint64_t* layer_end, size_t n_layers,
                                qimax_graph** out) {
  if (!c || !out) return QIMAX_EINVAL;
  *out = nullptr;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (c->rec) return fail(c, QIMAX_ESTATE, "a recording is already in progress");
  if (m && (!gate || !q0 || !q1)) return fail(c, QIMAX_EINVAL, "instruction arrays are NULL");
  std::vector<uint64_t> ends;
  if (layer_end && n_layers) ends.assign(layer_end, layer_end + n_layers);
  else ends.push_back(m);
  for (size_t l = 0; l < ends.size(); ++l)
    if (ends[l] > m || (l && ends[l] < ends[l - 1])) return fail(c, QIMAX_EINVAL, "layer ends out of order");
  if (ends.back() != m) return fail(c, QIMAX_EINVAL, "the last layer must end at m");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  // The step runs before it is recorded, with the same sort variants as the recording (no
  // exploration), until every buffer is large enough for the recording. A step moves the term
  // buffers between their roles (the current terms and the two pass outputs: a cycle of at
  // most three), so a buffer can meet a larger role only after up to three runs: the warm-up
  // ends after three runs in a row that grew nothing.
  c->tune_frozen = true;
  auto run_step = [&]() -> qimax_status {
    QCHK(qimax_reset(c));
    uint64_t a0 = 0;
    for (size_t l = 0; l < ends.size(); ++l) {
      QCHK(qimax_apply_circuit(c, gate + a0, q0 + a0, q1 + a0, theta ? theta + a0 : nullptr, ends[l] - a0));
      a0 = ends[l];
    }
    return flush_pending(c);
  };
  for (int runs = 0, quiet = 0; quiet < 3 && runs < 9; ++runs) {
    const uint64_t gen = c->buf_gen;
    const qimax_status s0 = run_step();
    if (s0 != QIMAX_OK) {
      c->tune_frozen = false;
      return s0;
    }
    quiet = c->buf_gen == gen ? quiet + 1 : 0;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  qimax_graph* g = new qimax_graph;
  g->ctx = c;
  const qimax_stats st0 = c->st;
  std::vector<uint64_t> upd0 = c->gen_updates;
  upd0.resize(c->n, 0);
  const bool prof_on = c->prof.on;
  c->prof.on = false;  // no timing events inside a recording
  const uint64_t gen0 = c->buf_gen;
  c->rec = g;
  qimax_status s = rec_resume(c);
  if (s == QIMAX_OK) s = run_step();
  if (s == QIMAX_OK) s = rec_cut(c);
  if (c->rec_capturing) {  // a failure inside a captured part: drop it
    hipGraph_t junk = nullptr;
    (void)hipStreamEndCapture(c->stream, &junk);
    if (junk) (void)hipGraphDestroy(junk);
    c->rec_capturing = false;
  }
  c->rec = nullptr;
  c->prof.on = prof_on;
  c->tune_frozen = false;
  if (s == QIMAX_OK && c->buf_gen != gen0)
    s = fail(c, QIMAX_ESTATE, "the context's buffers changed while recording: run the step once first");
  if (hipStreamSynchronize(c->stream) != hipSuccess && s == QIMAX_OK) s = fail(c, QIMAX_EDEVICE, "recorded step failed");
  for (hipGraphExec_t x : g->runs) (void)hipGraphExecDestroy(x);
  g->runs.clear();
  if (s == QIMAX_OK) {
    hipError_t e = hipGraphCreate(&g->whole, 0);
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < g->parts.size() && e == hipSuccess; ++i) {
      hipGraphNode_t node = nullptr;
      e = hipGraphAddChildGraphNode(&node, g->whole, prev ? &prev : nullptr, prev ? 1 : 0, g->parts[i]);
      prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->whole, nullptr, nullptr, 0);
    if (e != hipSuccess) s = fail(c, QIMAX_EDEVICE, std::string("building the step graph: ") + hipGetErrorString(e));
  }
  if (s != QIMAX_OK) {
    const std::string msg = c->last_error;
    g->ctx = nullptr;  // nothing of it is in flight
    qimax_graph_destroy(g);
    if (!c->broken) (void)qimax_reset(c);
    c->last_error = msg;
    return s;
  }
  g->gen = c->buf_gen;
  g->epoch_end = c->epoch;
  g->mepoch_end = c->mepoch;
  g->keys = c->keys; g->w = c->w; g->seg = c->seg;
  for (int i = 0; i < 2; ++i) { g->pk[i] = c->pk[i]; g->pw[i] = c->pw[i]; g->pseg[i] = c->pseg[i]; }
  g->h_seg = c->h_seg;
  g->T = c->T;
  g->st_delta.passes = c->st.passes - st0.passes;
  g->st_delta.term_updates = c->st.term_updates - st0.term_updates;
  g->st_delta.images = c->st.images - st0.images;
  g->st_delta.sort_elems = c->st.sort_elems - st0.sort_elems;
  g->st_delta.rounds = c->st.rounds - st0.rounds;
  g->st_delta.alg_bytes = c->st.alg_bytes - st0.alg_bytes;
  g->upd_delta.assign(c->n, 0);
  for (uint32_t j = 0; j < c->n && j < c->gen_updates.size(); ++j) g->upd_delta[j] = c->gen_updates[j] - upd0[j];
  *out = g;
  return QIMAX_OK;
}

qimax_status qimax_graph_launch(qimax_graph* g) {
  if (!g || !g->ctx) return QIMAX_EINVAL;
  qimax_ctx* c = g->ctx;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (c->rec) return fail(c, QIMAX_ESTATE, "a recording is in progress");
  if (c->buf_gen != g->gen) return fail(c, QIMAX_ESTATE, "the context's buffers changed since the recording");
  // the recorded buffers must be the context's (in any of the roles a call swaps them through)
  auto same = [](std::initializer_list<const DevBuf*> x, std::initializer_list<const DevBuf*> y) {
    std::vector<void*> a, b;
    for (auto* d : x) a.push_back(d->p);
    for (auto* d : y) b.push_back(d->p);
    std::sort(a.begin(), a.end());
    std::sort(b.begin(), b.end());
    return a == b;
  };
  if (!same({&c->keys, &c->pk[0], &c->pk[1]}, {&g->keys, &g->pk[0], &g->pk[1]}) ||
      !same({&c->w, &c->pw[0], &c->pw[1]}, {&g->w, &g->pw[0], &g->pw[1]}) ||
      !same({&c->seg, &c->pseg[0], &c->pseg[1]}, {&g->seg, &g->pseg[0], &g->pseg[1]}))
    return fail(c, QIMAX_ESTATE, "the context's term buffers are not the recorded ones");
  // look-back status words carry the recorded epochs: clear them first
  if (c->mstatus.p) HIPCHK(c, launch_fill_u64((uint64_t*)c->mstatus.p, c->mstatus.bytes / 8, 0ull, c->stream), "clear status");
  if (c->sstatus.p) HIPCHK(c, launch_fill_u64((uint64_t*)c->sstatus.p, c->sstatus.bytes / 8, 0ull, c->stream), "clear status");
  HIPCHK(c, hipGraphLaunch(g->exec, c->stream), "hipGraphLaunch");
  c->keys = g->keys; c->w = g->w; c->seg = g->seg;
  for (int i = 0; i < 2; ++i) { c->pk[i] = g->pk[i]; c->pw[i] = g->pw[i]; c->pseg[i] = g->pseg[i]; }
  c->h_seg = g->h_seg;
  c->T = g->T;
  c->st.terms = c->T;
  c->pending.clear();
  // the replay leaves status words tagged with the recorded epochs: later rounds count on
  // from above them
  c->epoch = std::max(c->epoch, g->epoch_end);
  c->mepoch = std::max(c->mepoch, g->mepoch_end);
  c->st.passes += g->st_delta.passes;
  c->st.term_updates += g->st_delta.term_updates;
  c->st.images += g->st_delta.images;
  c->st.sort_elems += g->st_delta.sort_elems;
  c->st.rounds += g->st_delta.rounds;
  c->st.alg_bytes += g->st_delta.alg_bytes;
  if (c->gen_updates.size() != c->n) c->gen_updates.assign(c->n, 0);
  for (uint32_t j = 0; j < c->n; ++j) c->gen_updates[j] += g->upd_delta[j];
  return QIMAX_OK;
}

qimax_status qimax_group_circuit(qimax_ctx* c, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                                 const double* theta, size_t m, qimax_op* ops, double* ptm_buf, size_t cap,
                                 size_t* n_ops, size_t* n_u, size_t* n_v) {
  if (!c || !n_ops) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (m && (!gate || !q0 || !q1)) return fail(c, QIMAX_EINVAL, "instruction arrays are NULL");
  std::vector<HostOp> hops;
  QCHK(group_circuit(c, c->n, gate, q0, q1, theta, m, hops, n_u, n_v));
  *n_ops = hops.size();
  if (cap == 0) return QIMAX_OK;
  if (!ops || !ptm_buf) return fail(c, QIMAX_EINVAL, "ops / ptm_buf is NULL");
  size_t off = 0;
  for (size_t i = 0; i < hops.size() && i < cap; ++i) {
    ops[i].arity = (uint32_t)hops[i].arity;
    ops[i].q[0] = (uint32_t)hops[i].q0;
    ops[i].q[1] = (uint32_t)hops[i].q1;
    std::copy(hops[i].R.begin(), hops[i].R.end(), ptm_buf + off);
    ops[i].ptm = ptm_buf + off;
    off += hops[i].R.size();
  }
  return QIMAX_OK;
}

qimax_status qimax_num_terms(qimax_ctx* c, uint64_t* T) {
  if (!c || !T) return QIMAX_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  *T = c->T;
  return QIMAX_OK;
}

qimax_status qimax_get_generators(qimax_ctx* c, uint64_t* gen_off, uint64_t* keys, double* w, size_t cap,
                                  size_t* T) {
  if (!c || !T) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  QCHK(flush_pending(c));
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  *T = (size_t)c->T;
  if (cap < c->T) {
    if (gen_off) std::copy(c->h_seg.begin(), c->h_seg.end(), gen_off);
    return QIMAX_OK;
  }
  if (!gen_off || (c->T && (!keys || !w))) return fail(c, QIMAX_EINVAL, "output buffers are NULL");
  bool done = false;
  QCHK(export_terms(c, 0, c->T, c->n <= 32 ? 1u : 2u, keys, w, &done));
  if (done) {
    std::copy(c->h_seg.begin(), c->h_seg.end(), gen_off);
    return QIMAX_OK;
  }
  HostGens g;
  QCHK(fetch(c, g));
  std::copy(g.off.begin(), g.off.end(), gen_off);
  keys_to_words(g.key, c->n, keys);
  std::copy(g.w.begin(), g.w.end(), w);
  return QIMAX_OK;
}

qimax_status qimax_expect(qimax_ctx* c, const char* pauli, double* out) {
  if (!c || !pauli || !out) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (std::strlen(pauli) != c->n) return fail(c, QIMAX_EINVAL, "pauli must be exactly n letters");
  std::vector<std::vector<int>> Ps;
  QCHK(parse_paulis(c, pauli, 1, Ps));
  return expect_strings(c, Ps, out);
}

qimax_status qimax_expect_many(qimax_ctx* c, const char* paulis, size_t k, double* out) {
  if (!c || (k && (!paulis || !out))) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  std::vector<std::vector<int>> Ps;
  QCHK(parse_paulis(c, paulis, k, Ps));
  if (k == 0) return QIMAX_OK;
  return expect_strings(c, Ps, out);
}

qimax_status qimax_prob_zero_all(qimax_ctx* c, double* p0) {
  if (!c || !p0) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  QCHK(flush_pending(c));
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  std::vector<double> z(c->n);
  bool cliff = false;
  CliffordReducer red;
  QCHK(clifford_reducer(c, &cliff, red));
  if (cliff) {
    std::vector<int> P(c->n, 0);
    for (uint32_t q = 0; q < c->n; ++q) {
      std::fill(P.begin(), P.end(), 0);
      P[q] = 3;
      if (!red.expect(P, &z[q])) return fail(c, QIMAX_EDEVICE, "inconsistent generator phases");
    }
  } else {
    QCHK(expect_device(c, {}, true, z.data()));
  }
  for (uint32_t q = 0; q < c->n; ++q) p0[q] = 0.5 * (1.0 + z[q]);
  return QIMAX_OK;
}

qimax_status qimax_get_generators_xz(qimax_ctx* c, uint64_t* gen_off, uint64_t* x, uint64_t* z, double* w, size_t cap,
                                     size_t* T) {
  if (!c || !T) return QIMAX_EINVAL;
  if (c->broken) return fail(c, QIMAX_ESTATE, "context unusable after an earlier device error");
  QCHK(flush_pending(c));
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  *T = (size_t)c->T;
  if (gen_off) std::copy(c->h_seg.begin(), c->h_seg.end(), gen_off);
  if (cap < c->T) return QIMAX_OK;
  if (!gen_off || (c->T && (!x || !z || !w))) return fail(c, QIMAX_EINVAL, "output buffers are NULL");
  if (c->T == 0) return QIMAX_OK;
  const size_t tb = (size_t)c->T * 8;
  void* mem = nullptr;
  if (hipMalloc(&mem, 3 * tb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, QIMAX_ENOMEM, "get_generators_xz: hipMalloc of the readout buffers failed");
  }
  uint64_t* dx = (uint64_t*)mem;
  uint64_t* dz = dx + c->T;
  double* dw = (double*)(dz + c->T);
  hipError_t e = launch_keys_to_xz(c->KC, c->keys.p, c->T, c->n, dx, dz, c->stream);
  if (e == hipSuccess) {
    if (c->WP == 64) e = hipMemcpyAsync(dw, c->w.p, tb, hipMemcpyDeviceToDevice, c->stream);
    else e = launch_weights_to_f64(c->WP, c->w.p, dw, c->T, c->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(x, dx, tb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(z, dz, tb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(w, dw, tb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(mem);
  if (e != hipSuccess) return hip_fail(c, e, "get_generators_xz");
  return QIMAX_OK;
}

namespace {

// The comparison of qimax_compare. With a scratch area (no_alloc), the tile arrays and the
// accumulators live there and nothing is allocated on the device; deferred operators are then
// refused instead of applied (applying them allocates).
qimax_status compare_impl(qimax_ctx* a, qimax_ctx* b, double tau, double* diff_norm, double* ref_norm,
                          uint64_t* n_tau_diff, bool no_alloc) {
  if (!a || !b || !diff_norm || !ref_norm || !n_tau_diff) return QIMAX_EINVAL;
  if (a->n != b->n) return fail(a, QIMAX_EINVAL, "compare: contexts of different n");
  if (a->device != b->device) return fail(a, QIMAX_EINVAL, "compare: contexts on different devices");
  if (a->broken || b->broken) return fail(a, QIMAX_ESTATE, "context unusable after an earlier device error");
  if (no_alloc) {
    if (!a->pending.empty() || !b->pending.empty())
      return fail(a, QIMAX_ESTATE, "compare_noalloc: a context holds deferred operators (call qimax_flush first)");
  } else {
    QCHK(flush_pending(a));
    qimax_status sb = flush_pending(b);
    if (sb != QIMAX_OK) return fail(a, sb, std::string("compare: ") + b->last_error);
  }
  int prev_dev = -1;
  HIPCHK(a, hipGetDevice(&prev_dev), "hipGetDevice");
  if (prev_dev != a->device) HIPCHK(a, hipSetDevice(a->device), "hipSetDevice");
  struct Restore {
    int dev, prev;
    ~Restore() {
      if (prev != dev) (void)hipSetDevice(prev);
    }
  } restore{a->device, prev_dev};
  HIPCHK(a, hipStreamSynchronize(a->stream), "hipStreamSynchronize");
  HIPCHK(a, hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  const uint32_t n = a->n;
  const uint64_t tile = compare_tile();
  // tiles of one side's segments, side a then side b
  HostTiling ta, tb;
  make_tiling(a->h_seg, tile, ta);
  make_tiling(b->h_seg, tile, tb);
  const size_t na = ta.begin.size(), nb = tb.begin.size(), nt = na + nb;
  std::vector<uint64_t> host_u64;
  host_u64.insert(host_u64.end(), a->h_seg.begin(), a->h_seg.end());
  host_u64.insert(host_u64.end(), b->h_seg.begin(), b->h_seg.end());
  host_u64.insert(host_u64.end(), ta.begin.begin(), ta.begin.end());
  host_u64.insert(host_u64.end(), tb.begin.begin(), tb.begin.end());
  host_u64.insert(host_u64.end(), ta.end.begin(), ta.end.end());
  host_u64.insert(host_u64.end(), tb.end.begin(), tb.end.end());
  std::vector<uint32_t> segs(ta.seg);
  segs.insert(segs.end(), tb.seg.begin(), tb.seg.end());
  const size_t ou = host_u64.size() * 8, os = align256(ou), oacc = os + align256(std::max<size_t>(segs.size(), 1) * 4);
  const size_t ocnt = oacc + align256((size_t)n * 16), total = ocnt + align256((size_t)n * 8);
  void* mem = nullptr;
  if (no_alloc) {
    size_t cap = 0;
    HIPCHK(a, compare_scratch(a->device, &mem, &cap), "compare_noalloc scratch");
    if (total > cap)
      return fail(a, QIMAX_ETOOLARGE, "compare_noalloc: " + std::to_string(total) + " bytes of tiles and sums exceed the " +
                                          std::to_string(cap) + "-byte scratch (" + std::to_string(nt) + " tiles)");
  } else if (hipMalloc(&mem, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(a, QIMAX_ENOMEM, "compare: hipMalloc failed");
  }
  uint8_t* m = (uint8_t*)mem;
  const uint64_t* d_aoff = (const uint64_t*)m;
  const uint64_t* d_boff = d_aoff + (n + 1);
  const uint64_t* d_beg = d_boff + (n + 1);
  const uint64_t* d_end = d_beg + nt;
  const uint32_t* d_seg = (const uint32_t*)(m + os);
  double* acc = (double*)(m + oacc);
  unsigned long long* cnt = (unsigned long long*)(m + ocnt);
  hipStream_t st = a->stream;
  hipError_t e = hipMemcpyAsync(m, host_u64.data(), ou, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !segs.empty()) e = hipMemcpyAsync(m + os, segs.data(), segs.size() * 4, hipMemcpyHostToDevice, st);
  // the sums and counters start at zero (a fill kernel: no memset node if the stream is captured)
  if (e == hipSuccess) e = launch_fill_u64((uint64_t*)acc, (total - oacc) / 8, 0ull, st);
  // pass 0 over a's terms (searched in b), pass 1 over b's (the reference) searched in a
  if (e == hipSuccess)
    e = launch_compare(a->KC, a->WP, b->WP, a->keys.p, a->w.p, b->keys.p, b->w.p, d_boff, d_beg, d_end, d_seg,
                       (uint32_t)na, 0, tau, acc, cnt, st);
  if (e == hipSuccess)
    e = launch_compare(a->KC, b->WP, a->WP, b->keys.p, b->w.p, a->keys.p, a->w.p, d_aoff, d_beg + na, d_end + na,
                       d_seg + na, (uint32_t)nb, 1, tau, acc, cnt, st);
  std::vector<double> h_acc(2 * (size_t)n);
  std::vector<unsigned long long> h_cnt(n);
  if (e == hipSuccess) e = hipMemcpyAsync(h_acc.data(), acc, (size_t)n * 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h_cnt.data(), cnt, (size_t)n * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (!no_alloc) (void)hipFree(mem);
  if (e != hipSuccess) return hip_fail(a, e, no_alloc ? "compare_noalloc" : "compare");
  for (uint32_t j = 0; j < n; ++j) {
    diff_norm[j] = std::sqrt(h_acc[2 * j]);
    ref_norm[j] = std::sqrt(h_acc[2 * j + 1]);
    n_tau_diff[j] = h_cnt[j];
  }
  return QIMAX_OK;
}

}  // namespace

qimax_status qimax_compare(qimax_ctx* a, qimax_ctx* b, double tau, double* diff_norm, double* ref_norm,
                           uint64_t* n_tau_diff) {
  return compare_impl(a, b, tau, diff_norm, ref_norm, n_tau_diff, false);
}

qimax_status qimax_compare_noalloc(qimax_ctx* a, qimax_ctx* b, double tau, double* diff_norm, double* ref_norm,
                                   uint64_t* n_tau_diff) {
  return compare_impl(a, b, tau, diff_norm, ref_norm, n_tau_diff, true);
}

qimax_status qimax_get_tuning(const qimax_ctx* c, qimax_tune_entry* out, size_t cap, size_t* n) {
  if (!c || !n || (cap && !out)) return QIMAX_EINVAL;
  size_t i = 0;
  for (const auto& kv : c->tune) {
    if (i < cap) {
      const uint32_t k = kv.first;  // see the size class of a round in run_round
      qimax_tune_entry& e = out[i];
      e.key_bytes = 4u << ((k >> 8) & 3u);
      e.weight_bits = (k & 64u) ? 64u : 32u;
      e.log2_images = k & 63u;
      e.dense_candidate = (k >> 20) & 1u;
      e.best = kv.second.best;
      e.tried = (uint32_t)kv.second.tried;
      for (int j = 0; j < 6; ++j) e.ms[j] = j < TuneState::kCand ? kv.second.ms[j] : 0.f;
    }
    ++i;
  }
  *n = i;
  return QIMAX_OK;
}

qimax_status qimax_get_stats(const qimax_ctx* c, qimax_stats* out) {
  if (!c || !out) return QIMAX_EINVAL;
  *out = c->st;
  out->terms = c->T;
  out->peak_bytes = c->peak_bytes;
  out->alloc_bytes = c->alloc_bytes;
  return QIMAX_OK;
}

qimax_status qimax_profile(qimax_ctx* c, int enable) {
  if (!c) return QIMAX_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  prof_resolve(&c->prof);
  if (enable) prof_reset(&c->prof);
  c->prof.on = enable != 0;
  return QIMAX_OK;
}

qimax_status qimax_profile_only(qimax_ctx* c, const char* kernel) {
  if (!c) return QIMAX_EINVAL;
  if (!kernel || !kernel[0]) {
    c->prof.mask = ~0u;
    return QIMAX_OK;
  }
  for (int i = 0; i < kKNum; ++i)
    if (std::strcmp(kernel, kernel_kind_name(i)) == 0) {
      c->prof.mask = 1u << i;
      return QIMAX_OK;
    }
  return fail(c, QIMAX_EINVAL, std::string("unknown kernel name ") + kernel);
}

qimax_status qimax_profile_read(qimax_ctx* c, qimax_kernel_time* out, size_t cap, size_t* n) {
  if (!c || !n) return QIMAX_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  prof_resolve(&c->prof);
  size_t k = 0;
  for (int i = 0; i < kKNum; ++i) {
    if (!c->prof.launches[i]) continue;
    if (out && k < cap) {
      out[k].name = kernel_kind_name(i);
      out[k].launches = c->prof.launches[i];
      out[k].total_ms = c->prof.ms[i];
      out[k].alg_bytes = c->prof.bytes[i];
    }
    ++k;
  }
  *n = k;
  return QIMAX_OK;
}

qimax_status qimax_get_generator_updates(const qimax_ctx* c, uint64_t* out, size_t n) {
  if (!c || !out || n < c->n) return QIMAX_EINVAL;
  for (uint32_t j = 0; j < c->n; ++j) out[j] = j < c->gen_updates.size() ? c->gen_updates[j] : 0;
  return QIMAX_OK;
}

qimax_status qimax_copy_probe(size_t bytes, int reps, double* ms) {
  if (bytes < 8 || reps < 1 || !ms) return QIMAX_EINVAL;
  const uint64_t n = bytes / 8;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n * 8) != hipSuccess || hipMalloc(&b, n * 8) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return QIMAX_ENOMEM;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)launch_copy_u64((const uint64_t*)a, (uint64_t*)b, n, nullptr);  // warm-up
  (void)hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps; ++r) (void)launch_copy_u64((const uint64_t*)a, (uint64_t*)b, n, nullptr);
  (void)hipEventRecord(e1, nullptr);
  hipError_t e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  *ms = (double)t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  return e == hipSuccess ? QIMAX_OK : QIMAX_EDEVICE;
}

qimax_status qimax_sync(qimax_ctx* c) {
  if (!c) return QIMAX_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return QIMAX_OK;
}

const char* qimax_last_error(const qimax_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->last_error.c_str();
}

void qimax_destroy(qimax_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->keys, &c->w, &c->seg, &c->pk[0], &c->pk[1], &c->pw[0], &c->pw[1], &c->pseg[0],
                    &c->pseg[1], &c->ik[0], &c->ik[1], &c->iw[0], &c->iw[1], &c->cnt, &c->off, &c->scan_tmp,
                    &c->hist, &c->hist_off, &c->blk_begin, &c->blk_end, &c->blk_seg, &c->seg_blk, &c->blk_cnt,
                    &c->blk_off, &c->img_seg, &c->desc, &c->desc2, &c->err, &c->f64tmp, &c->gr_in, &c->gr_out, &c->ghist, &c->sbase, &c->sstatus, &c->tile_ctr, &c->mstatus, &c->dtile[0], &c->dtile[1], &c->dtile[2], &c->ptab, &c->akeys, &c->asign, &c->img_cnt, &c->dense_acc, &c->chunk_cnt, &c->chunk_start, &c->grp_cnt,
                    &c->chunk_off};
  for (DevBuf* b : bufs) dev_free(c, *b);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (int i = 0; i < 2; ++i)
    if (c->stage[i]) (void)hipHostFree(c->stage[i]);
  if (c->zres) (void)hipHostFree(c->zres);
  prof_destroy(&c->prof);
  for (hipEvent_t e : c->tune_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"

// ================================================================== batch engine (C ABI)

namespace {

// One circuit of a batch: its operators (stable storage), its planned passes with the merge
// threshold of each, and where it is in its life (queued -> active -> draining -> done).
struct BatchCirc {
  uint64_t id = 0;
  uint32_t n = 0;
  std::deque<HostOp> ops;
  std::vector<Pass> passes;
  std::vector<double> thr;
  size_t next = 0;
  int state = 0;  // 0 queued, 1 active, 2 draining (result taken; terms leave next round), 3 done
  uint64_t updates = 0;
  std::vector<uint64_t> res_off, res_key;
  std::vector<double> res_w;
};

}  // namespace

struct qimax_batch {
  qimax_ctx* c = nullptr;
  uint32_t max_n = 32;
  uint64_t next_id = 1;
  std::map<uint64_t, BatchCirc> circs;
  std::vector<uint64_t> order;  // circuits whose generators are in the term array, in order
  std::vector<uint64_t> queue;  // submitted, not yet admitted into the array
  std::vector<uint64_t> done;   // finished and not yet reported by poll
  std::vector<uint64_t> so{0};  // host segment offsets of the term array
  uint64_t rounds = 0;
};

namespace {

qimax_status bfail(qimax_batch* b, qimax_status s, const std::string& msg) {
  b->c->last_error = msg;
  return s;
}

// Plan every layer of a circuit into passes (the eps prune closes each layer).
qimax_status plan_circuit(qimax_batch* b, const qimax_circuit* q, double eps, BatchCirc& bc) {
  qimax_ctx* c = b->c;
  std::vector<std::pair<size_t, size_t>> layers;
  if (q->layer_end && q->n_layers) {
    size_t a = 0;
    for (size_t l = 0; l < q->n_layers; ++l) {
      const size_t e = (size_t)q->layer_end[l];
      if (e < a || e > q->m) return bfail(b, QIMAX_EINVAL, "layer_end must be non-decreasing and <= m");
      layers.push_back({a, e});
      a = e;
    }
    if (a != q->m) return bfail(b, QIMAX_EINVAL, "the last layer_end must equal m");
  } else {
    layers.push_back({0, q->m});
  }
  std::vector<const HostOp*> pending;
  for (size_t l = 0; l < layers.size(); ++l) {
    const size_t a = layers[l].first, e = layers[l].second;
    std::vector<HostOp> ops;
    QCHK(group_circuit(c, bc.n, q->gate + a, q->q0 + a, q->q1 + a, q->theta ? q->theta + a : nullptr, e - a, ops,
                       nullptr, nullptr));
    std::vector<const HostOp*> all = pending;
    for (auto& op : ops) {
      op.group += (int64_t)l << 32;  // layers in order (a layer has fewer than 2^32 groups)
      bc.ops.push_back(std::move(op));
      all.push_back(&bc.ops.back());
    }
    std::vector<Pass> passes;
    plan_passes(all, passes, pending);
    for (size_t i = 0; i < passes.size(); ++i) {
      bc.passes.push_back(passes[i]);
      bc.thr.push_back(i + 1 == passes.size() ? eps : 0.0);
    }
  }
  if (!pending.empty()) {  // trailing Clifford operators: one permutation-only pass
    Pass p;
    p.A = pending;
    count_clifford_groups(p, {});
    bc.passes.push_back(p);
    bc.thr.push_back(0.0);
  }
  return QIMAX_OK;
}

void initial_result(BatchCirc& bc) {
  bc.res_off.resize(bc.n + 1);
  bc.res_w.assign(bc.n, 1.0);
  for (uint32_t j = 0; j <= bc.n; ++j) bc.res_off[j] = j;
  std::vector<u128> k(bc.n);
  for (uint32_t j = 0; j < bc.n; ++j) k[j] = (u128)3 << (2 * (bc.n - 1 - j));
  bc.res_key.resize((size_t)bc.n * (bc.n <= 32 ? 1 : 2));
  keys_to_words(k, bc.n, bc.res_key.data());
}

// Admit the queued circuits: their Z_j terms go to the end of the term array.
qimax_status admit(qimax_batch* b) {
  if (b->queue.empty()) return QIMAX_OK;
  qimax_ctx* c = b->c;
  const uint64_t T = b->so.back();
  uint64_t add = 0;
  std::vector<uint32_t> nq;
  std::vector<uint64_t> dst;
  for (uint64_t id : b->queue) {
    BatchCirc& bc = b->circs[id];
    nq.push_back(bc.n);
    dst.push_back(T + add);
    add += bc.n;
  }
  QCHK(ensure_keep(c, c->keys, (T + add) * c->kb, T * c->kb));
  QCHK(ensure_keep(c, c->w, (T + add) * c->wb, T * c->wb));
  QCHK(ensure(c, c->gr_in, nq.size() * 4));  // the grouping buffers, free between calls
  QCHK(ensure(c, c->gr_out, dst.size() * 8));
  HIPCHK(c, hipMemcpyAsync(c->gr_in.p, nq.data(), nq.size() * 4, hipMemcpyHostToDevice, c->stream), "admit");
  HIPCHK(c, hipMemcpyAsync(c->gr_out.p, dst.data(), dst.size() * 8, hipMemcpyHostToDevice, c->stream), "admit");
  HIPCHK(c, launch_init_many(c->KC, c->WP, c->keys.p, c->w.p, (const uint32_t*)c->gr_in.p,
                             (const uint64_t*)c->gr_out.p, (uint32_t)nq.size(), c->stream), "init");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (uint64_t id : b->queue) {
    BatchCirc& bc = b->circs[id];
    bc.state = 1;
    b->order.push_back(id);
    for (uint32_t j = 0; j < bc.n; ++j) b->so.push_back(b->so.back() + 1);
  }
  b->queue.clear();
  return QIMAX_OK;
}

// Copy a finished circuit's generators (segments [s0, s0+n) of the committed array) to the host.
qimax_status take_result(qimax_batch* b, BatchCirc& bc, size_t s0) {
  qimax_ctx* c = b->c;
  // a round returns once its offsets are in, while its compaction may still write the
  // terms: wait for the stream before copying them (the copies below are not ordered after
  // the library's non-blocking stream)
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  const uint64_t a = b->so[s0], e = b->so[s0 + bc.n];
  bc.res_off.resize(bc.n + 1);
  for (uint32_t j = 0; j <= bc.n; ++j) bc.res_off[j] = b->so[s0 + j] - a;
  bc.res_w.resize(e - a);
  const uint32_t n_words = bc.n <= 32 ? 1u : 2u;
  bc.res_key.resize((e - a) * n_words);
  bool done = false;
  QCHK(export_terms(c, a, e - a, n_words, bc.res_key.data(), bc.res_w.data(), &done));
  if (done) return QIMAX_OK;
  std::vector<u128> k;
  HIPCHK(c, keys_to_host(c, (const uint8_t*)c->keys.p + a * c->kb, e - a, k), "result");
  keys_to_words(k, bc.n, bc.res_key.data());
  if (e == a) return QIMAX_OK;
  if (c->WP == 64) {
    HIPCHK(c, hipMemcpy(bc.res_w.data(), (double*)c->w.p + a, (e - a) * 8, hipMemcpyDeviceToHost), "result");
  } else {
    std::vector<float> w32(e - a);
    HIPCHK(c, hipMemcpy(w32.data(), (float*)c->w.p + a, (e - a) * 4, hipMemcpyDeviceToHost), "result");
    for (size_t i = 0; i < w32.size(); ++i) bc.res_w[i] = w32[i];
  }
  return QIMAX_OK;
}

size_t active_count(const qimax_batch* b) {
  size_t k = 0;
  for (uint64_t id : b->order)
    if (b->circs.at(id).state == 1) ++k;
  return k + b->queue.size();
}

}  // namespace

extern "C" {

qimax_status qimax_batch_create(const qimax_opts* opts, uint32_t max_n, qimax_batch** out) {
  if (!out) return QIMAX_EINVAL;
  *out = nullptr;
  if (max_n > 64) return QIMAX_ETOOLARGE;
  qimax_ctx* c = nullptr;
  // the batch's context: its key class fits max_n, buffers, stream
  const uint32_t cls = max_n <= 16 ? 16 : (max_n <= 32 ? 32 : 64);
  qimax_status s = qimax_create(cls, opts, &c);
  if (s != QIMAX_OK) return s;
  qimax_batch* b = new (std::nothrow) qimax_batch;
  if (!b) {
    qimax_destroy(c);
    return QIMAX_ENOMEM;
  }
  b->c = c;
  b->max_n = cls;
  c->T = 0;
  c->h_seg.assign(1, 0);
  *out = b;
  return QIMAX_OK;
}

qimax_status qimax_batch_submit(qimax_batch* b, const qimax_circuit* q, uint64_t* id) {
  if (!b || !q || !id) return QIMAX_EINVAL;
  qimax_ctx* c = b->c;
  if (c->broken) return bfail(b, QIMAX_ESTATE, "batch unusable after an earlier device error");
  if (q->n < 1 || q->n > b->max_n)
    return bfail(b, q->n < 1 ? QIMAX_EINVAL : QIMAX_ETOOLARGE, "circuit n must be 1..max_n of the batch");
  if (q->m && (!q->gate || !q->q0 || !q->q1)) return bfail(b, QIMAX_EINVAL, "instruction arrays are NULL");
  if (!(q->prune_eps >= 0.0) || !std::isfinite(q->prune_eps)) return bfail(b, QIMAX_EINVAL, "prune_eps must be >= 0");
  BatchCirc bc;
  bc.id = b->next_id;
  bc.n = q->n;
  QCHK(plan_circuit(b, q, q->prune_eps, bc));
  const uint64_t cid = b->next_id++;
  if (bc.passes.empty()) {  // nothing to propagate: the result is Z_0 .. Z_{n-1}
    initial_result(bc);
    bc.state = 3;
    b->done.push_back(cid);
  } else {
    b->queue.push_back(cid);
  }
  b->circs.emplace(cid, std::move(bc));
  *id = cid;
  return QIMAX_OK;
}

qimax_status qimax_batch_step(qimax_batch* b, size_t* n_active) {
  if (!b) return QIMAX_EINVAL;
  qimax_ctx* c = b->c;
  BusyTimer bt(c);
  if (c->broken) return bfail(b, QIMAX_ESTATE, "batch unusable after an earlier device error");
  QCHK(admit(b));
  // one entry per circuit in the array: its next pass, or a drop of a finished circuit
  std::vector<RoundEntry> entries;
  std::vector<uint32_t> seg_entry;
  bool any = false;
  for (uint64_t id : b->order) {
    BatchCirc& bc = b->circs.at(id);
    RoundEntry en;
    en.n = bc.n;
    if (bc.state == 1) {
      en.pass = &bc.passes[bc.next];
      en.thr = bc.thr[bc.next];
      any = true;
    } else {
      en.drop = true;
    }
    for (uint32_t j = 0; j < bc.n; ++j) seg_entry.push_back((uint32_t)entries.size());
    entries.push_back(en);
  }
  if (!any) {  // only finished circuits left in the array: empty it
    for (uint64_t id : b->order) {
      BatchCirc& bc = b->circs.at(id);
      if (bc.state == 4) b->circs.erase(id);
      else bc.state = 3;
    }
    b->order.clear();
    b->so.assign(1, 0);
    c->T = 0;
    if (n_active) *n_active = active_count(b);
    return QIMAX_OK;
  }
  QCHK(ensure(c, c->seg, b->so.size() * 8));
  HIPCHK(c, hipMemcpyAsync(c->seg.p, b->so.data(), b->so.size() * 8, hipMemcpyHostToDevice, c->stream), "offsets");
  std::vector<uint64_t> so_out, so_img, upd;
  QCHK(run_round(c, entries, seg_entry, c->keys.p, c->w.p, (const uint64_t*)c->seg.p, b->so, 0, so_out, so_img,
                 &upd));
  std::swap(c->keys, c->pk[0]);
  std::swap(c->w, c->pw[0]);
  std::swap(c->seg, c->pseg[0]);
  b->so = so_out;
  c->T = so_out.back();
  b->rounds += 1;
  // finished circuits hand over their result; dropped ones leave the segment list
  std::vector<uint64_t> keep_order, erase;
  std::vector<uint64_t> keep_so{0};
  size_t s0 = 0;
  for (size_t e = 0; e < b->order.size(); ++e) {
    BatchCirc& bc = b->circs.at(b->order[e]);
    bc.updates += upd[e];
    bool leaves = false;
    if (bc.state == 1) {
      if (!bc.passes[bc.next].E.empty()) c->st.passes += 1;
      bc.next += 1;
      if (bc.next == bc.passes.size()) {
        QCHK(take_result(b, bc, s0));
        bc.state = 2;
        b->done.push_back(bc.id);
      }
    } else {  // dropped this round: no terms left in the array
      leaves = true;
      if (bc.state == 4) erase.push_back(bc.id);
      else bc.state = 3;
    }
    if (!leaves) {
      keep_order.push_back(bc.id);
      for (uint32_t j = 0; j < bc.n; ++j) keep_so.push_back(keep_so.back() + (b->so[s0 + j + 1] - b->so[s0 + j]));
    }
    s0 += bc.n;
  }
  for (uint64_t id : erase) b->circs.erase(id);
  bool still_active = false;
  for (uint64_t id : keep_order) still_active |= b->circs.at(id).state == 1;
  if (!still_active) {  // every remaining circuit has handed over its result: empty the array
    for (uint64_t id : keep_order) b->circs.at(id).state = 3;
    keep_order.clear();
    keep_so.assign(1, 0);
    c->T = 0;
  }
  // the dropped circuits hold no terms any more, so the kept segments stay contiguous
  b->order.swap(keep_order);
  b->so.swap(keep_so);
  if (n_active) *n_active = active_count(b);
  return QIMAX_OK;
}

qimax_status qimax_batch_run(qimax_batch* b) {
  if (!b) return QIMAX_EINVAL;
  size_t act = 1;
  while (act) QCHK(qimax_batch_step(b, &act));
  return QIMAX_OK;
}

qimax_status qimax_batch_poll(qimax_batch* b, uint64_t* ids, size_t cap, size_t* n) {
  if (!b || !n) return QIMAX_EINVAL;
  *n = b->done.size();
  if (!ids || cap < b->done.size()) return QIMAX_OK;
  std::copy(b->done.begin(), b->done.end(), ids);
  b->done.clear();
  return QIMAX_OK;
}

qimax_status qimax_batch_fetch(qimax_batch* b, uint64_t id, uint64_t* gen_off, uint64_t* keys, double* w, size_t cap,
                               size_t* T) {
  if (!b || !T) return QIMAX_EINVAL;
  auto it = b->circs.find(id);
  if (it == b->circs.end()) return bfail(b, QIMAX_EINVAL, "unknown circuit id");
  BatchCirc& bc = it->second;
  if (bc.state < 2) return bfail(b, QIMAX_ESTATE, "circuit not finished");
  *T = bc.res_w.size();
  if (cap < bc.res_w.size()) return QIMAX_OK;
  if (!gen_off || (*T && (!keys || !w))) return bfail(b, QIMAX_EINVAL, "output buffers are NULL");
  std::copy(bc.res_off.begin(), bc.res_off.end(), gen_off);
  std::copy(bc.res_key.begin(), bc.res_key.end(), keys);
  std::copy(bc.res_w.begin(), bc.res_w.end(), w);
  if (bc.state == 3) {
    b->circs.erase(it);
  } else {
    bc.res_off.clear(); bc.res_key.clear(); bc.res_w.clear();
    bc.state = 4;  // taken; its terms leave the array next round, then the record goes
  }
  return QIMAX_OK;
}

qimax_status qimax_batch_info(const qimax_batch* b, qimax_batch_info_t* out) {
  if (!b || !out) return QIMAX_EINVAL;
  out->queued = b->queue.size();
  out->active = 0;
  for (uint64_t id : b->order)
    if (b->circs.at(id).state == 1) ++out->active;
  out->finished = b->done.size();
  out->rounds = b->rounds;
  out->terms = b->so.back();
  out->term_updates = b->c->st.term_updates;
  out->alloc_bytes = b->c->alloc_bytes;
  out->peak_bytes = b->c->peak_bytes;
  return QIMAX_OK;
}

qimax_status qimax_batch_circuit_updates(const qimax_batch* b, uint64_t id, uint64_t* updates) {
  if (!b || !updates) return QIMAX_EINVAL;
  auto it = b->circs.find(id);
  if (it == b->circs.end()) return QIMAX_EINVAL;
  *updates = it->second.updates;
  return QIMAX_OK;
}

qimax_ctx* qimax_batch_context(qimax_batch* b) { return b ? b->c : nullptr; }

const char* qimax_batch_last_error(const qimax_batch* b) { return b ? b->c->last_error.c_str() : ""; }

void qimax_batch_destroy(qimax_batch* b) {
  if (!b) return;
  qimax_destroy(b->c);
  delete b;
}

}  // extern "C"
