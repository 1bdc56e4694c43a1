// HIP kernels for gfx950 (wave64): generator init, fan-out count, scans, term expansion,
// segmented LSD radix sort, segmented reduce + prune + compaction, grouping (PTM
// composition). Every global write is bounds-checked against the size its launcher was
// given; a violation raises an error bit instead of writing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qimax_internal.h"

namespace qimax {
namespace {

static_assert(kSortBlock == kRadix, "one thread per radix digit in the scatter kernel");

// ------------------------------------------------------------------------------ keys
// A key is the paper's base-4 Pauli index; qubit q's digit is at bit pos = 2(n-1-q).
template <typename K>
__device__ __forceinline__ uint32_t get_d(K k, uint32_t pos) {
  return (uint32_t)(k >> pos) & 3u;
}
template <typename K>
__device__ __forceinline__ K set_d(K k, uint32_t pos, uint32_t d) {
  return (k & ~((K)3 << pos)) | ((K)d << pos);
}

template <typename K>
__device__ __forceinline__ K apply_perm(K key, const PermDesc& p, uint32_t& neg) {
  uint32_t in = get_d(key, p.pa);
  if (p.arity == 2) in = (in << 2) | get_d(key, p.pb);
  const uint64_t word = (in < 8) ? p.lo : p.hi;
  const uint32_t e = (uint32_t)(word >> ((in & 7u) * 8u)) & 0xFFu;
  neg ^= (e >> 4) & 1u;
  const uint32_t o = e & 15u;
  if (p.arity == 2) {
    key = set_d(key, p.pa, o >> 2);
    key = set_d(key, p.pb, o & 3u);
  } else {
    key = set_d(key, p.pa, o);
  }
  return key;
}

// Mask of the low bit of every 2-bit digit.
template <typename K>
__device__ __forceinline__ K even_bits() {
  if constexpr (sizeof(K) > 8) return ((K)0x5555555555555555ull << 64) | (K)0x5555555555555555ull;
  else return (K)0x5555555555555555ull;
}

template <typename K>
__device__ __forceinline__ int popc_k(K x) {
  if constexpr (sizeof(K) > 8) return __popcll((uint64_t)x) + __popcll((uint64_t)(x >> 64));
  else if constexpr (sizeof(K) == 8) return __popcll(x);
  else return __popc(x);
}

// Number of Y digits of a key (hi bit set, lo bit clear).
template <typename K>
__device__ __forceinline__ uint32_t y_count(K key) {
  return (uint32_t)popc_k((key >> 1) & ~key & even_bits<K>());
}

// Image of a key under a compiled Clifford chain (tables staged in LDS by the caller): the
// product of the images of its bytes. Entry b of byte k holds the image key and, in tn, its
// sign (bit 0) and its number of Y digits mod 4 (bits 1-2). With x = lo ^ hi and z = hi the
// planes of a digit key and P = i^(x.z) X^x Z^z, an ordered product of images P_j is
// i^e P(xor of the keys) with e = sum_j y_j + 2 sum_{i<j} z_i.x_j - y(product) (mod 4); the
// images commute, so e is 0 or 2. The cross term only matters mod 2: the z plane of the
// product so far ANDed with each image's x plane, accumulated by XOR, counted once.
template <typename K>
__device__ __forceinline__ K apply_table(K key, const K* __restrict__ tk, const uint8_t* __restrict__ tn,
                                         uint32_t& neg) {
  K acc = 0, cross = 0;
  uint32_t e = 0;
#pragma unroll
  for (int k = 0; k < (int)sizeof(K); ++k) {
    const uint32_t b = (uint32_t)(key >> (8 * k)) & 0xFFu;
    if (b == 0) continue;  // four identities map to identity
    const K img = tk[k * 256 + b];
    const uint32_t t = tn[k * 256 + b];
    neg ^= t & 1u;
    e += t >> 1;
    cross ^= (acc >> 1) & (img ^ (img >> 1));
    acc ^= img;
  }
  e += 2u * ((uint32_t)popc_k(cross & even_bits<K>()) & 1u) - y_count(acc);
  neg ^= (e >> 1) & 1u;
  return acc;
}

// Stage a chain table into LDS (all threads of the block take part).
template <typename K>
__device__ __forceinline__ void stage_table(const ChainTable& t, K* sk, uint8_t* sn) {
  const K* gk = (const K*)t.tab_key;
  for (int i = threadIdx.x; i < (int)sizeof(K) * 256; i += blockDim.x) {
    sk[i] = gk[i];
    sn[i] = t.tab_neg[i];
  }
}

// The XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ uint32_t xcd_id() {
  uint32_t x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & (kXcds - 1);
}

// Block index -> tile for launches of independent tiles: blocks are dealt to the XCDs in turn,
// so block i of XCD x takes tile x * q + min(x, r) + i (q, r: n / kXcds, n % kXcds) and
// neighbouring tiles run on one XCD at about the same time; the partial cache lines where
// their outputs meet then merge in that XCD's L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t x = b & (kXcds - 1), i = b / kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + min(x, r) + i;
}

// First tile b >= target with b a segment's first tile (seg_blk[0..S] is non-decreasing and
// ends with the tile count).
__device__ __forceinline__ uint32_t seg_boundary_at_or_after(const uint32_t* seg_blk, uint32_t S, uint32_t target) {
  uint32_t lo = 0, hi = S;  // seg_blk[hi] >= target
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (seg_blk[mid] >= target) hi = mid; else lo = mid + 1;
  }
  return seg_blk[lo];
}

template <typename K>
__device__ __forceinline__ uint32_t local2(K key, uint32_t pa, uint32_t pb) {
  return (get_d(key, pa) << 2) | get_d(key, pb);
}

template <int WP> struct WTraits;
template <> struct WTraits<64> { using W = double; };
template <> struct WTraits<32> { using W = float; };

// ------------------------------------------------------------------------ block scans
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive scan over a block of NT threads (NT a multiple of 64). sh: NT/64 words.
// OR of v over the block (every thread gets it); sh holds NT/64 values.
template <int NT, typename K>
__device__ __forceinline__ K block_or(K v, K* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    if constexpr (sizeof(K) <= 8) {
      v |= (K)__shfl_xor((unsigned long long)v, o, 64);
    } else {
      const uint64_t lo = __shfl_xor((unsigned long long)(uint64_t)v, o, 64);
      const uint64_t hi = __shfl_xor((unsigned long long)(uint64_t)(v >> 64), o, 64);
      v |= ((K)hi << 64) | (K)lo;
    }
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  K r = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r |= sh[w];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* sh, uint64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t incl = wave_incl_scan(v);
  if (lane == 63) sh[wid] = incl;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint64_t x = sh[w];
    if (w < wid) pre += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return pre + incl - v;
}

// ------------------------------------------------------------------------------ init
template <typename K, typename W>
__global__ void k_init(K* keys, W* w, uint64_t* seg_off, uint32_t n) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    keys[j] = (K)3 << (2u * (n - 1u - j));  // Z on qubit j
    w[j] = (W)1;
    seg_off[j] = j;
  }
  if (j == 0) seg_off[n] = n;
}

// ------------------------------------------------------------------------------ scans
template <typename TI>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const TI* __restrict__ in, uint64_t N,
                                                            uint64_t* __restrict__ part) {
  __shared__ uint64_t sh[kScanBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kScanBlock + threadIdx.x;
    if (i < N) s += (uint64_t)in[i];
  }
  uint64_t tot;
  block_excl_scan<kScanBlock>(s, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of part[0..nb) in place by one block; part[nb] = total.
__global__ void __launch_bounds__(kScanBlock) k_scan_partials(uint64_t* part, uint64_t nb) {
  __shared__ uint64_t sh[kScanBlock / 64];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < nb; base += kScanTile) {
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t i = base + (uint64_t)threadIdx.x * kScanItems + k;
      v[k] = (i < nb) ? part[i] : 0;
      s += v[k];
    }
    uint64_t tot;
    uint64_t pre = block_excl_scan<kScanBlock>(s, sh, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const uint64_t i = base + (uint64_t)threadIdx.x * kScanItems + k;
      if (i < nb) part[i] = pre;
      pre += v[k];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

template <typename TI>
__global__ void __launch_bounds__(kScanBlock) k_scan_down(const TI* __restrict__ in, uint64_t N,
                                                          const uint64_t* __restrict__ part,
                                                          uint64_t* __restrict__ out) {
  __shared__ uint64_t sh[kScanBlock / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    v[k] = (i < N) ? (uint64_t)in[i] : 0;
    s += v[k];
  }
  uint64_t tot;
  uint64_t pre = block_excl_scan<kScanBlock>(s, sh, &tot) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + k;
    if (i < N) out[i] = pre;
    pre += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[N] = part[gridDim.x];
}

__global__ void k_zero_one(uint64_t* out) { out[0] = 0; }

__global__ void k_gather_u64(const uint64_t* __restrict__ src, const uint64_t* __restrict__ idx,
                             uint64_t* __restrict__ dst, uint32_t S1) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S1) dst[s] = src[idx[s]];
}

__global__ void k_gather_u64_by_u32(const uint64_t* __restrict__ src, const uint32_t* __restrict__ idx,
                                    uint64_t* __restrict__ dst, uint32_t S1) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S1) dst[s] = src[idx[s]];
}

// ----------------------------------------------------------------------------- expand
// Block b produces images [b*kExpandTile, min((b+1)*kExpandTile, T_img)). The parents
// covering that range are found by binary search on the image offsets `off`
// (off[p] = first image of parent p, off[T_in] = T_img); image g of parent p is the
// (g - off[p])-th entry of the Cartesian product over the pass's expanding operators
// (mixed-radix over their per-term nonzero counts), i.e. one term of the flatten.
__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* a, uint64_t lo, uint64_t hi,
                                                    uint64_t x) {
  // first index i in [lo, hi) with a[i] > x (hi if none)
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// upper_bound by one wave: first index i in [lo, hi) with a[i] > x (hi if none), a sorted
// non-decreasing. Each round probes 64 evenly spaced elements at once and keeps the interval
// between the last probe <= x and the first probe > x, so n elements take ceil(log64 n)
// rounds of one parallel load instead of log2 n dependent loads.
template <typename Pred>
__device__ __forceinline__ uint64_t wave_first_true(uint64_t lo, uint64_t hi, const Pred& pred) {
  // first i in [lo, hi) with pred(i) (hi if none), pred monotone (false..false true..true)
  const int lane = threadIdx.x & 63;
  while (true) {
    const uint64_t n = hi - lo;
    if (n == 0) return lo;
    const uint64_t step = n <= 64 ? 1 : (n + 63) / 64;
    const uint64_t i = lo + (uint64_t)lane * step;
    const bool gt = i < hi ? pred(i) : true;
    const uint64_t m = __ballot(gt);
    const int first = m ? __ffsll((long long)m) - 1 : 64;
    if (step == 1) return first == 64 ? hi : lo + (uint64_t)first;
    if (first == 0) return lo;
    const uint64_t nlo = lo + (uint64_t)(first - 1) * step + 1;
    const uint64_t nhi = first == 64 ? hi : min(lo + (uint64_t)first * step, hi);
    lo = nlo;
    hi = nhi;
  }
}

__device__ __forceinline__ uint64_t wave_upper_bound(const uint64_t* __restrict__ a, uint64_t lo, uint64_t hi,
                                                     uint64_t x) {
  return wave_first_true(lo, hi, [&](uint64_t i) { return a[i] > x; });
}

// q = r / c and rem = r - q c for an image count 1 <= c <= 16, with m = ceil(2^32 / c): the
// high word of r m exceeds r / c by r (m - 2^32 / c) / 2^32 < 1, so it is the quotient or one
// more, which one correction step settles (integer division has no instruction on the chip).
__device__ __forceinline__ uint32_t div_count(uint32_t r, uint32_t c, uint32_t m, uint32_t& rem) {
  if (c == 1) {
    rem = 0;
    return r;
  }
  uint32_t q = __umulhi(r, m);
  int32_t k = (int32_t)(r - q * c);
  if (k < 0) {
    --q;
    k += (int32_t)c;
  }
  rem = (uint32_t)k;
  return q;
}

// Image number r (mixed radix over the operators' column counts, first operator fastest) of
// a term under the expanding operators: key and weight updated in place.
template <typename K, int WP>
__device__ __forceinline__ void expand_ops(K& key, typename WTraits<WP>::W& wv, uint32_t r, const PassArgs& pa,
                                           const Exp1Desc* E1s, const Exp2Desc* E2s, uint32_t* err) {
  for (uint32_t e = 0; e < pa.nE1; ++e) {
    const Exp1Desc& E = E1s[e];
    const uint32_t d = get_d(key, E.pos);
    const uint32_t c = E.cnt[d];
    if (c == 0) { atomicOr(err, kErrIndex | kErrExpand); break; }
    uint32_t k;
    r = div_count(r, c, E.rcp[d], k);
    key = set_d(key, E.pos, E.out[d][k]);
    if constexpr (WP == 64) wv *= E.val[d][k]; else wv *= E.valf[d][k];
  }
  for (uint32_t e = 0; e < pa.nE2; ++e) {
    const Exp2Desc& E = E2s[e];
    const uint32_t in = local2(key, E.pa, E.pb);
    const uint32_t c = E.cnt[in];
    if (c == 0) { atomicOr(err, kErrIndex | kErrExpand); break; }
    uint32_t k;
    r = div_count(r, c, E.rcp[in], k);
    const uint32_t o = E.out[in][k];
    key = set_d(key, E.pa, o >> 2);
    key = set_d(key, E.pb, o & 3u);
    if constexpr (WP == 64) wv *= E.val[in][k]; else wv *= E.valf[in][k];
  }
}

// A term's image under the A chain (table or op list) and its fan-out f = prod of the
// expanding operators' column counts (0 for a dropped entry; errors as in the count).
template <typename K>
__device__ __forceinline__ uint64_t a_chain_and_fanout(K& key, uint32_t& neg, const PassArgs& pa, const K* tk,
                                                        const uint8_t* tn, uint32_t* err,
                                                        const Exp1Desc* E1s = nullptr) {
  if (pa.drop) return 0;
  if (pa.useA) key = apply_table(key, tk, tn, neg);
  else for (uint32_t a = 0; a < pa.nA; ++a) key = apply_perm(key, pa.A[a], neg);
  if (!E1s) E1s = pa.E1;
  uint64_t f = 1;
  for (uint32_t e = 0; e < pa.nE1 && f <= 0xFFFFFFFFull; ++e) f *= E1s[e].cnt[get_d(key, E1s[e].pos)];
  for (uint32_t e = 0; e < pa.nE2 && f <= 0xFFFFFFFFull; ++e) f *= pa.E2[e].cnt[local2(key, pa.E2[e].pa, pa.E2[e].pb)];
  if (f > 0xFFFFFFFFull) {
    atomicOr(err, kErrFanout);
    f = 0;
  }
  return f;
}

template <typename K, int WP>
__global__ void __launch_bounds__(kExpandBlock)
k_expand(const K* __restrict__ keys, const uint8_t* __restrict__ asign, const typename WTraits<WP>::W* __restrict__ w,
         uint64_t T_in, const uint64_t* __restrict__ off, uint64_t T_img, Tiling tl, const PassArgs* __restrict__ pas,
         const uint32_t* __restrict__ seg_entry, const uint64_t* __restrict__ seg_in, K* __restrict__ keys_out,
         typename WTraits<WP>::W* __restrict__ w_out, uint32_t* __restrict__ ghist, uint32_t n_pass, uint32_t hp_begin,
         uint32_t* err, uint64_t narrow_lim) {
  using W = typename WTraits<WP>::W;
  constexpr int kWaves = kExpandBlock / 64;
  constexpr int kWin = kExpandTile + 1;
  constexpr int kTab = (int)sizeof(K) * 256;
  // dynamic LDS: offset window (relative to the tile's first image), image -> parent map,
  // the chain tables that this pass uses, then its expanding operators' descriptors
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t blk = blockIdx.x;
  const uint32_t seg = tl.blk_seg[blk];
  const PassArgs pa = pas[seg_entry[seg]];
  int32_t* win = (int32_t*)lds;
  uint16_t* pmap = (uint16_t*)(lds + kWin * 4);
  uint8_t* cur = lds + kExpandLdsHead;
  K* tbk = (K*)cur;
  cur += pa.useB ? kTab * sizeof(K) : 0;
  uint8_t* tbn = cur;
  cur += pa.useB ? kTab : 0;
  uint64_t* edesc = (uint64_t*)cur;
  __shared__ uint64_t bounds[2];
  // digit counts of the images for the sort passes hp_begin .. n_pass-1 (one copy per wave),
  // added to the segment's histograms ghist[(seg*n_pass + p)*256 + d] at the end
  const uint32_t n_hp = ghist ? n_pass - hp_begin : 0u;
  // this block's images: one segment-aligned tile of at most kExpandTile
  const uint64_t g0 = tl.blk_begin[blk];
  const uint64_t g1 = min(tl.blk_end[blk], T_img);
  if (g0 >= g1) return;
  if (pa.useB) stage_table(pa.tB, tbk, tbn);
  // the expanding operators' descriptors, read many times per image, go to LDS
  const uint32_t e1w = pa.nE1 * (uint32_t)(sizeof(Exp1Desc) / 8), e2w = pa.nE2 * (uint32_t)(sizeof(Exp2Desc) / 8);
  for (uint32_t i = threadIdx.x; i < e1w; i += kExpandBlock) edesc[i] = ((const uint64_t*)pa.E1)[i];
  for (uint32_t i = threadIdx.x; i < e2w; i += kExpandBlock) edesc[e1w + i] = ((const uint64_t*)pa.E2)[i];
  const Exp1Desc* E1s = (const Exp1Desc*)edesc;
  const Exp2Desc* E2s = (const Exp2Desc*)(edesc + e1w);
  uint32_t* hh = (uint32_t*)(edesc + e1w + e2w);
  for (uint32_t i = threadIdx.x; i < n_hp * kWaves * kRadix; i += kExpandBlock) hh[i] = 0u;
  uint32_t* hw = hh + (threadIdx.x >> 6) * n_hp * kRadix;
  // parents of the first and last image: wave 0 and wave 1 search the segment's parents
  // (off is the global image offset of every parent; the segment's are seg_in[seg] ..)
  if (threadIdx.x < 128) {
    const uint64_t lo = seg_in[seg], hi = seg_in[seg + 1] + 1;
    const uint64_t x = threadIdx.x < 64 ? g0 : g1 - 1;
    const uint64_t p = wave_upper_bound(off, lo, hi, x) - 1;
    if ((threadIdx.x & 63) == 0) bounds[threadIdx.x >> 6] = p;
  }
  __syncthreads();
  const uint64_t plo = bounds[0], phi = bounds[1];
  const uint64_t nwin = phi - plo + 2;  // off[plo .. phi+1]
  // (offsets below 2^31 keep every window entry minus g0 within 32 bits; narrow_lim = 2^31,
  // 0 forces the search in global memory, for tests)
  const bool in_lds = nwin <= (uint64_t)kWin && T_img < narrow_lim;
  if (in_lds) {
    for (uint64_t k = threadIdx.x; k < nwin; k += kExpandBlock) win[k] = (int32_t)((int64_t)off[plo + k] - (int64_t)g0);
    __syncthreads();
    // image -> parent map of the tile: window parent j covers images [g0 + win[j], g0 + win[j+1])
    const int32_t n_t = (int32_t)(g1 - g0);
    for (uint32_t j = threadIdx.x; j + 1 < (uint32_t)nwin; j += kExpandBlock) {
      const int32_t a = max(win[j], 0), b = min(win[j + 1], n_t);
      for (int32_t g = a; g < b; ++g) pmap[g] = (uint16_t)j;
    }
  }
  __syncthreads();
  // the items in two halves (fewer registers live at once); in each, parents of every item
  // first, then every parent load in flight, then the arithmetic
  constexpr int kHalf = kExpandItems / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint64_t par[kHalf];
    uint32_t rk[kHalf];
#pragma unroll
    for (int it = 0; it < kHalf; ++it) {
      const uint64_t g = min(g0 + (uint64_t)(h * kHalf + it) * kExpandBlock + threadIdx.x, g1 - 1);
      uint64_t p, start;
      if (in_lds) {
        const uint32_t j = pmap[g - g0];
        p = plo + j;
        start = (uint64_t)((int64_t)g0 + win[j]);
      } else {
        p = upper_bound_u64(off, plo, phi + 2, g) - 1;
        start = off[p];
      }
      par[it] = p;
      rk[it] = (uint32_t)(g - start);
    }
    K kp[kHalf];
    W wp[kHalf];
    uint32_t sp[kHalf];
#pragma unroll
    for (int it = 0; it < kHalf; ++it) {
      const uint64_t p = min(par[it], T_in - 1);  // T_in >= 1: this tile has images
      kp[it] = keys[p];
      wp[it] = w[p];
      sp[it] = asign[p];
    }
#pragma unroll
    for (int it = 0; it < kHalf; ++it) {
      const uint64_t g = g0 + (uint64_t)(h * kHalf + it) * kExpandBlock + threadIdx.x;
      if (g >= g1) break;
      if (par[it] >= T_in) {
        atomicOr(err, kErrIndex | kErrExpand);
        continue;
      }
      K key = kp[it];  // the parent's image under the A chain (and its sign), from the count
      W wv = wp[it];
      uint32_t neg = sp[it];
      expand_ops<K, WP>(key, wv, rk[it], pa, E1s, E2s, err);
      if (pa.useB) key = apply_table(key, tbk, tbn, neg);
      else for (uint32_t b = 0; b < pa.nB; ++b) key = apply_perm(key, pa.B[b], neg);
      if (neg) wv = -wv;
      keys_out[g] = key;
      w_out[g] = wv;
      for (uint32_t p = 0; p < n_hp; ++p) atomicAdd(&hw[p * kRadix + ((uint32_t)(key >> (8u * (hp_begin + p))) & 255u)], 1u);
    }
  }
  if (n_hp) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_hp * kRadix; i += kExpandBlock) {
      uint32_t c = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) c += hh[w * n_hp * kRadix + i];
      const uint32_t p = hp_begin + i / kRadix, d = i % kRadix;
      if (c) atomicAdd(&ghist[((uint64_t)seg * n_pass + p) * kRadix + d], c);
    }
  }
}

// A round of small segments (every segment at most kChunkCap terms and images), one block
// per segment: the A chain and fan-out of each term (as the count), their scan in LDS, and
// the images (as the expansion), written to the segment's own chunk [s*kChunkCap, +n_img)
// of keys_out / w_out. The chunk tiling (tiles = segments) goes to blk_begin, blk_end,
// blk_seg, seg_blk (S + 1 entries) and the image count of segment s to img_cnt[s].
constexpr int kSmallBlock = 256;
template <typename K, int WP>
__global__ void __launch_bounds__(kSmallBlock)
k_expand_small(const K* __restrict__ keys, const typename WTraits<WP>::W* __restrict__ w,
               const uint64_t* __restrict__ seg_in, uint32_t S, const PassArgs* __restrict__ pas,
               const uint32_t* __restrict__ seg_entry, K* __restrict__ keys_out,
               typename WTraits<WP>::W* __restrict__ w_out, uint32_t* __restrict__ img_cnt,
               uint64_t* __restrict__ blk_begin, uint64_t* __restrict__ blk_end, uint32_t* __restrict__ blk_seg,
               uint32_t* __restrict__ seg_blk, uint32_t* err) {
  using W = typename WTraits<WP>::W;
  constexpr int kTabN = sizeof(K) <= 8 ? (int)sizeof(K) * 256 : 1;  // no tables for 16-byte keys
  constexpr uint32_t kPer = kChunkCap / kSmallBlock;                 // scan run per thread
  __shared__ K tk[kTabN];
  __shared__ uint8_t tn[kTabN];
  __shared__ K akey[kChunkCap];
  __shared__ uint32_t off[kChunkCap + 1];
  __shared__ uint8_t negs[kChunkCap];
  __shared__ uint16_t pmap[kChunkCap];
  __shared__ uint64_t scan_sh[kSmallBlock / 64];
  __shared__ uint32_t nimg_sh;
  const uint32_t s = blockIdx.x;
  const PassArgs pa = pas[seg_entry[s]];
  const uint64_t a0 = seg_in[s];
  const uint64_t n64 = seg_in[s + 1] - a0;
  const uint64_t c0 = (uint64_t)s * kChunkCap;
  if (threadIdx.x == 0) {
    blk_begin[s] = c0;
    blk_seg[s] = s;
    seg_blk[s] = s;
    if (s + 1 == S) seg_blk[S] = S;
  }
  if (n64 > (uint64_t)kChunkCap) {  // the caller's bound did not hold
    if (threadIdx.x == 0) {
      atomicOr(err, kErrIndex | kErrFanout);
      blk_end[s] = c0;
      img_cnt[s] = 0;
    }
    return;
  }
  const uint32_t n = (uint32_t)n64;
  if (pa.useA && !pa.drop) {
    stage_table(pa.tA, tk, tn);
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < n; i += kSmallBlock) {
    K key = keys[a0 + i];
    uint32_t neg = 0;
    const uint64_t f = a_chain_and_fanout(key, neg, pa, tk, tn, err);
    akey[i] = key;
    negs[i] = (uint8_t)(neg & 1u);
    off[i] = (uint32_t)min<uint64_t>(f, kChunkCap + 1);  // larger: flagged by the total below
  }
  __syncthreads();
  // exclusive scan of the fan-outs: thread t sums the run [t*kPer, (t+1)*kPer)
  {
    const uint32_t r0 = min(threadIdx.x * kPer, n), r1 = min(r0 + kPer, n);
    uint64_t sum = 0;
    for (uint32_t i = r0; i < r1; ++i) sum += off[i];
    uint64_t tot;
    uint64_t run = block_excl_scan<kSmallBlock>(sum, scan_sh, &tot);
    __syncthreads();  // every run read before any is overwritten
    for (uint32_t i = r0; i < r1; ++i) {
      const uint32_t f = off[i];
      off[i] = (uint32_t)min<uint64_t>(run, kChunkCap);
      run += f;
    }
    if (threadIdx.x == 0) {
      if (tot > (uint64_t)kChunkCap) atomicOr(err, kErrIndex | kErrFanout);
      nimg_sh = tot > (uint64_t)kChunkCap ? 0u : (uint32_t)tot;
      off[n] = nimg_sh;
    }
  }
  __syncthreads();
  const uint32_t n_img = nimg_sh;
  // image -> parent map
  for (uint32_t j = threadIdx.x; j < n; j += kSmallBlock) {
    const uint32_t e = min(off[j + 1], n_img);
    for (uint32_t g = off[j]; g < e; ++g) pmap[g] = (uint16_t)j;
  }
  if (pa.useB) {
    __syncthreads();  // the A table is no longer read
    stage_table(pa.tB, tk, tn);
  }
  __syncthreads();
  for (uint32_t g = threadIdx.x; g < n_img; g += kSmallBlock) {
    const uint32_t j = pmap[g];
    K key = akey[j];
    W wv = w[a0 + j];
    uint32_t neg = negs[j];
    expand_ops<K, WP>(key, wv, g - off[j], pa, pa.E1, pa.E2, err);
    if (pa.useB) key = apply_table(key, tk, tn, neg);
    else for (uint32_t b = 0; b < pa.nB; ++b) key = apply_perm(key, pa.B[b], neg);
    if (neg) wv = -wv;
    keys_out[c0 + g] = key;
    w_out[c0 + g] = wv;
  }
  if (threadIdx.x == 0) {
    blk_end[s] = c0 + n_img;
    img_cnt[s] = n_img;
  }
}

// ----------------------------------------------------------------------- radix sort
// Histogram position of (block b, digit d) in the flat array whose exclusive scan gives
// the scatter bases: segment-major, then digit, then block within the segment. Since
// segments are contiguous in the array being sorted, the scan value is
// seg_begin + (count of smaller digits in the segment) + (count of d in earlier blocks).
__device__ __forceinline__ uint64_t hist_pos(const Tiling& tl, uint32_t b, uint32_t d) {
  const uint32_t s = tl.blk_seg[b];
  const uint32_t f = tl.seg_blk[s];
  const uint32_t nb = tl.seg_blk[s + 1] - f;
  return (uint64_t)kRadix * f + (uint64_t)d * nb + (b - f);
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock) k_sort_hist(const K* __restrict__ keys, uint32_t shift,
                                                          Tiling tl, uint64_t* __restrict__ hist,
                                                          uint64_t hist_size, uint32_t* err) {
  // One counter copy per quarter wave, rows one word longer than the radix: lanes of different
  // quarters that count the same digit hit different LDS banks, so a skewed digit (many lanes
  // on one counter) serializes at most the 16 lanes of a quarter.
  constexpr int kCopies = 4 * (kSortBlock / 64), kRow = kRadix + 1;
  __shared__ uint32_t h[kCopies * kRow];
  // consecutive tiles on one XCD: their counts of a digit are neighbouring words of hist
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  if (tl.n_dev && b >= *tl.n_dev) return;  // launched for a bound on the tile count
  uint32_t* const hq = h + (threadIdx.x >> 4) * kRow;
  for (int k = threadIdx.x; k < kCopies * kRow; k += kSortBlock) h[k] = 0;
  __syncthreads();
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t n = (uint32_t)(end - begin);  // at most kSortTile
  K kr[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {  // every load in flight before the first use
    const uint32_t li = r * kSortBlock + threadIdx.x;
    kr[r] = keys[n ? begin + min(li, n - 1) : 0];
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r)  // no early exit: the loads above stay in flight together
    if (r * kSortBlock + threadIdx.x < n) atomicAdd(&hq[(uint32_t)(kr[r] >> shift) & (kRadix - 1)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kCopies; ++q) c += h[q * kRow + d];
    const uint64_t pos = hist_pos(tl, b, d);
    if (pos < hist_size) hist[pos] = c; else atomicOr(err, kErrIndex | kErrSort);
  }
}

// Status words of the single-sweep radix pass: [epoch:16][flag:2][value:46] per (tile, digit).
constexpr uint64_t kStAgg = 1ull << 46;   // value = this tile's count of the digit
constexpr uint64_t kStPre = 2ull << 46;   // value = inclusive prefix over the segment's tiles so far
constexpr uint64_t kStValMask = (1ull << 46) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

// The flag and the count share one 64-bit word, so relaxed device-scope atomics suffice: a
// reader that sees the flag also sees the count, and no other data is published with it.
__device__ __forceinline__ uint64_t st_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One stable LSD pass over a segment-aligned tile. kSweep = false: the destination of each
// (tile, digit) comes from the scanned per-tile histograms (hist_off). kSweep = true: tiles are
// claimed in order through tile_ctr, each publishes its digit counts and looks back over the
// earlier tiles of its segment for their prefix (decoupled look-back), and the digit's base
// within the segment comes from the upfront histogram (base).
template <typename K, typename W, bool kSweep>
__global__ void __launch_bounds__(kSortBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_sort_scatter(const K* __restrict__ keys_in, const W* __restrict__ w_in, K* __restrict__ keys_out,
               W* __restrict__ w_out, uint64_t T, uint32_t shift, Tiling tl,
               const uint64_t* __restrict__ hist_off, const uint32_t* __restrict__ ghist_p, uint32_t gstride,
               const uint64_t* __restrict__ seg_off, uint64_t* __restrict__ status, uint32_t* __restrict__ tile_ctr,
               uint64_t epoch, uint32_t* err) {
  constexpr int kWaves = kSortBlock / 64;
  constexpr int kRounds = kSortItems;                 // rounds per wave
  constexpr int kWaveSpan = 64 * kRounds;             // tile elements per wave
  constexpr int kWords = sizeof(K) > 8 ? 2 : 1;
  // Four blocks per CU: under 40 KB of LDS and 128 VGPRs per thread. The digit of a sorted
  // slot is read back from the staged key word (one-word keys) and kept in registers for the
  // weights; two-word keys keep it in LDS, since the digit may lie in either word.
  constexpr bool kDigLds = kWords > 1;
  static_assert(kSortBlock == kRadix && kRounds % 4 == 0, "one thread per digit; four digits a word");
  __shared__ uint64_t stage[kSortTile];               // key words, then weights (as raw 64-bit)
  __shared__ uint8_t sdig[kDigLds ? kSortTile : 1];   // digit of each sorted slot (two-word keys)
  __shared__ uint32_t wrun[kWaves][kRadix];            // per-wave running digit counts, then slot bases
  __shared__ uint32_t wdummy[kWaves][64];              // target of the lanes that lead no digit
  __shared__ uint64_t gdst[kRadix];                    // destination of tile slot j of digit d: gdst[d] + j
  __shared__ uint64_t scan_sh[kSortBlock / 64];
  __shared__ uint32_t tile_sh;

  uint32_t b = blockIdx.x;
  if constexpr (kSweep) {
    // launched for a bound on the tile count: the first n_dev blocks claim the n_dev tiles
    if (tl.n_dev && b >= *tl.n_dev) return;
    // Tiles are claimed in order. With per-XCD ranges, a block claims from the range of its
    // own XCD first (whole segments, so every look-back chain and every pair of neighbouring
    // digit runs stays on one XCD and its L2), then from the others; every tile is claimed
    // once whatever the placement of the blocks (there are at least as many blocks as tiles).
    if (threadIdx.x == 0) {
      uint32_t got = 0xFFFFFFFFu;
      if (tl.xrange) {
        const uint32_t x = xcd_id();
        for (int j = 0; j < kXcds; ++j) {
          const uint32_t y = (x + j) & (kXcds - 1);
          const uint32_t a = tl.xrange[y], len = tl.xrange[y + 1] - a;
          if (len == 0) continue;
          const uint32_t k = atomicAdd(tile_ctr + y, 1u);
          if (k < len) { got = a + k; break; }
        }
      } else {
        got = atomicAdd(tile_ctr, 1u);
      }
      tile_sh = got;
    }
    __syncthreads();
    b = tile_sh;
    if (b == 0xFFFFFFFFu) return;  // every tile was claimed already
  } else {
    // independent tiles: consecutive tiles on one XCD, where neighbouring tiles' digit runs meet
    b = xcd_tile(b, gridDim.x);
  }
  if (tl.n_dev && b >= *tl.n_dev) return;  // past the tiles that exist
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t n_tile = (uint32_t)(end - begin);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // sweep: the segment's count of this thread's digit (all tiles) and the segment start
  uint64_t seg_cnt = 0, seg_begin = 0;
  if constexpr (kSweep) {
    const uint32_t s = tl.blk_seg[b];
    seg_cnt = ghist_p[(uint64_t)s * gstride + threadIdx.x];
    seg_begin = seg_off[s];
  }
  for (int k = threadIdx.x; k < kWaves * kRadix; k += kSortBlock) (&wrun[0][0])[k] = 0;
  __syncthreads();

  K key[kRounds];
  // the wave-local rank of each tile element waits in the (not yet used) staging area, so
  // that it holds no registers across the look-back and the scan
  uint16_t* const rk = reinterpret_cast<uint16_t*>(stage);
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  // the tile's elements from a block-uniform base with 32-bit index arithmetic; slots past the
  // tile re-read its last element
  const uint64_t ld_base = n_tile ? begin : 0;
  const uint32_t ld_last = n_tile ? n_tile - 1 : 0;
  const K* __restrict__ kb = keys_in + ld_base;
  // all key loads first, with no branch, so that every load of the thread is in flight at once
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = wid * kWaveSpan + r * 64 + lane;
    key[r] = kb[min(li, ld_last)];
  }
  // Ranking: the lanes of a round that share this lane's digit are those where no bit of the
  // digit differs (a ballot per bit, folded with the bit spread over the word); the lowest of
  // them adds their number to the wave's digit counter (the others add nothing to a dummy
  // word, so no branch) and passes the counter's old value on.
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = wid * kWaveSpan + r * 64 + lane;  // tile-local index, stable order
    const bool valid = li < n_tile;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (kRadix - 1);
    const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
    uint32_t dlo = ~(uint32_t)vm, dhi = ~(uint32_t)(vm >> 32);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const int spread = __builtin_amdgcn_sbfe((int)d, bit, 1);
      const uint64_t bb = __builtin_amdgcn_ballot_w64(spread != 0);
      dlo |= (uint32_t)bb ^ (uint32_t)spread;
      dhi |= (uint32_t)(bb >> 32) ^ (uint32_t)spread;
    }
    const uint64_t mk = ~(((uint64_t)dhi << 32) | dlo);
    const int leader = __ffsll((long long)mk) - 1;  // lowest lane with this digit
    const bool lead_me = valid && lane == leader;
    const uint32_t bs = atomicAdd(lead_me ? &wrun[wid][d] : &wdummy[wid][lane], lead_me ? (uint32_t)__popcll(mk) : 0u);
    const uint32_t v = __shfl(bs, leader < 0 ? 0 : leader, 64) + (uint32_t)__popcll(mk & lt);
    if (valid) rk[li] = (uint16_t)v;
  }
  __syncthreads();
  // per-digit totals of the tile and wave prefixes
  uint32_t tile_cnt = 0;
  const int d = threadIdx.x;  // kSortBlock == kRadix
  uint32_t wpre[kWaves];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    wpre[w] = tile_cnt;
    tile_cnt += wrun[w][d];
  }
  uint64_t gbase = 0;
  if constexpr (kSweep) {
    // publish this tile's count, then collect the prefix of the earlier tiles of the segment
    uint64_t* my = status + (uint64_t)b * kRadix + d;
    const uint32_t s = tl.blk_seg[b];
    const uint32_t first = tl.seg_blk[s];
    const uint64_t ep = epoch << 48;
    st_store(my, ep | (b == first ? kStPre : kStAgg) | tile_cnt);
    uint64_t excl = 0;
    if (b != first) {
      uint32_t t = b - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t v = st_load(status + (uint64_t)t * kRadix + d);
        const bool ready = (v >> 48) == epoch && (v & (kStAgg | kStPre));
        if (!ready) {
          if (++spins > kSpinLimit) { atomicOr(err, kErrSpin); break; }
          continue;
        }
        excl += v & kStValMask;
        if ((v & kStPre) || t == first) break;
        --t;
      }
      st_store(my, ep | kStPre | (excl + tile_cnt));
    }
    gbase = excl;
  }
  // one scan gives the tile-local digit starts (low 16 bits: a tile holds at most 4096 < 2^16
  // elements) and, in a sweep, the segment-wide start of every digit (high bits)
  uint64_t tot;
  const uint64_t ds2 = block_excl_scan<kSortBlock>((seg_cnt << 16) | tile_cnt, scan_sh, &tot);
  const uint32_t ds = (uint32_t)(ds2 & 0xFFFFu);
  if constexpr (kSweep) gbase += seg_begin + (ds2 >> 16);
  else gbase = tile_cnt ? hist_off[hist_pos(tl, b, d)] : 0;
  // slot j of digit d (ds <= j < ds + tile_cnt) goes to gbase + (j - ds); modular arithmetic
  // keeps the difference exact for the digits that occur
  gdst[d] = gbase - ds;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wrun[w][d] = ds + wpre[w];  // slot base of (wave, digit)
  __syncthreads();
  // tile-local sorted position of every element of the thread
  uint32_t pos[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = wid * kWaveSpan + r * 64 + lane;
    const uint32_t dd = (uint32_t)(key[r] >> shift) & (kRadix - 1);
    pos[r] = li < n_tile ? wrun[wid][dd] + rk[li] : 0xFFFFFFFFu;
  }
  __syncthreads();
  // stage keys at those positions (one 64-bit word of the key per round)
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (pos[r] != 0xFFFFFFFFu) {
      const uint32_t dd = (uint32_t)(key[r] >> shift) & (kRadix - 1);
      if (pos[r] < (uint32_t)kSortTile) {
        stage[pos[r]] = (uint64_t)key[r];
        if constexpr (kDigLds) sdig[pos[r]] = (uint8_t)dd;
      } else {
        atomicOr(err, kErrIndex | kErrSort);
      }
    }
  }
  // the weights are needed only once the keys are out: their loads fly during the key
  // stores (loaded this late, they do not share registers with the keys)
  W wv[kRounds];
  const W* __restrict__ wb = w_in + ld_base;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t li = wid * kWaveSpan + r * 64 + lane;
    wv[r] = wb[min(li, ld_last)];
  }
  __syncthreads();
  // write keys out in sorted tile order (coalesced within each digit run); the digits of this
  // thread's slots are kept, four to a register, for the weights
  uint32_t dpk[kRounds / 4];
#pragma unroll
  for (int q = 0; q < kRounds / 4; ++q) dpk[q] = 0;
#pragma unroll
  for (int word = 0; word < kWords; ++word) {
    if (word) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRounds; ++r)
        if (pos[r] < (uint32_t)kSortTile) stage[pos[r]] = (uint64_t)(key[r] >> (64 * word));
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t j = r * kSortBlock + threadIdx.x;
      if (j < n_tile) {
        uint32_t dd;
        if constexpr (kDigLds) dd = sdig[j];
        else dd = (uint32_t)(stage[j] >> shift) & (kRadix - 1);
        if (word == 0) dpk[r >> 2] |= dd << (8 * (r & 3));
        const uint64_t dst = gdst[dd] + j;
        if (dst < T) {
          if constexpr (kWords == 1) keys_out[dst] = (K)stage[j];
          else ((uint64_t*)keys_out)[2 * dst + word] = stage[j];
        } else {
          atomicOr(err, kErrIndex | kErrSort);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (pos[r] < (uint32_t)kSortTile) {
      if constexpr (sizeof(W) == 8) stage[pos[r]] = __double_as_longlong(wv[r]);
      else stage[pos[r]] = (uint64_t)__float_as_uint(wv[r]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t j = r * kSortBlock + threadIdx.x;
    if (j < n_tile) {
      const uint32_t dd = (dpk[r >> 2] >> (8 * (r & 3))) & (kRadix - 1);
      const uint64_t dst = gdst[dd] + j;
      W v;
      if constexpr (sizeof(W) == 8) v = __longlong_as_double((long long)stage[j]);
      else v = __uint_as_float((uint32_t)stage[j]);
      if (dst < T) w_out[dst] = v;
    }
  }
}

// Fan-out count and its exclusive scan in one sweep: tiles of input terms are claimed in
// order; each computes f = prod nnz(PTM column) for its terms (the A chain applied first),
// publishes its total and looks back over the earlier tiles for its global offset, then
// writes off[i] = first image of term i (off[T_in] = image count, from the last tile).
template <typename K>
__global__ void __launch_bounds__(256) k_count_scan(const K* __restrict__ keys, Tiling tl,
                                                    const PassArgs* __restrict__ pas,
                                                    const uint32_t* __restrict__ seg_entry, uint64_t* __restrict__ off,
                                                    uint64_t T_in, uint64_t* __restrict__ status,
                                                    uint32_t* __restrict__ ctr, uint64_t epoch, uint32_t* err,
                                                    K* __restrict__ akeys, uint8_t* __restrict__ asign,
                                                    uint64_t narrow_lim) {
  constexpr int kItems = kSortTile / 256;  // input tiles hold at most kSortTile terms
  constexpr int kTabN = sizeof(K) <= 8 ? (int)sizeof(K) * 256 : 1;  // no tables for 16-byte keys
  __shared__ K tk[kTabN];
  __shared__ uint8_t tn[kTabN];
  __shared__ uint32_t sf[kSortTile + kSortTile / kItems];  // fan-outs (< 2^32); one pad word per run of items
  __shared__ uint64_t scan_sh[4];
  __shared__ uint64_t base_sh;
  __shared__ uint32_t tile_sh;
  if (threadIdx.x == 0) tile_sh = atomicAdd(ctr, 1u);
  __syncthreads();
  const uint32_t b = tile_sh;  // launched with exactly n_blocks blocks
  const PassArgs pa = pas[seg_entry[tl.blk_seg[b]]];
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t n = (uint32_t)(end - begin);
  auto pad = [](uint32_t li) { return li + li / kItems; };
  K kr[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {  // every load in flight before the first use
    const uint32_t li = r * 256 + threadIdx.x;
    kr[r] = keys[n ? begin + min(li, n - 1) : 0];
  }
  if (pa.useA && !pa.drop) {
    stage_table(pa.tA, tk, tn);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint32_t li = r * 256 + threadIdx.x;
    if (li >= n) break;
    K key = kr[r];
    uint32_t neg = 0;
    const uint64_t f = a_chain_and_fanout(key, neg, pa, tk, tn, err);
    sf[pad(li)] = (uint32_t)f;
    // the A chain is applied once per term here; the expand kernel starts from this image
    akeys[begin + li] = key;
    asign[begin + li] = (uint8_t)(neg & 1u);
  }
  __syncthreads();
  // each thread sums a run of kItems consecutive terms; block scan of the run sums
  const uint32_t l0 = threadIdx.x * kItems;
  uint64_t sum = 0;
#pragma unroll
  for (int k2 = 0; k2 < kItems; ++k2)
    if (l0 + k2 < n) sum += sf[pad(l0 + k2)];
  uint64_t tot;
  const uint64_t pre = block_excl_scan<256>(sum, scan_sh, &tot);
  if (threadIdx.x == 0) {
    const uint64_t ep = epoch << 48;
    st_store(status + b, ep | (b == 0 ? kStPre : kStAgg) | tot);
    uint64_t excl = 0;
    if (b > 0) {
      uint32_t t = b - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t v = st_load(status + t);
        const bool ready = (v >> 48) == epoch && (v & (kStAgg | kStPre));
        if (!ready) {
          if (++spins > kSpinLimit) { atomicOr(err, kErrSpin); break; }
          continue;
        }
        excl += v & kStValMask;
        if ((v & kStPre) || t == 0) break;
        --t;
      }
      st_store(status + b, ep | kStPre | (excl + tot));
    }
    base_sh = excl;
    if (b + 1 == tl.n_blocks) off[T_in] = excl + tot;
  }
  __syncthreads();
  const uint64_t base = base_sh;
  if (tot < narrow_lim) {
    // offsets within the tile fit 32 bits (narrow_lim = 2^32; 0 forces the other branch, for
    // tests): they go back through LDS for coalesced stores
    uint32_t run = (uint32_t)pre;
#pragma unroll
    for (int k2 = 0; k2 < kItems; ++k2) {
      if (l0 + k2 < n) {
        const uint32_t v = sf[pad(l0 + k2)];
        sf[pad(l0 + k2)] = run;
        run += v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t li = r * 256 + threadIdx.x;
      if (li < n) off[begin + li] = base + sf[pad(li)];
    }
  } else {
    // (a tile with 2^32 images or more) each thread writes the offsets of its own run
    uint64_t run = base + pre;
#pragma unroll
    for (int k2 = 0; k2 < kItems; ++k2) {
      if (l0 + k2 < n) {
        off[begin + l0 + k2] = run;
        run += sf[pad(l0 + k2)];
      }
    }
  }
}

// Count and expansion in one launch, for rounds whose fan-out bound is at most
// kFuseMaxFanout: tiles of kFuseTile input terms are claimed in order; each applies its terms'
// A chain and counts their fan-outs, scans them in LDS, looks back over the earlier tiles for
// its first image (decoupled look-back, as the count), and then writes every image
// (expansion and B chain) straight to its position, with the digit counts of up to
// kExpandHistPasses global sort passes. img_seg[s] receives the first image of segment s
// (written by the tile that starts it, or for segments without terms by the next tile, or the
// last tile for the trailing ones) and img_seg[S] the image count. The images come out in the
// same order as from the count and expansion launches.
constexpr int kFuseBlock = 512, kFuseItems = 4, kFuseTile = kFuseBlock * kFuseItems;
constexpr int kFuseChunk = 2048;  // images per window of the image -> parent map
template <typename K, int WP>
__global__ void __launch_bounds__(kFuseBlock)
k_count_expand(const K* __restrict__ keys, const typename WTraits<WP>::W* __restrict__ w, Tiling tl,
               const PassArgs* __restrict__ pas, const uint32_t* __restrict__ seg_entry, uint64_t* __restrict__ status,
               uint32_t* __restrict__ ctr, uint64_t epoch, uint64_t* __restrict__ img_seg, K* __restrict__ keys_out,
               typename WTraits<WP>::W* __restrict__ w_out, uint64_t out_cap, uint32_t* __restrict__ ghist,
               uint32_t n_pass, uint32_t hp_begin, uint32_t* err) {
  using W = typename WTraits<WP>::W;
  constexpr int kTabN = sizeof(K) <= 8 ? (int)sizeof(K) * 256 : 1;  // no tables for 16-byte keys
  constexpr int kWaves = kFuseBlock / 64;
  __shared__ K tk[kTabN];
  __shared__ uint8_t tn[kTabN];
  __shared__ K akey[kFuseTile];
  __shared__ uint8_t aneg[kFuseTile];
  __shared__ uint32_t loff[kFuseTile + 1];
  __shared__ uint16_t pmap[kFuseChunk];
  __shared__ uint32_t hh[kExpandHistPasses * kRadix];  // one copy per block (LDS for 3 blocks per CU)
  __shared__ uint64_t scan_sh[kWaves];
  __shared__ uint64_t base_sh;
  __shared__ uint32_t tile_sh;
  // the expanding single-qubit operators' descriptors, read for every image, in LDS (a fan-out
  // bound of 16 leaves at most four operators that expand; more, with columns of one entry,
  // are read from global memory)
  constexpr int kE1Lds = 4, kE1Words = (int)(sizeof(Exp1Desc) / 8);
  __shared__ uint64_t e1sh[kE1Lds * kE1Words];
  if (threadIdx.x == 0) tile_sh = atomicAdd(ctr, 1u);
  __syncthreads();
  const uint32_t b = tile_sh;  // launched with exactly n_blocks blocks
  const uint32_t seg = tl.blk_seg[b];
  const PassArgs pa = pas[seg_entry[seg]];
  const bool e1lds = pa.nE1 <= (uint32_t)kE1Lds;
  if (e1lds)
    for (uint32_t i = threadIdx.x; i < pa.nE1 * (uint32_t)kE1Words; i += kFuseBlock)
      e1sh[i] = ((const uint64_t*)pa.E1)[i];
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t n = (uint32_t)min<uint64_t>(end - begin, (uint64_t)kFuseTile);
  const uint32_t n_hp = ghist ? n_pass - hp_begin : 0u;
  K kr[kFuseItems];
#pragma unroll
  for (int r = 0; r < kFuseItems; ++r) {  // every load in flight before the first use
    const uint32_t li = r * kFuseBlock + threadIdx.x;
    kr[r] = keys[n ? begin + min(li, n - 1) : 0];
  }
  if (pa.useA && !pa.drop) stage_table(pa.tA, tk, tn);
  __syncthreads();  // A table and descriptors staged
#pragma unroll
  for (int r = 0; r < kFuseItems; ++r) {
    const uint32_t li = r * kFuseBlock + threadIdx.x;
    if (li >= n) break;
    K key = kr[r];
    uint32_t neg = 0;
    uint64_t f = e1lds ? a_chain_and_fanout(key, neg, pa, tk, tn, err, (const Exp1Desc*)e1sh)
                       : a_chain_and_fanout(key, neg, pa, tk, tn, err);
    if (f > (uint64_t)kFuseMaxFanout) {  // the caller's bound did not hold
      atomicOr(err, kErrIndex | kErrFanout);
      f = 0;
    }
    akey[li] = key;
    aneg[li] = (uint8_t)(neg & 1u);
    loff[li] = (uint32_t)f;
  }
  for (uint32_t i = threadIdx.x; i < n_hp * kRadix; i += kFuseBlock) hh[i] = 0u;
  __syncthreads();
  // each thread scans a run of kFuseItems consecutive terms
  const uint32_t l0 = threadIdx.x * kFuseItems;
  uint32_t fv[kFuseItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k2 = 0; k2 < kFuseItems; ++k2) {
    fv[k2] = l0 + k2 < n ? loff[l0 + k2] : 0u;
    sum += fv[k2];
  }
  uint64_t tot;
  const uint64_t pre = block_excl_scan<kFuseBlock>(sum, scan_sh, &tot);
  {
    uint32_t run = (uint32_t)pre;
#pragma unroll
    for (int k2 = 0; k2 < kFuseItems; ++k2) {
      if (l0 + k2 < n) loff[l0 + k2] = run;
      run += fv[k2];
    }
  }
  if (threadIdx.x == 0) {
    loff[n] = (uint32_t)tot;
    const uint64_t ep = epoch << 48;
    st_store(status + b, ep | (b == 0 ? kStPre : kStAgg) | tot);
    uint64_t excl = 0;
    if (b > 0) {
      uint32_t t = b - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t v = st_load(status + t);
        const bool ready = (v >> 48) == epoch && (v & (kStAgg | kStPre));
        if (!ready) {
          if (++spins > kSpinLimit) { atomicOr(err, kErrSpin); break; }
          continue;
        }
        excl += v & kStValMask;
        if ((v & kStPre) || t == 0) break;
        --t;
      }
      st_store(status + b, ep | kStPre | (excl + tot));
    }
    base_sh = excl;
    // the segments this tile starts (with any empty ones before it), and after the last tile
    // the trailing empty segments and the total
    for (uint32_t q = seg + 1; q-- > 0 && tl.seg_blk[q] == b;) img_seg[q] = excl;
    if (b + 1 == tl.n_blocks)
      for (uint32_t q = tl.n_segs; q > seg && tl.seg_blk[q] == tl.n_blocks; --q) img_seg[q] = excl + tot;
  }
  if (pa.useB) {
    __syncthreads();  // the A table is no longer read
    stage_table(pa.tB, tk, tn);
  }
  __syncthreads();
  const uint64_t base = base_sh;
  const uint32_t n_img = (uint32_t)tot;
  if (base + n_img > out_cap) {
    if (threadIdx.x == 0 && n_img) atomicOr(err, kErrIndex | kErrExpand);
    return;
  }
  uint32_t* hw = hh;
  for (uint32_t c0 = 0; c0 < n_img; c0 += kFuseChunk) {
    const uint32_t c1 = min(c0 + (uint32_t)kFuseChunk, n_img);
    for (uint32_t j = threadIdx.x; j < n; j += kFuseBlock) {
      const uint32_t a = max(loff[j], c0), e = min(loff[j + 1], c1);
      for (uint32_t g = a; g < e; ++g) pmap[g - c0] = (uint16_t)j;
    }
    __syncthreads();
    // kFuseUnroll images per thread at a time: their parents' weight loads all in flight
    // before the first is used
    constexpr int kFuseUnroll = 4;
    for (uint32_t g0 = c0 + threadIdx.x; g0 < c1; g0 += kFuseUnroll * kFuseBlock) {
      uint32_t jj[kFuseUnroll];
      W wp[kFuseUnroll];
#pragma unroll
      for (int u = 0; u < kFuseUnroll; ++u) {
        const uint32_t g = min(g0 + (uint32_t)u * kFuseBlock, c1 - 1);
        jj[u] = pmap[g - c0];
        wp[u] = w[begin + jj[u]];
      }
#pragma unroll
      for (int u = 0; u < kFuseUnroll; ++u) {
        const uint32_t g = g0 + (uint32_t)u * kFuseBlock;
        if (g >= c1) break;
        const uint32_t j = jj[u];
        K key = akey[j];
        W wv = wp[u];
        uint32_t neg = aneg[j];
        if (e1lds) expand_ops<K, WP>(key, wv, g - loff[j], pa, (const Exp1Desc*)e1sh, pa.E2, err);
        else expand_ops<K, WP>(key, wv, g - loff[j], pa, pa.E1, pa.E2, err);
        if (pa.useB) key = apply_table(key, tk, tn, neg);
        else for (uint32_t q = 0; q < pa.nB; ++q) key = apply_perm(key, pa.B[q], neg);
        if (neg) wv = -wv;
        keys_out[base + g] = key;
        w_out[base + g] = wv;
        for (uint32_t p = 0; p < n_hp; ++p) atomicAdd(&hw[p * kRadix + ((uint32_t)(key >> (8u * (hp_begin + p))) & 255u)], 1u);
      }
    }
    __syncthreads();  // the map is rebuilt for the next window
  }
  if (n_hp) {
    for (uint32_t i = threadIdx.x; i < n_hp * kRadix; i += kFuseBlock) {
      const uint32_t c = hh[i];
      const uint32_t p = hp_begin + i / kRadix, d = i % kRadix;
      if (c) atomicAdd(&ghist[((uint64_t)seg * n_pass + p) * kRadix + d], c);
    }
  }
}

// --------------------------------------------------------------- run accumulators
// Equal keys are adjacent inside a segment after the sort. The thread that owns the
// first element of a run (its head) sums the run in array order (deterministic), then
// keeps it when |sum| > thr. FP32 runs are summed with the TwoSum-compensated
// (Kahan-Babuska) recurrence, or in FP64 and rounded once.
template <typename W>
struct RunSum {
  W s = 0;
  W c = 0;
  __device__ __forceinline__ void add(W x) {
    const W t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ W value() const { return s + c; }
};

template <typename W>
struct PlainSum {  // in W, array order
  W s = 0;
  __device__ __forceinline__ void add(W x) { s += x; }
  __device__ __forceinline__ W value() const { return s; }
};

struct F64Sum {  // FP32 weights accumulated in FP64, rounded once
  double s = 0;
  __device__ __forceinline__ void add(float x) { s += (double)x; }
  __device__ __forceinline__ float value() const { return (float)s; }
};

// kMode 0: count the kept runs of each tile (blk_cnt); 1: write them at the scanned
// offsets (blk_off); 2: single sweep - tiles are claimed in order, each publishes its
// count and looks back over the earlier tiles for its output offset (written to blk_off,
// with the total at blk_off[n_blocks]), then writes.
// After the merge (one block): the segment output offsets seg_off_out[s] = blk_off[seg_blk[s]]
// (all 0 when there are no tiles) and the packed readback area (see MergeFin).
// The end of a publishing kernel (one block): every thread's result words reach memory before
// the sequence word is stored, so a host that sees the sequence word may read them all.
__device__ __forceinline__ void publish_seq(const MergeFin& fin, uint32_t S) {
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) *(volatile uint64_t*)&fin.result[2 * (uint64_t)S + 3] = fin.seq;
}

__global__ void k_merge_publish(Tiling tl, const uint64_t* __restrict__ blk_off, uint64_t* __restrict__ seg_off_out,
                                MergeFin fin, const uint32_t* __restrict__ err, int none) {
  const uint32_t S = tl.n_segs;
  for (uint32_t s = threadIdx.x; s <= S; s += blockDim.x) {
    const uint64_t v = none ? 0ull : blk_off[tl.seg_blk[s]];
    seg_off_out[s] = v;
    fin.result[s] = v;
    fin.result[S + 1 + s] = fin.img_seg[s];
  }
  if (threadIdx.x == 0) fin.result[2 * (uint64_t)S + 2] = *err;
  publish_seq(fin, S);
}


// ----------------------------------------------------------------- chunk-local sort
// After stable global passes over the top m digits, every segment is grouped into buckets of
// equal top digits, in order. Chunk c starts at the first bucket boundary at or after the
// start of nominal tile c (the segment start for its first tile), so chunks are runs of whole
// buckets; each chunk (at most kChunkCap elements) is sorted in LDS, stably, which completes a
// stable sort of the segment: stable 8-bit passes bring equal top m+1 digits together within
// each bucket, and each element of the resulting small groups moves to its rank in its group.
// A bucket too large for
// a chunk raises kErrRedo (not an error: the caller sorts the round again with global passes
// only).
constexpr int kChunkBlock = 512;  // threads of a chunk-local sort (8 waves)
constexpr uint64_t kChunkPlaced = ~0ull;          // chunk_start of a chunk written in place
template <typename K, typename W>
__global__ void __launch_bounds__(kChunkBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_chunk_sort(const K* __restrict__ keys_in, const W* __restrict__ w_in, K* __restrict__ keys_out, W* __restrict__ w_out,
             uint64_t out_cap, Tiling tc, uint32_t n_pass, uint32_t m, const PassArgs* __restrict__ pas,
             const uint32_t* __restrict__ seg_entry, int fp64_acc, ChunkOut co, uint32_t* err) {
  constexpr int kItems = kChunkCap / kChunkBlock, kWaves = kChunkBlock / 64;
  __shared__ __align__(16) K sk[kChunkCap];  // (also the staging area of the output weights)
  __shared__ uint16_t sidx[kChunkCap];
  __shared__ uint16_t sbk[kChunkCap];
  __shared__ __align__(16) uint32_t wrun[2][kWaves][kRadix];
  __shared__ uint32_t wdummy[kWaves][64];
  __shared__ __align__(16) uint32_t dbase[kWaves][kRadix];
  __shared__ uint64_t scan_sh[kWaves];
  __shared__ uint64_t cb[2];
  __shared__ uint32_t nb_sh, fallback_sh;
  __shared__ uint32_t gmax_sh[kWaves], gmin_sh[kWaves];
  __shared__ __align__(16) uint8_t vary_sh[kWaves * sizeof(K)];
  __shared__ uint32_t blk_sh;
  __shared__ uint64_t base_sh;
  __shared__ K prev_sh;
  // a look-back that waits claims chunks in order (so that every chunk it waits for is
  // running or done); one that only looks once takes the block's own index
  uint32_t blk = blockIdx.x;
  if (co.defer_spins) {
    if (threadIdx.x == 0) blk_sh = atomicAdd(co.ticket, 1u);
    __syncthreads();
    blk = blk_sh;
  }
  const uint32_t nc = tc.n_dev ? *tc.n_dev : tc.n_blocks;
  if (blk >= nc) return;
  // The chunk's output offset: publish its kept count and look back over the earlier chunks
  // for their prefix (decoupled look-back; status words [epoch:16][flag:2][value:46]). The
  // wait for an earlier chunk that has not published yet is short: past co.defer_spins polls the chunk
  // is deferred (its runs go to its own range, and a later launch moves them), so that one
  // slow chunk does not hold every later one on the chip. Returns the offset, or kDeferred.
  constexpr uint64_t kDeferred = ~0ull;
  auto lookback = [&](uint64_t tot, uint64_t start) -> uint64_t {
    if (threadIdx.x == 0) {
      const uint64_t ep = co.epoch << 48;
      st_store(co.status + blk, ep | (blk == 0 ? kStPre : kStAgg) | tot);
      uint64_t excl = 0;
      bool resolved = true;
      if (blk > 0) {
        uint32_t t = blk - 1;
        uint32_t spins = 0;
        while (true) {
          const uint64_t v = st_load(co.status + t);
          const bool ready = (v >> 48) == co.epoch && (v & (kStAgg | kStPre));
          if (!ready) {
            if (++spins > co.defer_spins) { resolved = false; break; }
            continue;
          }
          excl += v & kStValMask;
          if ((v & kStPre) || t == 0) break;
          --t;
        }
        if (resolved) st_store(co.status + blk, ep | kStPre | (excl + tot));
      }
      co.chunk_cnt[blk] = (uint32_t)tot;
      co.chunk_start[blk] = resolved ? kChunkPlaced : start;
      base_sh = resolved ? excl : kDeferred;
    }
    __syncthreads();
    return base_sh;
  };
  auto none = [&]() { lookback(0, 0); };  // this chunk keeps nothing (empty, or handed to the fallback)
  const uint64_t a = tc.blk_begin[blk], b = tc.blk_end[blk];
  if (a >= b) {
    none();
    return;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // The window [a, a + kChunkCap) of the segment goes to LDS first (with the key before it);
  // the chunk bounds are found there (wave 0 from the tile start, wave 1 from the tile end),
  // in global memory only where a bucket reaches past the window. Its loads (clamped to the
  // image arrays, co.in_len elements) are issued before the segment bounds are looked up.
  K kr[kItems];
  {
    const uint32_t ln = (uint32_t)(min(co.in_len, a + (uint64_t)kChunkCap) - a);  // >= b - a >= 1
#pragma unroll
    for (int r = 0; r < kItems; ++r) kr[r] = keys_in[a + min((uint32_t)(r * kChunkBlock + threadIdx.x), ln - 1)];
  }
  const K before = (threadIdx.x == 0 && a > 0) ? keys_in[a - 1] : (K)0;
  const uint32_t s = tc.blk_seg[blk];
  const uint64_t seg_lo = tc.blk_begin[tc.seg_blk[s]], seg_hi = tc.blk_end[tc.seg_blk[s + 1] - 1];
  const uint32_t top_shift = 8u * (n_pass - m);
  auto top = [&](K key) -> K { return m == 0 ? (K)0 : (K)(key >> top_shift); };
  const uint64_t wend = min(seg_hi, a + (uint64_t)kChunkCap);
  const uint32_t wn = (uint32_t)(wend - a);  // >= b - a >= 1
  {
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = r * kChunkBlock + threadIdx.x;
      if (j < wn) sk[j] = kr[r];
    }
    if (threadIdx.x == 0) prev_sh = before;
  }
  __syncthreads();
  if (threadIdx.x < 128) {
    const bool at_end = threadIdx.x >= 64;
    const uint64_t x = at_end ? b : a;
    uint64_t r = x;
    if (x != seg_lo && x != seg_hi) {
      // (b - 1 - a < b - a <= the nominal tile, inside the window)
      const K t = top(at_end ? sk[b - 1 - a] : prev_sh);
      // a bucket holding x-1 ends before x + kChunkCap unless it is too large for a chunk
      const uint64_t lim = min(seg_hi, x + (uint64_t)kChunkCap), lim_w = min(lim, wend);
      r = wave_first_true(x, lim_w, [&](uint64_t i) { return top(sk[i - a]) != t; });
      if (r == lim_w && lim_w < lim) r = wave_first_true(lim_w, lim, [&](uint64_t i) { return top(keys_in[i]) != t; });
      if (r == lim && lim < seg_hi && lane == 0) atomicOr(err, kErrRedo);
    }
    if (lane == 0) cb[threadIdx.x >> 6] = r;
  }
  __syncthreads();
  const uint64_t c0 = cb[0], c1 = cb[1];
  if (c1 <= c0) {  // every element of the tile belongs to an earlier chunk
    none();
    return;
  }
  if (c1 - c0 > (uint64_t)kChunkCap) {
    if (threadIdx.x == 0) atomicOr(err, kErrRedo);
    none();
    return;
  }
  const uint32_t n = (uint32_t)(c1 - c0);
  {
    // the chunk's keys to the front of sk: from the window, or from global memory where the
    // chunk reaches past it
    const bool in_win = c1 <= wend;
    K kr[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = min((uint32_t)(r * kChunkBlock + threadIdx.x), n - 1);
      kr[r] = in_win ? sk[(uint32_t)(c0 - a) + j] : keys_in[c0 + j];
    }
    __syncthreads();  // every window read before the first write
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
      const uint32_t j = r * kChunkBlock + threadIdx.x;
      if (j < n) {
        sk[j] = kr[r];
        sidx[j] = (uint16_t)j;
      }
    }
  }
  __syncthreads();
  // the n elements in equal wave spans of whole 64-element rounds
  const uint32_t span = (n + kWaves * 64 - 1) / (kWaves * 64) * 64, nr = span / 64;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  // the rounds of a wave run in pairs; a pair wholly past the span is skipped (no branch
  // inside a pair, so LDS operations of different rounds overlap)
  static_assert(kItems % 2 == 0, "rounds in pairs");
  auto rounds = [&](auto&& body) {
#pragma unroll
    for (int r2 = 0; r2 < kItems; r2 += 2) {
      if ((uint32_t)r2 < nr) {
        body(r2);
        body(r2 + 1);
      }
    }
  };
  // per-wave digit counters, double-buffered by pass parity (a wave clears its row of the
  // other buffer for the next pass), so that a pass needs only two block barriers
  for (int i = threadIdx.x; i < 2 * kWaves * kRadix; i += kChunkBlock) (&wrun[0][0][0])[i] = 0;
  // bucket of every element (runs of equal top digits, numbered in order): heads, block scan
  {
    const uint32_t j0 = threadIdx.x * kItems;
    uint32_t cnt = 0;
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      const uint32_t j = j0 + t;
      if (j < n && (j == 0 || top(sk[j]) != top(sk[j - 1]))) ++cnt;
    }
    uint64_t tot;
    uint32_t id = (uint32_t)block_excl_scan<kChunkBlock>(cnt, scan_sh, &tot);
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      const uint32_t j = j0 + t;
      if (j < n) {
        if (j == 0 || top(sk[j]) != top(sk[j - 1])) ++id;
        sbk[j] = (uint16_t)(id - 1);
      }
    }
    if (threadIdx.x == 0) nb_sh = (uint32_t)tot;
  }
  __syncthreads();
  const uint32_t nb = nb_sh;
  // One stable LDS radix pass: the digit of an element comes from dig(key, bucket); key,
  // original index and bucket move together.
  uint32_t pass_no = 0;
  // nbits: digits are below 2^nbits (a bit no lane sets leaves the ballot masks unchanged)
  auto radix_pass = [&](auto&& dig, uint32_t nbits) {
    const int pb = pass_no++ & 1;
    K key[kItems];
    uint16_t ix[kItems], bk[kItems];
    uint32_t rank[kItems], pk[kItems];  // pk: digit | leader lane << 8 | lanes below with that digit << 16
    // every read of the pass first (clamped indices), then the ranking
    rounds([&](int r) {
      const uint32_t li = min(wid * span + r * 64 + lane, n - 1);
      key[r] = sk[li];
      ix[r] = sidx[li];
      bk[r] = sbk[li];
    });
    rounds([&](int r) {
      const uint32_t li = wid * span + r * 64 + lane;  // stable order: wave span, round, lane
      const bool valid = (uint32_t)r < nr && li < n;    // rounds past nr belong to the next wave
      const uint32_t d = dig(key[r], (uint32_t)bk[r]) & (kRadix - 1);
      // lanes whose digit differs from this lane's in some bit: OR of (ballot of the bit) XOR
      // (this lane's bit spread over the mask)
      const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
      uint32_t dlo = ~(uint32_t)vm, dhi = ~(uint32_t)(vm >> 32);
#pragma unroll
      for (int bit = 0; bit < kRadixBits; ++bit) {
        if ((uint32_t)bit >= nbits) break;
        const int spread = __builtin_amdgcn_sbfe((int)d, bit, 1);  // 0 or all ones
        const uint64_t bb = __builtin_amdgcn_ballot_w64(spread != 0);
        dlo |= (uint32_t)bb ^ (uint32_t)spread;
        dhi |= (uint32_t)(bb >> 32) ^ (uint32_t)spread;
      }
      const uint64_t mk = ~(((uint64_t)dhi << 32) | dlo);
      // the leader of each digit group reserves its slots (every lane issues the atomic, the
      // others adding 0 to a slot of their own); a wave's LDS atomics complete in issue order
      const int leader = __ffsll((long long)mk) - 1;
      const bool lead_me = valid && lane == leader;
      rank[r] = atomicAdd(lead_me ? &wrun[pb][wid][d] : &wdummy[wid][lane], lead_me ? (uint32_t)__popcll(mk) : 0u);
      pk[r] = d | ((uint32_t)(leader < 0 ? 0 : leader) << 8) | ((uint32_t)__popcll(mk & lt) << 16);
    });
    rounds([&](int r) { rank[r] = __shfl(rank[r], (pk[r] >> 8) & 63u, 64); });
    rounds([&](int r) { rank[r] += pk[r] >> 16; });
    __syncthreads();
    {
      // every wave scans all 256 digit totals itself (lane l: digits 4l..4l+3) and keeps, in
      // its own row of dbase, where its elements of each digit start
      uint32_t tot[4] = {0, 0, 0, 0}, pre[4] = {0, 0, 0, 0};
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint4 c = *(const uint4*)&wrun[pb][w][4 * lane];
        const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (w < wid) pre[j] += cw[j];
          tot[j] += cw[j];
        }
      }
      const uint32_t lane_sum = tot[0] + tot[1] + tot[2] + tot[3];
      uint32_t run = (uint32_t)(wave_incl_scan((uint64_t)lane_sum) - lane_sum);
      uint4 base;
      base.x = run + pre[0]; run += tot[0];
      base.y = run + pre[1]; run += tot[1];
      base.z = run + pre[2]; run += tot[2];
      base.w = run + pre[3];
      *(uint4*)&dbase[wid][4 * lane] = base;
      *(uint4*)&wrun[pb ^ 1][wid][4 * lane] = make_uint4(0u, 0u, 0u, 0u);
    }
    rounds([&](int r) {
      if ((uint32_t)r < nr && wid * span + r * 64 + lane < n) {
        const uint32_t dst = dbase[wid][pk[r] & 255u] + rank[r];
        sk[dst] = key[r];
        sidx[dst] = ix[r];
        sbk[dst] = bk[r];
      }
    });
    __syncthreads();
  };
  // Few buckets: one pass by the digit just below the bucket digits, one by the bucket number
  // (skipped for a single bucket), which leaves groups of equal top m+1 digits in order.
  // Many buckets (fewer than 16 elements each on average): the buckets are the groups. The
  // groups are then sorted by ranking inside each group (stable); a group above kMaxGroup
  // elements sends the chunk through stable passes over every digit instead (same order).
  constexpr uint32_t kMaxGroup = 32;
  const bool two_pass = nb <= (uint32_t)kRadix && m > 0 && m < n_pass;
  const uint32_t g_shift = two_pass ? top_shift - 8u : top_shift;
  auto gkey = [&](K key) -> K { return (two_pass || m > 0) ? (K)(key >> g_shift) : (K)0; };
  if (two_pass) {
    radix_pass([&](K key, uint32_t) { return (uint32_t)(key >> g_shift); }, kRadixBits);
    if (nb > 1) radix_pass([&](K, uint32_t bkt) { return bkt; }, 32u - (uint32_t)__clz((int)(nb - 1)));
  }
  // Groups of equal gkey: thread t holds the sorted positions [t*kItems, (t+1)*kItems). Every
  // element finds its group [gs, ge) from a block max-scan of the group heads before it and a
  // min-scan of the heads after it (positions past n count as heads); with every group at most
  // kMaxGroup long, it counts the smaller keys of its group (equal keys by position: stable) and
  // moves to gs + that rank. A longer group sends the chunk to the fallback.
  {
    const uint32_t j0 = threadIdx.x * kItems;
    K kk[kItems];
    uint16_t ii[kItems];
    bool hd[kItems];
    const K prevk = (j0 > 0 && j0 - 1 < n) ? sk[j0 - 1] : (K)0;
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      const uint32_t j = j0 + t;
      const bool valid = j < n;
      kk[t] = valid ? sk[j] : (K)0;
      ii[t] = valid ? sidx[j] : (uint16_t)0;
      hd[t] = !valid || j == 0 || gkey(kk[t]) != gkey(t ? kk[t - 1] : prevk);
    }
    uint32_t last_head = 0, first_head = kChunkCap;
#pragma unroll
    for (int t = 0; t < kItems; ++t)
      if (hd[t]) last_head = j0 + t;
#pragma unroll
    for (int t = kItems - 1; t >= 0; --t)
      if (hd[t]) first_head = j0 + t;
    // wave scans: the last head in earlier lanes (max), the first head in later lanes (min)
    uint32_t lo_max = last_head, hi_min = first_head;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(lo_max, d, 64);
      const uint32_t v = __shfl_down(hi_min, d, 64);
      if (lane >= d) lo_max = max(lo_max, u);
      if (lane + d < 64) hi_min = min(hi_min, v);
    }
    if (lane == 63) gmax_sh[wid] = lo_max;
    if (lane == 0) gmin_sh[wid] = hi_min;
    if (threadIdx.x == 0) fallback_sh = 0;
    uint32_t before = __shfl_up(lo_max, 1, 64), after = __shfl_down(hi_min, 1, 64);
    if (lane == 0) before = 0;
    if (lane == 63) after = kChunkCap;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      if (w < wid) before = max(before, gmax_sh[w]);
      if (w > wid) after = min(after, gmin_sh[w]);
    }
    // group bounds packed per item: start | end << 16 (positions below 2^13)
    uint32_t gb[kItems];
    uint32_t run = before;
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      if (hd[t]) run = j0 + t;
      gb[t] = run;
    }
    run = after;
#pragma unroll
    for (int t = kItems - 1; t >= 0; --t) {
      gb[t] |= min(run, n) << 16;
      if (hd[t]) run = j0 + t;
    }
    bool big = false;
#pragma unroll
    for (int t = 0; t < kItems; ++t)
      if (j0 + t < n && (gb[t] >> 16) - (gb[t] & 0xFFFFu) > kMaxGroup) big = true;
    if (big) fallback_sh = 1;
    __syncthreads();
    if (!fallback_sh) {
      uint32_t dst[kItems];
#pragma unroll
      for (int t = 0; t < kItems; ++t) {
        const uint32_t j = j0 + t, gs = gb[t] & 0xFFFFu, ge = gb[t] >> 16;
        uint32_t r = 0;
        if (j < n && ge - gs > 1)
          for (uint32_t i = gs; i < ge; ++i) {
            const K v = sk[i];
            r += (v < kk[t] || (v == kk[t] && i < j)) ? 1u : 0u;
          }
        dst[t] = gs + r;
      }
      __syncthreads();  // every rank counted before any element moves
#pragma unroll
      for (int t = 0; t < kItems; ++t) {
        if (j0 + t < n && dst[t] != j0 + t) {
          sk[dst[t]] = kk[t];
          sidx[dst[t]] = ii[t];
        }
      }
      __syncthreads();
    }
  }
  if (fallback_sh) {
    // stable passes over the digits that vary inside the chunk (a constant digit leaves a
    // stable pass's order unchanged)
    K vary = 0;
    for (uint32_t j = threadIdx.x; j < n; j += kChunkBlock) vary |= sk[j] ^ sk[0];
    vary = block_or<kChunkBlock>(vary, (K*)vary_sh);
    for (uint32_t p = 0; p < n_pass; ++p)
      if ((uint32_t)(vary >> (8u * p)) & 255u) radix_pass([&](K key, uint32_t) { return (uint32_t)(key >> (8u * p)); }, kRadixBits);
  }
  // Merge in place: runs of equal keys lie in one chunk (equal keys share their top digits).
  // The thread owning a run's head sums it in array order and keeps it when |sum| > thr; the
  // kept runs are counted for the chunk's offset and written in order.
  const double thr = pas[seg_entry[s]].thr;
  const uint32_t j0 = threadIdx.x * kItems;  // this thread's run of sorted positions
  W wr[kItems], sums[kItems];
  K kt[kItems];
#pragma unroll
  for (int t = 0; t < kItems; ++t) wr[t] = w_in[c0 + sidx[min(j0 + t, n - 1)]];  // every gather in flight
#pragma unroll
  for (int t = 0; t < kItems; ++t) kt[t] = sk[min(j0 + t, n - 1)];
  const K k_before = (j0 > 0 && j0 <= n) ? sk[j0 - 1] : (K)0;
  const K k_after = j0 + kItems < n ? sk[j0 + kItems] : (K)0;
  // Each run is summed left to right by the thread holding its head (its tail past this
  // thread's items read from global memory) and its sum kept at its last item in this thread
  // (static register indices only).
  uint32_t keep_mask = 0, keep = 0;
  auto sum_runs = [&](auto proto) {
    auto acc = proto;
    bool active = false;
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      const uint32_t j = j0 + t;
      const bool valid = j < n;
      const bool head = valid && (j == 0 || kt[t] != (t ? kt[t - 1] : k_before));
      const bool cont = j + 1 < n && (t + 1 < kItems ? kt[t + 1] : k_after) == kt[t];
      if (head) {
        acc = proto;
        active = true;
      }
      if (active && valid) {
        acc.add(wr[t]);
        if (t + 1 == kItems && cont)
          for (uint32_t i = j0 + kItems; i < n && sk[i] == kt[t]; ++i) acc.add(w_in[c0 + sidx[i]]);
        if (!cont || t + 1 == kItems) {
          const W v = acc.value();
          sums[t] = v;
          if (fabs((double)v) > thr) {
            keep_mask |= 1u << t;
            ++keep;
          }
          active = false;
        }
      }
    }
  };
  if constexpr (sizeof(W) == 8) sum_runs(PlainSum<W>{});
  else if (fp64_acc) sum_runs(F64Sum{});
  else sum_runs(RunSum<float>{});
  uint64_t tot;
  const uint64_t pre = block_excl_scan<kChunkBlock>(keep, scan_sh, &tot);
  const uint64_t base = lookback(tot, c0);
  // every kept run straight to its output position, or (deferred) to the front of the chunk's
  // own range of the scratch arrays
  K* kd = keys_out;
  W* wd = w_out;
  uint64_t ob = base;  // output position of the chunk's first kept run
  if (base == kDeferred) {
    kd = (K*)co.tmp_keys;
    wd = (W*)co.tmp_w;
    ob = c0;
  } else if (base + tot > out_cap) {
    if (threadIdx.x == 0 && tot) atomicOr(err, kErrIndex | kErrMerge);
    return;
  }
  // The kept runs leave through LDS, which the sort no longer needs (the look-back's barrier
  // follows every read of it): staged at their rank in the chunk, then stored by consecutive
  // threads, so that a wave's stores fill whole lines instead of touching one element every
  // kItems slots per lane. Keys first, then the weights in passes of what the key area holds.
  const uint32_t nt = (uint32_t)tot;
  {
    uint32_t q = (uint32_t)pre;
#pragma unroll
    for (int t = 0; t < kItems; ++t)
      if (keep_mask & (1u << t)) sk[q++] = kt[t];
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < nt; j += kChunkBlock) kd[ob + j] = sk[j];
  constexpr uint32_t kWCap = (uint32_t)(sizeof(K) * kChunkCap / sizeof(W));
  W* const sws = reinterpret_cast<W*>(sk);
  for (uint32_t p0 = 0; p0 < nt; p0 += kWCap) {
    __syncthreads();  // every read of the staging area before it is rewritten
    uint32_t q = (uint32_t)pre;
#pragma unroll
    for (int t = 0; t < kItems; ++t)
      if (keep_mask & (1u << t)) {
        if (q >= p0 && q - p0 < kWCap) sws[q - p0] = sums[t];
        ++q;
      }
    __syncthreads();
    const uint32_t pn = min(nt - p0, kWCap);
    for (uint32_t j = threadIdx.x; j < pn; j += kChunkBlock) wd[ob + p0 + j] = sws[j];
  }
}

// After the chunk-local sort and merge (one block): chunk_off = exclusive scan of the kept
// counts of the chunks (n_dev or n_blocks of tc), the segment output offsets
// seg_off_out[s] = chunk_off[seg_blk[s]], and the packed readback area (see MergeFin), whose
// image offsets are fin.img_seg, or the scan of img_cnt when set; a total above out_cap is
// reported in the error word there (the compaction then writes nothing).
constexpr int kPublishBlock = 1024;
__global__ void __launch_bounds__(kPublishBlock) k_chunk_publish(Tiling tc, const uint32_t* __restrict__ chunk_cnt,
                                                                 uint64_t* __restrict__ chunk_off,
                                                                 uint64_t* __restrict__ seg_off_out, MergeFin fin,
                                                                 const uint32_t* __restrict__ img_cnt, uint64_t out_cap,
                                                                 const uint32_t* __restrict__ err) {
  __shared__ uint64_t sh[kPublishBlock / 64];
  __shared__ uint64_t total_sh;
  const uint32_t nc = tc.n_dev ? *tc.n_dev : tc.n_blocks;
  // thread t scans the run [t*per, (t+1)*per) serially: one block scan for all the runs
  const uint32_t per = (nc + kPublishBlock - 1) / kPublishBlock;
  const uint32_t r0 = min(threadIdx.x * per, nc), r1 = min(r0 + per, nc);
  // (eight loads in flight at a time: the run is read twice)
  constexpr uint32_t kBatch = 8;
  uint64_t sum = 0;
  for (uint32_t i0 = r0; i0 < r1; i0 += kBatch) {
    uint32_t v[kBatch];
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) v[u] = i0 + u < r1 ? chunk_cnt[i0 + u] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) sum += v[u];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan<kPublishBlock>(sum, sh, &tot);
  for (uint32_t i0 = r0; i0 < r1; i0 += kBatch) {
    uint32_t v[kBatch];
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) v[u] = i0 + u < r1 ? chunk_cnt[i0 + u] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) {
      if (i0 + u < r1) chunk_off[i0 + u] = run;
      run += v[u];
    }
  }
  if (threadIdx.x == 0) {
    chunk_off[nc] = tot;
    total_sh = tot;
  }
  __syncthreads();
  const uint32_t S = tc.n_segs;
  for (uint32_t q = threadIdx.x; q <= S; q += kPublishBlock) {
    const uint64_t v = chunk_off[min(tc.seg_blk[q], nc)];
    seg_off_out[q] = v;
    fin.result[q] = v;
    if (!img_cnt) fin.result[S + 1 + q] = fin.img_seg[q];
  }
  if (img_cnt) {  // image offsets of the segments from their counts (same serial-run scan)
    const uint32_t ps = (S + kPublishBlock - 1) / kPublishBlock;
    const uint32_t q0 = min(threadIdx.x * ps, S), q1 = min(q0 + ps, S);
    uint64_t isum = 0;
    for (uint32_t q = q0; q < q1; ++q) isum += img_cnt[q];
    uint64_t itot;
    uint64_t irun = block_excl_scan<kPublishBlock>(isum, sh, &itot);
    for (uint32_t q = q0; q < q1; ++q) {
      fin.result[S + 1 + q] = irun;
      irun += img_cnt[q];
    }
    if (threadIdx.x == 0) fin.result[2 * (uint64_t)S + 1] = itot;
  }
  if (threadIdx.x == 0) fin.result[2 * (uint64_t)S + 2] = *err | (total_sh > out_cap ? kErrIndex | kErrMerge : 0u);
  publish_seq(fin, S);
}

// Moves the kept runs of every deferred chunk from the front of its range (in the scratch
// arrays) to its output offset; the other chunks wrote theirs in place already.
template <typename K, typename W>
__global__ void __launch_bounds__(256) k_chunk_compact(const K* __restrict__ keys_in, const W* __restrict__ w_in,
                                                       K* __restrict__ keys_out, W* __restrict__ w_out, Tiling tc,
                                                       const uint32_t* __restrict__ chunk_cnt,
                                                       const uint64_t* __restrict__ chunk_start,
                                                       const uint64_t* __restrict__ chunk_off, uint64_t out_cap,
                                                       uint32_t* err) {
  const uint32_t blk = blockIdx.x;
  if (tc.n_dev && blk >= *tc.n_dev) return;
  const uint64_t src = chunk_start[blk];
  if (src == kChunkPlaced) return;
  const uint32_t cnt = chunk_cnt[blk];
  const uint64_t dst = chunk_off[blk];
  if (dst + cnt > out_cap || cnt > (uint32_t)kChunkCap) {
    if (threadIdx.x == 0 && cnt) atomicOr(err, kErrIndex | kErrMerge);
    return;
  }
  // every load of a thread's share in flight before its stores (a chunk keeps at most
  // kChunkCap terms: kChunkCap / 256 per thread)
  constexpr int kPer = kChunkCap / 256;
  K kv[kPer];
  W wv[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const uint32_t i = r * 256 + threadIdx.x;
    if (i < cnt) {
      kv[r] = keys_in[src + i];
      wv[r] = w_in[src + i];
    }
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const uint32_t i = r * 256 + threadIdx.x;
    if (i < cnt) {
      keys_out[dst + i] = kv[r];
      w_out[dst + i] = wv[r];
    }
  }
}

// ------------------------------------------------------------ persistent small passes
// Consecutive passes of one circuit whose segments stay small (at most kChunkCap terms and
// images each, by the host's fan-out bound) in one launch: one block per segment keeps its
// terms in a slot of kChunkCap in global memory (L2-resident at these sizes) and, pass after
// pass, applies the A chain and counts the fan-outs, scans them in LDS, forms the images
// (expansion and B chain: keys to LDS, weights to a scratch slot), sorts the keys stably in
// LDS (LSD passes over the digits that vary), sums each run of equal keys in array order,
// prunes, and writes the kept terms to the other slot. These are the images, the order and
// the sums of the round-by-round small path, so the results agree bit for bit; only the
// launches and the host's waits between the passes are gone. cnt[(p*S + s)*3 + {0,1,2}]
// receives segment s's input terms, images and kept terms in pass p.
constexpr int kGroupBlock = 512;
template <typename K, int WP>
__global__ void __launch_bounds__(kGroupBlock) k_small_passes(
    const K* __restrict__ keys_in, const typename WTraits<WP>::W* __restrict__ w_in,
    const uint64_t* __restrict__ seg_in, uint32_t S, const PassArgs* __restrict__ pas, uint32_t n_grp,
    K* __restrict__ kslot0, typename WTraits<WP>::W* __restrict__ wslot0, K* __restrict__ kslot1,
    typename WTraits<WP>::W* __restrict__ wslot1, typename WTraits<WP>::W* __restrict__ wimg,
    uint32_t* __restrict__ cnt, int fp64_acc, uint32_t* err) {
  using W = typename WTraits<WP>::W;
  constexpr int kTabN = (int)sizeof(K) * 256;
  constexpr int kItems = kChunkCap / kGroupBlock, kWaves = kGroupBlock / 64;
  __shared__ K tk[kTabN];
  __shared__ uint8_t tn[kTabN];
  __shared__ K akey[kChunkCap];
  __shared__ uint8_t negs[kChunkCap];
  __shared__ uint32_t off[kChunkCap + 1];
  __shared__ uint16_t pmap[kChunkCap];
  __shared__ K sk[kChunkCap];
  __shared__ uint16_t sidx[kChunkCap];
  __shared__ __align__(16) uint32_t wrun[kWaves][kRadix];
  __shared__ __align__(16) uint32_t dbase[kWaves][kRadix];
  __shared__ uint32_t wdummy[kWaves][64];
  __shared__ uint64_t scan_sh[kWaves];
  __shared__ uint32_t nimg_sh;
  __shared__ __align__(16) uint8_t vary_sh[kWaves * sizeof(K)];
  const uint32_t s = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t slot0 = (uint64_t)s * kChunkCap;
  const K* kin = keys_in + seg_in[s];
  const W* win = w_in + seg_in[s];
  uint64_t n64 = seg_in[s + 1] - seg_in[s];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (uint32_t p = 0; p < n_grp; ++p) {
    const PassArgs pa = pas[p];
    K* kout = ((p & 1u) ? kslot1 : kslot0) + slot0;
    W* wout = ((p & 1u) ? wslot1 : wslot0) + slot0;
    uint32_t* cp = cnt + ((uint64_t)p * S + s) * 3;
    if (n64 > (uint64_t)kChunkCap || pa.drop) {  // the caller's bound did not hold
      if (threadIdx.x == 0) {
        atomicOr(err, kErrIndex | kErrFanout);
        cp[0] = cp[1] = cp[2] = 0;
      }
      n64 = 0;
      kin = kout;
      win = wout;
      continue;
    }
    const uint32_t n = (uint32_t)n64;
    // ---- A chain and fan-out of every term, their scan (as the round's count)
    if (pa.useA) stage_table(pa.tA, tk, tn);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += kGroupBlock) {
      K key = kin[i];
      uint32_t neg = 0;
      const uint64_t f = a_chain_and_fanout(key, neg, pa, tk, tn, err);
      akey[i] = key;
      negs[i] = (uint8_t)(neg & 1u);
      off[i] = (uint32_t)min<uint64_t>(f, kChunkCap + 1);  // larger: flagged by the total below
    }
    __syncthreads();
    {
      const uint32_t r0 = min(threadIdx.x * (uint32_t)kItems, n), r1 = min(r0 + (uint32_t)kItems, n);
      uint64_t sum = 0;
      for (uint32_t i = r0; i < r1; ++i) sum += off[i];
      uint64_t tot;
      uint64_t run = block_excl_scan<kGroupBlock>(sum, scan_sh, &tot);
      for (uint32_t i = r0; i < r1; ++i) {  // (each thread rewrites only its own run)
        const uint32_t f = off[i];
        off[i] = (uint32_t)min<uint64_t>(run, kChunkCap);
        run += f;
      }
      if (threadIdx.x == 0) {
        if (tot > (uint64_t)kChunkCap) atomicOr(err, kErrIndex | kErrFanout);
        nimg_sh = tot > (uint64_t)kChunkCap ? 0u : (uint32_t)tot;
        off[n] = nimg_sh;
      }
    }
    __syncthreads();
    const uint32_t n_img = nimg_sh;
    for (uint32_t j = threadIdx.x; j < n; j += kGroupBlock) {
      const uint32_t e = min(off[j + 1], n_img);
      for (uint32_t g = off[j]; g < e; ++g) pmap[g] = (uint16_t)j;
    }
    __syncthreads();  // (the A table is no longer read)
    if (pa.useB) {
      stage_table(pa.tB, tk, tn);
      __syncthreads();
    }
    // ---- the images (as the expansion): keys to LDS with their positions, weights to wimg
    for (uint32_t g = threadIdx.x; g < n_img; g += kGroupBlock) {
      const uint32_t j = pmap[g];
      K key = akey[j];
      W wv = win[j];
      uint32_t neg = negs[j];
      expand_ops<K, WP>(key, wv, g - off[j], pa, pa.E1, pa.E2, err);
      if (pa.useB) key = apply_table(key, tk, tn, neg);
      else for (uint32_t q = 0; q < pa.nB; ++q) key = apply_perm(key, pa.B[q], neg);
      if (neg) wv = -wv;
      sk[g] = key;
      sidx[g] = (uint16_t)g;
      wimg[slot0 + g] = wv;
    }
    for (int i = threadIdx.x; i < kWaves * kRadix; i += kGroupBlock) (&wrun[0][0])[i] = 0;
    __syncthreads();
    // ---- stable LSD passes in LDS over the digits that vary (a constant digit leaves a
    // stable pass's order unchanged); elements in equal wave spans of whole 64-element rounds
    if (n_img > 1) {
      K vary = 0;
      for (uint32_t j = threadIdx.x; j < n_img; j += kGroupBlock) vary |= sk[j] ^ sk[0];
      vary = block_or<kGroupBlock>(vary, (K*)vary_sh);
      const uint32_t span = (n_img + kWaves * 64 - 1) / (kWaves * 64) * 64, nr = span / 64;
      for (uint32_t dp = 0; dp < (uint32_t)sizeof(K); ++dp) {
        if (!((uint32_t)(vary >> (8u * dp)) & 255u)) continue;
        K key[kItems];
        uint16_t ix[kItems];
        uint32_t rank[kItems], pk[kItems];
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t li = min(wid * span + r * 64 + lane, n_img - 1);
          key[r] = sk[li];
          ix[r] = sidx[li];
        }
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          const uint32_t li = wid * span + r * 64 + lane;  // stable order: wave span, round, lane
          const bool valid = (uint32_t)r < nr && li < n_img;
          const uint32_t d = (uint32_t)(key[r] >> (8u * dp)) & (kRadix - 1);
          // lanes with this lane's digit: no bit of the digit differs
          const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
          uint32_t dlo = ~(uint32_t)vm, dhi = ~(uint32_t)(vm >> 32);
#pragma unroll
          for (int bit = 0; bit < kRadixBits; ++bit) {
            const int spread = __builtin_amdgcn_sbfe((int)d, bit, 1);
            const uint64_t bb = __builtin_amdgcn_ballot_w64(spread != 0);
            dlo |= (uint32_t)bb ^ (uint32_t)spread;
            dhi |= (uint32_t)(bb >> 32) ^ (uint32_t)spread;
          }
          const uint64_t mk = ~(((uint64_t)dhi << 32) | dlo);
          const int leader = __ffsll((long long)mk) - 1;
          const bool lead_me = valid && lane == leader;
          rank[r] = atomicAdd(lead_me ? &wrun[wid][d] : &wdummy[wid][lane], lead_me ? (uint32_t)__popcll(mk) : 0u);
          pk[r] = d | ((uint32_t)(leader < 0 ? 0 : leader) << 8) | ((uint32_t)__popcll(mk & lt) << 16);
        }
#pragma unroll
        for (int r = 0; r < kItems; ++r) rank[r] = __shfl(rank[r], (pk[r] >> 8) & 63u, 64) + (pk[r] >> 16);
        __syncthreads();
        {
          // every wave scans all 256 digit totals (lane l: digits 4l..4l+3) for its bases
          uint32_t tot[4] = {0, 0, 0, 0}, pre[4] = {0, 0, 0, 0};
#pragma unroll
          for (int w = 0; w < kWaves; ++w) {
            const uint4 cw4 = *(const uint4*)&wrun[w][4 * lane];
            const uint32_t cw[4] = {cw4.x, cw4.y, cw4.z, cw4.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (w < wid) pre[j] += cw[j];
              tot[j] += cw[j];
            }
          }
          const uint32_t lane_sum = tot[0] + tot[1] + tot[2] + tot[3];
          uint32_t run = (uint32_t)(wave_incl_scan((uint64_t)lane_sum) - lane_sum);
          uint4 base;
          base.x = run + pre[0]; run += tot[0];
          base.y = run + pre[1]; run += tot[1];
          base.z = run + pre[2]; run += tot[2];
          base.w = run + pre[3];
          *(uint4*)&dbase[wid][4 * lane] = base;
        }
        __syncthreads();  // every count read before the counters are cleared and keys move
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
          if ((uint32_t)r < nr && wid * span + r * 64 + lane < n_img) {
            const uint32_t dst = dbase[wid][pk[r] & 255u] + rank[r];
            sk[dst] = key[r];
            sidx[dst] = ix[r];
          }
        }
        for (int i = threadIdx.x; i < kWaves * kRadix; i += kGroupBlock) (&wrun[0][0])[i] = 0;
        __syncthreads();
      }
    }
    // ---- runs of equal keys summed in array order by the thread holding their head, pruned
    // (thread t holds sorted positions [t*kItems, (t+1)*kItems); a run's sum is kept at its last
    // item in the thread), then written in order to the other slot
    const double thr = pa.thr;
    const uint32_t j0 = threadIdx.x * kItems;
    W wr[kItems], sums[kItems];
    K kt[kItems];
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      const uint32_t j = min(j0 + t, n_img ? n_img - 1 : 0u);
      kt[t] = sk[j];
      wr[t] = n_img ? wimg[slot0 + sidx[j]] : (W)0;
    }
    const K k_before = (j0 > 0 && j0 <= n_img) ? sk[j0 - 1] : (K)0;
    const K k_after = j0 + kItems < n_img ? sk[j0 + kItems] : (K)0;
    uint32_t keep_mask = 0, keep = 0;
    auto sum_runs = [&](auto proto) {
      auto acc = proto;
      bool active = false;
#pragma unroll
      for (int t = 0; t < kItems; ++t) {
        const uint32_t j = j0 + t;
        const bool valid = j < n_img;
        const bool head = valid && (j == 0 || kt[t] != (t ? kt[t - 1] : k_before));
        const bool cont = j + 1 < n_img && (t + 1 < kItems ? kt[t + 1] : k_after) == kt[t];
        if (head) {
          acc = proto;
          active = true;
        }
        if (active && valid) {
          acc.add(wr[t]);
          if (t + 1 == kItems && cont)
            for (uint32_t i = j0 + kItems; i < n_img && sk[i] == kt[t]; ++i) acc.add(wimg[slot0 + sidx[i]]);
          if (!cont || t + 1 == kItems) {
            const W v = acc.value();
            sums[t] = v;
            if (fabs((double)v) > thr) {
              keep_mask |= 1u << t;
              ++keep;
            }
            active = false;
          }
        }
      }
    };
    if constexpr (sizeof(W) == 8) sum_runs(PlainSum<W>{});
    else if (fp64_acc) sum_runs(F64Sum{});
    else sum_runs(RunSum<float>{});
    uint64_t tot;
    uint32_t o = (uint32_t)block_excl_scan<kGroupBlock>(keep, scan_sh, &tot);
#pragma unroll
    for (int t = 0; t < kItems; ++t) {
      if (!(keep_mask & (1u << t))) continue;
      kout[o] = kt[t];
      wout[o] = sums[t];
      ++o;
    }
    if (threadIdx.x == 0) {
      cp[0] = n;
      cp[1] = n_img;
      cp[2] = (uint32_t)tot;
    }
    __syncthreads();  // the kept terms (global, this block's) before the next pass reads them
    kin = kout;
    win = wout;
    n64 = tot;
  }
}

// After k_small_passes: segment s's kept terms (its slot, cnt_last[s*3 + 2] of them) copied to
// the pass output at the sum of the earlier segments' counts; seg_off receives the offsets.
template <typename K, typename W>
__global__ void __launch_bounds__(256) k_small_gather(const K* __restrict__ kslot, const W* __restrict__ wslot,
                                                      const uint32_t* __restrict__ cnt_last, uint32_t S,
                                                      K* __restrict__ keys_out, W* __restrict__ w_out,
                                                      uint64_t* __restrict__ seg_off) {
  __shared__ uint64_t base_sh;
  const uint32_t s = blockIdx.x;
  if (threadIdx.x == 0) {
    uint64_t b = 0;
    for (uint32_t q = 0; q < s; ++q) b += cnt_last[q * 3 + 2];
    base_sh = b;
    seg_off[s] = b;
    if (s + 1 == S) seg_off[S] = b + cnt_last[s * 3 + 2];
  }
  __syncthreads();
  const uint64_t base = base_sh, src = (uint64_t)s * kChunkCap;
  const uint32_t m = min(cnt_last[s * 3 + 2], (uint32_t)kChunkCap);
  for (uint32_t i = threadIdx.x; i < m; i += 256) {
    keys_out[base + i] = kslot[src + i];
    w_out[base + i] = wslot[src + i];
  }
}

// ------------------------------------------------------------------ dense accumulation
// The dense alternative to sorting (the paper's fixed-size weight tensor of its v2 mode,
// Sec. V): for a round whose keys index a small space (4^n per generator), every image adds
// its weight into the slot of its key in a dense array per segment, and a scan of the array in
// index order (which is key order) keeps the nonzero sums. The sums are taken in 64-bit fixed
// point (2^-kDenseFracBits units): integer additions commute, so the result does not depend
// on the order in which images arrive, and each image is rounded once by at most 2^-57.
constexpr int kDenseFracBits = 56;   // |partial sum| < 2^(63-56) = 128
constexpr int kDenseTile = 4096;     // dense slots per compaction tile

template <typename K, typename W>
__global__ void __launch_bounds__(256) k_dense_scatter(const K* __restrict__ keys, const W* __restrict__ w, Tiling tl,
                                                       unsigned long long* __restrict__ acc, uint64_t per_seg,
                                                       uint32_t* err) {
  const uint32_t b = blockIdx.x;
  if (tl.n_dev && b >= *tl.n_dev) return;
  const uint64_t a0 = tl.blk_begin[b], a1 = tl.blk_end[b];
  unsigned long long* base = acc + (uint64_t)tl.blk_seg[b] * per_seg;
  for (uint64_t i = a0 + threadIdx.x; i < a1; i += 256) {
    const uint64_t k = (uint64_t)keys[i];
    const double v = (double)w[i];
    if (k >= per_seg || !(fabs(v) < 64.0)) {  // outside the dense space, or too large for it
      atomicOr(err, kErrIndex | kErrMerge);
      continue;
    }
    const long long q = __double2ll_rn(ldexp(v, kDenseFracBits));
    atomicAdd(base + k, (unsigned long long)q);
  }
}

// Tiles of kDenseTile slots, tiles_per_seg per segment, claimed in order: each keeps the slots
// whose sum exceeds thr in magnitude (and is nonzero), finds its output offset by look-back
// over the earlier tiles, and writes its kept terms (key = slot index) in key order.
template <typename K, typename W>
__global__ void __launch_bounds__(256) k_dense_compact(const unsigned long long* __restrict__ acc, uint64_t per_seg,
                                                       uint32_t tiles_per_seg, uint32_t n_tiles, double thr,
                                                       uint32_t* __restrict__ ticket, uint64_t* __restrict__ status,
                                                       uint64_t epoch, uint64_t* __restrict__ tile_off,
                                                       K* __restrict__ keys_out, W* __restrict__ w_out,
                                                       uint64_t out_cap, uint32_t* err) {
  constexpr int kItems = kDenseTile / 256;
  __shared__ uint64_t scan_sh[4];
  __shared__ uint64_t base_sh;
  __shared__ uint32_t tile_sh;
  if (threadIdx.x == 0) tile_sh = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint32_t t = tile_sh;
  if (t >= n_tiles) return;
  const uint32_t s = t / tiles_per_seg;
  const uint64_t lo = (uint64_t)(t - s * tiles_per_seg) * kDenseTile;
  const uint64_t n = min<uint64_t>(kDenseTile, per_seg - lo);
  const unsigned long long* src = acc + (uint64_t)s * per_seg + lo;
  // each thread a run of kItems consecutive slots
  const uint32_t j0 = threadIdx.x * kItems;
  W vals[kItems];
  uint32_t keep_mask = 0, keep = 0;
#pragma unroll
  for (int k2 = 0; k2 < kItems; ++k2) {
    const uint32_t j = j0 + k2;
    double v = 0.0;
    if (j < n) v = ldexp((double)(long long)src[j], -kDenseFracBits);
    vals[k2] = (W)v;
    if (v != 0.0 && fabs(v) > thr) {
      keep_mask |= 1u << k2;
      ++keep;
    }
  }
  uint64_t tot;
  const uint64_t pre = block_excl_scan<256>(keep, scan_sh, &tot);
  if (threadIdx.x == 0) {
    const uint64_t ep = epoch << 48;
    st_store(status + t, ep | (t == 0 ? kStPre : kStAgg) | tot);
    uint64_t excl = 0;
    if (t > 0) {
      uint32_t u = t - 1;
      uint32_t spins = 0;
      while (true) {
        const uint64_t v = st_load(status + u);
        const bool ready = (v >> 48) == epoch && (v & (kStAgg | kStPre));
        if (!ready) {
          if (++spins > kSpinLimit) { atomicOr(err, kErrSpin); break; }
          continue;
        }
        excl += v & kStValMask;
        if ((v & kStPre) || u == 0) break;
        --u;
      }
      st_store(status + t, ep | kStPre | (excl + tot));
    }
    tile_off[t] = excl;
    if (t + 1 == n_tiles) tile_off[n_tiles] = excl + tot;
    base_sh = excl;
  }
  __syncthreads();
  const uint64_t base = base_sh;
  if (base + tot > out_cap) {
    if (threadIdx.x == 0 && tot) atomicOr(err, kErrIndex | kErrMerge);
    return;
  }
  uint64_t o = base + pre;
#pragma unroll
  for (int k2 = 0; k2 < kItems; ++k2) {
    if (!(keep_mask & (1u << k2))) continue;
    keys_out[o] = (K)(lo + j0 + k2);
    w_out[o] = vals[k2];
    ++o;
  }
}

// One block after the compaction: segment s's output starts at the offset of its first tile;
// the packed readback area as after the chunk-local merge.
__global__ void __launch_bounds__(256) k_dense_finish(const uint64_t* __restrict__ tile_off, uint32_t tiles_per_seg,
                                                      uint32_t S, uint64_t* __restrict__ seg_off_out, MergeFin fin,
                                                      uint64_t out_cap, const uint32_t* __restrict__ err) {
  const uint64_t total = tile_off[(uint64_t)S * tiles_per_seg];
  for (uint32_t q = threadIdx.x; q <= S; q += 256) {
    const uint64_t v = tile_off[(uint64_t)q * tiles_per_seg];
    seg_off_out[q] = v;
    fin.result[q] = v;
    fin.result[S + 1 + q] = fin.img_seg[q];
  }
  if (threadIdx.x == 0) fin.result[2 * (uint64_t)S + 2] = *err | (total > out_cap ? kErrIndex | kErrMerge : 0u);
  publish_seq(fin, S);
}

// Digit histograms of the radix passes p_begin .. n_pass-1 at once, per segment:
// ghist[(s*n_pass + p)*256 + d].
template <typename K>
__global__ void __launch_bounds__(kSortBlock) k_sort_upsweep(const K* __restrict__ keys, Tiling tl, uint32_t n_pass,
                                                             uint32_t p_begin, uint32_t* __restrict__ ghist) {
  constexpr int kWaves = sizeof(K) <= 8 ? kSortBlock / 64 : 1;  // private copies per wave
  constexpr int kMaxPass = (int)sizeof(K);
  __shared__ uint32_t h[kWaves][kMaxPass][kRadix];
  const int wid = (threadIdx.x >> 6) % kWaves;
  for (int i = threadIdx.x; i < kWaves * kMaxPass * kRadix; i += kSortBlock) (&h[0][0][0])[i] = 0;
  __syncthreads();
  const uint32_t b = blockIdx.x;
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t n = (uint32_t)(end - begin);  // at most kSortTile
  K kr[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {  // every load in flight before the first use
    const uint32_t li = r * kSortBlock + threadIdx.x;
    kr[r] = keys[n ? begin + min(li, n - 1) : 0];
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {  // no early exit: the loads above stay in flight together
    if (r * kSortBlock + threadIdx.x < n)
      for (uint32_t p = p_begin; p < n_pass; ++p) atomicAdd(&h[wid][p][(uint32_t)(kr[r] >> (8 * p)) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t s = tl.blk_seg[b];
  for (uint32_t i = p_begin * kRadix + threadIdx.x; i < n_pass * kRadix; i += kSortBlock) {
    const uint32_t p = i / kRadix, dd = i % kRadix;
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += h[w][p][dd];
    if (c) atomicAdd(&ghist[((uint64_t)s * n_pass + p) * kRadix + dd], c);
  }
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------------ merge
// Sum of a run starting at tile-local index li: from the staged tile (key_at / sw) while the
// run stays inside the tile, then from global memory up to the segment end: the elements are
// added in array order whatever the tiling, so results do not depend on it.
template <typename Acc, typename W, typename K, typename KeyAt, typename WAt>
__device__ __forceinline__ W run_sum_tile(const KeyAt& key_at, const WAt& w_at, uint32_t li, uint32_t n_tile,
                                          const K* __restrict__ keys, const W* __restrict__ w, uint64_t begin,
                                          uint64_t seg_end, K key) {
  Acc a;
  a.add(w_at(li));
  uint32_t j = li + 1;
  for (; j < n_tile && key_at(1 + j) == key; ++j) a.add(w_at(j));
  if (j == n_tile)
    for (uint64_t g = begin + j; g < seg_end && keys[g] == key; ++g) a.add(w[g]);
  return a.value();
}

template <typename K, typename W, int kMode>
__global__ void __launch_bounds__(kSortBlock)
k_merge(const K* __restrict__ keys, const W* __restrict__ w, Tiling tl, const PassArgs* __restrict__ pas,
        const uint32_t* __restrict__ seg_entry, int fp64_acc, uint32_t* __restrict__ blk_cnt,
        uint64_t* __restrict__ blk_off, K* __restrict__ keys_out, W* __restrict__ w_out, uint64_t out_cap,
        uint64_t* __restrict__ status, uint32_t* __restrict__ tile_ctr, uint64_t epoch, uint32_t* err) {
  constexpr bool kLds = sizeof(K) <= 8;  // 16-byte keys are read from global memory
  // A thread takes kSortItems consecutive elements, so a wave reads LDS with a stride of
  // kSortItems elements: one pad element after every 16 spreads those reads over the banks.
  auto pad = [](uint32_t i) -> uint32_t { return i + (i >> 4); };
  constexpr int kPadded = kSortTile + kSortTile / 16 + 1;
  __shared__ K sk[kLds ? kPadded : 1];
  __shared__ W sw[kPadded];
  __shared__ uint64_t scan_sh[kSortBlock / 64];
  __shared__ uint64_t base_sh;
  uint32_t b = blockIdx.x;
  if constexpr (kMode == 2) {
    // launched for a bound on the tile count: the first n_dev blocks claim the n_dev tiles
    if (tl.n_dev && b >= *tl.n_dev) {
      if (b == 0 && threadIdx.x == 0) blk_off[0] = 0;  // no tiles: every offset is 0
      return;
    }
    if (threadIdx.x == 0) base_sh = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    b = (uint32_t)base_sh;
    __syncthreads();
  }
  const uint32_t n_tiles = tl.n_dev ? *tl.n_dev : tl.n_blocks;
  if (b >= n_tiles) {  // past the tiles that exist
    if constexpr (kMode == 2) {
      if (n_tiles == 0 && b == 0 && threadIdx.x == 0) blk_off[0] = 0;  // no images: every offset is 0
    }
    return;
  }
  const uint64_t begin = tl.blk_begin[b], end = tl.blk_end[b];
  const uint32_t s = tl.blk_seg[b];
  const double thr = pas[seg_entry[s]].thr;
  const uint64_t seg_begin = tl.blk_begin[tl.seg_blk[s]];
  const uint64_t seg_end = tl.blk_end[tl.seg_blk[s + 1] - 1];
  const uint32_t n_tile = (uint32_t)(end - begin);
  // key(i) for i in [-1, n_tile): sk[0] holds the key before the tile (if inside the segment);
  // weights in sw. Coalesced loads, all in flight before the first LDS store.
  {
    K kr[kLds ? kSortItems : 1];
    W wr[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kSortBlock + threadIdx.x;
      const uint64_t gi = n_tile ? begin + min(li, n_tile - 1) : 0;
      if constexpr (kLds) kr[r] = keys[gi];
      wr[r] = w[gi];
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const uint32_t li = r * kSortBlock + threadIdx.x;
      if (li < n_tile) {
        if constexpr (kLds) sk[pad(1 + li)] = kr[r];
        sw[pad(li)] = wr[r];
      }
    }
    if constexpr (kLds) {
      if (threadIdx.x == 0 && begin > seg_begin) sk[0] = keys[begin - 1];
    }
    __syncthreads();
  }
  auto key_at = [&](uint32_t i1) -> K {  // i1 = tile-local index + 1
    if constexpr (kLds) return sk[pad(i1)];
    else return keys[begin + i1 - 1];
  };
  auto w_at = [&](uint32_t i) -> W { return sw[pad(i)]; };
  const uint32_t i0 = threadIdx.x * kSortItems;
  uint32_t keep = 0;
  uint32_t keep_mask = 0;
  W sums[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    sums[k] = 0;
    const uint32_t li = i0 + k;
    if (li >= n_tile) continue;
    const uint64_t gi = begin + li;
    const K key = key_at(1 + li);
    const bool head = (gi == seg_begin) || (key_at(li) != key);
    if (!head) continue;
    W v;
    if constexpr (sizeof(W) == 8) {
      v = run_sum_tile<PlainSum<W>>(key_at, w_at, li, n_tile, keys, w, begin, seg_end, key);
    } else {
      if (fp64_acc) v = run_sum_tile<F64Sum>(key_at, w_at, li, n_tile, keys, w, begin, seg_end, key);
      else v = run_sum_tile<RunSum<float>>(key_at, w_at, li, n_tile, keys, w, begin, seg_end, key);
    }
    if (fabs((double)v) > thr) {
      sums[k] = v;
      keep_mask |= 1u << k;
      ++keep;
    }
  }
  uint64_t tot;
  const uint64_t pre = block_excl_scan<kSortBlock>(keep, scan_sh, &tot);
  if constexpr (kMode == 0) {
    if (threadIdx.x == 0) blk_cnt[b] = (uint32_t)tot;
  } else {
    if constexpr (kMode == 2) {
      if (threadIdx.x == 0) {
        const uint64_t ep = epoch << 48;
        st_store(status + b, ep | (b == 0 ? kStPre : kStAgg) | tot);
        uint64_t excl = 0;
        if (b > 0) {
          uint32_t t = b - 1;
          uint32_t spins = 0;
          while (true) {
            const uint64_t v = st_load(status + t);
            const bool ready = (v >> 48) == epoch && (v & (kStAgg | kStPre));
            if (!ready) {
              if (++spins > kSpinLimit) { atomicOr(err, kErrSpin); break; }
              continue;
            }
            excl += v & kStValMask;
            if ((v & kStPre) || t == 0) break;
            --t;
          }
          st_store(status + b, ep | kStPre | (excl + tot));
        }
        base_sh = excl;
        blk_off[b] = excl;
        if (b + 1 == n_tiles) blk_off[n_tiles] = excl + tot;
      }
      __syncthreads();
    }
    const uint64_t ob = kMode == 2 ? base_sh : blk_off[b];  // output position of the tile's first kept run
    if constexpr (kLds) {
      // The kept runs leave through the tile's LDS arrays (every read of them came before the
      // scan's barriers): staged at their rank in the tile, then stored by consecutive threads,
      // so that a wave's stores fill whole lines instead of touching one element every
      // kSortItems slots per lane.
      K kk[kSortItems];
#pragma unroll
      for (int k = 0; k < kSortItems; ++k) kk[k] = key_at(1 + i0 + k);
      __syncthreads();
      uint32_t q = (uint32_t)pre;
#pragma unroll
      for (int k = 0; k < kSortItems; ++k)
        if (keep_mask & (1u << k)) {
          sk[pad(q)] = kk[k];
          sw[pad(q)] = sums[k];
          ++q;
        }
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < (uint32_t)tot; j += kSortBlock) {
        const uint64_t o = ob + j;
        if (o < out_cap) {
          keys_out[o] = sk[pad(j)];
          w_out[o] = sw[pad(j)];
        } else {
          atomicOr(err, kErrIndex | kErrMerge);
        }
      }
    } else {
      uint64_t o = ob + pre;
#pragma unroll
      for (int k = 0; k < kSortItems; ++k) {
        if (!(keep_mask & (1u << k))) continue;
        if (o < out_cap) {
          keys_out[o] = key_at(1 + i0 + k);
          w_out[o] = sums[k];
        } else {
          atomicOr(err, kErrIndex | kErrMerge);
        }
        ++o;
      }
    }
  }
}

// One thread per (job, byte position, byte value): push that 4-qubit Pauli string through
// the job's chain one op at a time.
template <typename K>
__global__ void k_build_tables(const TableJob* __restrict__ jobs) {
  const TableJob jb = jobs[blockIdx.y];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sizeof(K) * 256) return;
  K key = (K)(i & 255u) << (8 * (i >> 8));
  uint32_t neg = 0;
  for (uint32_t o = 0; o < jb.n_ops; ++o) key = apply_perm(key, jb.ops[o], neg);
  ((K*)jb.tab_key)[i] = key;
  jb.tab_neg[i] = (uint8_t)(neg | ((y_count(key) & 3u) << 1));  // see apply_table
}

// Z_j of freshly admitted circuits, written at the end of the term array: for entry c,
// nq[c] terms starting at dst[c].
template <typename K, typename W>
__global__ void k_init_many(K* keys, W* w, const uint32_t* __restrict__ nq, const uint64_t* __restrict__ dst,
                            uint32_t n_circ) {
  const uint32_t c = blockIdx.x;
  if (c >= n_circ) return;
  const uint32_t n = nq[c];
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    keys[dst[c] + j] = (K)3 << (2u * (n - 1u - j));
    w[dst[c] + j] = (W)1;
  }
}

template <int WP>
__global__ void k_weights_to_f64(const typename WTraits<WP>::W* __restrict__ w, double* __restrict__ out,
                                 uint64_t T) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T) out[i] = (double)w[i];
}

// -------------------------------------------------------------------- grouping pass
// The 4x4 transfer matrix R[out][in] of one gate (Pauli order I, X, Y, Z): the closed
// form of (1/2) Tr(P_out U P_in U^dagger), i.e. diag(1, M) with M the SO(3) rotation of
// the Bloch vector that U performs (Sec. II-C; Alg. 1 composes these per qubit).
__device__ void gate_ptm(uint32_t code, double th, double R[4][4]) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) R[a][b] = (a == b) ? 1.0 : 0.0;
  // rotation about axis ax in {1,2,3} by angle t: the two other axes (u, v) in cyclic
  // order turn as u -> cos t u + sin t v, v -> cos t v - sin t u
  auto rot = [&](int ax, double t) {
    double sn, cs;
    sincos(t, &sn, &cs);
    const int u = ax % 3 + 1, v = u % 3 + 1;
    R[u][u] = cs; R[v][v] = cs; R[v][u] = sn; R[u][v] = -sn;
  };
  switch (code) {
    case 0:  // H: X <-> Z, Y -> -Y
      R[1][1] = 0; R[3][3] = 0; R[3][1] = 1; R[1][3] = 1; R[2][2] = -1; break;
    case 1:  // S: X -> Y, Y -> -X
      R[1][1] = 0; R[2][2] = 0; R[2][1] = 1; R[1][2] = -1; break;
    case 2:  // S^dagger: X -> -Y, Y -> X
      R[1][1] = 0; R[2][2] = 0; R[2][1] = -1; R[1][2] = 1; break;
    case 3: rot(3, M_PI / 4); break;   // T
    case 4: rot(3, -M_PI / 4); break;  // T^dagger
    case 5:  // SX: Y -> Z, Z -> -Y
      R[2][2] = 0; R[3][3] = 0; R[3][2] = 1; R[2][3] = -1; break;
    case 6: R[2][2] = -1; R[3][3] = -1; break;  // X
    case 7: R[1][1] = -1; R[3][3] = -1; break;  // Y
    case 8: R[1][1] = -1; R[2][2] = -1; break;  // Z
    case 9: rot(1, th); break;   // RX
    case 10: rot(2, th); break;  // RY
    case 11: rot(3, th); break;  // RZ
    default: break;
  }
}

// One wave per chain (Alg. 1 composes the gates of one wire of a U_k, in gate order): lane l
// multiplies the gates of its contiguous slice of the chain in order, then the 64 partial
// products are combined by a tree in LDS, the later slice always on the left (matrix products
// are associative; only the rounding order differs from a serial product). A chain of
// #Repeats x 3 rotations (the |XYZ + chain> workload at 10^5 repeats) thus takes about
// len / 64 serial steps instead of len.
constexpr int kComposeWaves = 4;
__global__ void __launch_bounds__(64 * kComposeWaves)
k_compose_ptm(const uint8_t* __restrict__ gate, const double* __restrict__ theta, const uint32_t* __restrict__ idx,
              const uint32_t* __restrict__ chain_off, uint32_t n_chains, double* __restrict__ out) {
  __shared__ double part[kComposeWaves][64][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t c = blockIdx.x * kComposeWaves + wid;
  const bool valid = c < n_chains;  // a wave past the last chain still takes part in the barriers
  const uint32_t a = valid ? chain_off[c] : 0u, len = valid ? chain_off[c + 1] - a : 0u;
  const uint32_t k0 = a + (uint32_t)(((uint64_t)len * lane) / 64), k1 = a + (uint32_t)(((uint64_t)len * (lane + 1)) / 64);
  double R[4][4], G[4][4], P[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
  for (uint32_t k = k0; k < k1; ++k) {
    const uint32_t gi = idx[k];
    gate_ptm(gate[gi], theta[gi], G);
    // a later gate acts on the images of the earlier ones: R <- G R
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double sum = 0.0;
        for (int t = 0; t < 4; ++t) sum += G[i][t] * R[t][j];
        P[i][j] = sum;
      }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) R[i][j] = P[i][j];
  }
  for (int i = 0; i < 16; ++i) part[wid][lane][i] = R[i >> 2][i & 3];
  for (int step = 1; step < 64; step <<= 1) {
    __syncthreads();
    if ((lane & (2 * step - 1)) == 0) {
      const double* L = part[wid][lane + step];  // the later slice
      const double* Rr = part[wid][lane];
      double Q[16];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          double sum = 0.0;
          for (int t = 0; t < 4; ++t) sum += L[i * 4 + t] * Rr[t * 4 + j];
          Q[i * 4 + j] = sum;
        }
      for (int i = 0; i < 16; ++i) part[wid][lane][i] = Q[i];
    }
  }
  __syncthreads();
  if (valid && lane < 16) out[(uint64_t)c * 16 + lane] = part[wid][0][lane];
}

inline uint32_t grid_for(uint64_t n, uint32_t block) { return (uint32_t)((n + block - 1) / block); }

}  // namespace

// ============================================================================ launchers

const char* kernel_kind_name(int k) {
  static const char* names[kKNum] = {"init", "count", "scan", "expand", "sort_hist", "sort_scatter",
                                     "merge_count", "merge_write", "compose_ptm", "chunk_sort", "count_expand",
                                     "dense_merge", "chunk_finish", "small_passes"};
  return (k >= 0 && k < kKNum) ? names[k] : "?";
}

hipEvent_t prof_begin(Prof* p, hipStream_t s, int kind) {
  if (!p || !p->on || !((p->mask >> kind) & 1u)) return nullptr;
  hipEvent_t e = nullptr;
  if (!p->pool.empty()) {
    e = p->pool.back();
    p->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, s) != hipSuccess) return nullptr;
  return e;
}

void prof_end(Prof* p, hipStream_t s, hipEvent_t a, int kind, double bytes, uint32_t count) {
  if (!p || !p->on || !a) return;
  hipEvent_t b = nullptr;
  if (!p->pool.empty()) {
    b = p->pool.back();
    p->pool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    return;
  }
  if (hipEventRecord(b, s) != hipSuccess) return;
  p->recs.push_back({kind, a, b, bytes, count});
}

void prof_resolve(Prof* p) {
  if (!p) return;
  size_t keep = 0;  // records whose end event has not completed stay for a later call
  for (auto& r : p->recs) {
    if (hipEventQuery(r.b) == hipErrorNotReady) {
      p->recs[keep++] = r;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p->launches[r.kind] += r.count;
      p->ms[r.kind] += ms;
      p->bytes[r.kind] += r.bytes;
    }
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->recs.resize(keep);
}

void prof_reset(Prof* p) {
  if (!p) return;
  for (int k = 0; k < kKNum; ++k) {
    p->launches[k] = 0;
    p->ms[k] = 0;
    p->bytes[k] = 0;
  }
}

void prof_destroy(Prof* p) {
  if (!p) return;
  for (auto& r : p->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : p->pool) (void)hipEventDestroy(e);
  p->recs.clear();
  p->pool.clear();
}

#define QIMAX_DISPATCH_K(KC, ...)                                    \
  do {                                                               \
    if ((KC) == 0) { using K = uint32_t; __VA_ARGS__; }              \
    else if ((KC) == 1) { using K = uint64_t; __VA_ARGS__; }         \
    else { using K = unsigned __int128; __VA_ARGS__; }               \
  } while (0)

hipError_t launch_init(int KC, int WP, void* keys, void* w, uint64_t* seg_off, uint32_t n, hipStream_t s,
                       Prof* prof) {
  hipEvent_t ev = prof_begin(prof, s, kKInit);
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64) k_init<K, double><<<grid_for(n, 64), 64, 0, s>>>((K*)keys, (double*)w, seg_off, n);
    else k_init<K, float><<<grid_for(n, 64), 64, 0, s>>>((K*)keys, (float*)w, seg_off, n);
  });
  prof_end(prof, s, ev, kKInit, 0.0);
  return hipGetLastError();
}

hipError_t launch_count_scan(int KC, const void* keys, uint64_t T, const Tiling& tl, const PassArgs* pas,
                             const uint32_t* seg_entry, uint64_t* off, uint64_t* status, uint32_t* ctr, uint64_t epoch,
                             uint32_t* err, void* akeys, uint8_t* asign, hipStream_t s, Prof* prof, bool wide) {
  if (T == 0 || tl.n_blocks == 0) {
    k_zero_one<<<1, 1, 0, s>>>(off);
    return hipGetLastError();
  }
  hipEvent_t ev = prof_begin(prof, s, kKCount);
  QIMAX_DISPATCH_K(KC, {
    k_count_scan<K><<<tl.n_blocks, 256, 0, s>>>((const K*)keys, tl, pas, seg_entry, off, T, status, ctr, epoch, err,
                                                 (K*)akeys, asign, wide ? 0ull : (1ull << 32));
  });
  prof_end(prof, s, ev, kKCount, (double)T * (2 * (4 << KC) + 9));
  return hipGetLastError();
}

size_t scan_tmp_words(uint64_t N) { return (size_t)((N + kScanTile - 1) / kScanTile) + 2; }

template <typename TI>
static hipError_t scan_impl(const TI* in, uint64_t* out, uint64_t N, uint64_t* tmp, hipStream_t s, Prof* prof) {
  hipEvent_t ev = prof_begin(prof, s, kKScan);
  if (N == 0) {
    k_zero_one<<<1, 1, 0, s>>>(out);
  } else {
    const uint64_t nb = (N + kScanTile - 1) / kScanTile;
    k_scan_reduce<TI><<<(uint32_t)nb, kScanBlock, 0, s>>>(in, N, tmp);
    k_scan_partials<<<1, kScanBlock, 0, s>>>(tmp, nb);
    k_scan_down<TI><<<(uint32_t)nb, kScanBlock, 0, s>>>(in, N, tmp, out);
  }
  prof_end(prof, s, ev, kKScan, (double)N * sizeof(TI) + (double)(N + 1) * 8);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, uint64_t* out, uint64_t N, uint64_t* tmp, hipStream_t s,
                           Prof* prof) {
  return scan_impl<uint32_t>(in, out, N, tmp, s, prof);
}
hipError_t launch_scan_u64(const uint64_t* in, uint64_t* out, uint64_t N, uint64_t* tmp, hipStream_t s,
                           Prof* prof) {
  return scan_impl<uint64_t>(in, out, N, tmp, s, prof);
}

hipError_t launch_gather_u64(const uint64_t* src_off, const uint64_t* idx, uint64_t* dst, uint32_t S1, hipStream_t s,
                             Prof* prof) {
  (void)prof;
  k_gather_u64<<<grid_for(S1, 64), 64, 0, s>>>(src_off, idx, dst, S1);
  return hipGetLastError();
}

hipError_t launch_expand(int KC, int WP, const void* keys, const uint8_t* asign, const void* w, uint64_t T_in,
                         const uint64_t* off,
                         uint64_t T_img, const Tiling& tl, const PassArgs* pas, const uint32_t* seg_entry,
                         const uint64_t* seg_in, bool any_tables, size_t e_bytes, void* keys_out, void* w_out,
                         uint32_t* ghist, uint32_t n_pass, uint32_t hp_begin, uint32_t* err, hipStream_t s,
                         Prof* prof, bool wide) {
  if (T_img == 0 || tl.n_blocks == 0) return hipSuccess;
  const uint64_t narrow = wide ? 0ull : (1ull << 31);
  if (ghist && (hp_begin > n_pass || n_pass - hp_begin > kExpandHistPasses)) return hipErrorInvalidValue;
  const size_t hist = ghist ? (size_t)(n_pass - hp_begin) * (kExpandBlock / 64) * kRadix * 4 : 0;
  hipEvent_t ev = prof_begin(prof, s, kKExpand);
  QIMAX_DISPATCH_K(KC, {
    const size_t tab = sizeof(K) * 256 * (sizeof(K) + 1);  // a B-chain table (A chains: done by the count)
    const size_t lds = kExpandLdsHead + (any_tables ? tab : 0) +
                       e_bytes + hist + 64;
    if (WP == 64)
      k_expand<K, 64><<<tl.n_blocks, kExpandBlock, lds, s>>>((const K*)keys, asign, (const double*)w, T_in, off, T_img, tl,
                                                              pas, seg_entry, seg_in, (K*)keys_out, (double*)w_out,
                                                              ghist, n_pass, hp_begin, err, narrow);
    else
      k_expand<K, 32><<<tl.n_blocks, kExpandBlock, lds, s>>>((const K*)keys, asign, (const float*)w, T_in, off, T_img, tl,
                                                              pas, seg_entry, seg_in, (K*)keys_out, (float*)w_out,
                                                              ghist, n_pass, hp_begin, err, narrow);
  });
  const double per = (4 << KC) + (WP == 64 ? 8 : 4);
  prof_end(prof, s, ev, kKExpand, per * (double)(T_in + T_img) + 8.0 * (double)T_in);
  return hipGetLastError();
}

size_t fuse_tile() { return (size_t)kFuseTile; }

hipError_t launch_small_passes(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in,
                               const uint64_t* seg_in, uint32_t S, const PassArgs* pas, uint32_t n_grp,
                               void* const kslot[2], void* const wslot[2], void* wimg, uint32_t* cnt,
                               void* keys_out, void* w_out, uint64_t* seg_off_out, uint32_t* err, hipStream_t s,
                               Prof* prof) {
  if (S == 0 || n_grp == 0 || KC > 1) return hipErrorInvalidValue;  // keys of 4 or 8 bytes
  hipEvent_t ev = prof_begin(prof, s, kKSmallPasses);
  const int last = (int)((n_grp - 1) & 1u);
  const uint32_t* cnt_last = cnt + (uint64_t)(n_grp - 1) * S * 3;
#define QIMAX_SMALL_PASSES(K)                                                                                     \
  if (WP == 64) {                                                                                                 \
    k_small_passes<K, 64><<<S, kGroupBlock, 0, s>>>((const K*)keys_in, (const double*)w_in, seg_in, S, pas, n_grp, \
                                                    (K*)kslot[0], (double*)wslot[0], (K*)kslot[1], (double*)wslot[1], \
                                                    (double*)wimg, cnt, fp64_acc, err);                           \
    k_small_gather<K, double><<<S, 256, 0, s>>>((const K*)kslot[last], (const double*)wslot[last], cnt_last, S,    \
                                                (K*)keys_out, (double*)w_out, seg_off_out);                       \
  } else {                                                                                                        \
    k_small_passes<K, 32><<<S, kGroupBlock, 0, s>>>((const K*)keys_in, (const float*)w_in, seg_in, S, pas, n_grp,  \
                                                    (K*)kslot[0], (float*)wslot[0], (K*)kslot[1], (float*)wslot[1], \
                                                    (float*)wimg, cnt, fp64_acc, err);                            \
    k_small_gather<K, float><<<S, 256, 0, s>>>((const K*)kslot[last], (const float*)wslot[last], cnt_last, S,      \
                                               (K*)keys_out, (float*)w_out, seg_off_out);                         \
  }
  if (KC == 0) { QIMAX_SMALL_PASSES(uint32_t) } else { QIMAX_SMALL_PASSES(uint64_t) }
#undef QIMAX_SMALL_PASSES
  prof_end(prof, s, ev, kKSmallPasses, 0.0);  // bytes: added by the caller once the counts are back
  return hipGetLastError();
}

hipError_t launch_count_expand(int KC, int WP, const void* keys, const void* w, uint64_t T_in, const Tiling& tl,
                               const PassArgs* pas, const uint32_t* seg_entry, uint64_t* status, uint32_t* ctr,
                               uint64_t epoch, uint64_t* img_seg, void* keys_out, void* w_out, uint64_t out_cap,
                               uint32_t* ghist, uint32_t n_pass, uint32_t hp_begin, uint32_t* err, hipStream_t s,
                               Prof* prof) {
  if (tl.n_blocks == 0) return hipErrorInvalidValue;  // a round with no input terms takes another path
  if (ghist && (hp_begin > n_pass || n_pass - hp_begin > kExpandHistPasses)) return hipErrorInvalidValue;
  hipEvent_t ev = prof_begin(prof, s, kKCountExpand);
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64)
      k_count_expand<K, 64><<<tl.n_blocks, kFuseBlock, 0, s>>>((const K*)keys, (const double*)w, tl, pas, seg_entry,
                                                               status, ctr, epoch, img_seg, (K*)keys_out,
                                                               (double*)w_out, out_cap, ghist, n_pass, hp_begin, err);
    else
      k_count_expand<K, 32><<<tl.n_blocks, kFuseBlock, 0, s>>>((const K*)keys, (const float*)w, tl, pas, seg_entry,
                                                               status, ctr, epoch, img_seg, (K*)keys_out,
                                                               (float*)w_out, out_cap, ghist, n_pass, hp_begin, err);
  });
  // bytes: every input term read; the images' bytes are added by the caller once known
  const double per = (4 << KC) + (WP == 64 ? 8 : 4);
  prof_end(prof, s, ev, kKCountExpand, per * (double)T_in);
  return hipGetLastError();
}

hipError_t launch_expand_small(int KC, int WP, const void* keys, const void* w, const uint64_t* seg_in, uint32_t S,
                               uint64_t T_in, const PassArgs* pas, const uint32_t* seg_entry, void* keys_out,
                               void* w_out, uint32_t* img_cnt, const TileJob2& tiles, uint32_t* err, hipStream_t s,
                               Prof* prof) {
  if (S == 0) return hipSuccess;
  hipEvent_t ev = prof_begin(prof, s, kKExpand);
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64)
      k_expand_small<K, 64><<<S, kSmallBlock, 0, s>>>((const K*)keys, (const double*)w, seg_in, S, pas, seg_entry,
                                                      (K*)keys_out, (double*)w_out, img_cnt, tiles.blk_begin,
                                                      tiles.blk_end, tiles.blk_seg, tiles.seg_blk, err);
    else
      k_expand_small<K, 32><<<S, kSmallBlock, 0, s>>>((const K*)keys, (const float*)w, seg_in, S, pas, seg_entry,
                                                      (K*)keys_out, (float*)w_out, img_cnt, tiles.blk_begin,
                                                      tiles.blk_end, tiles.blk_seg, tiles.seg_blk, err);
  });
  const double per = (4 << KC) + (WP == 64 ? 8 : 4);
  prof_end(prof, s, ev, kKExpand, per * (double)T_in);  // the images' bytes are added once known
  return hipGetLastError();
}

hipError_t launch_sort_pass(int KC, int WP, const void* keys_in, const void* w_in, void* keys_out, void* w_out,
                            uint64_t T, uint32_t shift, const Tiling& tl, uint64_t* hist, uint64_t* hist_off,
                            uint64_t* tmp, uint32_t* err, hipStream_t s, Prof* prof) {
  if (T == 0 || tl.n_blocks == 0) return hipSuccess;
  const uint64_t hsize = (uint64_t)kRadix * tl.n_blocks;
  const double kb = 4 << KC, wb = WP == 64 ? 8 : 4;
  QIMAX_DISPATCH_K(KC, {
    hipEvent_t ev = prof_begin(prof, s, kKSortHist);
    k_sort_hist<K><<<tl.n_blocks, kSortBlock, 0, s>>>((const K*)keys_in, shift, tl, hist, hsize, err);
    prof_end(prof, s, ev, kKSortHist, kb * (double)T + 8.0 * (double)hsize);
    hipError_t e = scan_impl<uint64_t>(hist, hist_off, hsize, tmp, s, prof);
    if (e != hipSuccess) return e;
    ev = prof_begin(prof, s, kKSortScatter);
    if (WP == 64)
      k_sort_scatter<K, double, false><<<tl.n_blocks, kSortBlock, 0, s>>>(
          (const K*)keys_in, (const double*)w_in, (K*)keys_out, (double*)w_out, T, shift, tl, hist_off, nullptr, 0,
          nullptr, nullptr, nullptr, 0, err);
    else
      k_sort_scatter<K, float, false><<<tl.n_blocks, kSortBlock, 0, s>>>(
          (const K*)keys_in, (const float*)w_in, (K*)keys_out, (float*)w_out, T, shift, tl, hist_off, nullptr, 0,
          nullptr, nullptr, nullptr, 0, err);
    prof_end(prof, s, ev, kKSortScatter, 2.0 * (kb + wb) * (double)T);
  });
  return hipGetLastError();
}

hipError_t launch_sort_sweep(int KC, int WP, void* const keys[2], void* const w[2], uint64_t T, uint32_t key_bits,
                             uint32_t p_begin, bool upsweep, const Tiling& tl, const uint64_t* seg_off,
                             uint32_t* ghist, uint64_t* status, uint32_t* tile_ctr, uint64_t* epoch, uint32_t* err,
                             int* cur, hipStream_t s, Prof* prof) {
  *cur = 0;
  if (T == 0 || tl.n_blocks == 0) return hipSuccess;
  const uint32_t n_pass = (key_bits + kRadixBits - 1) / kRadixBits;
  const double kb = 4 << KC, wb = WP == 64 ? 8 : 4;
  QIMAX_DISPATCH_K(KC, {
    hipEvent_t ev = nullptr;
    if (upsweep) {
      ev = prof_begin(prof, s, kKSortHist);
      k_sort_upsweep<K><<<tl.n_blocks, kSortBlock, 0, s>>>((const K*)keys[0], tl, n_pass, p_begin, ghist);
      prof_end(prof, s, ev, kKSortHist, kb * (double)T);
    }
    // the digit passes run back to back: one pair of events times them all (fewer event
    // records on the host), and the average launch is their time over the passes
    ev = prof_begin(prof, s, kKSortScatter);
    for (uint32_t p = p_begin; p < n_pass; ++p) {
      *epoch += 1;  // the caller keeps *epoch + n_pass below 2^16 (clearing status on wrap)
      const int c = *cur;
      if (WP == 64)
        k_sort_scatter<K, double, true><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys[c], (const double*)w[c], (K*)keys[c ^ 1], (double*)w[c ^ 1], T, 8u * p, tl, nullptr,
            ghist + (uint64_t)p * kRadix, n_pass * kRadix, seg_off, status, tile_ctr + (uint64_t)p * kXcds, *epoch,
            err);
      else
        k_sort_scatter<K, float, true><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys[c], (const float*)w[c], (K*)keys[c ^ 1], (float*)w[c ^ 1], T, 8u * p, tl, nullptr,
            ghist + (uint64_t)p * kRadix, n_pass * kRadix, seg_off, status, tile_ctr + (uint64_t)p * kXcds, *epoch,
            err);
      *cur ^= 1;
    }
    if (n_pass > p_begin)
      prof_end(prof, s, ev, kKSortScatter, 2.0 * (kb + wb) * (double)T * (n_pass - p_begin), n_pass - p_begin);
  });
  return hipGetLastError();
}

hipError_t launch_chunk_sort_merge(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in, void* keys_out,
                                   void* w_out, uint64_t T, const Tiling& tc, uint32_t n_pass, uint32_t m,
                                   const PassArgs* pas, const uint32_t* seg_entry, const ChunkOut& co, uint32_t* err,
                                   hipStream_t s, Prof* prof) {
  if (tc.n_blocks == 0) {
    if (co.img_cnt) return hipErrorInvalidValue;  // chunks are the segments: S is 0 too
    k_merge_publish<<<1, 256, 0, s>>>(tc, nullptr, co.seg_off_out, co.fin, err, 1);
    return hipGetLastError();
  }
  const double kb = 4 << KC, wb = WP == 64 ? 8 : 4;
  hipEvent_t ev = prof_begin(prof, s, kKChunkSort);
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64)
      k_chunk_sort<K, double><<<tc.n_blocks, kChunkBlock, 0, s>>>((const K*)keys_in, (const double*)w_in,
                                                                  (K*)keys_out, (double*)w_out, T, tc, n_pass, m, pas,
                                                                  seg_entry, fp64_acc, co, err);
    else
      k_chunk_sort<K, float><<<tc.n_blocks, kChunkBlock, 0, s>>>((const K*)keys_in, (const float*)w_in, (K*)keys_out,
                                                                 (float*)w_out, T, tc, n_pass, m, pas, seg_entry,
                                                                 fp64_acc, co, err);
  });
  // bytes: every image read; the kept terms' bytes are added by the caller once known
  prof_end(prof, s, ev, kKChunkSort, (kb + wb) * (double)T);
  ev = prof_begin(prof, s, kKChunkFinish);
  k_chunk_publish<<<1, kPublishBlock, 0, s>>>(tc, co.chunk_cnt, co.chunk_off, co.seg_off_out, co.fin, co.img_cnt, T,
                                              err);
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64)
      k_chunk_compact<K, double><<<tc.n_blocks, 256, 0, s>>>((const K*)co.tmp_keys, (const double*)co.tmp_w,
                                                             (K*)keys_out, (double*)w_out, tc, co.chunk_cnt,
                                                             co.chunk_start, co.chunk_off, T, err);
    else
      k_chunk_compact<K, float><<<tc.n_blocks, 256, 0, s>>>((const K*)co.tmp_keys, (const float*)co.tmp_w,
                                                            (K*)keys_out, (float*)w_out, tc, co.chunk_cnt,
                                                            co.chunk_start, co.chunk_off, T, err);
  });
  // bytes: the chunk counts and offsets (the moved runs are not known here)
  prof_end(prof, s, ev, kKChunkFinish, 12.0 * (double)tc.n_blocks);
  return hipGetLastError();
}

size_t dense_tile() { return (size_t)kDenseTile; }

hipError_t launch_dense_merge(int KC, int WP, const void* keys_in, const void* w_in, uint64_t T_img, const Tiling& tl,
                              uint64_t per_seg, uint32_t S, void* acc, double thr, uint32_t* ticket, uint64_t* status,
                              uint64_t epoch, uint64_t* tile_off, void* keys_out, void* w_out, uint64_t out_cap,
                              uint64_t* seg_off_out, const MergeFin& fin, uint32_t* err, hipStream_t s, Prof* prof) {
  if (KC != 0 || S == 0 || per_seg == 0) return hipErrorInvalidValue;  // 32-bit keys only (n <= 16)
  const uint64_t slots = (uint64_t)S * per_seg;
  const uint32_t tps = (uint32_t)((per_seg + kDenseTile - 1) / kDenseTile);
  const uint32_t n_tiles = tps * S;
  hipEvent_t ev = prof_begin(prof, s, kKDense);
  k_fill_u64<<<grid_for(slots, 256), 256, 0, s>>>((uint64_t*)acc, slots, 0ull);
  if (tl.n_blocks) {
    if (WP == 64)
      k_dense_scatter<uint32_t, double><<<tl.n_blocks, 256, 0, s>>>((const uint32_t*)keys_in, (const double*)w_in, tl,
                                                                    (unsigned long long*)acc, per_seg, err);
    else
      k_dense_scatter<uint32_t, float><<<tl.n_blocks, 256, 0, s>>>((const uint32_t*)keys_in, (const float*)w_in, tl,
                                                                   (unsigned long long*)acc, per_seg, err);
  }
  if (WP == 64)
    k_dense_compact<uint32_t, double><<<n_tiles, 256, 0, s>>>((const unsigned long long*)acc, per_seg, tps, n_tiles,
                                                              thr, ticket, status, epoch, tile_off, (uint32_t*)keys_out,
                                                              (double*)w_out, out_cap, err);
  else
    k_dense_compact<uint32_t, float><<<n_tiles, 256, 0, s>>>((const unsigned long long*)acc, per_seg, tps, n_tiles, thr,
                                                             ticket, status, epoch, tile_off, (uint32_t*)keys_out,
                                                             (float*)w_out, out_cap, err);
  // bytes: images read, every slot written (cleared), read back; the kept terms added later
  const double wb = WP == 64 ? 8 : 4;
  prof_end(prof, s, ev, kKDense, (4.0 + wb) * (double)T_img + 16.0 * (double)slots);
  k_dense_finish<<<1, 256, 0, s>>>(tile_off, tps, S, seg_off_out, fin, out_cap, err);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_fill_u64<<<grid_for(n, 256), 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_merge(int KC, int WP, int fp64_acc, const void* keys_in, const void* w_in, uint64_t T,
                        const Tiling& tl, const PassArgs* pas, const uint32_t* seg_entry, void* keys_out, void* w_out,
                        uint64_t out_cap, uint64_t* seg_off_out, uint32_t* blk_cnt, uint64_t* blk_off, uint64_t* tmp,
                        uint64_t* status, uint32_t* tile_ctr, uint64_t epoch, uint32_t* err, const MergeFin* fin,
                        hipStream_t s, Prof* prof) {
  if (tl.n_blocks == 0 && fin) {
    k_merge_publish<<<1, 256, 0, s>>>(tl, nullptr, seg_off_out, *fin, err, 1);
    return hipGetLastError();
  }
  if (tl.n_blocks == 0) {
    // no terms at all: every segment offset is zero
    k_zero_one<<<1, 1, 0, s>>>(blk_off);
    k_gather_u64_by_u32<<<grid_for(tl.n_segs + 1, 64), 64, 0, s>>>(blk_off, tl.seg_blk, seg_off_out,
                                                                   tl.n_segs + 1);
    return hipGetLastError();
  }
  const double kb = 4 << KC, wb = WP == 64 ? 8 : 4;
  QIMAX_DISPATCH_K(KC, {
    if (status) {  // single sweep
      if (!fin) k_fill_u32<<<1, 64, 0, s>>>(tile_ctr, 1, 0u);  // with fin: zeroed by the caller
      hipEvent_t ev = prof_begin(prof, s, kKMergeWrite);
      if (WP == 64)
        k_merge<K, double, 2><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const double*)w_in, tl, pas, seg_entry, fp64_acc, nullptr, blk_off, (K*)keys_out,
            (double*)w_out, out_cap, status, tile_ctr, epoch, err);
      else
        k_merge<K, float, 2><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const float*)w_in, tl, pas, seg_entry, fp64_acc, nullptr, blk_off, (K*)keys_out,
            (float*)w_out, out_cap, status, tile_ctr, epoch, err);
      // the written terms are added by the caller once their count is back on the host
      prof_end(prof, s, ev, kKMergeWrite, (kb + wb) * (double)T);
    } else {
      hipEvent_t ev = prof_begin(prof, s, kKMergeCount);
      if (WP == 64)
        k_merge<K, double, 0><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const double*)w_in, tl, pas, seg_entry, fp64_acc, blk_cnt, nullptr, nullptr, nullptr, 0,
            nullptr, nullptr, 0, err);
      else
        k_merge<K, float, 0><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const float*)w_in, tl, pas, seg_entry, fp64_acc, blk_cnt, nullptr, nullptr, nullptr, 0,
            nullptr, nullptr, 0, err);
      prof_end(prof, s, ev, kKMergeCount, (kb + wb) * (double)T);
      hipError_t e = scan_impl<uint32_t>(blk_cnt, blk_off, tl.n_blocks, tmp, s, prof);
      if (e != hipSuccess) return e;
      ev = prof_begin(prof, s, kKMergeWrite);
      if (WP == 64)
        k_merge<K, double, 1><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const double*)w_in, tl, pas, seg_entry, fp64_acc, blk_cnt, blk_off, (K*)keys_out,
            (double*)w_out, out_cap, nullptr, nullptr, 0, err);
      else
        k_merge<K, float, 1><<<tl.n_blocks, kSortBlock, 0, s>>>(
            (const K*)keys_in, (const float*)w_in, tl, pas, seg_entry, fp64_acc, blk_cnt, blk_off, (K*)keys_out,
            (float*)w_out, out_cap, nullptr, nullptr, 0, err);
      prof_end(prof, s, ev, kKMergeWrite, (kb + wb) * (double)T);
    }
  });
  if (fin)  // offsets and the packed readback area
    k_merge_publish<<<1, 256, 0, s>>>(tl, blk_off, seg_off_out, *fin, err, 0);
  else
    k_gather_u64_by_u32<<<grid_for(tl.n_segs + 1, 64), 64, 0, s>>>(blk_off, tl.seg_blk, seg_off_out, tl.n_segs + 1);
  return hipGetLastError();
}

// Device memory <- mapped host memory, 16 bytes per thread and step.
__global__ void k_pull(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_pull(const void* src, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16) return hipErrorInvalidValue;
  const uint64_t n16 = bytes / 16;
  k_pull<<<std::min<uint32_t>(grid_for(n16, 256), 256), 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_build_tables(int KC, const TableJob* jobs, uint32_t n_jobs, hipStream_t s, Prof* prof) {
  (void)prof;
  if (n_jobs == 0) return hipSuccess;
  QIMAX_DISPATCH_K(KC, { k_build_tables<K><<<dim3((uint32_t)sizeof(K), n_jobs), 256, 0, s>>>(jobs); });
  return hipGetLastError();
}

// Terms as the C-ABI hands them out: each key as n_words little-endian 64-bit words (the
// second word of a key of at most 8 bytes is 0), each weight as FP64.
template <typename K, typename W>
__global__ void __launch_bounds__(256) k_export(const K* __restrict__ keys, const W* __restrict__ w, uint64_t T,
                                                uint32_t n_words, uint64_t* __restrict__ words,
                                                double* __restrict__ wd) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= T) return;
  const K k = keys[i];
  if (n_words == 2) {
    words[2 * i] = (uint64_t)k;
    if constexpr (sizeof(K) > 8) words[2 * i + 1] = (uint64_t)(k >> 64);
    else words[2 * i + 1] = 0;
  } else {
    words[i] = (uint64_t)k;
  }
  wd[i] = (double)w[i];
}

hipError_t launch_export(int KC, int WP, const void* keys, const void* w, uint64_t T, uint32_t n_words,
                         uint64_t* words, double* wd, hipStream_t s) {
  if (T == 0) return hipSuccess;
  const uint64_t nb = (T + 255) / 256;
  if (nb > 0x7FFFFFFFull || (n_words != 1 && n_words != 2)) return hipErrorInvalidValue;
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64) k_export<K, double><<<(uint32_t)nb, 256, 0, s>>>((const K*)keys, (const double*)w, T, n_words, words, wd);
    else k_export<K, float><<<(uint32_t)nb, 256, 0, s>>>((const K*)keys, (const float*)w, T, n_words, words, wd);
  });
  return hipGetLastError();
}

hipError_t launch_init_many(int KC, int WP, void* keys, void* w, const uint32_t* nq, const uint64_t* dst,
                            uint32_t n_circ, hipStream_t s) {
  if (n_circ == 0) return hipSuccess;
  QIMAX_DISPATCH_K(KC, {
    if (WP == 64) k_init_many<K, double><<<n_circ, 64, 0, s>>>((K*)keys, (double*)w, nq, dst, n_circ);
    else k_init_many<K, float><<<n_circ, 64, 0, s>>>((K*)keys, (float*)w, nq, dst, n_circ);
  });
  return hipGetLastError();
}

// Even blocks build tiling j0, odd blocks tiling j1, each tiling in gridDim/2 parts (see
// make_tiling_part); j0's lead part also stores the offsets in img_seg.
constexpr uint32_t kTileLdsSegs = 2048;  // segments a tiling block keeps in LDS (more: one block)

// Part `part` of n_parts blocks building one tiling (segment-aligned tiles of at most job.tile
// elements; cap tiles written, the ones past the actual count empty) from the segment
// offsets so[s] = off[seg_in[s]] (so[s] = seg_in[s] when off is null). Every part scans the
// per-segment tile counts itself, keeping them and the offsets in LDS (n_parts must be 1
// when S exceeds kTileLdsSegs), and writes tiles part*256 + i, stepping by n_parts*256;
// part 0 also writes seg_blk, n_dev, xrange, the offsets to img_seg (unless null) and the
// error bits.
__device__ __forceinline__ void make_tiling_part(const uint64_t* __restrict__ off, const uint64_t* __restrict__ seg_in,
                                                 uint32_t S, uint64_t* __restrict__ img_seg, const TileJob2& job,
                                                 uint64_t limit, uint32_t* err, uint32_t part, uint32_t n_parts) {
  __shared__ uint32_t sblk[kTileLdsSegs + 1];
  __shared__ uint64_t sso[kTileLdsSegs + 1];
  __shared__ uint64_t sh[4];
  __shared__ uint64_t carry_sh;
  const uint64_t tile = job.tile;
  const uint32_t cap = job.cap;
  const bool in_lds = S <= kTileLdsSegs, lead = part == 0;
  auto so = [&](uint32_t s) { return off ? off[seg_in[s]] : seg_in[s]; };
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (uint32_t base = 0; base < S; base += 256) {
    const uint32_t s = base + threadIdx.x;
    uint64_t len = 0;
    if (s < S) {
      const uint64_t a = so(s), b = so(s + 1);
      len = b - a;
      if (in_lds) {
        sso[s] = a;
        if (s + 1 == S) sso[S] = b;
      }
      if (lead && img_seg) {
        img_seg[s] = a;
        if (s + 1 == S) img_seg[S] = b;
      }
    }
    const uint64_t nt = (len + tile - 1) / tile;
    uint64_t tot;
    const uint64_t pre = block_excl_scan<256>(nt, sh, &tot);
    const uint64_t carry = carry_sh;
    if (s < S) {
      if (in_lds) sblk[s] = (uint32_t)(carry + pre);
      if (lead) job.seg_blk[s] = (uint32_t)(carry + pre);
    }
    __syncthreads();
    if (threadIdx.x == 0) carry_sh = carry + tot;
    __syncthreads();
  }
  if (S == 0 && threadIdx.x == 0) {
    if (in_lds) sso[0] = so(0);
    if (lead && img_seg) img_seg[0] = so(0);
  }
  const uint64_t total_img = so(S);
  const uint32_t total = (uint32_t)min<uint64_t>(carry_sh, cap);
  if (lead && threadIdx.x == 0) {
    // more tiles or elements than the capacity: the bound was not an upper bound (tiles are
    // clamped below so that nothing reads past the buffers; the pass reports the error)
    if (carry_sh > cap || total_img > limit) atomicOr(err, kErrIndex | kErrFanout);
    job.seg_blk[S] = total;
    *job.n_dev = total;
  }
  if (in_lds && threadIdx.x == 0) sblk[S] = total;
  __syncthreads();
  const uint32_t* blk_of = in_lds ? sblk : job.seg_blk;
  if (lead && threadIdx.x <= kXcds)
    job.xrange[threadIdx.x] =
        threadIdx.x == kXcds
            ? total
            : min(total, seg_boundary_at_or_after(blk_of, S,
                                                  (uint32_t)(((uint64_t)threadIdx.x * total + kXcds - 1) / kXcds)));
  for (uint32_t t = part * 256 + threadIdx.x; t < cap; t += n_parts * 256) {
    if (t < total) {
      uint32_t lo = 0, hi = S;  // last segment s with seg_blk[s] <= t (non-empty)
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (blk_of[mid] <= t) lo = mid; else hi = mid;
      }
      const uint64_t s0 = in_lds ? sso[lo] : so(lo), s1 = in_lds ? sso[lo + 1] : so(lo + 1);
      const uint64_t b0 = s0 + (uint64_t)(t - blk_of[lo]) * tile;
      job.blk_begin[t] = min(b0, limit);
      job.blk_end[t] = min(min(b0 + tile, s1), limit);
      job.blk_seg[t] = lo;
    } else {
      job.blk_begin[t] = 0;
      job.blk_end[t] = 0;
      job.blk_seg[t] = 0;
    }
  }
}

__global__ void __launch_bounds__(256) k_make_tiles2(const uint64_t* __restrict__ off,
                                                     const uint64_t* __restrict__ seg_in, uint32_t S,
                                                     uint64_t* __restrict__ img_seg, TileJob2 j0, TileJob2 j1,
                                                     uint64_t limit, uint32_t* err) {
  const uint32_t part = blockIdx.x >> 1, n_parts = gridDim.x >> 1;
  if ((blockIdx.x & 1) == 0) make_tiling_part(off, seg_in, S, img_seg, j0, limit, err, part, n_parts);
  else make_tiling_part(off, seg_in, S, nullptr, j1, limit, err, part, n_parts);
}

// The first launch of a round. Blocks [0, n_tparts) build the tiling of the input terms (see
// make_tiling_part; segments at seg_in[0..S], T terms), block 0 after clearing the error
// word. The other blocks clear the tile counters and digit histograms and copy the round's
// descriptors (n16 16-byte words) from mapped host memory to the device.
__global__ void __launch_bounds__(256) k_round_start(const uint4* __restrict__ blob_host, uint4* __restrict__ blob_dev,
                                                     uint64_t n16, uint32_t* __restrict__ err,
                                                     uint32_t* __restrict__ ctr, uint32_t n_ctr,
                                                     uint32_t* __restrict__ ghist, uint64_t nh,
                                                     const uint64_t* __restrict__ seg_in, uint32_t S, TileJob2 job,
                                                     uint64_t T, uint32_t n_tparts) {
  if (blockIdx.x < n_tparts) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0u;
    make_tiling_part(nullptr, seg_in, S, nullptr, job, T, err, blockIdx.x, n_tparts);
    return;
  }
  const uint64_t stride = (uint64_t)(gridDim.x - n_tparts) * blockDim.x;
  const uint64_t i0 = (uint64_t)(blockIdx.x - n_tparts) * blockDim.x + threadIdx.x;
  for (uint64_t i = i0; i < n_ctr; i += stride) ctr[i] = 0u;
  for (uint64_t i = i0; i < nh; i += stride) ghist[i] = 0u;
  for (uint64_t i = i0; i < n16; i += stride) blob_dev[i] = blob_host[i];
}

// Clears the round's error word, tile counters and digit histograms (one launch).
__global__ void k_round_prep(uint32_t* __restrict__ err, uint32_t* __restrict__ ctr, uint32_t n_ctr,
                             uint32_t* __restrict__ ghist, uint64_t nh) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *err = 0u;
  if (i < n_ctr) ctr[i] = 0u;
  for (uint64_t j = i; j < nh; j += (uint64_t)gridDim.x * blockDim.x) ghist[j] = 0u;
}

__global__ void k_copy_u64(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

// Blocks building one tiling of cap tiles: about 1024 tiles each, at most 64, one when the
// segments do not fit a block's LDS.
static uint32_t tiling_parts(uint32_t S, uint32_t cap) {
  if (S > kTileLdsSegs) return 1;
  return std::min<uint32_t>(cap / 1024 + 1, 64);
}

hipError_t launch_make_tiles2(const uint64_t* off, const uint64_t* seg_in, uint32_t S, uint64_t* img_seg,
                              const TileJob2& j0, const TileJob2& j1, uint64_t limit, uint32_t* err, hipStream_t s) {
  k_make_tiles2<<<2 * tiling_parts(S, std::max(j0.cap, j1.cap)), 256, 0, s>>>(off, seg_in, S, img_seg, j0, j1,
                                                                               limit, err);
  return hipGetLastError();
}

hipError_t launch_round_start(const void* blob_host, void* blob_dev, size_t blob_bytes, uint32_t* err, uint32_t* ctr,
                              uint32_t n_ctr, uint32_t* ghist, uint64_t nh, const uint64_t* seg_in, uint32_t S,
                              const TileJob2& job, uint64_t T, hipStream_t s) {
  if (blob_bytes % 16 || ((uintptr_t)blob_host | (uintptr_t)blob_dev) % 16) return hipErrorInvalidValue;
  const uint64_t n16 = blob_bytes / 16;
  const uint64_t work = std::max<uint64_t>(std::max<uint64_t>(nh, n16), n_ctr);
  const uint32_t g = (uint32_t)std::min<uint64_t>(grid_for(std::max<uint64_t>(work, 1), 256), 1024);
  const uint32_t tp = tiling_parts(S, job.cap);
  k_round_start<<<tp + g, 256, 0, s>>>((const uint4*)blob_host, (uint4*)blob_dev, n16, err, ctr, n_ctr, ghist, nh,
                                       seg_in, S, job, T, tp);
  return hipGetLastError();
}

hipError_t launch_round_prep(uint32_t* err, uint32_t* ctr, uint32_t n_ctr, uint32_t* ghist, uint64_t nh,
                             hipStream_t s) {
  const uint64_t n = std::max<uint64_t>(nh, n_ctr);
  k_round_prep<<<(uint32_t)std::min<uint64_t>(grid_for(std::max<uint64_t>(n, 1), 256), 1024), 256, 0, s>>>(
      err, ctr, n_ctr, ghist, nh);
  return hipGetLastError();
}

hipError_t launch_copy_u64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_copy_u64<<<std::min<uint64_t>(grid_for(n, 256), 65536), 256, 0, s>>>(in, out, n);
  return hipGetLastError();
}

hipError_t launch_weights_to_f64(int WP, const void* w, double* out, uint64_t T, hipStream_t s, Prof* prof) {
  (void)prof;
  if (T == 0) return hipSuccess;
  if (WP == 64) k_weights_to_f64<64><<<grid_for(T, 256), 256, 0, s>>>((const double*)w, out, T);
  else k_weights_to_f64<32><<<grid_for(T, 256), 256, 0, s>>>((const float*)w, out, T);
  return hipGetLastError();
}

hipError_t launch_compose_ptm(const uint8_t* gate, const double* theta, const uint32_t* idx,
                              const uint32_t* chain_off, uint32_t n_chains, double* ptm_out, hipStream_t s,
                              Prof* prof) {
  if (n_chains == 0) return hipSuccess;
  hipEvent_t ev = prof_begin(prof, s, kKCompose);
  k_compose_ptm<<<grid_for(n_chains, kComposeWaves), 64 * kComposeWaves, 0, s>>>(gate, theta, idx, chain_off,
                                                                                    n_chains, ptm_out);
  prof_end(prof, s, ev, kKCompose, 0.0);
  return hipGetLastError();
}

}  // namespace qimax
