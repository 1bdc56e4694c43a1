// Readout kernels for gfx950, off the propagation loop: the generators' keys as x/z bit
// words, a per-generator comparison of two term lists (the stated error of an FP32 result
// against an FP64 one), and expectation values <psi|P|psi> = Tr(rho P) with
// rho = 2^-n prod_j (I + G_j) (paper, eq. (2)) from a device statevector: a random vector is
// projected onto the common +1 eigenspace of the generators, one (I + G_j)/2 at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "qimax_internal.h"

namespace qimax {
namespace {

inline uint32_t blocks_for(uint64_t n, uint32_t block) { return (uint32_t)((n + block - 1) / block); }

// -------------------------------------------------------------------------- x / z words
// Base-4 digit d of qubit q sits at bit 2(n-1-q) of a key; bit q of x is set for X and Y,
// bit q of z for Y and Z.
template <typename K>
__global__ void k_keys_to_xz(const K* __restrict__ keys, uint64_t T, uint32_t n, uint64_t* __restrict__ x,
                             uint64_t* __restrict__ z) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const K k = keys[i];
  uint64_t xs = 0, zs = 0;
  for (uint32_t q = 0; q < n; ++q) {
    const uint32_t d = (uint32_t)(k >> (2 * (n - 1 - q))) & 3u;
    xs |= (uint64_t)(d == 1u || d == 2u) << q;
    zs |= (uint64_t)(d >= 2u) << q;
  }
  x[i] = xs;
  z[i] = zs;
}

// ----------------------------------------------------------------------------- compare
// Tiles of one side's segments (each tile inside one segment). For every element of side
// `a`, its key is searched in the same segment of side `b`: matched pairs add (wa - wb)^2,
// unmatched ones wa^2 (the other side's weight is 0). With count_ref set the pass is the
// second one (a = the reference list): it adds every wa^2 to the reference norm and only the
// unmatched elements to the difference. A key on whose side |w| > tau differs is counted.
constexpr int kCmpBlock = 256, kCmpItems = 16, kCmpTile = kCmpBlock * kCmpItems;

template <typename K>
__device__ __forceinline__ uint64_t lower_bound_k(const K* __restrict__ a, uint64_t lo, uint64_t hi, K key) {
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K, typename WA, typename WB>
__global__ void __launch_bounds__(kCmpBlock)
k_compare(const K* __restrict__ ka, const WA* __restrict__ wa, const K* __restrict__ kb, const WB* __restrict__ wb,
          const uint64_t* __restrict__ b_off, const uint64_t* __restrict__ t_begin, const uint64_t* __restrict__ t_end,
          const uint32_t* __restrict__ t_seg, int count_ref, double tau, double* __restrict__ acc,
          unsigned long long* __restrict__ cnt) {
  __shared__ uint64_t rng[2];
  __shared__ double red[2][kCmpBlock / 64];
  __shared__ unsigned long long redc[kCmpBlock / 64];
  const uint32_t t = blockIdx.x, s = t_seg[t];
  const uint64_t a0 = t_begin[t], a1 = t_end[t];
  const uint64_t lo = b_off[s], hi = b_off[s + 1];
  // the part of b's segment that can hold this tile's keys
  if (threadIdx.x == 0) rng[0] = lower_bound_k(kb, lo, hi, ka[a0]);
  if (threadIdx.x == 1) rng[1] = lower_bound_k(kb, lo, hi, ka[a1 - 1]) + 1;
  __syncthreads();
  const uint64_t r0 = rng[0], r1 = min(rng[1], hi);
  double d2 = 0.0, ref2 = 0.0;
  unsigned long long nd = 0;
  for (int r = 0; r < kCmpItems; ++r) {
    const uint64_t i = a0 + (uint64_t)r * kCmpBlock + threadIdx.x;
    if (i >= a1) break;
    const K key = ka[i];
    const double x = (double)wa[i];
    const uint64_t p = lower_bound_k(kb, r0, r1, key);
    const bool hit = p < r1 && kb[p] == key;
    const double y = hit ? (double)wb[p] : 0.0;
    if (count_ref) {
      ref2 += x * x;
      if (!hit) {
        d2 += x * x;
        nd += fabs(x) > tau;
      }
    } else {
      d2 += (x - y) * (x - y);
      nd += (fabs(x) > tau) != (fabs(y) > tau);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    ref2 += __shfl_xor(ref2, o, 64);
    nd += __shfl_xor(nd, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = d2;
    red[1][wid] = ref2;
    redc[wid] = nd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sd = 0.0, sr = 0.0;
    unsigned long long sc = 0;
    for (int w = 0; w < kCmpBlock / 64; ++w) {
      sd += red[0][w];
      sr += red[1][w];
      sc += redc[w];
    }
    atomicAdd(&acc[2 * s], sd);
    if (count_ref) atomicAdd(&acc[2 * s + 1], sr);
    atomicAdd(&cnt[s], sc);
  }
}

// ---------------------------------------------------------------------- statevector
// Basis state index i: qubit q is bit (n-1-q). A Pauli string with x mask xm, z mask zm
// (over those bits) and ny letters Y acts as P|i> = i^ny (-1)^{popcount(i & zm)} |i ^ xm>,
// so (P v)[k] = i^ny (-1)^{popcount((k ^ xm) & zm)} v[k ^ xm].

__device__ __forceinline__ uint64_t mix64(uint64_t x) {  // splitmix64 finaliser
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_sv_random(double2* __restrict__ v, uint64_t D, uint64_t seed) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  const uint64_t a = mix64(seed ^ (2 * i)), b = mix64(seed ^ (2 * i + 1));
  v[i] = make_double2((double)(a >> 11) * 0x1.0p-53 - 0.5, (double)(b >> 11) * 0x1.0p-53 - 0.5);
}

// out[k] = sum over terms t of c_t (-1)^{popcount((k ^ x_t) & z_t)} v[k ^ x_t], the terms'
// masks and complex coefficients (w_t i^{ny_t}) staged through LDS in chunks.
constexpr int kSvBlock = 256, kSvChunk = 256;
__global__ void __launch_bounds__(kSvBlock) k_sv_apply(const double2* __restrict__ v, double2* __restrict__ out,
                                                      uint64_t D, const uint64_t* __restrict__ xm,
                                                      const uint64_t* __restrict__ zm, const double2* __restrict__ cf,
                                                      uint64_t T) {
  __shared__ uint64_t sx[kSvChunk], sz[kSvChunk];
  __shared__ double2 sc[kSvChunk];
  const uint64_t k = (uint64_t)blockIdx.x * kSvBlock + threadIdx.x;
  double re = 0.0, im = 0.0;
  for (uint64_t t0 = 0; t0 < T; t0 += kSvChunk) {
    const uint32_t nt = (uint32_t)min<uint64_t>(kSvChunk, T - t0);
    __syncthreads();
    if (threadIdx.x < nt) {
      sx[threadIdx.x] = xm[t0 + threadIdx.x];
      sz[threadIdx.x] = zm[t0 + threadIdx.x];
      sc[threadIdx.x] = cf[t0 + threadIdx.x];
    }
    __syncthreads();
    if (k < D) {
      for (uint32_t u = 0; u < nt; ++u) {
        const uint64_t src = k ^ sx[u];
        const double2 a = v[src];
        const double2 c = sc[u];
        const double sg = (__popcll(src & sz[u]) & 1) ? -1.0 : 1.0;
        re += sg * (c.x * a.x - c.y * a.y);
        im += sg * (c.x * a.y + c.y * a.x);
      }
    }
  }
  if (k < D) out[k] = make_double2(re, im);
}

// v = (v + g) / 2, the projection (I + G) / 2 applied given g = G v.
__global__ void k_sv_half_sum(double2* __restrict__ v, const double2* __restrict__ g, uint64_t D) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D) return;
  const double2 a = v[i], b = g[i];
  v[i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
}

// acc[0] += sum |v|^2, acc[1] += Re sum conj(v) (P v), acc[2] += Im of it (one string), or
// with zall set acc[1 + q] += sum |v_i|^2 (1 - 2 bit_q(i)) for every qubit q (<Z_q>, unnormalised).
constexpr uint32_t kSvMaxQubits = 32;  // statevectors hold at most 2^kSvMaxQubits amplitudes
__global__ void __launch_bounds__(kSvBlock) k_sv_reduce(const double2* __restrict__ v, uint64_t D, uint32_t n,
                                                       uint64_t xm, uint64_t zm, double2 c, int zall,
                                                       double* __restrict__ acc) {
  __shared__ double sh[kSvBlock / 64][1 + kSvMaxQubits];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double nv = 0.0, pr = 0.0, pi = 0.0;
  double zq[kSvMaxQubits];
  const uint32_t nz = zall ? min(n, kSvMaxQubits) : 0u;
#pragma unroll
  for (uint32_t q = 0; q < kSvMaxQubits; ++q) zq[q] = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * kSvBlock + threadIdx.x; i < D; i += (uint64_t)gridDim.x * kSvBlock) {
    const double2 a = v[i];
    const double p2 = a.x * a.x + a.y * a.y;
    nv += p2;
    if (zall) {
#pragma unroll
      for (uint32_t q = 0; q < kSvMaxQubits; ++q)
        if (q < nz) zq[q] += ((i >> (n - 1 - q)) & 1u) ? -p2 : p2;
    } else {
      const uint64_t src = i ^ xm;
      const double2 b = v[src];
      const double sg = (__popcll(src & zm) & 1) ? -1.0 : 1.0;
      const double br = sg * (c.x * b.x - c.y * b.y), bi = sg * (c.x * b.y + c.y * b.x);  // (P v)[i]
      pr += a.x * br + a.y * bi;
      pi += a.x * bi - a.y * br;
    }
  }
  auto wsum = [](double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
  };
  nv = wsum(nv);
  if (lane == 0) sh[wid][0] = nv;
  if (zall) {
#pragma unroll
    for (uint32_t q = 0; q < kSvMaxQubits; ++q) {
      const double s = wsum(zq[q]);
      if (lane == 0 && q < nz) sh[wid][1 + q] = s;
    }
  } else {
    pr = wsum(pr);
    pi = wsum(pi);
    if (lane == 0) {
      sh[wid][1] = pr;
      sh[wid][2] = pi;
    }
  }
  __syncthreads();
  const uint32_t nacc = zall ? 1 + nz : 3;
  if (threadIdx.x < nacc) {
    double s = 0.0;
    for (int w = 0; w < kSvBlock / 64; ++w) s += sh[w][threadIdx.x];
    atomicAdd(&acc[threadIdx.x], s);
  }
}

// Terms of a generator as statevector operators: x / z masks over the basis-index bits and
// the coefficient w * i^(number of Y letters).
template <typename K, typename W>
__global__ void k_sv_terms(const K* __restrict__ keys, const W* __restrict__ w, uint64_t T, uint32_t n,
                           uint64_t* __restrict__ xm, uint64_t* __restrict__ zm, double2* __restrict__ cf) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const K k = keys[i];
  uint64_t xs = 0, zs = 0;
  uint32_t ny = 0;
  for (uint32_t q = 0; q < n; ++q) {
    const uint32_t d = (uint32_t)(k >> (2 * (n - 1 - q))) & 3u;
    const uint64_t bit = 1ull << (n - 1 - q);
    if (d == 1u || d == 2u) xs |= bit;
    if (d >= 2u) zs |= bit;
    ny += d == 2u;
  }
  const double v = (double)w[i];
  const double2 ph[4] = {make_double2(v, 0.0), make_double2(0.0, v), make_double2(-v, 0.0), make_double2(0.0, -v)};
  xm[i] = xs;
  zm[i] = zs;
  cf[i] = ph[ny & 3u];
}

}  // namespace

hipError_t launch_sv_terms(int KC, int WP, const void* keys, const void* w, uint64_t T, uint32_t n, uint64_t* xm,
                           uint64_t* zm, void* cf, hipStream_t s) {
  if (T == 0) return hipSuccess;
  const uint32_t g = blocks_for(T, 256);
#define QIMAX_SVT(K)                                                                                              \
  do {                                                                                                            \
    if (WP == 64) k_sv_terms<K, double><<<g, 256, 0, s>>>((const K*)keys, (const double*)w, T, n, xm, zm, (double2*)cf); \
    else k_sv_terms<K, float><<<g, 256, 0, s>>>((const K*)keys, (const float*)w, T, n, xm, zm, (double2*)cf);  \
  } while (0)
  if (KC == 0) QIMAX_SVT(uint32_t);
  else if (KC == 1) QIMAX_SVT(uint64_t);
  else QIMAX_SVT(unsigned __int128);
#undef QIMAX_SVT
  return hipGetLastError();
}

hipError_t launch_keys_to_xz(int KC, const void* keys, uint64_t T, uint32_t n, uint64_t* x, uint64_t* z,
                             hipStream_t s) {
  if (T == 0) return hipSuccess;
  if (KC == 0) k_keys_to_xz<uint32_t><<<blocks_for(T, 256), 256, 0, s>>>((const uint32_t*)keys, T, n, x, z);
  else if (KC == 1) k_keys_to_xz<uint64_t><<<blocks_for(T, 256), 256, 0, s>>>((const uint64_t*)keys, T, n, x, z);
  else
    k_keys_to_xz<unsigned __int128><<<blocks_for(T, 256), 256, 0, s>>>((const unsigned __int128*)keys, T, n, x, z);
  return hipGetLastError();
}

size_t compare_tile() { return (size_t)kCmpTile; }

// Device memory of qimax_compare_noalloc (the comparison's tile arrays, accumulators and
// counters), held by every GPU the library runs on until the process ends. Host code never
// passes the array's name to a kernel or copy: it uses the address hipGetSymbolAddress
// returns for the current device.
constexpr size_t kCompareScratchBytes = (size_t)4 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) uint8_t scratch[kCompareScratchBytes];

hipError_t compare_scratch(int device, void** ptr, size_t* bytes) {
  static std::mutex mu;
  static void* addr[kScratchDevices] = {};
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  *bytes = kCompareScratchBytes;
  return hipSuccess;
}

hipError_t launch_compare(int KC, int WPa, int WPb, const void* ka, const void* wa, const void* kb, const void* wb,
                          const uint64_t* b_off, const uint64_t* t_begin, const uint64_t* t_end, const uint32_t* t_seg,
                          uint32_t n_tiles, int count_ref, double tau, double* acc, unsigned long long* cnt,
                          hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
#define QIMAX_CMP(K, WA, WB)                                                                                     \
  k_compare<K, WA, WB><<<n_tiles, kCmpBlock, 0, s>>>((const K*)ka, (const WA*)wa, (const K*)kb, (const WB*)wb, \
                                                      b_off, t_begin, t_end, t_seg, count_ref, tau, acc, cnt)
#define QIMAX_CMP_W(K)                                      \
  do {                                                      \
    if (WPa == 64 && WPb == 64) QIMAX_CMP(K, double, double); \
    else if (WPa == 64) QIMAX_CMP(K, double, float);          \
    else if (WPb == 64) QIMAX_CMP(K, float, double);          \
    else QIMAX_CMP(K, float, float);                          \
  } while (0)
  if (KC == 0) QIMAX_CMP_W(uint32_t);
  else if (KC == 1) QIMAX_CMP_W(uint64_t);
  else QIMAX_CMP_W(unsigned __int128);
#undef QIMAX_CMP_W
#undef QIMAX_CMP
  return hipGetLastError();
}

hipError_t launch_sv_random(void* v, uint64_t D, uint64_t seed, hipStream_t s) {
  k_sv_random<<<blocks_for(D, 256), 256, 0, s>>>((double2*)v, D, seed);
  return hipGetLastError();
}

hipError_t launch_sv_project(void* v, void* tmp, uint64_t D, const uint64_t* xm, const uint64_t* zm, const void* cf,
                             uint64_t T, hipStream_t s) {
  k_sv_apply<<<blocks_for(D, kSvBlock), kSvBlock, 0, s>>>((const double2*)v, (double2*)tmp, D, xm, zm,
                                                          (const double2*)cf, T);
  k_sv_half_sum<<<blocks_for(D, 256), 256, 0, s>>>((double2*)v, (const double2*)tmp, D);
  return hipGetLastError();
}

hipError_t launch_sv_reduce(const void* v, uint64_t D, uint32_t n, uint64_t xm, uint64_t zm, double c_re,
                            double c_im, int zall, double* acc, hipStream_t s) {
  const uint32_t grid = (uint32_t)std::min<uint64_t>(blocks_for(D, kSvBlock), 4096);
  k_sv_reduce<<<grid, kSvBlock, 0, s>>>((const double2*)v, D, n, xm, zm, make_double2(c_re, c_im), zall, acc);
  return hipGetLastError();
}

}  // namespace qimax
