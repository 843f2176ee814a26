// Global operators (Table 2): operators that read every pixel of an image
// and produce a few values.  Each kernel streams the image once in 16-byte
// chunks (a row split into chunks across the 256 threads of a work-group,
// four rows a grid size apart loaded together, so that every lane has four
// independent loads in flight), reduces inside the wave with lane
// exchanges, and combines work-groups with one global atomic per wave (per
// bin for the histogram).  The caller's result buffer is
// initialised by a small kernel in the same stream, so the sequence can be
// captured into a HIP graph.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <mutex>

#include "dev_reduce.hpp"
#include "gen_abi.h"
#include "global.h"
#include "hvx_desc.h"

namespace hvx {

constexpr int kGThreads = 256;

// Launch shapes, measured on a 16384 x 16384 image.  The histogram combines
// work-groups through 256 different counters and runs best on many 256-thread
// groups with two rows in flight.  Min/max and the sums combine through two
// words each: same-address atomics serialise, so those kernels reduce a
// whole 1024-thread group in LDS first and launch one group per CU.
constexpr int kRThreads = 1024;
constexpr int kRGroups = 256;
static_assert(kRGroups <= kMMSubKeys, "one counting key per group");

static int global_grid(const GlobalImg& im, int rows_in_flight, int cap) {
  const int g = (im.h + rows_in_flight - 1) / rows_in_flight;
  return g < cap ? g : cap;
}

// Calls f(chunk, valid elements) for every 16-byte chunk of the image
// (PER elements per chunk) that this thread of an NT-thread group reads.
// Rows y, y + G, ..., y + (K - 1) G (G the grid size) are loaded together;
// together the work-groups cover every row once.
template <int PER, int NT, int K, class F>
__device__ __forceinline__ void stream_image(const GlobalImg& im, F&& f) {
  const int G = gridDim.x;
  const int chunks = (im.w + PER - 1) / PER;
  for (int y = blockIdx.x; y < im.h; y += K * G) {
    for (int c = threadIdx.x; c < chunks; c += NT) {
      uint4 q[K];
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (y + k * G < im.h) q[k] = *(const uint4*)(im.base + (size_t)(y + k * G) * im.pitch + 16 * c);
      const int n = min(PER, im.w - PER * c);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (y + k * G < im.h) f(q[k], n);
    }
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int n, uint32_t a, uint32_t b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i == 0 ? a : b;
}

// ---- histogram of a U8 image ------------------------------------------------
// Bin of value v: (v - offset) * num_bins / range for offset <= v < offset +
// range, none otherwise.  With y = (v - offset) * num_bins * 256 (mod 2^32),
// formed as one 24-bit multiply-add v * B + D, the bin is the high word of
// y * m for m = ceil(2^24 / range) (0 for range 1): y and m fit 24 bits, so
// both products run on the full-rate 24-bit multiplier, and the quotient is
// exact because (v - offset) * num_bins * (m * range - 2^24) < 2^16 * 2^8.
// v lies in the interval exactly when y < R = range * num_bins * 256 (below
// the offset y wraps past 2^32 - 2^24).  The 256-bin histogram over [0, 256)
// takes the byte itself.  Pixels outside the interval, and the bytes past
// the row's end in its last chunk, go to a spare counter (index 256), so that
// every lane adds for every byte without a branch.  Each wave counts into its
// own LDS sub-histogram, held as kCopies interleaved copies (copy c of bin b
// at word b * kCopies + c, lane l adding to copy l mod kCopies): lanes that
// draw the same bin, or bins in the same bank, collide less (measured on
// uniform random bytes: 78 / 71 / 66 / 66 us for 1 / 2 / 4 / 8 copies).
struct HistBins {
  uint32_t B, D, R, m;
};

template <bool kIdentity>
__global__ __launch_bounds__(kGThreads) void k_histogram(GlobalImg im, int num_bins, HistBins hb,
                                                         uint32_t* __restrict__ counts) {
  constexpr int kSlots = 257, kCopies = 4;
  __shared__ uint32_t sub[kGThreads / 64][kSlots * kCopies];
  const int t = threadIdx.x, wv = t >> 6;
  for (int k = t; k < (kGThreads / 64) * kSlots * kCopies; k += kGThreads) (&sub[0][0])[k] = 0;
  __syncthreads();
  uint32_t* mine = sub[wv] + (t & (kCopies - 1));
  const uint32_t B = hb.B & 0xFFFFFFu, m = hb.m & 0xFFFFFFu;
  stream_image<16, kGThreads, 2>(im, [&](const uint4& q, int n) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t v = (wd[k >> 2] >> (8 * (k & 3))) & 0xFFu;
      uint32_t b;
      if constexpr (kIdentity) {
        b = k < n ? v : 256u;
      } else {
        const uint32_t y = v * B + hb.D;
        const uint32_t h = (uint32_t)(((uint64_t)(y & 0xFFFFFFu) * m) >> 32);
        b = (k < n && y < hb.R) ? h : 256u;
      }
      atomicAdd(&mine[b * kCopies], 1u);
    }
  });
  __syncthreads();
  for (int b = t; b < num_bins; b += kGThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kGThreads / 64; ++w)
#pragma unroll
      for (int c = 0; c < kCopies; ++c) s += sub[w][b * kCopies + c];
    if (s) atomicAdd(&counts[b], s);
  }
}

hipError_t launch_histogram(const GlobalImg& im, int num_bins, int offset, int range, uint32_t* counts,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((num_bins + 255) / 256), dim3(256), 0, s, counts, num_bins, 0u, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || im.w <= 0 || im.h <= 0) return e;
  HistBins hb;
  hb.B = (uint32_t)num_bins << 8;
  hb.D = 0u - (uint32_t)offset * hb.B;
  hb.R = (uint32_t)range * hb.B;
  hb.m = range == 1 ? 0u : (uint32_t)(((1u << 24) + (uint32_t)range - 1) / (uint32_t)range);
  const dim3 grid(global_grid(im, 2, 2048));
  if (offset == 0 && range == 256 && num_bins == 256)
    hipLaunchKernelGGL(k_histogram<true>, grid, dim3(kGThreads), 0, s, im, num_bins, hb, counts);
  else
    hipLaunchKernelGGL(k_histogram<false>, grid, dim3(kGThreads), 0, s, im, num_bins, hb, counts);
  return hipGetLastError();
}

// ---- histogram equalisation of a U8 image ----------------------------------------
// From the 256-bin histogram: cdf(v) by an LDS scan, cdf_min the cdf at the
// first nonzero bin, and lut[v] = round((cdf(v) - cdf_min) * 255 / (N -
// cdf_min)) clamped to 0..255, or v itself for an image of one value.
__global__ __launch_bounds__(256) void k_eq_lut(const uint32_t* __restrict__ hist, uint8_t* __restrict__ lut,
                                                 long long n) {
  __shared__ unsigned long long cdf[256];
  __shared__ int first;
  const int t = threadIdx.x;
  if (t == 0) first = 256;
  cdf[t] = hist[t];
  __syncthreads();
  if (hist[t] != 0) atomicMin(&first, t);
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scan
    const unsigned long long add = t >= d ? cdf[t - d] : 0ull;
    __syncthreads();
    cdf[t] += add;
    __syncthreads();
  }
  const long long cmin = (long long)cdf[first < 256 ? first : 0];
  const long long den = n - cmin;
  int v = t;
  if (den > 0) {
    const long long num = ((long long)cdf[t] - cmin) * 255;
    long long r = num >= 0 ? (2 * num + den) / (2 * den) : 0;
    v = (int)(r > 255 ? 255 : r);
  }
  lut[t] = (uint8_t)v;
}

// out = lut[in], 16 bytes per lane per step; rows strided over the grid.  A
// thread reads and writes the same chunk, so in place is allowed.
__global__ __launch_bounds__(kGThreads) void k_apply_lut(GlobalImg im, const uint8_t* __restrict__ lut,
                                                         uint8_t* out, int64_t out_pitch) {
  __shared__ uint8_t tab[256];
  tab[threadIdx.x] = lut[threadIdx.x];
  __syncthreads();
  const int chunks = (im.w + 15) >> 4;
  for (int y = blockIdx.x; y < im.h; y += gridDim.x) {
    const uint8_t* row = im.base + (size_t)y * im.pitch;
    uint8_t* orow = out + (size_t)y * out_pitch;
    for (int c = threadIdx.x; c < chunks; c += kGThreads) {
      const uint4 q = *(const uint4*)(row + 16 * c);
      const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
      uint32_t o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        o[j] = (uint32_t)tab[wd[j] & 0xFF] | (uint32_t)tab[(wd[j] >> 8) & 0xFF] << 8 |
               (uint32_t)tab[(wd[j] >> 16) & 0xFF] << 16 | (uint32_t)tab[wd[j] >> 24] << 24;
      }
      // streamed past the caches: nothing here reads the output again
      typedef unsigned int u4v __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(u4v{o[0], o[1], o[2], o[3]}, (u4v*)(orow + 16 * c));
    }
  }
}

hipError_t launch_equalize_mapping(const GlobalImg& im, void* workspace, hipStream_t s) {
  static_assert(kEqHistBytes <= (int)kEqualizeScratchBytes, "the fixed workspace holds the counts and the mapping");
  uint32_t* hist = (uint32_t*)workspace;
  uint8_t* lut = (uint8_t*)workspace + 256 * 4;
  hipError_t e = launch_histogram(im, 256, 0, 256, hist, s);
  if (e != hipSuccess || im.w <= 0 || im.h <= 0) return e;
  hipLaunchKernelGGL(k_eq_lut, dim3(1), dim3(256), 0, s, (const uint32_t*)hist, lut, (long long)im.w * im.h);
  return hipGetLastError();
}

hipError_t launch_equalize_hist(const GlobalImg& im, uint8_t* out, int64_t out_pitch, void* workspace,
                                hipStream_t s) {
  const uint8_t* lut = (const uint8_t*)workspace + 256 * 4;
  hipError_t e = launch_equalize_mapping(im, workspace, s);
  if (e != hipSuccess || im.w <= 0 || im.h <= 0) return e;
  hipLaunchKernelGGL(k_apply_lut, dim3(im.h < 2048 ? im.h : 2048), dim3(kGThreads), 0, s, im, lut, out, out_pitch);
  return hipGetLastError();
}

// ---- EqualizeHist without a caller workspace ------------------------------------
// For callers that cannot allocate: the histogram and the mapping live in a
// fixed device array, `scratch`, one copy per GPU, held until the process
// ends.  In host code the array's name is only a host-side stand-in, so it
// is never passed to a kernel: its device address is resolved once per
// device (with that device current) and kept.  Every call on a GPU shares
// that GPU's copy; the histogram part is cleared by a kernel at the start
// of each call, and calls that overlap on one GPU race.
static __device__ __align__(256) uint8_t scratch[kEqualizeScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t equalize_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> l(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// ---- smallest and largest element of a U8 or S16 image ------------------------
template <bool S16>
__global__ __launch_bounds__(kRThreads) void k_min_max(GlobalImg im, int32_t* __restrict__ out) {
  constexpr int kPer = S16 ? 8 : 16;  // elements per 16-byte chunk
  __shared__ int part[2][kRThreads / 64];
  int mn = INT_MAX, mx = INT_MIN;
  const int t = threadIdx.x;
  stream_image<kPer, kRThreads, 4>(im, [&](const uint4& q, int n) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int v = S16 ? (int)(int16_t)(wd[k >> 1] >> (16 * (k & 1))) : (int)((wd[k >> 2] >> (8 * (k & 3))) & 0xFF);
      if (k < n) {
        mn = min(mn, v);
        mx = max(mx, v);
      }
    }
  });
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off));
    mx = max(mx, __shfl_xor(mx, off));
  }
  if ((t & 63) == 0) {
    part[0][t >> 6] = mn;
    part[1][t >> 6] = mx;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kRThreads / 64; ++w) {
      mn = min(mn, part[0][w]);
      mx = max(mx, part[1][w]);
    }
    // the result only moves one way: a group that cannot improve it skips
    // the atomic (a stale read only costs an unneeded atomic)
    if (mn < __atomic_load_n(&out[0], __ATOMIC_RELAXED)) atomicMin(&out[0], mn);
    if (mx > __atomic_load_n(&out[1], __ATOMIC_RELAXED)) atomicMax(&out[1], mx);
  }
}

// Number of elements of the 32-bit word w equal to the element value whose
// copies fill `splat` (SWAR: an element of x = w ^ splat is zero exactly
// where w matches; adding 0x7F.. to its low bits sets its top bit unless the
// element is zero, and no carry crosses an element), added to acc.
template <bool S16>
__device__ __forceinline__ uint32_t count_eq(uint32_t w, uint32_t splat, uint32_t acc) {
  const uint32_t lo = S16 ? 0x7FFF7FFFu : 0x7F7F7F7Fu, hi = S16 ? 0x80008000u : 0x80808080u;
  const uint32_t x = w ^ splat;
  const uint32_t y = ((x & lo) + lo) | x;
  return acc + (uint32_t)__popc(~y & hi);
}

// One pass for the smallest and the largest value and how many pixels take
// each.  Every lane keeps a running (value, count) pair per extreme: for each
// 16-byte chunk it takes the chunk's extremes, restarts a count when the
// value improves, and adds the chunk's matches counted word-wise.  The pairs
// are merged across the wave and the group, then into the group's own
// 64-bit key of each extreme (at most kMMSubKeys groups run, so no two share
// a key and the compare-and-swap never retries; see kMMSubKeys).
template <bool S16>
__global__ __launch_bounds__(kRThreads) void k_min_max_count(GlobalImg im, unsigned long long* __restrict__ keys) {
  constexpr int kPer = S16 ? 8 : 16;
  __shared__ int part[4][kRThreads / 64];
  int mn = S16 ? 32767 : 255, mx = S16 ? -32768 : 0;
  uint32_t cmn = 0, cmx = 0;
  const int t = threadIdx.x;
  stream_image<kPer, kRThreads, 4>(im, [&](const uint4& q, int n) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
    if (n == kPer) {
      int a = S16 ? 32767 : 255, b = S16 ? -32768 : 0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int v = S16 ? (int)(int16_t)(wd[k >> 1] >> (16 * (k & 1))) : (int)((wd[k >> 2] >> (8 * (k & 3))) & 0xFF);
        a = min(a, v);
        b = max(b, v);
      }
      cmn = a < mn ? 0u : cmn;
      cmx = b > mx ? 0u : cmx;
      mn = min(mn, a);
      mx = max(mx, b);
      const uint32_t sl = S16 ? ((uint32_t)mn & 0xFFFFu) * 0x10001u : (uint32_t)mn * 0x01010101u;
      const uint32_t sh = S16 ? ((uint32_t)mx & 0xFFFFu) * 0x10001u : (uint32_t)mx * 0x01010101u;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cmn = count_eq<S16>(wd[j], sl, cmn);
        cmx = count_eq<S16>(wd[j], sh, cmx);
      }
    } else {  // the last chunk of a row: element by element
      for (int k = 0; k < n; ++k) {
        const int v = S16 ? (int)(int16_t)(wd[k >> 1] >> (16 * (k & 1))) : (int)((wd[k >> 2] >> (8 * (k & 3))) & 0xFF);
        cmn = v < mn ? 1u : cmn + (v == mn ? 1u : 0u);
        cmx = v > mx ? 1u : cmx + (v == mx ? 1u : 0u);
        mn = min(mn, v);
        mx = max(mx, v);
      }
    }
  });
  wave_merge_extremes(mn, cmn, mx, cmx);
  if ((t & 63) == 0) {
    part[0][t >> 6] = mn;
    part[1][t >> 6] = (int)cmn;
    part[2][t >> 6] = mx;
    part[3][t >> 6] = (int)cmx;
  }
  __syncthreads();
  if (t == 0) {
    unsigned long long kmin = kMinKeyInit, kmax = kMaxKeyInit;
    for (int w = 0; w < kRThreads / 64; ++w) {
      kmin = mm_merge(kmin, mm_key(part[0][w], (uint32_t)part[1][w]), true);
      kmax = mm_merge(kmax, mm_key(part[2][w], (uint32_t)part[3][w]), false);
    }
    const int sub = blockIdx.x % kMMSubKeys;
    merge_key(&keys[sub], kmin, true);
    merge_key(&keys[kMMSubKeys + sub], kmax, false);
  }
}

// The sub-keys merged into {min, max, count of min, count of max} at the
// front of the result.
// (One wave: each lane merges every 64th key, then the lanes merge by
// exchange.)
__global__ __launch_bounds__(64) void k_unpack_keys(int32_t* __restrict__ mm) {
  const unsigned long long* k = (const unsigned long long*)((uint8_t*)mm + kMMKeyOffset);
  const int lane = threadIdx.x;
  unsigned long long kmin = kMinKeyInit, kmax = kMaxKeyInit;
  for (int i = lane; i < kMMSubKeys; i += 64) {
    kmin = mm_merge(kmin, k[i], true);
    kmax = mm_merge(kmax, k[kMMSubKeys + i], false);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    kmin = mm_merge(kmin, __shfl_xor(kmin, off), true);
    kmax = mm_merge(kmax, __shfl_xor(kmax, off), false);
  }
  if (lane == 0) {
    mm[0] = mm_value(kmin);
    mm[1] = mm_value(kmax);
    mm[2] = (int32_t)(uint32_t)kmin;
    mm[3] = (int32_t)(uint32_t)kmax;
  }
}

__global__ __launch_bounds__(256) void k_init_keys(int32_t* __restrict__ mm) {
  unsigned long long* k = (unsigned long long*)((uint8_t*)mm + kMMKeyOffset);
  for (int i = threadIdx.x; i < 2 * kMMSubKeys; i += blockDim.x) k[i] = i < kMMSubKeys ? kMinKeyInit : kMaxKeyInit;
}

hipError_t launch_min_max_count(const GlobalImg& im, int32_t* result, hipStream_t s) {
  unsigned long long* keys = (unsigned long long*)((uint8_t*)result + kMMKeyOffset);
  hipLaunchKernelGGL(k_init_keys, dim3(1), dim3(256), 0, s, result);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (im.w > 0 && im.h > 0) {
    const dim3 grid(global_grid(im, 4, kRGroups));
    if (im.bpp == 2) hipLaunchKernelGGL(k_min_max_count<true>, grid, dim3(kRThreads), 0, s, im, keys);
    else hipLaunchKernelGGL(k_min_max_count<false>, grid, dim3(kRThreads), 0, s, im, keys);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_unpack_keys, dim3(1), dim3(64), 0, s, result);
  return hipGetLastError();
}

// MinMaxLoc: the (x, y) of pixels equal to mm[0] (into lmin) and to mm[1]
// (into lmax), two words per location, at most `cap` of each list, in no
// particular order; mm[4], mm[5] count the reserved slots (the exact counts
// come from k_min_max_count).  One 1024-thread group per CU streams K rows a
// grid apart per step, one 16-byte chunk per lane and row.  Each lane marks
// its matches, the counts are scanned across the wave and summed over the
// group in LDS, and one thread reserves the group's slots of each list with
// a single atomic; then every lane writes its entries.  Once both lists are
// full the groups stop (thread 0 reads the counters and the decision goes
// through LDS, so the whole group leaves together).
template <bool S16>
__global__ __launch_bounds__(kRThreads) void k_extreme_locs(GlobalImg im, int32_t* __restrict__ mm,
                                                            uint32_t* __restrict__ lmin, uint32_t* __restrict__ lmax,
                                                            uint32_t cap) {
  constexpr int kPer = S16 ? 8 : 16, K = 4, NW = kRThreads / 64;
  __shared__ uint32_t wtot[2][NW];  // wave totals, then their exclusive prefix
  __shared__ uint32_t gbase[2];     // the group's first slot of each list (cap: none)
  __shared__ int stop;
  const int lo = mm[0], hi = mm[1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int chunks = (im.w + kPer - 1) / kPer;
  const int G = gridDim.x;
  for (int y = blockIdx.x; y < im.h; y += K * G) {
    if (t == 0)
      stop = (uint32_t)__atomic_load_n(&mm[4], __ATOMIC_RELAXED) >= cap &&
             (uint32_t)__atomic_load_n(&mm[5], __ATOMIC_RELAXED) >= cap;
    __syncthreads();
    if (stop) return;
    for (int cb = 0; cb < chunks; cb += kRThreads) {
      const int c = cb + t;
      uint32_t m[2][K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        m[0][k] = m[1][k] = 0;
        const int yy = y + k * G;
        if (c < chunks && yy < im.h) {
          const uint4 q = *(const uint4*)(im.base + (size_t)yy * im.pitch + 16 * c);
          const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
          const int n = min(kPer, im.w - kPer * c);
#pragma unroll
          for (int e = 0; e < kPer; ++e) {
            const int v = S16 ? (int)(int16_t)(wd[e >> 1] >> (16 * (e & 1))) : (int)((wd[e >> 2] >> (8 * (e & 3))) & 0xFF);
            m[0][k] |= (e < n && v == lo) ? 1u << e : 0u;
            m[1][k] |= (e < n && v == hi) ? 1u << e : 0u;
          }
        }
      }
      uint32_t cnt[2], inc[2];
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        cnt[l] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) cnt[l] += (uint32_t)__popc(m[l][k]);
        inc[l] = cnt[l];  // inclusive scan across the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t u = (uint32_t)__shfl_up((int)inc[l], off);
          if (lane >= off) inc[l] += u;
        }
        if (lane == 63) wtot[l][wv] = inc[l];
      }
      __syncthreads();
      if (t < 2) {  // exclusive prefix over the waves, one reservation per list
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
          const uint32_t x = wtot[t][w];
          wtot[t][w] = run;
          run += x;
        }
        uint32_t base = cap;
        if (run && (uint32_t)__atomic_load_n(&mm[4 + t], __ATOMIC_RELAXED) < cap)
          base = (uint32_t)atomicAdd(&mm[4 + t], (int)run);
        gbase[t] = base;
      }
      __syncthreads();
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        uint32_t i = gbase[l] + wtot[l][wv] + inc[l] - cnt[l];
        if (gbase[l] >= cap || i >= cap) continue;
        uint32_t* out = l ? lmax : lmin;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          uint32_t mk = m[l][k];
          while (mk && i < cap) {
            const int e = __ffs(mk) - 1;
            mk &= mk - 1;
            out[2 * i] = (uint32_t)(kPer * c + e);
            out[2 * i + 1] = (uint32_t)(y + k * G);
            ++i;
          }
        }
      }
      __syncthreads();  // wtot and gbase are rewritten by the next step
    }
  }
}

hipError_t launch_extreme_locs(const GlobalImg& im, int32_t* result, uint32_t* lmin, uint32_t* lmax, uint32_t cap,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)result + 4, 2, 0u, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || im.w <= 0 || im.h <= 0 || cap == 0) return e;
  const dim3 grid(global_grid(im, 4, kRGroups));
  if (im.bpp == 2) hipLaunchKernelGGL(k_extreme_locs<true>, grid, dim3(kRThreads), 0, s, im, result, lmin, lmax, cap);
  else hipLaunchKernelGGL(k_extreme_locs<false>, grid, dim3(kRThreads), 0, s, im, result, lmin, lmax, cap);
  return hipGetLastError();
}

hipError_t launch_min_max_loc(const GlobalImg& im, int32_t* result, uint32_t* lmin, uint32_t* lmax, uint32_t cap,
                              hipStream_t s) {
  hipError_t e = launch_min_max_count(im, result, s);
  if (e != hipSuccess) return e;
  return launch_extreme_locs(im, result, lmin, lmax, cap, s);
}

// Slot counters of the location lists clamped to the capacity: the number of
// locations each list holds.
__global__ void k_clamp_slots(int32_t* __restrict__ mm, uint32_t cap) {
  if (threadIdx.x < 2) {
    const uint32_t v = (uint32_t)mm[4 + threadIdx.x];
    mm[4 + threadIdx.x] = (int32_t)(v < cap ? v : cap);
  }
}

hipError_t launch_clamp_slots(int32_t* result, uint32_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_clamp_slots, dim3(1), dim3(64), 0, s, result, cap);
  return hipGetLastError();
}

hipError_t launch_min_max(const GlobalImg& im, int32_t* min_max, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)min_max, 2, (uint32_t)INT_MAX,
                     (uint32_t)INT_MIN);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || im.w <= 0 || im.h <= 0) return e;
  const dim3 grid(global_grid(im, 4, kRGroups));
  if (im.bpp == 2) hipLaunchKernelGGL(k_min_max<true>, grid, dim3(kRThreads), 0, s, im, min_max);
  else hipLaunchKernelGGL(k_min_max<false>, grid, dim3(kRThreads), 0, s, im, min_max);
  return hipGetLastError();
}

// ---- mean and standard deviation of a U8 image ----------------------------------
// Exact sums S1 = sum v and S2 = sum v^2 (64-bit), then one thread forms
// mean = S1 / N and stddev = sqrt(S2 / N - mean^2) in double precision.
// result: u64 S1, u64 S2, f32 mean, f32 stddev.
__global__ __launch_bounds__(kRThreads) void k_sums(GlobalImg im, unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long part[2][kRThreads / 64];
  unsigned long long s1 = 0, s2 = 0;
  const int t = threadIdx.x;
  stream_image<16, kRThreads, 4>(im, [&](const uint4& q, int n) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
    uint32_t a = 0, b = 0;  // at most 16 * 255^2 < 2^21
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t v = k < n ? (wd[k >> 2] >> (8 * (k & 3))) & 0xFF : 0u;
      a += v;
      b += v * v;
    }
    s1 += a;
    s2 += b;
  });
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  if ((t & 63) == 0) {
    part[0][t >> 6] = s1;
    part[1][t >> 6] = s2;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kRThreads / 64; ++w) {
      s1 += part[0][w];
      s2 += part[1][w];
    }
    atomicAdd(&sums[0], s1);
    atomicAdd(&sums[1], s2);
  }
}

__global__ void k_mean_std_final(unsigned long long* __restrict__ sums, double n) {
  if (threadIdx.x != 0) return;
  const double mean = (double)sums[0] / n;
  const double var = (double)sums[1] / n - mean * mean;
  float* f = (float*)(sums + 2);
  f[0] = (float)mean;
  f[1] = (float)sqrt(var > 0.0 ? var : 0.0);
}

hipError_t launch_mean_std_dev(const GlobalImg& im, void* result, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)result, 6, 0u, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || im.w <= 0 || im.h <= 0) return e;
  hipLaunchKernelGGL(k_sums, dim3(global_grid(im, 4, kRGroups)), dim3(kRThreads), 0, s, im,
                     (unsigned long long*)result);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mean_std_final, dim3(1), dim3(64), 0, s, (unsigned long long*)result,
                     (double)im.w * (double)im.h);
  return hipGetLastError();
}

// ---- first and last steps of global operators reduced inside fused kernels ----
// The fused kernels merge their partial results into the operator's result
// buffer; these kernels set its starting value before and form the final
// values after, in the same stream.

// ---- partial results of the generated reducing kernels ----------------------
// Every work-group of such a kernel wrote the partial results of its tile to
// its own slot (red_end_partial); here each of up to kMergeGroups groups
// combines a contiguous range of slots and merges that into the results with
// one atomic (per bin, per word) or compare-and-swap, as the kernel's groups
// did directly before: the results start from launch_reduce_init's values
// and end with launch_reduce_finish.  Few groups, so same-address atomics
// stay few.
constexpr int kMergeGroups = 256;
constexpr int kMergeThreads = 256;

__global__ __launch_bounds__(kMergeThreads) void k_merge_partials(const GProg* __restrict__ P, const IOTable io,
                                                                  const uint32_t* __restrict__ ws, int nslots,
                                                                  int slot_words) {
  __shared__ unsigned long long part[2][kMergeThreads / 64];
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int s0 = (int)((long long)blockIdx.x * nslots / gridDim.x);
  const int s1 = (int)((long long)(blockIdx.x + 1) * nslots / gridDim.x);
  int off = 0;
  for (int oi = 0; oi < P->nops; ++oi) {
    const GOp& o = P->ops[oi];
    if (!is_reduce_op(o.kind)) continue;
    void* out = io.ptr[P->vals[o.out].io];
    if (o.kind == OP_HISTOGRAM || o.kind == OP_EQHIST) {
      for (int b = t; b < o.p0; b += kMergeThreads) {
        // eight slots' loads in flight at a time
        uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int sl = s0;
        for (; sl + 8 <= s1; sl += 8) {
#pragma unroll
          for (int u = 0; u < 8; ++u) c[u] += ws[(size_t)(sl + u) * slot_words + off + b];
        }
        for (; sl < s1; ++sl) c[0] += ws[(size_t)sl * slot_words + off + b];
        const uint32_t sum = c[0] + c[1] + c[2] + c[3] + c[4] + c[5] + c[6] + c[7];
        if (sum) atomicAdd((uint32_t*)out + b, sum);
      }
    } else {
      // this thread's slots, then the wave, then the group
      unsigned long long a, b;
      if (o.kind == OP_SUMS) {
        a = b = 0;
      } else if (o.kind == OP_MINMAX) {
        a = (unsigned)INT_MAX;
        b = (unsigned)INT_MIN;
      } else {
        a = kMinKeyInit;
        b = kMaxKeyInit;
      }
      for (int sl = s0 + t; sl < s1; sl += kMergeThreads) {
        const uint32_t* w = ws + (size_t)sl * slot_words + off;
        if (o.kind == OP_MINMAX) {
          a = (unsigned)min((int)(unsigned)a, (int)w[0]);
          b = (unsigned)max((int)(unsigned)b, (int)w[1]);
        } else {
          const unsigned long long x = w[0] | (unsigned long long)w[1] << 32;
          const unsigned long long y = w[2] | (unsigned long long)w[3] << 32;
          if (o.kind == OP_SUMS) {
            a += x;
            b += y;
          } else {
            a = mm_merge(a, x, true);
            b = mm_merge(b, y, false);
          }
        }
      }
#pragma unroll
      for (int sh = 32; sh > 0; sh >>= 1) {
        const unsigned long long x = __shfl_xor(a, sh), y = __shfl_xor(b, sh);
        if (o.kind == OP_SUMS) {
          a += x;
          b += y;
        } else if (o.kind == OP_MINMAX) {
          a = (unsigned)min((int)(unsigned)a, (int)(unsigned)x);
          b = (unsigned)max((int)(unsigned)b, (int)(unsigned)y);
        } else {
          a = mm_merge(a, x, true);
          b = mm_merge(b, y, false);
        }
      }
      if (lane == 0) {
        part[0][wv] = a;
        part[1][wv] = b;
      }
      __syncthreads();
      if (t == 0 && s1 > s0) {
        for (int w = 1; w < kMergeThreads / 64; ++w) {
          if (o.kind == OP_SUMS) {
            a += part[0][w];
            b += part[1][w];
          } else if (o.kind == OP_MINMAX) {
            a = (unsigned)min((int)(unsigned)a, (int)(unsigned)part[0][w]);
            b = (unsigned)max((int)(unsigned)b, (int)(unsigned)part[1][w]);
          } else {
            a = mm_merge(a, part[0][w], true);
            b = mm_merge(b, part[1][w], false);
          }
        }
        if (o.kind == OP_SUMS) {
          atomicAdd((unsigned long long*)out, a);
          atomicAdd((unsigned long long*)out + 1, b);
        } else if (o.kind == OP_MINMAX) {
          atomicMin((int32_t*)out, (int)(unsigned)a);
          atomicMax((int32_t*)out + 1, (int)(unsigned)b);
        } else {
          unsigned long long* keys = (unsigned long long*)((uint8_t*)out + kMMKeyOffset);
          const int sub = blockIdx.x % kMMSubKeys;
          merge_key(&keys[sub], a, true);
          merge_key(&keys[kMMSubKeys + sub], b, false);
        }
      }
      __syncthreads();
    }
    off += red_block_words(o.kind, o.p0);
  }
}

hipError_t launch_merge_partials(const GProg* dev_prog, const IOTable& io, const uint32_t* ws, int nslots,
                                 int slot_words, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const int groups = nslots < kMergeGroups ? nslots : kMergeGroups;
  hipLaunchKernelGGL(k_merge_partials, dim3(groups), dim3(kMergeThreads), 0, s, dev_prog, io, ws, nslots, slot_words);
  return hipGetLastError();
}

hipError_t launch_reduce_init(int kind, void* result, int num_bins, hipStream_t s) {
  switch (kind) {
    case OP_HISTOGRAM:
    case OP_EQHIST: {
      const int n = kind == OP_EQHIST ? 256 : num_bins;
      hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, (uint32_t*)result, n, 0u, 0u);
      break;
    }
    case OP_MINMAX:
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)result, 2, (uint32_t)INT_MAX,
                         (uint32_t)INT_MIN);
      break;
    case OP_MMCOUNT: hipLaunchKernelGGL(k_init_keys, dim3(1), dim3(256), 0, s, (int32_t*)result); break;
    case OP_SUMS: hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)result, 6, 0u, 0u); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_words(void* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, (uint32_t*)p, n, 0u, 0u);
  return hipGetLastError();
}

hipError_t launch_reduce_finish(int kind, void* result, long long npix, hipStream_t s) {
  switch (kind) {
    case OP_EQHIST:
      hipLaunchKernelGGL(k_eq_lut, dim3(1), dim3(256), 0, s, (const uint32_t*)result, (uint8_t*)result + 256 * 4,
                         npix);
      break;
    case OP_MMCOUNT: hipLaunchKernelGGL(k_unpack_keys, dim3(1), dim3(64), 0, s, (int32_t*)result); break;
    case OP_SUMS:
      hipLaunchKernelGGL(k_mean_std_final, dim3(1), dim3(64), 0, s, (unsigned long long*)result, (double)npix);
      break;
    default: return hipSuccess;
  }
  return hipGetLastError();
}

}  // namespace hvx
