// Grouping of a long list by bucket key (the transaxial line of an event)
// for the projector pair by line.  A counting sort with one global atomic
// per element (its rank in its bucket) runs at the rate the memory side
// executes returning atomics, ~1e10/s: 46 ms for 5e8 events.  Here the key
// is split into two 9-bit digits and each digit is counted per workgroup in
// LDS (8192 elements per workgroup): pass 1 distributes the elements by
// their high digit, pass 2 distributes each high-digit range by the low
// digit.  A workgroup reserves its range for every digit value it holds
// with one global atomic, so a pass issues about (elements / 8192) x 512
// global atomics instead of one per element.  The order inside a bucket is
// not fixed (ranks come from LDS atomics).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lm_host.hpp"
#include "lm_sort.hpp"

namespace {

constexpr int kDigit = 9;
constexpr unsigned kRadix = 1u << kDigit;   // values of a digit
constexpr int kThreads = 256;
constexpr int kPer = 32;                    // elements per thread
constexpr int kChunk = kThreads * kPer;     // elements per workgroup

inline unsigned blocks_of(long long n) { return (unsigned)((n + kChunk - 1) / kChunk); }

// hi_tot[h] += the elements of the workgroup's chunk with high digit h.
__global__ __launch_bounds__(kThreads) void k_hi_count(const unsigned *__restrict__ key, long long n, unsigned nb,
                                                       const int *flag, unsigned *hi_tot) {
  __shared__ unsigned h[kRadix];
  if (flag && !*flag) return;
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads) h[i] = 0u;
  __syncthreads();
  const long long e0 = (long long)blockIdx.x * kChunk + threadIdx.x;
#pragma unroll 8
  for (int j = 0; j < kPer; ++j) {
    const long long e = e0 + (long long)j * kThreads;
    if (e < n) {
      const unsigned k = key[e];
      if (k < nb) atomicAdd(&h[k >> kDigit], 1u);
    }
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads)
    if (h[i]) atomicAdd(hi_tot + i, h[i]);
}

// Exclusive prefix sum of cnt[0 .. m) into off[0 .. m] (one workgroup of
// 1024 threads, each summing a contiguous segment).
__global__ __launch_bounds__(1024) void k_prefix(const unsigned *cnt, long long m, const int *flag, unsigned *off) {
  __shared__ unsigned part[1024];
  if (flag && !*flag) return;
  const int t = threadIdx.x;
  const long long seg = (m + 1023) / 1024;
  const long long a = std::min(m, t * seg), b = std::min(m, a + seg);
  unsigned sum = 0;
  for (long long i = a; i < b; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned add = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  unsigned run = part[t] - sum;
  for (long long i = a; i < b; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[m] = part[1023];
}

// Pass 1: the chunk's elements go to their high-digit range hi_off[h] ..,
// at a position reserved for the workgroup (hi_fill) plus their LDS rank.
template <class P>
__global__ __launch_bounds__(kThreads) void k_hi_place(const unsigned *__restrict__ key, const P *__restrict__ payload,
                                                       long long n, unsigned nb, const int *flag,
                                                       const unsigned *hi_off, unsigned *hi_fill,
                                                       unsigned *__restrict__ tkey, P *__restrict__ tpay) {
  __shared__ unsigned h[kRadix], base[kRadix];
  if (flag && !*flag) return;
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads) h[i] = 0u;
  __syncthreads();
  const long long e0 = (long long)blockIdx.x * kChunk + threadIdx.x;
  unsigned kk[kPer], rk[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const long long e = e0 + (long long)j * kThreads;
    kk[j] = e < n ? key[e] : nb;
    rk[j] = kk[j] < nb ? atomicAdd(&h[kk[j] >> kDigit], 1u) : 0u;
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads)
    base[i] = h[i] ? hi_off[i] + atomicAdd(hi_fill + i, h[i]) : 0u;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (kk[j] >= nb) continue;
    const long long e = e0 + (long long)j * kThreads;
    const unsigned pos = base[kk[j] >> kDigit] + rk[j];
    tkey[pos] = kk[j];
    tpay[pos] = payload ? payload[e] : (P)e;
  }
}

// Pass 2 chunks: high-digit range h is cut into chunks of kChunk elements;
// chunk_off[h] = the first chunk of range h (exclusive prefix of the chunk
// counts, nhi + 1 entries; one workgroup).
__global__ __launch_bounds__(1024) void k_chunks(const unsigned *hi_off, unsigned nhi, const int *flag,
                                                 unsigned *chunk_off) {
  __shared__ unsigned c[kRadix + 1];
  if (flag && !*flag) return;
  for (unsigned i = threadIdx.x; i < nhi; i += blockDim.x)
    c[i] = (hi_off[i + 1] - hi_off[i] + kChunk - 1) / kChunk;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned run = 0;
    for (unsigned i = 0; i < nhi; ++i) {
      chunk_off[i] = run;
      run += c[i];
    }
    chunk_off[nhi] = run;
  }
}

// The high-digit range and the element range [a, b) of pass-2 chunk blk,
// or false past the last chunk.
__device__ __forceinline__ bool chunk_range(unsigned blk, const unsigned *hi_off, const unsigned *chunk_off,
                                            unsigned nhi, unsigned &hi, unsigned &a, unsigned &b) {
  if (blk >= chunk_off[nhi]) return false;
  unsigned lo = 0, up = nhi - 1;  // the last h with chunk_off[h] <= blk
  while (lo < up) {
    const unsigned mid = (lo + up + 1) >> 1;
    if (chunk_off[mid] <= blk) lo = mid;
    else up = mid - 1;
  }
  hi = lo;
  a = hi_off[hi] + (blk - chunk_off[hi]) * (unsigned)kChunk;
  b = min(hi_off[hi + 1], a + (unsigned)kChunk);
  return true;
}

// Pass 2 counts: bucket totals tot[key] from the chunks' LDS counts.
__global__ __launch_bounds__(kThreads) void k_lo_count(const unsigned *__restrict__ tkey, const unsigned *hi_off,
                                                       const unsigned *chunk_off, unsigned nhi, const int *flag,
                                                       unsigned *tot) {
  __shared__ unsigned h[kRadix];
  if (flag && !*flag) return;
  unsigned hi, a, b;
  if (!chunk_range(blockIdx.x, hi_off, chunk_off, nhi, hi, a, b)) return;
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads) h[i] = 0u;
  __syncthreads();
#pragma unroll 8
  for (int j = 0; j < kPer; ++j) {
    const unsigned p = a + threadIdx.x + (unsigned)j * kThreads;
    if (p < b) atomicAdd(&h[tkey[p] & (kRadix - 1)], 1u);
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads)
    if (h[i]) atomicAdd(tot + ((hi << kDigit) | i), h[i]);
}

// Pass 2 placement: out[off[key] + reserved + LDS rank] = payload.
template <class P>
__global__ __launch_bounds__(kThreads) void k_lo_place(const unsigned *__restrict__ tkey, const P *__restrict__ tpay,
                                                       const unsigned *hi_off, const unsigned *chunk_off,
                                                       unsigned nhi, const int *flag, const unsigned *off,
                                                       unsigned *fill, P *__restrict__ out) {
  __shared__ unsigned h[kRadix], base[kRadix];
  if (flag && !*flag) return;
  unsigned hi, a, b;
  if (!chunk_range(blockIdx.x, hi_off, chunk_off, nhi, hi, a, b)) return;
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads) h[i] = 0u;
  __syncthreads();
  unsigned lo[kPer], rk[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const unsigned p = a + threadIdx.x + (unsigned)j * kThreads;
    lo[j] = p < b ? (tkey[p] & (kRadix - 1)) : kRadix;
    rk[j] = lo[j] < kRadix ? atomicAdd(&h[lo[j]], 1u) : 0u;
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < kRadix; i += kThreads) {
    const unsigned k = (hi << kDigit) | i;
    base[i] = h[i] ? off[k] + atomicAdd(fill + k, h[i]) : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    if (lo[j] >= kRadix) continue;
    const unsigned p = a + threadIdx.x + (unsigned)j * kThreads;
    out[base[lo[j]] + rk[j]] = tpay[p];
  }
}

template <class P>
int group_impl(const unsigned *key, const P *payload, long long n, unsigned nb, const int *flag, P *out,
               unsigned *off, hipStream_t st) {
  LM_REQUIRE(n >= 0 && n < (1LL << 31) && nb >= 1 && nb <= lmk::kGroupMaxBuckets, LM_EINVAL,
             "grouping: %lld elements, %u buckets", n, nb);
  const unsigned nhi = (nb + kRadix - 1) >> kDigit;
  const unsigned nbk = nhi << kDigit;  // bucket counters, whole digits
  unsigned *hi_tot = nullptr, *hi_off = nullptr, *hi_fill = nullptr, *chunk_off = nullptr, *tot = nullptr,
           *fill = nullptr, *tkey = nullptr;
  P *tpay = nullptr;
  auto release = [&]() {  // release errors are not reported
    for (void *q : {(void *)hi_tot, (void *)hi_off, (void *)hi_fill, (void *)chunk_off, (void *)tot, (void *)fill,
                    (void *)tkey, (void *)tpay})
      if (q) (void)hipFreeAsync(q, st);
  };
  const size_t nn = (size_t)std::max<long long>(n, 1);
  hipError_t e = hipMallocAsync((void **)&hi_tot, kRadix * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&hi_off, (kRadix + 1) * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&hi_fill, kRadix * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&chunk_off, (kRadix + 1) * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&tot, nbk * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&fill, nbk * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&tkey, nn * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&tpay, nn * sizeof(P), st);
  if (e != hipSuccess) {
    release();
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return LM_ENOMEM;
    lmh::set_error("grouping temporaries: %s", hipGetErrorString(e));
    return LM_EHIP;
  }
  e = hipMemsetAsync(hi_tot, 0, kRadix * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMemsetAsync(hi_fill, 0, kRadix * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMemsetAsync(tot, 0, nbk * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMemsetAsync(fill, 0, nbk * sizeof(unsigned), st);
  const unsigned nblk = blocks_of(n);
  // pass-2 chunks: at most one partial chunk per high-digit range beyond n / kChunk
  const unsigned nchunk_max = nblk + nhi;
  if (e == hipSuccess && n > 0) {
    hipLaunchKernelGGL(k_hi_count, dim3(nblk), dim3(kThreads), 0, st, key, n, nb, flag, hi_tot);
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, st, hi_tot, (long long)nhi, flag, hi_off);
    hipLaunchKernelGGL((k_hi_place<P>), dim3(nblk), dim3(kThreads), 0, st, key, payload, n, nb, flag, hi_off,
                       hi_fill, tkey, tpay);
    hipLaunchKernelGGL(k_chunks, dim3(1), dim3(1024), 0, st, hi_off, nhi, flag, chunk_off);
    hipLaunchKernelGGL(k_lo_count, dim3(nchunk_max), dim3(kThreads), 0, st, tkey, hi_off, chunk_off, nhi, flag,
                       tot);
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, st, tot, (long long)nb, flag, off);
    hipLaunchKernelGGL((k_lo_place<P>), dim3(nchunk_max), dim3(kThreads), 0, st, tkey, tpay, hi_off, chunk_off,
                       nhi, flag, off, fill, out);
    e = hipGetLastError();
  } else if (e == hipSuccess) {
    e = hipMemsetAsync(off, 0, ((size_t)nb + 1) * sizeof(unsigned), st);
  }
  release();
  if (e != hipSuccess) {
    lmh::set_error("grouping: %s", hipGetErrorString(e));
    return LM_EHIP;
  }
  return LM_OK;
}

}  // namespace

namespace lmk {

size_t group_temp_bytes(long long n, unsigned nb, size_t payload_bytes) {
  const size_t nbk = (size_t)((nb + kRadix - 1) >> kDigit) << kDigit;
  return (size_t)std::max<long long>(n, 1) * (sizeof(unsigned) + payload_bytes) + 2 * nbk * sizeof(unsigned) +
         4 * (kRadix + 1) * sizeof(unsigned);
}

int group_by_key(const unsigned *key, const unsigned *payload, long long n, unsigned nb, const int *flag,
                 unsigned *out, unsigned *off, hipStream_t st) {
  return group_impl(key, payload, n, nb, flag, out, off, st);
}

int group_by_key(const unsigned *key, const unsigned long long *payload, long long n, unsigned nb, const int *flag,
                 unsigned long long *out, unsigned *off, hipStream_t st) {
  return group_impl(key, payload, n, nb, flag, out, off, st);
}

}  // namespace lmk
