// Grouping of a long list by a bucket key on the device (lm_sort.hip): the
// counting sort that orders events by transaxial line for the projector
// pair by line.
#pragma once

#include <hip/hip_runtime.h>

namespace lmk {

// Largest number of buckets group_by_key handles (two digits of 9 bits).
constexpr unsigned kGroupMaxBuckets = 1u << 18;

// Stream-ordered temporaries of group_by_key for n elements and nb buckets
// (bytes), its payload excluded.
size_t group_temp_bytes(long long n, unsigned nb, size_t payload_bytes);

// out[off[b] .. off[b + 1]) = the payloads of the elements with key b, for
// every bucket b < nb (their order inside a bucket is not fixed); elements
// with key >= nb are dropped; off has nb + 1 entries; payload NULL: the
// element's index is its payload.  n < 2^31, nb <= kGroupMaxBuckets.  When
// flag != NULL and *flag == 0 at run time, nothing is read or written (the
// keys may then be unset).  Two passes of per-workgroup
// counting in LDS, one per 9-bit digit of the key (most significant first),
// each reserving its ranges with one global atomic per workgroup and
// digit value instead of one per element.  Temporaries are allocated and
// freed stream-ordered; LM_ENOMEM when they do not fit (nothing enqueued).
int group_by_key(const unsigned *key, const unsigned *payload, long long n, unsigned nb, const int *flag,
                 unsigned *out, unsigned *off, hipStream_t st);
int group_by_key(const unsigned *key, const unsigned long long *payload, long long n, unsigned nb, const int *flag,
                 unsigned long long *out, unsigned *off, hipStream_t st);

}  // namespace lmk
