// Compile-time sorting network over N keys held in registers.
//
// Bitonic sort in the form where every comparator puts the smaller key at the
// lower index: a merge of two sorted halves first compares i with its mirror
// (i ^ (size-1)), then half-cleans with distance stride.  Because every
// comparator is min-to-lower, keys at positions >= N can be taken as +inf and
// every comparator touching them dropped: the network sorts any N, not only
// powers of two.  All loops have constant trip counts and unroll completely,
// so the key array never leaves registers.
#pragma once
#include <stdint.h>

namespace dfb {

constexpr int pow2_ceil(int n) { return n <= 1 ? 1 : 2 * pow2_ceil((n + 1) / 2); }

template <typename K>
__host__ __device__ __forceinline__ void compare_exchange(K& a, K& b) {
  const bool lt = a < b;  // one compare, two selects per word
  const K lo = lt ? a : b;
  const K hi = lt ? b : a;
  a = lo;
  b = hi;
}

template <typename K>
struct CompareExchange {
  __host__ __device__ __forceinline__ void operator()(K& a, K& b) const { compare_exchange(a, b); }
};

// The network with a given comparator ce(a, b): min to a, max to b.
template <int N, typename K, typename CE>
__host__ __device__ __forceinline__ void sort_network(K (&k)[N], CE ce) {
  constexpr int NP = pow2_ceil(N);
#pragma unroll
  for (int size = 2; size <= NP; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int c = 0; c < NP / 2; ++c) {
        const int lo = (c / stride) * (2 * stride) + (c % stride);
        const int hi = (stride == (size >> 1)) ? (lo ^ (size - 1)) : (lo + stride);
        if (hi < N) ce(k[lo], k[hi]);
      }
    }
  }
}

template <int N, typename K>
__host__ __device__ __forceinline__ void sort_network(K (&k)[N]) {
  sort_network<N>(k, CompareExchange<K>());
}

}  // namespace dfb
