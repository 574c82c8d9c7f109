// Sign correlations of the random bath vectors, the input of the
// high-temperature offset of the estimator (Section "A note on high
// temperatures"): for a bath vector v with Rademacher signs s,
// <v| sx_p |v> = 2^-nb sum_b s_b s_(b xor 2^p), with sx_p the Pauli X on bath
// bit p.  The sums are integers, accumulated exactly.
#include "internal.h"
#include "rng_device.h"

namespace rdm {

namespace {

constexpr int kSxThreads = 256;
constexpr int kSxMaxBlocks = 256;

// Mask of the bit positions i < 64 whose bit p is clear, p < 6.
__device__ __forceinline__ uint64_t low_half_mask(int p) {
  switch (p) {
    case 0: return 0x5555555555555555ull;
    case 1: return 0x3333333333333333ull;
    case 2: return 0x0F0F0F0F0F0F0F0Full;
    case 3: return 0x00FF00FF00FF00FFull;
    case 4: return 0x0000FFFF0000FFFFull;
    default: return 0x00000000FFFFFFFFull;
  }
}

// blockIdx.y = bath vector j; each thread takes sign words w = 64-index
// chunks of v_j with a grid stride; per bath bit p the block total goes to
// part[(j * gridDim.x + blockIdx.x) * nb + p].
__global__ void __launch_bounds__(kSxThreads) k_bath_sx(uint64_t seed, int nb, long long* part) {
  __shared__ long long red[kSxThreads / 64];
  const uint64_t key = rng_bath_key(seed, blockIdx.y);
  const uint64_t nw = nb >= 6 ? (1ull << (nb - 6)) : 1ull;
  // fewer than 64 bath indices: only the low 2^nb bits of word 0 are entries
  const uint64_t valid = nb >= 6 ? ~0ull : ((1ull << (1u << nb)) - 1ull);
  const int nvalid = nb >= 6 ? 64 : (1 << nb);
  const uint64_t stride = (uint64_t)gridDim.x * kSxThreads;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long* out = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * nb;
  for (int p = 0; p < nb; ++p) {
    long long acc = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * kSxThreads + threadIdx.x; w < nw; w += stride) {
      const uint64_t s = rng_bath_word(key, w) & valid;
      uint64_t t;  // t bit i = sign of entry (64 w + i) xor 2^p
      if (p < 6) {
        const uint64_t m = low_half_mask(p);
        const int sh = 1 << p;
        t = ((s >> sh) & m) | ((s & m) << sh);
      } else {
        t = rng_bath_word(key, w ^ (1ull << (p - 6)));
      }
      // __popcll is unsigned: take it as a signed count before subtracting
      const int differ = (int)__popcll((s ^ t) & valid);
      acc += nvalid - 2 * differ;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int i = 0; i < kSxThreads / 64; ++i) tot += red[i];
      out[p] = tot;
    }
    __syncthreads();
  }
}

}  // namespace

int bath_sx_blocks(int nb) {
  const long long nw = nb >= 6 ? (1ll << (nb - 6)) : 1;
  const long long b = (nw + kSxThreads - 1) / kSxThreads;
  return (int)(b < kSxMaxBlocks ? b : kSxMaxBlocks);
}

hipError_t launch_bath_sx(uint64_t seed, int nb, int nv, long long* part, hipStream_t st) {
  if (nb < 1 || nb > 40 || nv < 1 || nv > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bath_sx, dim3(bath_sx_blocks(nb), nv), dim3(kSxThreads), 0, st, seed, nb, part);
  return hipGetLastError();
}

}  // namespace rdm
