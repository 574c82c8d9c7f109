// Device side of the bath-vector rule: SplitMix64 (Steele, Lea & Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014) and the
// Rademacher sign words of the random bath vectors.
//
// Bath vector j has entry v_j[b] = (1 - 2 bit) 2^(-n_b/2), where bit is bit
// (b mod 64) of the 64-bit word sm64(key_j XOR (b div 64)) and
// key_j = sm64(seed XOR sm64(j)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rdm {

// One SplitMix64 output from state x.
static __device__ __forceinline__ uint64_t rng_sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static __device__ __forceinline__ uint64_t rng_bath_key(uint64_t seed, uint32_t j) {
  return rng_sm64(seed ^ rng_sm64((uint64_t)j));
}

// Signs of bath indices 64 w .. 64 w + 63 (bit i set: entry 64 w + i negative).
static __device__ __forceinline__ uint64_t rng_bath_word(uint64_t key, uint64_t w) {
  return rng_sm64(key ^ w);
}

}  // namespace rdm
