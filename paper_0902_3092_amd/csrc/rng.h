// Counter-based random numbers for packet streams: Philox4x32-10 (Salmon,
// Moraes, Dror & Shaw, SC'11), keyed by the run seed, counter = (packet id,
// block index).  No state lives in memory: a packet's stream is a function of
// (seed, packet id, draw index), so any packet can be traced on any lane, in
// any order, and a run can resume at a packet offset.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply each (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Draw d of a packet comes from block d/2: the 64-bit word (o[2h] << 32 |
// o[2h+1]), h = d % 2, whose top 52 bits x give (x + 1/2) / 2^52 in (0, 1).
struct Rng64 {
  uint32_t k0, k1;
  uint64_t pid;
  uint64_t d;
  double spare;

  __device__ __forceinline__ void init(uint32_t key0, uint32_t key1, uint64_t id) {
    k0 = key0;
    k1 = key1;
    pid = id;
    d = 0;
    spare = 0.0;
  }
  __device__ __forceinline__ static double unit(uint32_t hi, uint32_t lo) {
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return ((double)(x >> 12) + 0.5) * (1.0 / 4503599627370496.0);
  }
  __device__ __forceinline__ double next() {
    if (d & 1ull) {
      ++d;
      return spare;
    }
    uint64_t blk = d >> 1;
    uint32_t c0 = (uint32_t)pid, c1 = (uint32_t)(pid >> 32), c2 = (uint32_t)blk,
             c3 = (uint32_t)(blk >> 32);
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    spare = unit(c2, c3);
    ++d;
    return unit(c0, c1);
  }
  __device__ __forceinline__ uint64_t nd_value() const { return d; }
};

// FP32 streams: draw d uses output word d % 4 of block d / 4; its top 24 bits
// x give (x + 1/2) / 2^24 rounded to FP32, in (0, 1] (x = 2^24 - 1 rounds up
// to 1).
struct Rng32 {
  uint32_t k0, k1;
  uint64_t pid;
  uint32_t blk;
  uint32_t o1, o2, o3;
  uint32_t have;  // words left in o1..o3

  __device__ __forceinline__ void init(uint32_t key0, uint32_t key1, uint64_t id) {
    k0 = key0;
    k1 = key1;
    pid = id;
    blk = 0;
    have = 0;
  }
  __device__ __forceinline__ static float unit(uint32_t w) {
    return ((float)(w >> 8) + 0.5f) * (1.0f / 16777216.0f);
  }
  __device__ __forceinline__ float next() {
    if (have) {
      uint32_t w = o1;
      o1 = o2;
      o2 = o3;
      --have;
      return unit(w);
    }
    uint32_t c0 = (uint32_t)pid, c1 = (uint32_t)(pid >> 32), c2 = blk, c3 = 0;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    ++blk;
    o1 = c1;
    o2 = c2;
    o3 = c3;
    have = 3;
    return unit(c0);
  }
  __device__ __forceinline__ uint64_t draws() const { return (uint64_t)blk * 4 - have; }
};

}  // namespace mcrt
