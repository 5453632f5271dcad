// Device-side helpers shared by the traversal kernels: wave/block scans and
// reductions, the device-wide barrier, clocks and mask types.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "blest_internal.h"

namespace blest {

template <int SIGMA>
struct MaskOf;
template <>
struct MaskOf<8> {
  using T = uint8_t;
};
template <>
struct MaskOf<16> {
  using T = uint16_t;
};
template <>
struct MaskOf<32> {
  using T = uint32_t;
};

// Slice word layout: mask in the low bits, row above it.
template <class SliceT>
struct SliceFmt;
template <>
struct SliceFmt<uint32_t> {
  static constexpr int kRowShift = 8;
};
template <>
struct SliceFmt<uint64_t> {
  static constexpr int kRowShift = 32;
};

__device__ __forceinline__ unsigned long long dev_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63u); }

// Pointers to device (global) memory. Pointers read from an argument struct
// that lives on the stack reach a callee with no address space, and accesses
// through them become flat instructions, which also count against the
// LDS/scalar wait counter (so an LDS wait also waits for every load in
// flight). Hot loops access device memory through gptr<T>, which makes the
// compiler emit global loads, stores and atomics.
// (The host pass of the single-source compile only parses device code; there
// the qualifiers are dropped, since x86 has no generic address space that
// contains them.)
// cptr<T> points into the constant address space: memory no kernel writes
// while it runs, whose wave-uniform loads become scalar loads (waited on with
// the LDS/scalar counter instead of the vector-load counter).
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
using lptr = __attribute__((address_space(3))) T*;
template <class T>
using cptr = __attribute__((address_space(4))) T*;
#else
template <class T>
using gptr = T*;
template <class T>
using lptr = T*;
template <class T>
using cptr = T*;
#endif
template <class T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}
// A pointer the caller knows to be the same in every lane, made wave-uniform
// for the compiler (a pointer read through a function argument is not), so
// that loads through it with uniform indices can be scalar loads.
template <class T>
__device__ __forceinline__ cptr<T> to_const_uniform(T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (cptr<T>)reinterpret_cast<T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Same for LDS: pointers into a __shared__ array handed to a function that is
// not inlined stay ds_* accesses.
template <class T>
__device__ __forceinline__ lptr<T> to_lds(T* p) {
  return (lptr<T>)p;
}

// Wave index inside the block, known uniform to the compiler.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6)); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T x = __shfl_up(v, d, 64);
    if (lane >= d) v += x;
  }
  return v;
}

// Exclusive block scan of N int counters; tot[] receives the block totals.
// lds must hold N * (BLOCK / 64) ints. Contains two __syncthreads().
template <int BLOCK, int N>
__device__ __forceinline__ void block_exclusive_scan(const int (&v)[N], int (&excl)[N], int (&tot)[N], int* lds) {
  constexpr int W = BLOCK / 64;
  const int lane = lane_id(), w = static_cast<int>(threadIdx.x >> 6);
  int inc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    inc[k] = wave_inclusive_scan(v[k]);
    if (lane == 63) lds[k * W + w] = inc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int before = 0, all = 0;
    for (int i = 0; i < W; ++i) {
      int x = lds[k * W + i];
      before += (i < w) ? x : 0;
      all += x;
    }
    excl[k] = before + inc[k] - v[k];
    tot[k] = all;
  }
  __syncthreads();
}

// Block sum of N int64 values, result valid in thread 0. lds: N * (BLOCK/64) slots.
template <int BLOCK, int N>
__device__ __forceinline__ void block_sum64(long long (&v)[N], long long* lds) {
  constexpr int W = BLOCK / 64;
  const int lane = lane_id(), w = static_cast<int>(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    long long s = wave_sum(v[k]);
    if (lane == 0) lds[k * W + w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      long long s = 0;
      for (int i = 0; i < W; ++i) s += lds[k * W + i];
      v[k] = s;
    }
  }
  __syncthreads();
}

template <class P>
__device__ __forceinline__ unsigned long long ld_acquire_u64(P p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ unsigned long long ld_relaxed_u64(P p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ void add_u64(P p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P>
__device__ __forceinline__ unsigned long long fetch_add_u64(P p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 7u;
}

// Device-wide barrier for a cooperative (co-resident) grid.
//
// The eight XCDs of MI355X each have a private L2 that is not coherent with
// the others, so data written before the barrier must be written back to
// memory (buffer_wbl2) and readers must invalidate (buffer_inv) after it.
// Arrival is hierarchical: every wave waits for its own stores to be
// acknowledged (s_waitcnt 0), the block's thread 0 arrives on its XCD's
// counter, and the last block of each XCD -- whose L2 now holds every store
// of that XCD -- performs one agent-scope release (one L2 write-back per XCD
// instead of one per block) and arrives on the top-level counter. The last
// XCD leader acquires, resets the counter and bumps the generation; each XCD
// leader then forwards the release to its XCD's flag, which that XCD's blocks
// poll with relaxed loads before a single acquire fence. Blocks per XCD are
// counted at kernel start (barrier_register), so no dispatch order is
// assumed. Every spin is bounded by `timeout` device-clock ticks and by the
// error flag, so every wave leaves even if a block never arrives. Returns
// false (uniformly in the block) when the traversal must stop.
struct BarrierCtx {
  unsigned xcc;        // this block's XCD
  unsigned nlocal;     // blocks on this XCD
  unsigned nxcd;       // XCDs with blocks
  unsigned long long timeout;
};

__device__ __forceinline__ bool spin_until_changed(gptr<const unsigned> flag, unsigned old, gptr<Ctl> ctl,
                                                   unsigned long long t0, unsigned long long timeout) {

  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == old) {
    if (__hip_atomic_load(&ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (dev_ticks() - t0 > timeout) {
      __hip_atomic_store(&ctl->error[0], static_cast<int>(BLEST_ERR_TIMEOUT), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__device__ __forceinline__ bool grid_barrier(Ctl* ctl_in, const BarrierCtx& bc) {
  __shared__ int ok_flag;
  const gptr<Ctl> ctl = to_global(ctl_in);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned long long t0 = dev_ticks();
    const unsigned x = bc.xcc;
    const unsigned g = __hip_atomic_load(&ctl->xcd_gen[x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned p = __hip_atomic_fetch_add(&ctl->xcd_count[x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == bc.nlocal - 1) {
      __hip_atomic_store(&ctl->xcd_count[x][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned gg = __hip_atomic_load(&ctl->bar_gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned q = __hip_atomic_fetch_add(&ctl->bar_count[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (q == bc.nxcd - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&ctl->bar_count[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->bar_gen[0], gg + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = spin_until_changed(&ctl->bar_gen[0], gg, ctl, t0, bc.timeout);
      }
      __hip_atomic_store(&ctl->xcd_gen[x][0], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      ok = spin_until_changed(&ctl->xcd_gen[x][0], g, ctl, t0, bc.timeout);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (__hip_atomic_load(&ctl->error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    ok_flag = ok;
  }
  __syncthreads();
  return ok_flag != 0;
}

// Counts the blocks of this launch on each XCD. Must be the first grid-wide
// step of a persistent kernel; it uses a flat barrier on bar_count/bar_gen
// (one release RMW per block) because the per-XCD counts are not known yet.
// The host zeroes xcd_blocks/xcd_active before every launch.
__device__ __forceinline__ bool barrier_register(Ctl* ctl_in, BarrierCtx* bc, unsigned long long timeout) {
  const gptr<Ctl> ctl = to_global(ctl_in);
  __shared__ unsigned s_xcc, s_nlocal, s_nxcd;
  __shared__ int ok_flag;
  // every wave's stores are performed before workgroup 0's release, so the
  // registration also publishes what the workgroups wrote before it
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned x = xcc_id();
    const unsigned prevx = __hip_atomic_fetch_add(&ctl->xcd_blocks[x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prevx == 0) __hip_atomic_fetch_add(&ctl->xcd_active[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const unsigned long long t0 = dev_ticks();
    const unsigned gg = __hip_atomic_load(&ctl->bar_gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned q = __hip_atomic_fetch_add(&ctl->bar_count[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (q == gridDim.x - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&ctl->bar_count[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen[0], gg + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      ok = spin_until_changed(&ctl->bar_gen[0], gg, ctl, t0, timeout);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_xcc = x;
    s_nlocal = __hip_atomic_load(&ctl->xcd_blocks[x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_nxcd = __hip_atomic_load(&ctl->xcd_active[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok_flag = ok;
  }
  __syncthreads();
  bc->xcc = s_xcc;
  bc->nlocal = s_nlocal;
  bc->nxcd = s_nxcd;
  bc->timeout = timeout;
  return ok_flag != 0;
}

// Number of sigma-byte marks of a slice set that are set, as a sigma-bit word.
// Marks are 0 or 1 per byte; (x * 0x0102040810204080) >> 56 gathers the low
// bit of each of the 8 bytes of x into one byte, byte i -> bit i.
__device__ __forceinline__ uint32_t gather8(unsigned long long x) {
  return static_cast<uint32_t>((x * 0x0102040810204080ULL) >> 56);
}

template <int SIGMA>
__device__ __forceinline__ typename MaskOf<SIGMA>::T load_marks(gptr<const uint8_t> p) {
  if constexpr (SIGMA == 8) {
    return static_cast<uint8_t>(gather8(*(gptr<const unsigned long long>)p));
  } else if constexpr (SIGMA == 16) {
    const u64x2 x = *(gptr<const u64x2>)p;
    return static_cast<uint16_t>(gather8(x.x) | (gather8(x.y) << 8));
  } else {
    const u64x2 x = *(gptr<const u64x2>)p;
    const u64x2 y = *(gptr<const u64x2>)(p + 16);
    return gather8(x.x) | (gather8(x.y) << 8) | (gather8(y.x) << 16) | (gather8(y.y) << 24);
  }
}

template <int SIGMA>
__device__ __forceinline__ void clear_marks(gptr<uint8_t> p) {
  if constexpr (SIGMA == 8) {
    *(gptr<unsigned long long>)p = 0ULL;
  } else if constexpr (SIGMA == 16) {
    *(gptr<u64x2>)p = u64x2{0ULL, 0ULL};
  } else {
    *(gptr<u64x2>)p = u64x2{0ULL, 0ULL};
    *(gptr<u64x2>)(p + 16) = u64x2{0ULL, 0ULL};
  }
}

}  // namespace blest
