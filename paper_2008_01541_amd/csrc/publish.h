// Cross-workgroup publication inside one launch (dataflow Cholesky, solves):
// agent-coherent loads and stores, bounded flag waits that raise an error
// word, and the flag store after a workgroup's data stores have drained.
// Header-only: included by each kernel file that publishes or consumes.
#pragma once
#include "common.h"

namespace pdk {

__device__ inline double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void coherent_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long SPIN_LIMIT_DF = 1L << 24;

// Cross-workgroup publication protocol.  Tiles, tile inverses and solve
// vectors are written with agent-coherent (write-through) stores; after every
// thread's stores have completed (s_waitcnt vmcnt(0)) and a barrier, one
// thread stores the ready flag.  Consumers poll flags with agent-coherent
// loads.  Published data is immutable for the rest of the launch, its cache
// lines are never touched before publication by other workgroups (tiles are
// 128-byte aligned: leading dimensions are multiples of 16 doubles, and the
// owner reads its input tile with coherent loads), so plain cached loads of
// published data cannot see stale lines and no cache invalidation is needed.
__device__ inline void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

__device__ inline bool df_wait(const int* f, int epoch, int* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > SPIN_LIMIT_DF) {
      atomicExch(err, 1);
      return false;
    }
  }
  return true;
}

__device__ inline void publish_flag(int* f, int epoch) {
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pdk
