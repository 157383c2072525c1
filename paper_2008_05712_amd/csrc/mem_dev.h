// Device memory accessors shared by the force and reorganisation code.
//
// Argument blocks that a kernel reads from memory (the whole-step kernel's per-round blocks) carry
// generic pointers, for which the compiler emits FLAT instructions.  Those count on the LDS counter
// as well, so every wait for an LDS read would also wait for outstanding memory loads (a prefetched
// node tile among them), and their addresses take 64-bit vector arithmetic.  Every buffer here is
// device global memory, so it is accessed as such: GLOBAL instructions with a scalar base.  Vector
// values go through native vector types (HIP's float4 copy constructor takes a generic reference,
// which would turn the access back into a FLAT one).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gc {
namespace dev {

#define GC_GLOBAL(T) __attribute__((address_space(1))) T
typedef float gc_vf4 __attribute__((ext_vector_type(4)));
typedef int gc_vi4 __attribute__((ext_vector_type(4)));
typedef int gc_vi2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float4 gld(const float4* p) {
  const gc_vf4 v = *(const GC_GLOBAL(gc_vf4)*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 gld(const int4* p) {
  const gc_vi4 v = *(const GC_GLOBAL(gc_vi4)*)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int2 gld(const int2* p) {
  const gc_vi2 v = *(const GC_GLOBAL(gc_vi2)*)p;
  return make_int2(v.x, v.y);
}
// The first three words of a record, its fourth left zero (a load of three words: no register is
// written that nothing reads, which would make later reuse of that register wait for the load).
typedef float gc_vf3 __attribute__((ext_vector_type(3)));
__device__ __forceinline__ float4 gld_xyz(const float4* p) {
  const gc_vf3 v = *(const GC_GLOBAL(gc_vf3)*)p;
  return make_float4(v.x, v.y, v.z, 0.f);
}
__device__ __forceinline__ int32_t gld(const int32_t* p) { return *(const GC_GLOBAL(int32_t)*)p; }
__device__ __forceinline__ uint32_t gld(const uint32_t* p) { return *(const GC_GLOBAL(uint32_t)*)p; }

__device__ __forceinline__ void gst(float4* p, const float4 v) {
  const gc_vf4 w = {v.x, v.y, v.z, v.w};
  *(GC_GLOBAL(gc_vf4)*)p = w;
}
__device__ __forceinline__ uint64_t gld(const uint64_t* p) { return *(const GC_GLOBAL(uint64_t)*)p; }
__device__ __forceinline__ void gst(uint64_t* p, uint64_t v) { *(GC_GLOBAL(uint64_t)*)p = v; }
__device__ __forceinline__ void gst(int32_t* p, int32_t v) { *(GC_GLOBAL(int32_t)*)p = v; }
__device__ __forceinline__ void gst(uint32_t* p, uint32_t v) { *(GC_GLOBAL(uint32_t)*)p = v; }

// Relaxed device-scope atomic loads and stores (coherent across the XCDs' L2s).
__device__ __forceinline__ uint64_t aload(uint64_t* p) {
  return __hip_atomic_load((GC_GLOBAL(uint64_t)*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(uint64_t* p, uint64_t v) {
  __hip_atomic_store((GC_GLOBAL(uint64_t)*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t aload(int32_t* p) {
  return __hip_atomic_load((GC_GLOBAL(int32_t)*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(int32_t* p, int32_t v) {
  __hip_atomic_store((GC_GLOBAL(int32_t)*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dev
}  // namespace gc
