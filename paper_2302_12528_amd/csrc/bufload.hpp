// Raw buffer loads and stores (MUBUF) for the streaming kernels.
//
// A buffer resource describes [base, base + bytes); a load takes a per-lane byte offset (VGPR) and a
// wave-uniform byte offset (SGPR), so a kernel that walks a matrix keeps one 32-bit offset per lane
// and advances a scalar, instead of carrying a 64-bit address per load.  A load whose offset lies at
// or beyond `bytes` returns zeros without touching memory (a store there is dropped); kOob is such an
// offset for every resource made here (bytes < 2^31) and is how masked lanes are expressed.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lobpcg {

typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
typedef int32_t i32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

__device__ f32x4_t llvm_buffer_load_f32x4(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v4f32");
__device__ f64x2_t llvm_buffer_load_f64x2(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2f64");
__device__ float llvm_buffer_load_f32(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.f32");
__device__ double llvm_buffer_load_f64(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.f64");
__device__ i32x4_t llvm_buffer_load_i32x4(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v4i32");
__device__ i32x2_t llvm_buffer_load_i32x2(i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2i32");
__device__ void llvm_buffer_store_f32x4(f32x4_t v, i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.store.v4f32");
__device__ void llvm_buffer_store_f64x2(f64x2_t v, i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.store.v2f64");
__device__ void llvm_buffer_store_f32(float v, i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.store.f32");
__device__ void llvm_buffer_store_f64(double v, i32x4_t rsrc, int32_t voffset, int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.raw.buffer.store.f64");

constexpr int32_t kOob = 0x7ffffff0;   // past the end of every resource (bytes < 2^31 - 2^4)

// Resource word 3 for gfx9-family raw buffers: 32-bit data format, no swizzle, no index stride.
__device__ inline i32x4_t make_rsrc(const void* base, int64_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  i32x4_t r;
  r.x = (int32_t)(uint32_t)(a & 0xffffffffu);
  r.y = (int32_t)(uint32_t)((a >> 32) & 0xffffu);
  r.z = (int32_t)(uint32_t)bytes;
  r.w = 0x00020000;
  return r;
}

// 16 bytes into VW = 16 / sizeof(T) values.
template <typename T> struct Buf;
template <> struct Buf<float> {
  static __device__ inline void load16(i32x4_t r, int32_t v, int32_t s, float (&o)[4]) {
    const f32x4_t q = llvm_buffer_load_f32x4(r, v, s, 0);
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
  }
  static __device__ inline float load1(i32x4_t r, int32_t v, int32_t s) { return llvm_buffer_load_f32(r, v, s, 0); }
  static __device__ inline void store16(i32x4_t r, int32_t v, int32_t s, const float (&o)[4]) {
    llvm_buffer_store_f32x4(f32x4_t{o[0], o[1], o[2], o[3]}, r, v, s, 0);
  }
  static __device__ inline void store1(i32x4_t r, int32_t v, int32_t s, float o) { llvm_buffer_store_f32(o, r, v, s, 0); }
  static __device__ inline void load_idx(i32x4_t r, int32_t v, int32_t s, int32_t (&o)[4]) {
    const i32x4_t q = llvm_buffer_load_i32x4(r, v, s, 0);
    o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
  }
};
template <> struct Buf<double> {
  static __device__ inline void load16(i32x4_t r, int32_t v, int32_t s, double (&o)[2]) {
    const f64x2_t q = llvm_buffer_load_f64x2(r, v, s, 0);
    o[0] = q.x; o[1] = q.y;
  }
  static __device__ inline double load1(i32x4_t r, int32_t v, int32_t s) { return llvm_buffer_load_f64(r, v, s, 0); }
  static __device__ inline void store16(i32x4_t r, int32_t v, int32_t s, const double (&o)[2]) {
    llvm_buffer_store_f64x2(f64x2_t{o[0], o[1]}, r, v, s, 0);
  }
  static __device__ inline void store1(i32x4_t r, int32_t v, int32_t s, double o) { llvm_buffer_store_f64(o, r, v, s, 0); }
  static __device__ inline void load_idx(i32x4_t r, int32_t v, int32_t s, int32_t (&o)[2]) {
    const i32x2_t q = llvm_buffer_load_i32x2(r, v, s, 0);
    o[0] = q.x; o[1] = q.y;
  }
};

}  // namespace lobpcg
