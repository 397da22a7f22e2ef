// Shared device/host helpers: interleaved complex arithmetic for float and
// double, launch checking and the error channel of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace lsw {

template <typename T>
struct cplx;
template <>
struct cplx<double> {
  using type = double2;
};
template <>
struct cplx<float> {
  using type = float2;
};
template <typename T>
using C = typename cplx<T>::type;

template <typename T>
__host__ __device__ inline C<T> mk(T re, T im) {
  C<T> r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename T>
__host__ __device__ inline C<T> cadd(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ inline C<T> csub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ inline C<T> cmul(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__host__ __device__ inline C<T> cmulc(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__host__ __device__ inline C<T> cconj(C<T> a) { return mk<T>(a.x, -a.y); }
template <typename T>
__host__ __device__ inline C<T> cscale(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// acc += a * b
template <typename T>
__host__ __device__ inline C<T> cfma(C<T> acc, C<T> a, C<T> b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
  return acc;
}
template <typename T>
__host__ __device__ inline T cabs2(C<T> a) { return a.x * a.x + a.y * a.y; }

template <typename TO, typename TI>
__host__ __device__ inline C<TO> ccast(C<TI> a) { return mk<TO>((TO)a.x, (TO)a.y); }

// Workgroup barrier that orders LDS accesses only: outstanding global loads
// and stores stay in flight across it (a plain __syncthreads waits for them).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// thread-local message of the last failure of the C ABI
void set_error(const std::string& msg);
const char* get_error();

// v stored at byte offset off of the buffer rs; an offset past the buffer's
// size (the hardware's range check) drops the store, with no branch
template <typename T>
__device__ inline void store_or_drop(__amdgpu_buffer_rsrc_t rs, int off, C<T> v) {
  if constexpr (sizeof(C<T>) == 8) {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, off, 0, 0);
  } else {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), rs, off, 0, 0);
  }
}

}  // namespace lsw

#define LSW_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      lsw::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));           \
      return LS_E_DEVICE;                                                          \
    }                                                                              \
  } while (0)
