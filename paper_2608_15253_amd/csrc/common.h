// Shared definitions of libmmx (host and device).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mmx {

// Physical constants (the paper uses gamma0, mu0 and kB without values; the
// mumax3 gyromagnetic ratio, SI mu0 = 4 pi 1e-7 and the exact SI kB are used).
constexpr double kPi = 3.14159265358979323846;
constexpr double kGamma0 = 1.7595e11;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kKB = 1.380649e-23;
constexpr double kHbar = 6.62607015e-34 / (2.0 * kPi);  // exact SI h / 2 pi
constexpr double kQe = 1.602176634e-19;                 // exact SI elementary charge

constexpr int kMaxPass = 16;
constexpr int kTensorStride = 8;  // reals per frequency of the tensor spectrum

// aligned to its size, so that a complex value in LDS moves as one 8-byte
// (FP32) or 16-byte (FP64) access rather than two halves
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__host__ __device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__host__ __device__ inline cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }

// Synchronises the lanes of a one-wave workgroup around LDS exchanges.  A
// wave's memory accesses are performed in issue order, so ordering them at
// wavefront scope needs no wait instruction; unlike __syncthreads(), whose
// workgroup-scope fence waits for every outstanding global load and store,
// global loads issued before this point stay in flight across it.  Only for
// kernels launched with 64 threads per workgroup.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stockham plan of one transform length: radices applied in order; `prune`
// marks a first radix-2 pass whose upper half input is known to be zero.
struct FftPlan {
  int n;
  int npass;
  int prune;
  int radix[kMaxPass];
};

}  // namespace mmx
