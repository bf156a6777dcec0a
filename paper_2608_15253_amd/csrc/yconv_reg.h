// Column convolution of 2-D films with the columns held in registers (device
// code): y transform, tensor product and inverse y transform of N1 N2-point
// columns, one wave per NC = 64 / N1 spectrum columns.
//
// A column x[y], y = a + N2 b (a < N2, b < N1), has the spectrum
//   X[c + N1 d] = sum_a w_N2^(a d) w^(a c) sum_b x[a + N2 b] w_N1^(b c)
// (w = exp(-2 pi i / (N1 N2))).  Lane q of a column first holds the columns
// a = q, q + N1, ... and takes the N1-point transforms over b; the products
// Y[a][c] are transposed through LDS so that lane q then holds all a for
// c = q and takes the N2-point transform over a, which leaves it the spectrum
// rows ky = q + N1 d of all three components: the tensor product is local.
// The inverse runs the same steps backwards (N2-point over d, twiddle,
// transpose, N1-point over c).  Compared with the LDS Stockham kernel this
// moves each column through LDS twice instead of once per radix pass.  With
// a zero-padded (pruned) axis only b < N1/2 carries input and only those rows
// are written back.  The arithmetic differs from the Stockham kernel only in
// the order of the butterflies (round-off level).
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"

namespace mmx {

template <typename T, bool INV, int R>
__device__ inline void dft_reg(cpx<T>* v) {
  if constexpr (R == 2) Dft<T, INV>::r2(v);
  if constexpr (R == 4) Dft<T, INV>::r4(v);
  if constexpr (R == 8) Dft<T, INV>::r8(v);
  if constexpr (R == 12) Dft<T, INV>::r12(v);
  if constexpr (R == 16) Dft<T, INV>::r16(v);
  if constexpr (R == 24) Dft<T, INV>::r24(v);
  if constexpr (R == 32) Dft<T, INV>::r32(v);
}

template <typename T, int N1, int N2, bool PRUNE>
__global__ void __launch_bounds__(64) k_yconv_reg(YArgs<T> a) {
  static_assert(N2 % N1 == 0 && 64 % N1 == 0, "column split");
  constexpr int n = N1 * N2, NC = 64 / N1, S2 = N2 / N1, STR = N2 + 1;
  constexpr int NB = PRUNE ? N1 / 2 : N1;  // input rows (forward) = output rows (inverse) per a
  __shared__ cpx<T> E[NC * N1 * STR];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x, wc = lane / N1, q = lane - wc * N1;
  // neighbouring column tiles of a replica share cache lines of the spectrum
  // rows: keep them on one XCD
  int tile, by, rep;
  xcd_block(tile, by, rep);
  if (a.sw_tsw && tile == 0 && lane == 0) {
    const unsigned long long st = (a.sw_stepdev ? *a.sw_stepdev : 0ull) + a.sw_step;
    switch_check(a.sw_part, a.sw_tsw, *a.sw_nblk, a.sw_N, rep, (double)st * a.sw_dt);
  }
  const int kx = tile * NC + wc;
  const bool live = kx < a.Kx;
  const int Kx = a.Kx;
  // one component of one replica (nz = 1); offsets within the replica are
  // 32-bit on a workgroup-uniform base pointer (one address register per
  // access instead of a 64-bit pair)
  const unsigned plane = (unsigned)a.Sy * (unsigned)Kx;
  cpx<T>* __restrict__ S = a.S + (size_t)rep * 3 * plane;
  const unsigned off0 = (unsigned)q * (unsigned)Kx + (unsigned)kx;
  // element i of the replica's spectrum: 32-bit byte offset on the uniform base
  auto at = [&](unsigned i) -> cpx<T>& {
    return *reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(S) + i * (unsigned)sizeof(cpx<T>));
  };
  cpx<T>* Ew = E + wc * N1 * STR;
  // twiddle table exp(-2 pi i k / n) staged in LDS (broadcast reads)
  __shared__ cpx<T> twl[n];
  for (int i = lane; i < n; i += 64) twl[i] = a.tw[i];
  __syncthreads();
  const cpx<T>* tw = twl;
  cpx<T> X[3][N2];
  // forward, step 1 per component (the next component's loads are issued
  // before the transpose of the current one): N1-point transforms over b for
  // a = q + N1 s, twiddles, transpose so that lane q gathers Y[a][q], all a
  cpx<T> v[S2][N1];
  auto load = [&](int c) {
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b)
        v[s][b] = (b < NB && live)
                      ? at(off0 + (unsigned)c * plane + (unsigned)(N1 * s + N2 * b) * (unsigned)Kx)
                      : cpx<T>{0, 0};
  };
  load(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int av = q + N1 * s;
      dft_reg<T, false, N1>(v[s]);
      Ew[av] = v[s][0];
#pragma unroll
      for (int cc = 1; cc < N1; ++cc) Ew[cc * STR + av] = cmul(v[s][cc], tw[(av * cc) & (n - 1)]);
    }
    if (c < 2) load(c + 1);
    __syncthreads();
#pragma unroll
    for (int av = 0; av < N2; ++av) X[c][av] = Ew[q * STR + av];
    __syncthreads();
  }
  // forward, step 2: N2-point transforms over a -> rows ky = q + N1 d
#pragma unroll
  for (int c = 0; c < 3; ++c) dft_reg<T, false, N2>(X[c]);
  if (live) {
#pragma unroll
    for (int d = 0; d < N2; ++d) {
      const int ky = q + N1 * d;
      const bool lo = 2 * ky <= n;
      const int ty = lo ? ky : n - ky;
      const T sy = lo ? T(1) : T(-1);
      tensor_apply(a.Nt, (size_t)ty * Kx + kx, sy, T(1), sy, false, X[0][d], X[1][d],
                   X[2][d]);
    }
  }
  // inverse per component: N2-point transforms over d, conjugate twiddles,
  // transpose back, N1-point transforms over c for a = q + N1 s, store
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dft_reg<T, true, N2>(X[c]);
    Ew[q * STR] = X[c][0];
#pragma unroll
    for (int av = 1; av < N2; ++av) Ew[q * STR + av] = cmulc(X[c][av], tw[(av * q) & (n - 1)]);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int av = q + N1 * s;
      cpx<T> u[N1];
#pragma unroll
      for (int cc = 0; cc < N1; ++cc) u[cc] = Ew[cc * STR + av];
      dft_reg<T, true, N1>(u);
      if (live) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          at(off0 + (unsigned)c * plane + (unsigned)(N1 * s + N2 * b) * (unsigned)Kx) = u[b];
      }
    }
    __syncthreads();
  }
}

}  // namespace mmx
