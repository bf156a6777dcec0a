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
  cpx<T> X[3][N2];
  // forward, step 1 per component: N1-point transforms over b for a = q +
  // N1 s, twiddles, transpose so that lane q gathers Y[a][q], all a.  The
  // columns of component c + 1 are loaded into the second register set
  // before component c is transformed, and a scheduling barrier after each
  // transpose keeps the compiler from pulling the next transform (and with
  // it the wait for those loads) ahead of it.
  cpx<T> va[S2][N1], vb[S2][N1];
  // loads are unconditional (a lane past the last column reads the last
  // column and drops the value), so that no branch splits a batch of loads
  // and the waits for them can count exactly
  const unsigned offl = live ? off0 : (unsigned)q * (unsigned)Kx + (unsigned)(Kx - 1);
  auto load = [&](cpx<T> (&v)[S2][N1], int c) {
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        if (b < NB) {
          const cpx<T> x = at(offl + (unsigned)c * plane + (unsigned)(N1 * s + N2 * b) * (unsigned)Kx);
          v[s][b] = live ? x : cpx<T>{0, 0};
        } else {
          v[s][b] = cpx<T>{0, 0};
        }
      }
  };
  // twiddle table exp(-2 pi i k / n) staged in LDS (broadcast reads); its
  // loads go out first and the first component's right after them, so the
  // two global latencies overlap
  __shared__ cpx<T> twl[n];
  constexpr int TWL = (n + 63) / 64;
  cpx<T> twv[TWL];
#pragma unroll
  for (int j = 0; j < TWL; ++j)
    if (lane + 64 * j < n) twv[j] = a.tw[lane + 64 * j];
  load(va, 0);
#pragma unroll
  for (int j = 0; j < TWL; ++j)
    if (lane + 64 * j < n) twl[lane + 64 * j] = twv[j];
  wave_sync();
  const cpx<T>* tw = twl;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cpx<T>(&v)[S2][N1] = (c & 1) ? vb : va;
    if (c < 2) load((c & 1) ? va : vb, c + 1);
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int av = q + N1 * s;
      dft_reg<T, false, N1>(v[s]);
      Ew[av] = v[s][0];
#pragma unroll
      for (int cc = 1; cc < N1; ++cc) Ew[cc * STR + av] = cmul(v[s][cc], tw[(av * cc) & (n - 1)]);
    }
    wave_sync();
#pragma unroll
    for (int av = 0; av < N2; ++av) X[c][av] = Ew[q * STR + av];
    wave_sync();
    __builtin_amdgcn_sched_barrier(0);
  }
  // The transpose buffer is free now: the tile's tensor entries (xx, yy, zz,
  // xy of rows ty <= n/2 for its NC columns, [ty][column]) are copied into it
  // straight from global memory (LDS DMA, no registers) while the step-2
  // transforms run.  Fetched one row per lane as the product needs them, the
  // N2 dependent loads took a sixth of the kernel's time.
  constexpr int TROWS = n / 2 + 1, TENT = NC * TROWS;
  static_assert(TENT * sizeof(float4) <= sizeof(E), "tensor tile fits the transpose buffer");
  float4* Tl = reinterpret_cast<float4*>(E);
  {
    const int kx0 = tile * NC;
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the transpose reads of E are done
#pragma unroll
    for (int j = 0; j < (TENT + 63) / 64; ++j) {
      const int e = 64 * j + lane;
      if (e < TENT) {
        const int ty = e / NC, col = e - ty * NC;
        const int kc = min(kx0 + col, Kx - 1);  // columns past Kx: any valid entry, unused
        const T* src = a.Nt + ((size_t)ty * Kx + kc) * kTensorStride;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(Tl + 64 * j),
                                         16, 0, 0);
      }
    }
  }
  // forward, step 2: N2-point transforms over a -> rows ky = q + N1 d
#pragma unroll
  for (int c = 0; c < 3; ++c) dft_reg<T, false, N2>(X[c]);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the tensor entries are in LDS
  wave_sync();
  if (live) {
#pragma unroll
    for (int d = 0; d < N2; ++d) {
      const int ky = q + N1 * d;
      const bool lo = 2 * ky <= n;
      const int ty = lo ? ky : n - ky;
      const T sy = lo ? T(1) : T(-1);
      const float4 e4 = Tl[ty * NC + wc];
      const T ev[4] = {e4.x, e4.y, e4.z, e4.w};
      tensor_apply(ev, 0, sy, T(1), sy, false, X[0][d], X[1][d], X[2][d]);
    }
  }
  wave_sync();  // the inverse transposes overwrite E
  // inverse per component: N2-point transforms over d, conjugate twiddles,
  // transpose back, N1-point transforms over c for a = q + N1 s, store
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dft_reg<T, true, N2>(X[c]);
    Ew[q * STR] = X[c][0];
#pragma unroll
    for (int av = 1; av < N2; ++av) Ew[q * STR + av] = cmulc(X[c][av], tw[(av * q) & (n - 1)]);
    wave_sync();
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
    wave_sync();
  }
}

}  // namespace mmx
