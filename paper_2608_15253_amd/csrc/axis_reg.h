// Transforms of 3-D grids along y and z with the lines held in registers
// (device code), the split of yconv_reg.h applied to other axes:
//
//  k_ypass_reg  the y transform of one (component, plane) line per column,
//               forward (input rows y < ny, all Py spectrum rows out) or
//               inverse (all rows in, rows y < ny out); no tensor product.
//  k_zline_reg  the z transform of a pillar (ky, kx) of all three
//               components, the full symmetric tensor product per (kz, ky,
//               kx) and the inverse z transform, keeping the nz stored planes.
//
// A line x[j], j = a + N2 b (a < N2, b < N1), is split over N1 lanes: lane q
// takes the N1-point DFTs over b for a = q + N1 s, twiddles, one LDS
// transpose, and the N2-point DFT over a leaves it the outputs q + N1 d.
// One wave holds NC = 64 / N1 lines of consecutive kx, so each global access
// covers NC neighbouring columns of one row (plane).  With a zero-padded
// axis (PRUNE) only b < N1 / 2 carries input and only those outputs are
// written back.  The arithmetic equals the LDS Stockham passes up to the
// order of the butterflies.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "yconv_reg.h"

namespace mmx {

// y pass of 3-D grids: grid (ceil(Kx / NC), 3 nz, R), one wave per workgroup
template <typename T, int N1, int N2, bool INV, bool PRUNE>
__global__ void __launch_bounds__(64) k_ypass_reg(YArgs<T> a) {
  static_assert(N2 % N1 == 0 && 64 % N1 == 0, "line split");
  constexpr int n = N1 * N2, NC = 64 / N1, S2 = N2 / N1, STR = N2 + 1;
  constexpr int NB = PRUNE ? N1 / 2 : N1;  // rows y = a + N2 b kept (b < NB)
  __shared__ cpx<T> E[NC * N1 * STR];
  __shared__ cpx<T> twl[n];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x, wc = lane / N1, q = lane - wc * N1;
  int tile, line, rep;
  xcd_block(tile, line, rep);
  const int kx = tile * NC + wc;
  const bool live = kx < a.Kx;
  const unsigned Kx = (unsigned)a.Kx;
  // the (component, plane) line of the replica; 32-bit offsets on the
  // workgroup-uniform base
  cpx<T>* __restrict__ P = a.S + ((size_t)rep * 3 * a.nz + line) * (size_t)a.Sy * Kx;
  auto at = [&](unsigned row) -> cpx<T>& {
    return *reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(P) +
                                      (row * Kx + (unsigned)kx) * (unsigned)sizeof(cpx<T>));
  };
  // loads are unconditional (a lane past the last column reads the last
  // column; what it computes is never stored), so that no branch splits a
  // batch of loads; the twiddle table's loads go out first, the line's right
  // after them, and the table is written to LDS once both are in flight
  const unsigned kxl = live ? (unsigned)kx : Kx - 1;
  auto atl = [&](unsigned row) -> cpx<T> {
    return *reinterpret_cast<const cpx<T>*>(reinterpret_cast<const char*>(P) +
                                            (row * Kx + kxl) * (unsigned)sizeof(cpx<T>));
  };
  constexpr int TWL = (n + 63) / 64;
  cpx<T> twv[TWL];
#pragma unroll
  for (int j = 0; j < TWL; ++j)
    if (lane + 64 * j < n) twv[j] = a.tw[lane + 64 * j];
  cpx<T>* Ew = E + wc * N1 * STR;
  cpx<T> X[N2];
  cpx<T> v[INV ? 1 : S2][N1];
  if constexpr (!INV) {
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b)
        v[s][b] = (b < NB) ? atl((unsigned)(q + N1 * s + N2 * b)) : cpx<T>{0, 0};
  } else {
#pragma unroll
    for (int d = 0; d < N2; ++d) X[d] = atl((unsigned)(q + N1 * d));
  }
#pragma unroll
  for (int j = 0; j < TWL; ++j)
    if (lane + 64 * j < n) twl[lane + 64 * j] = twv[j];
  wave_sync();
  const cpx<T>* tw = twl;
  if constexpr (!INV) {
#pragma unroll
    for (int s = 0; s < S2; ++s) {
      const int av = q + N1 * s;
      dft_reg<T, false, N1>(v[s]);
      Ew[av] = v[s][0];
#pragma unroll
      for (int cc = 1; cc < N1; ++cc) Ew[cc * STR + av] = cmul(v[s][cc], tw[av * cc]);
    }
    wave_sync();
#pragma unroll
    for (int av = 0; av < N2; ++av) X[av] = Ew[q * STR + av];
    dft_reg<T, false, N2>(X);
    if (live) {
#pragma unroll
      for (int d = 0; d < N2; ++d) at((unsigned)(q + N1 * d)) = X[d];
    }
  } else {
    dft_reg<T, true, N2>(X);
    Ew[q * STR] = X[0];
#pragma unroll
    for (int av = 1; av < N2; ++av) Ew[q * STR + av] = cmulc(X[av], tw[av * q]);
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
        for (int b = 0; b < NB; ++b) at((unsigned)(av + N2 * b)) = u[b];
      }
    }
  }
}

// z pass of 3-D grids with the tensor product: grid (ceil(Kx / NC), Py, R),
// one wave per workgroup; the Pz = N1 N2 point pillar of component c at
// (ky, kx) is S[((r 3 + c) nz + z) Sy Kx + ky Kx + kx], z < nz
template <typename T, int N1, int N2, bool PRUNE>
__global__ void __launch_bounds__(64) k_zline_reg(YArgs<T> a) {
  static_assert(N2 % N1 == 0 && 64 % N1 == 0, "line split");
  constexpr int n = N1 * N2, NC = 64 / N1, S2 = N2 / N1, STR = N2 + 1;
  constexpr int NB = PRUNE ? N1 / 2 : N1;
  // the transpose buffer also takes the tile's tensor entries between the
  // forward and the inverse transposes: NC columns x (n/2 + 1) kz rows x the
  // 8 reals of a frequency, [tz][column] as two 16-byte halves
  constexpr int TROWS = n / 2 + 1, TENT = NC * TROWS;
  constexpr int ESZ = NC * N1 * STR > 4 * TENT ? NC * N1 * STR : 4 * TENT;
  __shared__ cpx<T> E[ESZ];
  __shared__ cpx<T> twl[n];
  if (a.done && *a.done) return;
  const int lane = threadIdx.x, wc = lane / N1, q = lane - wc * N1;
  int tile, ky, rep;
  xcd_block(tile, ky, rep);
  const int kx = tile * NC + wc;
  const bool live = kx < a.Kx;
  const unsigned Kx = (unsigned)a.Kx, plane = (unsigned)a.Sy * Kx, nz = (unsigned)a.nz;
  cpx<T>* __restrict__ P = a.S + (size_t)rep * 3 * nz * plane;
  // element (c, z) of this pillar: 32-bit byte offset on the uniform base
  auto at = [&](int c, unsigned z) -> cpx<T>& {
    const unsigned i = ((unsigned)c * nz + z) * plane + (unsigned)ky * Kx + (unsigned)kx;
    return *reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(P) + i * (unsigned)sizeof(cpx<T>));
  };
  // loads are unconditional (a lane past the last column reads the last
  // column; what it computes is never stored), so that no branch splits a
  // batch; component c + 1 is loaded into the second register set before
  // component c is transformed, and a scheduling barrier after each
  // transpose keeps the next transform (and its wait) behind it.  The z
  // pass arguments carry the z twiddles exp(-2 pi i k / Pz) in tw; their
  // loads go out first.
  const unsigned kxl = live ? (unsigned)kx : Kx - 1;
  auto atl = [&](int c, unsigned z) -> cpx<T> {
    const unsigned i = ((unsigned)c * nz + z) * plane + (unsigned)ky * Kx + kxl;
    return *reinterpret_cast<const cpx<T>*>(reinterpret_cast<const char*>(P) +
                                            i * (unsigned)sizeof(cpx<T>));
  };
  constexpr int TWL = (n + 63) / 64;
  cpx<T> twv[TWL];
#pragma unroll
  for (int j = 0; j < TWL; ++j)
    if (lane + 64 * j < n) twv[j] = a.tw[lane + 64 * j];
  cpx<T>* Ew = E + wc * N1 * STR;
  cpx<T> X[3][N2];
  cpx<T> va[S2][N1], vb[S2][N1];
  auto load = [&](cpx<T> (&v)[S2][N1], int c) {
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b)
        v[s][b] = (b < NB) ? atl(c, (unsigned)(q + N1 * s + N2 * b)) : cpx<T>{0, 0};
  };
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
      for (int cc = 1; cc < N1; ++cc) Ew[cc * STR + av] = cmul(v[s][cc], tw[av * cc]);
    }
    wave_sync();
#pragma unroll
    for (int av = 0; av < N2; ++av) X[c][av] = Ew[q * STR + av];
    wave_sync();
    __builtin_amdgcn_sched_barrier(0);
  }
  // the tile's tensor entries go straight from global memory into the free
  // transpose buffer (direct-to-LDS loads, no registers) while the step-2
  // transforms run, instead of N2 dependent loads per lane
  const bool ylo = 2 * ky <= a.Py;
  const int ty = ylo ? ky : a.Py - ky;
  static_assert(sizeof(T) == 4, "FP32 register passes");
  float4* Tl = reinterpret_cast<float4*>(E);
  {
    const int kx0 = tile * NC;
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the transpose reads of E are done
#pragma unroll
    for (int j = 0; j < (2 * TENT + 63) / 64; ++j) {
      const int e2 = 64 * j + lane;  // half h of entry e
      if (e2 < 2 * TENT) {
        const int e = e2 >> 1, h = e2 & 1;
        const int tz = e / NC, col = e - tz * NC;
        const int kc = min(kx0 + col, (int)Kx - 1);  // columns past Kx: any valid entry, unused
        const T* src = a.Nt + (((size_t)tz * a.Ty + ty) * Kx + kc) * kTensorStride + 4 * h;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(Tl + 64 * j),
                                         16, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) dft_reg<T, false, N2>(X[c]);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the tensor entries are in LDS
  wave_sync();
  if (live) {
    // lane q holds kz = q + N1 d of all three components: the product is local
    const T sy = ylo ? T(1) : T(-1);
#pragma unroll
    for (int d = 0; d < N2; ++d) {
      const int kz = q + N1 * d;
      const bool zlo = 2 * kz <= n;
      const int tz = zlo ? kz : n - kz;
      const T sz = zlo ? T(1) : T(-1);
      const float4 e0 = Tl[2 * (tz * NC + wc)], e1 = Tl[2 * (tz * NC + wc) + 1];
      const T ev[6] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y};
      tensor_apply(ev, 0, sy, sz, sy * sz, true, X[0][d], X[1][d], X[2][d]);
    }
  }
  wave_sync();  // the inverse transposes overwrite E
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dft_reg<T, true, N2>(X[c]);
    Ew[q * STR] = X[c][0];
#pragma unroll
    for (int av = 1; av < N2; ++av) Ew[q * STR + av] = cmulc(X[c][av], tw[av * q]);
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
        for (int b = 0; b < NB; ++b) at(c, (unsigned)(av + N2 * b)) = u[b];
      }
    }
    wave_sync();
  }
}

}  // namespace mmx
