// Row pass of the stochastic Heun stages with the rows held in registers
// (device code): inverse x transform of the demag spectrum, local fields,
// torque, predictor or corrector update, and the forward x transform of the
// state just written, for films whose half-length x transform has
// hx = NR * NR points (NR = 4 or 8).
//
// One wave holds RPW = 64 / NR grid rows; lane q of a row owns the packed
// positions k = q + NR d (d < NR), i.e. the cells x = 2k and 2k + 1, for all
// three components.  A transform of the row, X[c + NR d'] = sum_k x[k]
// w^(+-k (c + NR d')), splits k = a + NR b: lane q = a takes the NR-point
// DFT over b in registers, multiplies by w^(+-a c), the values are transposed
// through LDS so that lane c holds all a, and an NR-point DFT over a leaves
// lane c the outputs c + NR d'.  With the square split the outputs of the
// inverse transform sit in the lanes that own the cells, and the new state
// of those cells is already in the input layout of the forward transform,
// so a row crosses LDS once per direction (plus one exchange to pair X[k]
// with X[hx - k] for the real-to-complex split).  The cell arithmetic is the
// one of k_fields; only the butterfly order of the transforms differs.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "philox.h"
#include "yconv_reg.h"

namespace mmx {

template <typename T, int NR>
__device__ inline void row_transform_step(cpx<T> (&v)[3][NR], cpx<T>* E, int q,
                                          const cpx<T>* __restrict__ tw, int tw_stride,
                                          bool inv) {
  constexpr int STR = NR + 1;
  // NR-point DFTs over b (lane q = a), twiddles w^(+-a c), transpose
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (inv) dft_reg<T, true, NR>(v[c]); else dft_reg<T, false, NR>(v[c]);
#pragma unroll
    for (int cc = 1; cc < NR; ++cc) {
      const cpx<T> w = tw[((q * cc) & (NR * NR - 1)) * tw_stride];
      v[c][cc] = inv ? cmulc(v[c][cc], w) : cmul(v[c][cc], w);
    }
#pragma unroll
    for (int cc = 0; cc < NR; ++cc) E[(c * NR + cc) * STR + q] = v[c][cc];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int av = 0; av < NR; ++av) v[c][av] = E[(c * NR + q) * STR + av];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (inv) dft_reg<T, true, NR>(v[c]); else dft_reg<T, false, NR>(v[c]);
  }
}

template <typename T, int NR, int MODE>
__global__ void __launch_bounds__(64) k_rows_reg(FArgs<T> a) {
  static_assert(MODE == FM_HEUN1 || MODE == FM_HEUN2, "Heun stages only");
  constexpr int hx = NR * NR, RPW = 64 / NR, STR = NR + 1;
  __shared__ cpx<T> Es[RPW * 3 * NR * STR];
  __shared__ double red[64];
  const int lane = threadIdx.x, row = lane / NR, q = lane - row * NR;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, z = by, y = bx * RPW + row;
  const bool live = y < a.ny;
  cpx<T>* E = Es + row * 3 * NR * STR;
  const size_t rb = (size_t)r * 3 * a.N;
  const unsigned N = (unsigned)a.N;
  const int Kx = a.Kx;
  // spectrum row of component c: S[(((r 3 + c) nz + z) Sy + y) Kx + kx]
  cpx<T>* Srow = a.S + (((size_t)r * 3 * a.nz + z) * a.Sy + (live ? y : 0)) * Kx;
  const size_t cstride = (size_t)a.nz * a.Sy * Kx;
  const cpx<T>* __restrict__ tw = a.tw;  // exp(-2 pi i k / hx), k < hx
  // 1. inverse x transform of the demag spectrum: lane q loads the packed
  //    inputs Z[q + NR b] (complex-to-real combination of S[k], S[hx - k])
  cpx<T> v[3][NR];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int k = q + NR * b;
      cpx<T> Zv = {0, 0};
      if (live) {
        const cpx<T> Xk = Srow[c * cstride + k];
        cpx<T> Xc = Srow[c * cstride + (hx - k)];
        Xc.im = -Xc.im;
        const cpx<T> Ev = cadd(Xk, Xc);
        const cpx<T> D = csub(Xk, Xc);
        const cpx<T> O = cmulc(D, a.wpost[k]);  // D * conj(W^k)
        Zv = {Ev.re - O.im, Ev.im + O.re};
      }
      v[c][b] = Zv;
    }
  row_transform_step<T, NR>(v, E, q, tw, 1, true);
  // lane q now holds z[q + NR d] = H_demag at cells x = 2 (q + NR d) + {0, 1};
  // the row's field goes to LDS (real view, [c][x]) so that the cell loop
  // below holds one cell at a time and each lane takes the cells x = q + NR j
  T* Hs = reinterpret_cast<T*>(E);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      Hs[c * 2 * hx + 2 * (q + NR * d)] = v[c][d].re;
      Hs[c * 2 * hx + 2 * (q + NR * d) + 1] = v[c][d].im;
    }
  __syncthreads();
  const T dt = (T)a.dth;
  T sigma = 0;
  if ((a.terms & T_THERMAL) && a.Trep) {
    const double Tr = a.Trep[r];
    if (Tr > 0) sigma = (T)sqrt(a.sig2pref * Tr / a.dt_th);
  }
  const uint64_t step_now = a.stepdev ? *a.stepdev : a.step;
  const T* __restrict__ mr = a.m + rb;
  T* mout_r = a.mout + rb;
  T* k1_r = a.k1 + rb;
  double acc = 0;
#pragma unroll 2
  for (int j = 0; j < 2 * NR; ++j) {
    const int x = q + NR * j;
    T mn_out[3] = {0, 0, 0};
    if (live && x < a.nx) {
      const unsigned cell = (unsigned)x + (unsigned)a.nx * (unsigned)(y + a.ny * z);
      T mc[3];
      ld3(mr, N, cell, mc);
      T Hex[3], Hdm[3], Han[3], Hz[3];
      local_terms(a, mr, cell, x, y, z, mc, a.kbc, Hex, Hdm, Han, Hz);
      T H[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) H[c] = Hex[c] + Hdm[c] + Han[c] + Hz[c] + Hs[c * 2 * hx + x];
      if (sigma != T(0)) {
        T eta[3];
        thermal_eta<T>(a.seeds[r], (uint32_t)cell, step_now, eta);
#pragma unroll
        for (int c = 0; c < 3; ++c) H[c] += sigma * eta[c];
      }
      T kv[3];
      llg_torque(mc, H, a.gpm, a.alpha, kv);
      if (MODE == FM_HEUN1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mn_out[c] = mc[c] + dt * kv[c];
          k1_r[c * N + cell] = kv[c];
          mout_r[c * N + cell] = mn_out[c];
        }
      } else {
        T mo[3], k1v[3], mn[3];
        ld3(a.m0 + rb, N, cell, mo);
        ld3(k1_r, N, cell, k1v);
#pragma unroll
        for (int c = 0; c < 3; ++c) mn[c] = mo[c] + T(0.5) * dt * (k1v[c] + kv[c]);
        const T inv = T(1) / sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          mn_out[c] = mn[c] * inv;
          mout_r[c * N + cell] = mn_out[c];
        }
        acc += (double)mn_out[2];
      }
    }
    // the new state is the forward transform's input (zero beyond the last
    // cell); it replaces the field value of the same cell
#pragma unroll
    for (int c = 0; c < 3; ++c) Hs[c * 2 * hx + x] = mn_out[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < NR; ++d)
      v[c][d] = {Hs[c * 2 * hx + 2 * (q + NR * d)], Hs[c * 2 * hx + 2 * (q + NR * d) + 1]};
  __syncthreads();
  // 2. forward x transform of the new state; lane q ends with X[q + NR d']
  row_transform_step<T, NR>(v, E, q, tw, 1, false);
  // 3. real-to-complex split S[kx] = E + conj(W^kx) O, kx = q + NR d' and
  //    (lane 0) kx = hx; the partner X[hx - kx] comes through LDS
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < NR; ++d) E[c * hx + q + NR * d] = v[c][d];
  __syncthreads();
  if (live) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int d = 0; d <= NR; ++d) {
        const int kx = (d < NR) ? q + NR * d : hx;
        if (d == NR && q != 0) continue;
        const cpx<T> Zk = E[c * hx + (kx == hx ? 0 : kx)];
        cpx<T> Zc = E[c * hx + (kx == 0 ? 0 : hx - kx)];
        Zc.im = -Zc.im;
        const cpx<T> Ev = {T(0.5) * (Zk.re + Zc.re), T(0.5) * (Zk.im + Zc.im)};
        const cpx<T> O = {T(0.5) * (Zk.re - Zc.re), T(0.5) * (Zk.im - Zc.im)};
        const cpx<T> w = a.wpost[kx];
        Srow[c * cstride + kx] = {Ev.re + (w.re * O.im + w.im * O.re),
                                  Ev.im - (w.re * O.re - w.im * O.im)};
      }
    }
  }
  if (MODE == FM_HEUN2) {
    // per-workgroup sum of m_z (fixed order) for the switching detector
    red[lane] = acc;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
      if (lane < s) red[lane] += red[lane + s];
      __syncthreads();
    }
    if (lane == 0) {
      const size_t blk = (size_t)by * gridDim.x + bx;
      const size_t nblk = (size_t)gridDim.x * gridDim.y;
      a.partial[(size_t)r * nblk + blk] = red[0];
    }
  }
}

}  // namespace mmx
