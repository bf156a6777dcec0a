// Replica-resident stochastic Heun kernel for 2-D films (device code).
//
// One workgroup owns one replica for a run of steps.  The half spectrum of the
// replica's magnetisation (3 x ny x (Px/2+1) complex values) stays in LDS for
// the whole field evaluation: the x transforms of row chunks write into it,
// the y transform + tensor product + inverse works on column chunks in place,
// and the inverse x transform of row chunks feeds the local fields, torque and
// Heun update directly.  HBM is touched only for the magnetisation itself
// (stencil neighbours and the predictor state).  The corrector takes the
// predictor's slope from the predictor state, (m + m~)/2 + dt/2 k, with the
// epilogue of the three-kernel path (heun_correct), so no slope is stored.
// The local terms, torque and update are those of the three-kernel path; the
// transforms are LDS Stockham passes, so results agree with that path to
// round-off, not bit for bit.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "philox.h"

namespace mmx {

constexpr int kFusedBlock = 1024;
constexpr int kFusedMaxChunks = 8;

template <typename T>
struct HeunFusedArgs {
  FArgs<T> f;           // geometry, coefficients, thermal keys, tables
  FftPlan pxf, pxi, pyf, pyi;
  const cpx<T>* tw_x;
  const cpx<T>* wpost;
  const cpx<T>* tw_y;
  const T* Nt;          // [Ty][Kx][kTensorStride], 2-D: xx, yy, zz, xy used
  int Ty, Py;
  T* m;                 // state, updated in place
  T* ms;                // predictor state (stencil source of the corrector)
  double* tsw;          // switching times or null
  double dt;
  uint64_t step0;
  const unsigned long long* stepdev;  // if set, the step index is *stepdev + step0
  int nsteps;
  int C;                // grid rows per x chunk
  int W;                // spectrum columns per y chunk
  int nch;              // ceil(ny / C) <= kFusedMaxChunks
};

// Forward half of the demag convolution of the replica's state `src`
// (global): x transforms of row chunks into the LDS spectrum X, then the y
// transform, tensor product and inverse y transform of column chunks in place.
template <typename T>
__device__ inline void fused_forward(const HeunFusedArgs<T>& a, const T* __restrict__ src,
                                     size_t rb, cpx<T>* X, cpx<T>* A, cpx<T>* Bf,
                                     const cpx<T>* twx, const cpx<T>* wpost,
                                     const cpx<T>* twy) {
  const FArgs<T>& f = a.f;
  const int hx = f.hx, Kx = f.Kx, ny = f.ny, nx = f.nx, C = a.C;
  const int npair = (nx + 1) / 2;
  // phase 1: x forward transforms of row chunks into X
  for (int q = 0; q < a.nch; ++q) {
    const int y0 = q * C;
    for (int t = threadIdx.x; t < C * hx; t += blockDim.x) {
      const int l = udiv(t, hx), k = t - l * hx, y = y0 + l;
      cpx<T> v[3] = {{0, 0}, {0, 0}, {0, 0}};
      if (y < ny && k < npair) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int x = 2 * k + h;
          if (x >= nx) break;
          const size_t cell = (size_t)x + (size_t)nx * y;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T s = src[rb + (size_t)c * f.N + cell];
            if (h == 0) v[c].re = s; else v[c].im = s;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) A[(c * C + l) * hx + k] = v[c];
    }
    __syncthreads();
    const cpx<T>* Z = lds_fft<T, false>(A, Bf, 3 * C, a.pxf, twx);
    for (int t = threadIdx.x; t < 3 * C * Kx; t += blockDim.x) {
      const int line = t / Kx, kx = t - line * Kx;
      const int c = udiv(line, C), l = line - c * C, y = y0 + l;
      if (y >= ny) continue;
      const cpx<T> Zk = Z[line * hx + (kx == hx ? 0 : kx)];
      cpx<T> Zc = Z[line * hx + (kx == 0 ? 0 : hx - kx)];
      Zc.im = -Zc.im;
      const cpx<T> E = {T(0.5) * (Zk.re + Zc.re), T(0.5) * (Zk.im + Zc.im)};
      const cpx<T> O = {T(0.5) * (Zk.re - Zc.re), T(0.5) * (Zk.im - Zc.im)};
      const cpx<T> w = wpost[kx];
      X[((size_t)c * ny + y) * Kx + kx] = {E.re + (w.re * O.im + w.im * O.re),
                                           E.im - (w.re * O.re - w.im * O.im)};
    }
    __syncthreads();
  }
  // phase 2: y transform, tensor product, inverse y transform on column chunks
  const int W = a.W, Py = a.Py;
  for (int kx0 = 0; kx0 < Kx; kx0 += W) {
    for (int t = threadIdx.x; t < 3 * W * Py; t += blockDim.x) {
      const int w = umod(t, W), rest = udiv(t, W), y = umod(rest, Py), c = udiv(rest, Py);
      cpx<T> v = {0, 0};
      if (y < ny && kx0 + w < Kx) v = X[((size_t)c * ny + y) * Kx + kx0 + w];
      A[(c * W + w) * Py + y] = v;
    }
    __syncthreads();
    cpx<T>* Y = lds_fft<T, false>(A, Bf, 3 * W, a.pyf, twy);
    cpx<T>* scratch = (Y == A) ? Bf : A;
    for (int t = threadIdx.x; t < W * Py; t += blockDim.x) {
      const int w = umod(t, W), ky = udiv(t, W), kx = kx0 + w;
      if (kx >= Kx) continue;
      const bool lo = 2 * ky <= Py;
      const int ty = lo ? ky : Py - ky;
      const T sy = lo ? T(1) : T(-1);
      tensor_apply(a.Nt, (size_t)ty * Kx + kx, sy, T(1), sy, false, Y[(0 * W + w) * Py + ky],
                   Y[(1 * W + w) * Py + ky], Y[(2 * W + w) * Py + ky]);
    }
    __syncthreads();
    const cpx<T>* Yi = lds_fft<T, true>(Y, scratch, 3 * W, a.pyi, twy);
    for (int t = threadIdx.x; t < 3 * W * ny; t += blockDim.x) {
      const int w = umod(t, W), rest = udiv(t, W), y = umod(rest, ny), c = udiv(rest, ny);
      if (kx0 + w < Kx) X[((size_t)c * ny + y) * Kx + kx0 + w] = Yi[(c * W + w) * Py + y];
    }
    __syncthreads();
  }
}

// Inverse x transform of row chunk q from X; returns the real view of the
// demag field of the chunk's rows (line (c, l) at offset (c C + l) 2 hx).
template <typename T>
__device__ inline const T* fused_inverse_chunk(const HeunFusedArgs<T>& a, int q, const cpx<T>* X,
                                               cpx<T>* A, cpx<T>* Bf, const cpx<T>* twx,
                                               const cpx<T>* wpost) {
  const FArgs<T>& f = a.f;
  const int hx = f.hx, Kx = f.Kx, ny = f.ny, C = a.C;
  const int y0 = q * C;
  for (int t = threadIdx.x; t < 3 * C * hx; t += blockDim.x) {
    const int line = udiv(t, hx), k = t - line * hx;
    const int c = udiv(line, C), l = line - c * C, y = y0 + l;
    cpx<T> Zv = {0, 0};
    if (y < ny) {
      const cpx<T>* row = X + ((size_t)c * ny + y) * Kx;
      const cpx<T> Xk = row[k];
      cpx<T> Xc = row[hx - k];
      Xc.im = -Xc.im;
      const cpx<T> E = cadd(Xk, Xc);
      const cpx<T> D = csub(Xk, Xc);
      const cpx<T> O = cmulc(D, wpost[k]);
      Zv = {E.re - O.im, E.im + O.re};
    }
    A[line * hx + k] = Zv;
  }
  __syncthreads();
  return reinterpret_cast<const T*>(lds_fft<T, true>(A, Bf, 3 * C, a.pxi, twx));
}

template <typename T>
__global__ void __launch_bounds__(kFusedBlock) k_heun_fused(HeunFusedArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[kFusedBlock / 64];
  const FArgs<T>& f = a.f;
  const int hx = f.hx, Kx = f.Kx, ny = f.ny, nx = f.nx, C = a.C;
  const int r = blockIdx.x;
  const size_t rb = (size_t)r * 3 * f.N;
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* A = X + (size_t)3 * ny * Kx;
  const int scratch = max(3 * C * hx, 3 * a.W * a.Py);
  cpx<T>* Bf = A + scratch;
  cpx<T>* twx = Bf + scratch;
  cpx<T>* wp = twx + hx;
  cpx<T>* twy = wp + hx + 1;
  for (int i = threadIdx.x; i < hx; i += blockDim.x) twx[i] = a.tw_x[i];
  for (int i = threadIdx.x; i <= hx; i += blockDim.x) wp[i] = a.wpost[i];
  for (int i = threadIdx.x; i < a.Py; i += blockDim.x) twy[i] = a.tw_y[i];
  __syncthreads();
  const T dt = (T)a.dt;
  T sigma = 0;
  if ((f.terms & T_THERMAL) && f.Trep) {
    const double Tr = f.Trep[r];
    if (Tr > 0) sigma = (T)sqrt(f.sig2pref * Tr / a.dt);
  }
  const uint64_t seed = f.seeds ? f.seeds[r] : 0;
  const bool demag = (f.terms & T_DEMAG) != 0;
  const int t = threadIdx.x;
  const int l = t / nx, x = t - (t / nx) * nx;
  const bool active_col = t < C * nx;
  for (int s = 0; s < a.nsteps; ++s) {
    const uint64_t step = (a.stepdev ? *a.stepdev : 0ull) + a.step0 + (uint64_t)s;
    double mz_acc = 0.0;
    for (int stage = 0; stage < 2; ++stage) {
      // predictor: fields at m; corrector: fields at the predictor state ms
      const T* src = stage == 0 ? a.m : a.ms;
      if (demag) fused_forward(a, src, rb, X, A, Bf, twx, wp, twy);
      for (int q = 0; q < a.nch; ++q) {
        const T* Hd = demag ? fused_inverse_chunk(a, q, X, A, Bf, twx, wp) : nullptr;
        const int y = q * C + l;
        if (active_col && y < ny) {
          const size_t cell = (size_t)x + (size_t)nx * y;
          T mc[3];
          ld3(src + rb, (unsigned)f.N, (unsigned)cell, mc);
          T Hex[3], Hdm[3], Han[3], Hz[3];
          local_terms<T, false>(f, src + rb, (unsigned)cell, x, y, 0, mc, f.kbc, Hex, Hdm, Han, Hz);
          T Hdd[3] = {0, 0, 0};
          if (demag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Hdd[c] = Hd[(c * C + l) * 2 * hx + x];
          }
          T H[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) H[c] = Hex[c] + Hdm[c] + Han[c] + Hz[c] + Hdd[c];
          if (sigma != T(0)) {
            T eta[3];
            thermal_eta<T>(seed, (uint32_t)cell, step, eta);
#pragma unroll
            for (int c = 0; c < 3; ++c) H[c] += sigma * eta[c];
          }
          T k[3];
          llg_torque(mc, H, f.gpm, f.alpha, k);
          const T tau[3] = {0, 0, 0};
          if (stage == 0) {
            T k1v[3], mn[3];
            heun_predict(f, false, mc, H, k, tau, dt, k1v, mn);
#pragma unroll
            for (int c = 0; c < 3; ++c) a.ms[rb + (size_t)c * f.N + cell] = mn[c];
          } else {
            // own cell of m is read and written only by this thread here
            T mo[3], mn[3];
            const T k1v[3] = {0, 0, 0};
            ld3(a.m + rb, (unsigned)f.N, (unsigned)cell, mo);
            heun_correct(f, false, mc, H, k, tau, mo, k1v, dt, mn);
#pragma unroll
            for (int c = 0; c < 3; ++c) a.m[rb + (size_t)c * f.N + cell] = mn[c];
            if (f.nonfinite && !(fabs(mn[0]) + fabs(mn[1]) + fabs(mn[2]) <= T(3))) *f.nonfinite = 1;
            mz_acc += (double)mn[2];
          }
        }
        __syncthreads();
      }
    }
    if (a.tsw) {
      // replica mean of m_z after the step: wave sums, then a fixed-order sum
      double v = mz_acc;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((t & 63) == 0) red[t >> 6] = v;
      __syncthreads();
      if (t == 0) {
        double sum = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
        if (a.tsw[r] < 0 && sum / f.N < 0) a.tsw[r] = (double)(step + 1) * a.dt;
      }
      __syncthreads();
    }
  }
}

}  // namespace mmx
