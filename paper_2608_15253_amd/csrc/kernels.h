// Hot-path kernels of the effective-field + LLG step (device code).
//
// One field evaluation of a replica group is three launches (2-D films and
// 3-D blocks of at most 8 layers) or five (other 3-D blocks), all over every
// replica of the group at once:
//   k_xfwd   stage combine (RK45: m + dt sum a_sj k_j; optional
//            normalisation) fused with the real-to-complex x transform of the
//            zero-padded magnetisation (two real cells packed per complex
//            value, half-length Stockham FFT in LDS, even/odd split);
//   k_yconv  (2-D) y transform (pruned: rows >= ny are zero), product with the
//            parity-compressed real symmetric tensor spectrum, inverse y
//            transform, rows >= ny dropped;
//   k_yzconv (3-D, few layers) y transforms, z transform with the full
//            tensor product and inverse transforms in one pass;
//   k_ypass / k_zconv(_reg) / k_ypass  (other 3-D) the same split over y and z;
//   k_fields complex-to-real inverse x transform (outputs x < nx only) fused
//            with exchange, interfacial DMI, uniaxial anisotropy, Zeeman and
//            Brown thermal fields, the LLG torque and the integrator epilogue
//            (Heun predictor/corrector, RK45 stage store, embedded error
//            with a workgroup max reduction, energy partial sums).
// Spectrum layout: S[((r*3 + c)*nz + z)*Sy + y][kx], Sy = ny (2-D) or Py (3-D),
// kx < Kx = Px/2 + 1.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "philox.h"

namespace mmx {

enum : unsigned {
  T_EXCH = 1, T_DMI = 2, T_ANIS = 4, T_ZEEMAN = 8, T_DEMAG = 16, T_THERMAL = 32, T_STT = 64,
  T_DMI_BULK = 128, T_CUBIC = 256, T_RKKY = 512
};

enum FieldMode { FM_FIELD = 0, FM_TORQUE, FM_HEUN1, FM_HEUN2, FM_RKK, FM_RK7, FM_ENERGY };

constexpr int kBlock = 256;

// Device controller state of the adaptive integrator (FP64 time and error).
struct RkState {
  double t, dt, t_end, tol, dt_max, dt_min;
  unsigned long long err_bits;  // max error of the current attempt (bit pattern)
  double last_err;
  double dt_prop;  // the controller's last proposal before clipping to t_end
  long long accepted, rejected, n_replay, replay_idx;
  int done, accepted_flag, final_flag, nonfinite, dtmin_hit, pad;
};

// Copies a twiddle table into LDS (callers reach a barrier before using it).
template <typename T>
__device__ inline const cpx<T>* stage_table(cpx<T>* dst, const cpx<T>* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  return dst;
}

// Workgroups are dealt to the 8 XCDs round-robin in launch order.  This
// relabels a 3-D grid so that blocks with neighbouring logical indices
// (adjacent row or column tiles of one replica, which share cache lines)
// run on the same XCD and its L2.  A bijection on the blocks of the grid.
__device__ inline void xcd_block(int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y;
  const int nblk = gx * gy * gridDim.z;
  const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int per = nblk / 8;
  const int lg = lin < 8 * per ? (lin % 8) * per + lin / 8 : lin;
  bx = lg % gx;
  by = (lg / gx) % gy;
  bz = lg / (gx * gy);
}

// Moves elements t = 0 .. total-1 with v = ld(t); st(t, v), eight per thread
// at a time: the eight loads are issued before the first store, so their
// global-memory latencies overlap instead of adding up.  Whole workgroup of
// kBlock threads.
constexpr int kBatch = 8;
template <typename V, typename Ld, typename St>
__device__ inline void batched_move(int total, Ld ld, St st) {
  for (int base = 0; base < total; base += kBatch * kBlock) {
    V v[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int t = base + i * kBlock + (int)threadIdx.x;
      if (t < total) v[i] = ld(t);
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int t = base + i * kBlock + (int)threadIdx.x;
      if (t < total) st(t, v[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// x forward transform with stage combine
// ---------------------------------------------------------------------------
// Half spectrum rows y0 .. y0+L-1 (plane z of replica r) from the
// half-length complex transforms X of their packed cell pairs (line c L + l):
// the real-to-complex split S[kx] = E + conj(W^kx) O with W = exp(-2 pi i / Px).
template <typename T>
__device__ inline void xfwd_store(const cpx<T>* X, const cpx<T>* __restrict__ wpost,
                                  cpx<T>* __restrict__ S, int r, int z, int y0, int L, int hx,
                                  int Kx, int ny, int nz, int Sy, int xone) {
  const int nl = 3 * L;
  for (int t = threadIdx.x; t < nl * Kx; t += blockDim.x) {
    const int line = t / Kx, kx = t - line * Kx;
    const int c = udiv(line, L), l = line - c * L, y = y0 + l;
    if (y >= ny) continue;
    cpx<T> out;
    if (xone) {
      out = {X[line].re, T(0)};
    } else {
      const cpx<T> Zk = X[line * hx + (kx == hx ? 0 : kx)];
      cpx<T> Zc = X[line * hx + (kx == 0 ? 0 : hx - kx)];
      Zc.im = -Zc.im;
      const cpx<T> E = {T(0.5) * (Zk.re + Zc.re), T(0.5) * (Zk.im + Zc.im)};
      const cpx<T> O = {T(0.5) * (Zk.re - Zc.re), T(0.5) * (Zk.im - Zc.im)};
      const cpx<T> w = wpost[kx];
      out = {E.re + (w.re * O.im + w.im * O.re), E.im - (w.re * O.re - w.im * O.im)};
    }
    S[((((size_t)r * 3 + c) * nz + z) * Sy + y) * Kx + kx] = out;
  }
}

template <typename T>
struct XArgs {
  const T* m;
  const T* kk[6];
  T coef[6];
  int ncoef;
  const double* dtdev;
  double dth;
  T* mout;
  int normalise;
  int do_fft;
  cpx<T>* S;
  const cpx<T>* tw;
  const cpx<T>* wpost;
  FftPlan plan;
  int nx, ny, nz, N, Sy, Kx, hx, L, xone;
  const int* done;
  int* nonfinite;  // normalised combine: set to 1 if a combined state is not finite
  const T* msr;    // per-cell Ms_i / Ms scaling the transform input (null: uniform)
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_xfwd(XArgs<T> a) {
  if (a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int hx = a.hx, L = a.L, nl = 3 * L;
  cpx<T>* Bf = A + nl * hx;
  const cpx<T>* tw = a.do_fft ? stage_table(Bf + nl * hx, a.tw, hx) : nullptr;
  const cpx<T>* wpost = a.do_fft ? stage_table(Bf + nl * hx + hx, a.wpost, hx + 1) : nullptr;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, z = by, y0 = bx * L;
  const size_t rb = (size_t)r * 3 * a.N;
  const T dt = a.dtdev ? (T)(*a.dtdev) : (T)a.dth;
  const int npair = a.xone ? 1 : (a.nx + 1) / 2;
  // a pruned transform never reads k >= hx/2 = npair: those slots stay unfilled
  const int kw = (a.do_fft && !a.plan.prune) ? hx : npair;
  for (int t = threadIdx.x; t < L * kw; t += blockDim.x) {
    const int l = udiv(t, kw), k = t - l * kw, y = y0 + l;
    cpx<T> v[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (y < a.ny && k < npair) {
      // both cells' state and slope values are loaded before the sums (a
      // cell past the row end loads its partner and is dropped)
      T pm[2][3], pkv[2][6][3];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = (2 * k + h < a.nx) ? 2 * k + h : 2 * k;
        const size_t cell = (size_t)x + (size_t)a.nx * (y + (size_t)a.ny * z);
#pragma unroll
        for (int c = 0; c < 3; ++c) pm[h][c] = a.m[rb + (size_t)c * a.N + cell];
#pragma unroll
        for (int j = 0; j < 6; ++j)
          if (j < a.ncoef) {
#pragma unroll
            for (int c = 0; c < 3; ++c) pkv[h][j][c] = a.kk[j][rb + (size_t)c * a.N + cell];
          }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = 2 * k + h;
        if (x >= a.nx) break;
        const size_t cell = (size_t)x + (size_t)a.nx * (y + (size_t)a.ny * z);
        T mv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T s = pm[h][c];
#pragma unroll
          for (int j = 0; j < 6; ++j)
            if (j < a.ncoef) s += dt * a.coef[j] * pkv[h][j][c];
          mv[c] = s;
        }
        if (a.normalise) {
          const T inv = T(1) / sqrt(mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2]);
          mv[0] *= inv; mv[1] *= inv; mv[2] *= inv;
          if (a.nonfinite && !(fabs(mv[0]) + fabs(mv[1]) + fabs(mv[2]) <= T(3))) *a.nonfinite = 1;
        }
        if (a.mout) {
#pragma unroll
          for (int c = 0; c < 3; ++c) a.mout[rb + (size_t)c * a.N + cell] = mv[c];
        }
        if (a.msr) {  // the convolution acts on M = Ms_i m
          const T w = a.msr[cell];
          mv[0] *= w; mv[1] *= w; mv[2] *= w;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (h == 0) v[c].re = mv[c]; else v[c].im = mv[c];
        }
      }
    }
    if (a.do_fft) {
#pragma unroll
      for (int c = 0; c < 3; ++c) A[(c * L + l) * hx + k] = v[c];
    }
  }
  if (!a.do_fft) return;
  __syncthreads();
  const cpx<T>* X = lds_fft<T, false>(A, Bf, nl, a.plan, tw);
  xfwd_store(X, wpost, a.S, r, z, y0, L, hx, a.Kx, a.ny, a.nz, a.Sy, a.xone);
}

// ---------------------------------------------------------------------------
// spectral tensor product helpers
// ---------------------------------------------------------------------------
// H = N M at one frequency; Nt points at its kTensorStride reals (xx, yy,
// zz, xy, xz, yz); s.. restore the signs of the odd components per octant.
template <typename T>
__device__ inline void tensor_apply(const T* __restrict__ Nt, size_t idx, T sxy, T sxz, T syz,
                                    bool full, cpx<T>& X, cpx<T>& Y, cpx<T>& Z) {
  const T* __restrict__ n = Nt + idx * kTensorStride;
  const T nxx = n[0], nyy = n[1], nzz = n[2];
  const T nxy = sxy * n[3];
  cpx<T> hx = {nxx * X.re + nxy * Y.re, nxx * X.im + nxy * Y.im};
  cpx<T> hy = {nxy * X.re + nyy * Y.re, nxy * X.im + nyy * Y.im};
  cpx<T> hz = {nzz * Z.re, nzz * Z.im};
  if (full) {
    const T nxz = sxz * n[4], nyz = syz * n[5];
    hx.re += nxz * Z.re; hx.im += nxz * Z.im;
    hy.re += nyz * Z.re; hy.im += nyz * Z.im;
    hz.re += nxz * X.re + nyz * Y.re;
    hz.im += nxz * X.im + nyz * Y.im;
  }
  X = hx; Y = hy; Z = hz;
}

// ---------------------------------------------------------------------------
// 2-D: y transform + tensor product + inverse y transform
// ---------------------------------------------------------------------------
template <typename T>
struct YArgs {
  cpx<T>* S;
  const T* Nt;
  const cpx<T>* tw;
  FftPlan pf, pi;
  int ny, Py, Kx, W, Ty, Sy, nz, Pz, Tz, z;
  const int* done;
  const cpx<T>* twz;  // z twiddles exp(-2 pi i k / Pz) of the fused y-z pass
  // switching check of the previous Heun step, folded into the register
  // column kernel (sw_tsw null: none): the workgroup of column tile 0 of
  // each replica sums that replica's corrector partial sums of m_z
  const double* sw_part;
  double* sw_tsw;
  const int* sw_nblk;  // the corrector's workgroups per replica (device)
  int sw_N;
  double sw_dt;
  // the check's time is st sw_dt, st = (*sw_stepdev if set) + sw_step
  unsigned long long sw_step;
  const unsigned long long* sw_stepdev;
};

// Replica r's switching time: the first t after which the mean m_z (from
// the corrector's per-workgroup partial sums, summed in a fixed order) is
// negative.
__device__ inline void switch_check(const double* part, double* tsw, int nblk, int N, int r,
                                    double t) {
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)r * nblk + b];
  if (tsw[r] < 0 && s / N < 0) tsw[r] = t;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_yconv(YArgs<T> a) {
  if (a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int W = a.W, Py = a.Py, nl = 3 * W;
  cpx<T>* Bf = A + nl * Py;
  const cpx<T>* tw = stage_table(Bf + nl * Py, a.tw, Py);
  // neighbouring column tiles share the cache lines of the spectrum rows:
  // keep them on one XCD (one L2) instead of dealing them round robin
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, kx0 = bx * W;
  const size_t rbase = (size_t)r * 3;
  batched_move<cpx<T>>(
      nl * Py,
      [&](int t) {
        const int w = umod(t, W), rest = udiv(t, W), y = umod(rest, Py), c = udiv(rest, Py);
        cpx<T> v = {0, 0};
        if (y < a.ny && kx0 + w < a.Kx)
          v = a.S[(((rbase + c) * a.nz) * a.Sy + y) * a.Kx + kx0 + w];
        return v;
      },
      [&](int t, cpx<T> v) {
        const int w = umod(t, W), rest = udiv(t, W), y = umod(rest, Py), c = udiv(rest, Py);
        A[(c * W + w) * Py + y] = v;
      });
  __syncthreads();
  cpx<T>* X = lds_fft<T, false>(A, Bf, nl, a.pf, tw);
  cpx<T>* scratch = (X == A) ? Bf : A;
  for (int t = threadIdx.x; t < W * Py; t += blockDim.x) {
    const int w = umod(t, W), ky = udiv(t, W), kx = kx0 + w;
    if (kx >= a.Kx) continue;
    const bool lo = 2 * ky <= Py;
    const int ty = lo ? ky : Py - ky;
    const T sy = lo ? T(1) : T(-1);
    cpx<T>& Mx = X[(0 * W + w) * Py + ky];
    cpx<T>& My = X[(1 * W + w) * Py + ky];
    cpx<T>& Mz = X[(2 * W + w) * Py + ky];
    tensor_apply(a.Nt, (size_t)ty * a.Kx + kx, sy, T(1), sy, false, Mx, My, Mz);
  }
  __syncthreads();
  const cpx<T>* Y = lds_fft<T, true>(X, scratch, nl, a.pi, tw);
  for (int t = threadIdx.x; t < nl * a.ny; t += blockDim.x) {
    const int w = umod(t, W), rest = udiv(t, W), y = umod(rest, a.ny), c = udiv(rest, a.ny);
    if (kx0 + w < a.Kx)
      a.S[(((rbase + c) * a.nz) * a.Sy + y) * a.Kx + kx0 + w] = Y[(c * W + w) * Py + y];
  }
}

// ---------------------------------------------------------------------------
// 3-D: y transforms (forward pruned / inverse cropped) on z < nz planes
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ void __launch_bounds__(kBlock) k_ypass(YArgs<T> a) {
  if (a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  // lines of Py + 1 slots: the lanes of one global access (consecutive kx,
  // i.e. consecutive lines) then fall into different LDS banks
  const int W = a.W, Py = a.Py, ld = Py + 1;
  cpx<T>* Bf = A + W * ld;
  const cpx<T>* tw = stage_table(Bf + W * ld, a.tw, Py);
  int bx, by, bz;
  xcd_block(bx, by, bz);  // neighbouring column tiles on one XCD (shared lines)
  const int kx0 = bx * W;
  // one (component, z) plane of one replica: no product couples the
  // components here, so a workgroup takes W columns of a single one (wider
  // tiles, longer contiguous runs along kx)
  cpx<T>* __restrict__ P = a.S + ((size_t)bz * 3 * a.nz + by) * a.Sy * a.Kx + kx0;
  const int nin = INV ? Py : a.ny;
  batched_move<cpx<T>>(
      W * Py,
      [&](int t) {
        const int w = umod(t, W), y = udiv(t, W);
        cpx<T> v = {0, 0};
        if (y < nin && kx0 + w < a.Kx) v = P[(size_t)y * a.Kx + w];
        return v;
      },
      [&](int t, cpx<T> v) { A[umod(t, W) * ld + udiv(t, W)] = v; });
  __syncthreads();
  const cpx<T>* Y = lds_fft<T, INV>(A, Bf, W, INV ? a.pi : a.pf, tw, ld);
  const int nout = INV ? a.ny : Py;
  for (int t = threadIdx.x; t < W * nout; t += blockDim.x) {
    const int w = umod(t, W), y = udiv(t, W);
    if (kx0 + w < a.Kx) P[(size_t)y * a.Kx + w] = Y[w * ld + y];
  }
}

// 3-D: z transform + full tensor product + inverse z transform, per ky.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_zconv(YArgs<T> a) {
  if (a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int W = a.W, Pz = a.Pz, nl = 3 * W;
  cpx<T>* Bf = A + nl * Pz;
  const cpx<T>* tw = stage_table(Bf + nl * Pz, a.tw, Pz);
  int bx, by, bz;
  xcd_block(bx, by, bz);  // neighbouring column tiles on one XCD (shared lines)
  const int r = bz, ky = by, kx0 = bx * W;
  const size_t rbase = (size_t)r * 3;
  batched_move<cpx<T>>(
      nl * Pz,
      [&](int t) {
        const int w = umod(t, W), rest = udiv(t, W), z = umod(rest, Pz), c = udiv(rest, Pz);
        cpx<T> v = {0, 0};
        if (z < a.nz && kx0 + w < a.Kx)
          v = a.S[(((rbase + c) * a.nz + z) * a.Sy + ky) * a.Kx + kx0 + w];
        return v;
      },
      [&](int t, cpx<T> v) {
        const int w = umod(t, W), rest = udiv(t, W), z = umod(rest, Pz), c = udiv(rest, Pz);
        A[(c * W + w) * Pz + z] = v;
      });
  __syncthreads();
  cpx<T>* X = lds_fft<T, false>(A, Bf, nl, a.pf, tw);
  cpx<T>* scratch = (X == A) ? Bf : A;
  const bool ylo = 2 * ky <= a.Py;
  const int ty = ylo ? ky : a.Py - ky;
  const T sy = ylo ? T(1) : T(-1);
  for (int t = threadIdx.x; t < W * Pz; t += blockDim.x) {
    const int w = umod(t, W), kz = udiv(t, W), kx = kx0 + w;
    if (kx >= a.Kx) continue;
    const bool zlo = 2 * kz <= Pz;
    const int tz = zlo ? kz : Pz - kz;
    const T sz = zlo ? T(1) : T(-1);
    cpx<T>& Mx = X[(0 * W + w) * Pz + kz];
    cpx<T>& My = X[(1 * W + w) * Pz + kz];
    cpx<T>& Mz = X[(2 * W + w) * Pz + kz];
    tensor_apply(a.Nt, ((size_t)tz * a.Ty + ty) * a.Kx + kx, sy, sz, sy * sz, true, Mx, My,
                 Mz);
  }
  __syncthreads();
  const cpx<T>* Y = lds_fft<T, true>(X, scratch, nl, a.pi, tw);
  for (int t = threadIdx.x; t < nl * a.nz; t += blockDim.x) {
    const int w = umod(t, W), rest = udiv(t, W), z = umod(rest, a.nz), c = udiv(rest, a.nz);
    if (kx0 + w < a.Kx)
      a.S[(((rbase + c) * a.nz + z) * a.Sy + ky) * a.Kx + kx0 + w] = Y[(c * W + w) * Pz + z];
  }
}

// The z transform of one (ky, kx) pillar held as x[c][z] (planes z >= nz
// are zero padding and not stored) as a direct sum over the nz planes, the
// full tensor product per kz, and the inverse z transform as a direct sum
// evaluated only on the nz planes kept (accumulated into y, zero on entry).
// tw: exp(-2 pi i k / Pz), k < Pz.
template <typename T, int NZ>
__device__ inline void z_pillar(const YArgs<T>& a, const cpx<T>* __restrict__ tw, int ky, int kx,
                                const cpx<T> (&x)[3][NZ], cpx<T> (&y)[3][NZ]) {
  const int nz = a.nz, Pz = a.Pz, Kx = a.Kx;
  const bool ylo = 2 * ky <= a.Py;
  const int ty = ylo ? ky : a.Py - ky;
  const T sy = ylo ? T(1) : T(-1);
  // Pz <= 2 NZ: with few layers the tensor entries of every kz are loaded
  // before the first product, so their latencies overlap
  constexpr int KZ = 2 * NZ;
  constexpr bool kPre = NZ <= 4;
  T pre[kPre ? KZ : 1][6];
  if constexpr (kPre) {
#pragma unroll
    for (int kz = 0; kz < KZ; ++kz) {
      if (kz < Pz) {
        const int tz = (2 * kz <= Pz) ? kz : Pz - kz;
        const T* __restrict__ n = a.Nt + (((size_t)tz * a.Ty + ty) * Kx + kx) * kTensorStride;
#pragma unroll
        for (int i = 0; i < 6; ++i) pre[kz][i] = n[i];
      }
    }
  }
  auto step = [&](int kz, const T* __restrict__ n) {
    cpx<T> X[3] = {x[0][0], x[1][0], x[2][0]};
    int e = 0;  // kz z mod Pz
#pragma unroll
    for (int z = 1; z < NZ; ++z) {
      e += kz;
      if (e >= Pz) e -= Pz;
      if (z < nz) {
        const cpx<T> w = tw[e];
#pragma unroll
        for (int c = 0; c < 3; ++c) X[c] = cadd(X[c], cmul(x[c][z], w));
      }
    }
    const T sz = (2 * kz <= Pz) ? T(1) : T(-1);
    tensor_apply(n, 0, sy, sz, sy * sz, true, X[0], X[1], X[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c][0] = cadd(y[c][0], X[c]);
    e = 0;
#pragma unroll
    for (int z = 1; z < NZ; ++z) {
      e += kz;
      if (e >= Pz) e -= Pz;
      if (z < nz) {
        const cpx<T> w = tw[e];
#pragma unroll
        for (int c = 0; c < 3; ++c) y[c][z] = cadd(y[c][z], cmulc(X[c], w));
      }
    }
  };
  if constexpr (kPre) {
#pragma unroll
    for (int kz = 0; kz < KZ; ++kz)
      if (kz < Pz) step(kz, pre[kz]);
  } else {
    for (int kz = 0; kz < Pz; ++kz) {
      const int tz = (2 * kz <= Pz) ? kz : Pz - kz;
      step(kz, a.Nt + (((size_t)tz * a.Ty + ty) * Kx + kx) * kTensorStride);
    }
  }
}

// 3-D grids of few layers (nz <= NZ): one thread per (ky, kx) pillar holds
// its nz planes of all three components in registers (z_pillar).  Threads
// run along the contiguous (ky, kx) plane, so every access is a coalesced
// stream; the LDS kernel above moves a few hundred values per workgroup
// through several synchronised passes instead.
template <typename T, int NZ>
__global__ void __launch_bounds__(kBlock) k_zconv_reg(YArgs<T> a) {
  if (a.done && *a.done) return;
  const int nz = a.nz, Kx = a.Kx;
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= a.Py * Kx) return;
  const int ky = j / Kx, kx = j - ky * Kx;
  const size_t pstride = (size_t)a.Sy * Kx;
  cpx<T>* __restrict__ base = a.S + (size_t)blockIdx.y * 3 * nz * pstride + j;
  cpx<T> x[3][NZ], y[3][NZ];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
      x[c][z] = (z < nz) ? base[(size_t)(c * nz + z) * pstride] : cpx<T>{0, 0};
      y[c][z] = {0, 0};
    }
  z_pillar<T, NZ>(a, a.tw, ky, kx, x, y);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < NZ; ++z)
      if (z < nz) base[(size_t)(c * nz + z) * pstride] = y[c][z];
}

// 3-D grids of few layers, y and z in one pass: a workgroup holds W spectrum
// columns of one replica, all nz planes of all three components (3 nz W
// lines of Py + 1 slots in LDS); forward y transforms (rows >= ny are zero:
// pruned), then per (ky, kx) pillar the z transform, tensor product and
// inverse z transform in registers (z_pillar), then inverse y transforms
// keeping the ny rows stored.  HBM carries each stored row once in and once
// out, instead of the three passes of k_ypass / k_zconv_reg / k_ypass over
// the Py padded rows.
template <typename T, int NZ>
__global__ void __launch_bounds__(kBlock) k_yzconv(YArgs<T> a) {
  if (a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int W = a.W, Py = a.Py, nz = a.nz, ny = a.ny, ld = Py + 1, nl = 3 * nz * W;
  cpx<T>* Bf = A + nl * ld;
  const cpx<T>* tw = stage_table(Bf + nl * ld, a.tw, Py);
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int kx0 = bx * W;
  const size_t plane = (size_t)a.Sy * a.Kx;
  cpx<T>* __restrict__ S = a.S + (size_t)bz * 3 * nz * plane + kx0;
  // line (c nz + z) W + w holds column kx0 + w of plane z of component c
  for (int t = threadIdx.x; t < nl * ny; t += blockDim.x) {
    const int w = umod(t, W), rest = udiv(t, W), cz = rest / ny, y = rest - cz * ny;
    cpx<T> v = {0, 0};
    if (kx0 + w < a.Kx) v = S[cz * plane + (size_t)y * a.Kx + w];
    A[(cz * W + w) * ld + y] = v;
  }
  __syncthreads();
  cpx<T>* X = lds_fft<T, false>(A, Bf, nl, a.pf, tw, ld);
  cpx<T>* scratch = (X == A) ? Bf : A;
  for (int t = threadIdx.x; t < W * Py; t += blockDim.x) {
    const int w = umod(t, W), ky = udiv(t, W), kx = kx0 + w;
    if (kx >= a.Kx) continue;
    cpx<T> x[3][NZ], yv[3][NZ];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < NZ; ++z) {
        x[c][z] = (z < nz) ? X[((c * nz + z) * W + w) * ld + ky] : cpx<T>{0, 0};
        yv[c][z] = {0, 0};
      }
    z_pillar<T, NZ>(a, a.twz, ky, kx, x, yv);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < NZ; ++z)
        if (z < nz) X[((c * nz + z) * W + w) * ld + ky] = yv[c][z];
  }
  __syncthreads();
  const cpx<T>* Y = lds_fft<T, true>(X, scratch, nl, a.pi, tw, ld);
  for (int t = threadIdx.x; t < nl * ny; t += blockDim.x) {
    const int w = umod(t, W), rest = udiv(t, W), cz = rest / ny, y = rest - cz * ny;
    if (kx0 + w < a.Kx) S[cz * plane + (size_t)y * a.Kx + w] = Y[(cz * W + w) * ld + y];
  }
}

// ---------------------------------------------------------------------------
// inverse x transform + local fields + torque + integrator epilogue
// ---------------------------------------------------------------------------
template <typename T>
struct FArgs {
  int nx, ny, nz, N, Sy, Kx, hx, L, xone;
  int pbc[3];
  int nax[3];
  T idd2[3];  // 1/d^2 (exchange)
  T ih2[3];   // 1/(2d) (DMI)
  T hd[3];    // cell size (ghosts)
  T cex, cdmi, kbc, can, u[3], hz[3], gpm, alpha;
  // bulk DMI: field -(2 Db / mu0 Ms) curl m (cbulk), ghost factor Db / 2A (kbb);
  // cubic anisotropy 2 Kc1 / mu0 Ms, 2 Kc2 / mu0 Ms along the rows of cax;
  // RKKY: sigma / (mu0 Ms dz) between cell layers rkz0 and rkz1
  T cbulk, kbb, kc1h, kc2h, kc1, kc2, cax[3][3], crkky;
  double ecub;  // -2 / (mu0 Ms): turns the cubic energy density into the -m.H/2 sum
  int rkz0, rkz1;
  // per-cell exchange stiffness (null: uniform A): pair coupling by the
  // harmonic mean, field prefactor 2 / mu0 Ms, edge factors D/2 and Db/2 over A_i
  const T* Acell;
  T exs, dhalf, dbhalf;
  // further per-cell parameters (null: the group's uniform material), one
  // value per cell: Ms_i / Ms (transform input and energy weight), Ms / Ms_i
  // (local fields, spin-transfer b_J), gamma0 mu0 / (1 + alpha_i^2), alpha_i,
  // sqrt(alpha_i Ms / Ms_i) (thermal), 2 Ku_i / (mu0 Ms), D_i
  const T* msr;
  const T* mgi;
  const T* gpc;
  const T* alc;
  const T* sgc;
  const T* kuc;
  const T* dmc;
  T c2ms, Agrp;     // 2 / (mu0 Ms) and the group's uniform A
  double sigunit;   // 2 kB / (mu0^2 Ms V gamma0): sigma_i^2 = sigunit T alpha_i Ms / Ms_i / dt
  unsigned terms;
  const double* Trep;
  const uint64_t* seeds;
  double sig2pref;  // 2 alpha kB / (mu0^2 Ms V gamma0); sigma^2 = sig2pref T / dt
  uint64_t step;
  // if set, the step index is *stepdev + step (graph replays: a device
  // counter advanced once per captured run, step the offset within it)
  const unsigned long long* stepdev;
  double dt_th;
  const T* m;
  cpx<T>* S;
  FftPlan plan;
  const cpx<T>* tw;
  const cpx<T>* wpost;
  T* out;
  T* k1;
  const T* m0;
  T* mout;
  const T* kk[6];
  double e[7];
  const double* dtdev;
  double dth;
  RkState* st;
  double* partial;
  const int* done;
  const float* hext;  // if set (demag term off): Hd = hext_scale * hext + (0, 0, hext_mz m_z)
  T hext_scale, hext_mz;
  int fwd;            // Heun epilogues: also x-transform the new state into S
  // RK stage epilogue (FM_RKK with fwd): the next stage's state m0 + dt sum_j
  // cn[j] k_j (k_j from kk, the stage's own slope from registers at index
  // cstage), normalised if cnext == 2, is written to mnext and x-transformed
  T cn[6];
  int cnext, cstage;
  T* mnext;
  FftPlan plan_f;     // forward x plan (pruned like the one of k_xfwd)
  T* hd_out;          // if set: the exact demag field is also stored here
  int rot;            // Heun epilogues take the rotation (Depondt-Mertens) update
  const int* tgen;    // retire/refill: trial generation of each replica (noise word 3)
  const unsigned long long* tstart;  // and the first step of its running trial
  // Slonczewski spin-transfer torque: b_J = stt_c J[r] (A/m), fixed-layer unit
  // vector, polarisation, Lambda^2 and the field-like coefficient eps'
  int noprec;         // damping-only dynamics: the precession term is dropped
  int* nblk_out;      // Heun corrector: receives its workgroups per replica (partial-sum stride)
  int* nonfinite;     // set to 1 by a corrector whose new state is not finite (null: no check)
  const double* Jrep;
  double stt_c;
  T sttp[3], stt_P, stt_L2, stt_e2;
};

// The three components of a cell of one replica (component stride N).  With
// O32 the byte offsets are formed in 32 bits (the caller guarantees
// 3 N sizeof(T) < 2^32): with the replica's base pointer uniform across the
// workgroup the loads then take the scalar-base plus 32-bit vector-offset
// form instead of 64-bit address arithmetic per lane.
template <typename T, bool O32 = false>
__device__ inline void ld3(const T* __restrict__ mr, unsigned N, unsigned cell, T v[3]) {
  if constexpr (O32) {
    const char* b = reinterpret_cast<const char*>(mr);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[c] = *reinterpret_cast<const T*>(b + ((unsigned)c * N + cell) * (unsigned)sizeof(T));
  } else {
    v[0] = mr[cell];
    v[1] = mr[N + cell];
    v[2] = mr[2 * N + cell];
  }
}

// Exchange (six-point Laplacian), interfacial DMI (central differences), both
// with periodic wrap or free-edge ghosts m_edge -/+ D_a (D/2A)(z x n) x m at
// open x/y edges (Neumann along z), uniaxial anisotropy and Zeeman field of
// the cell at (x, y, z) with magnetisation mc; neighbours read from m.
// Cubic anisotropy field (added to Han) and energy density at mc.
template <typename T>
__device__ inline void cubic_terms(const FArgs<T>& a, const T mc[3], T Hc[3], T& dens) {
  T mi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    mi[i] = mc[0] * a.cax[i][0] + mc[1] * a.cax[i][1] + mc[2] * a.cax[i][2];
  const T s0 = mi[0] * mi[0], s1 = mi[1] * mi[1], s2 = mi[2] * mi[2];
  const T g[3] = {a.kc1h * mi[0] * (s1 + s2) + a.kc2h * mi[0] * s1 * s2,
                  a.kc1h * mi[1] * (s0 + s2) + a.kc2h * mi[1] * s0 * s2,
                  a.kc1h * mi[2] * (s0 + s1) + a.kc2h * mi[2] * s0 * s1};
#pragma unroll
  for (int c = 0; c < 3; ++c) Hc[c] = -(g[0] * a.cax[0][c] + g[1] * a.cax[1][c] + g[2] * a.cax[2][c]);
  dens = a.kc1 * (s0 * s1 + s1 * s2 + s2 * s0) + a.kc2 * s0 * s1 * s2;
}

// Exchange (six-point Laplacian), interfacial DMI (central differences), both
// with periodic wrap or free-edge ghosts m_edge -/+ D_a g at open edges, g =
// (D/2A)(z x n) x m (x and y) + (Db/2A) e_a x m (every axis; Neumann when both
// vanish), uniaxial anisotropy and Zeeman field of the cell at (x, y, z) with
// magnetisation mc; neighbours read from m.  EXT adds bulk DMI (into Hdm),
// cubic anisotropy (into Han) and RKKY (into Hex); kernels that never see
// those terms instantiate it without.
template <typename T, bool EXT = true, bool O32 = false>
__device__ inline void local_terms(const FArgs<T>& a, const T* __restrict__ mr, unsigned cell,
                                   int x, int y, int z, const T mc[3], T kbc, T Hex[3],
                                   T Hdm[3], T Han[3], T Hz[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) { Hex[c] = 0; Hdm[c] = 0; Han[c] = 0; Hz[c] = 0; }
  const int coord[3] = {x, y, z};
  const unsigned stride[3] = {1u, (unsigned)a.nx, (unsigned)(a.nx * a.ny)};
  const unsigned N = (unsigned)a.N;
  const bool bulk = EXT && (a.terms & T_DMI_BULK);
  const T* __restrict__ Ac = EXT ? a.Acell : nullptr;
  T kbb = EXT ? a.kbb : T(0);
  T Ai = 0;
  if (Ac) {  // the cell's own stiffness sets its edge conditions
    Ai = Ac[cell];
    kbc = Ai > T(0) ? a.dhalf / Ai : T(0);
    kbb = Ai > T(0) ? a.dbhalf / Ai : T(0);
  }
  const T* __restrict__ Dc = EXT ? a.dmc : nullptr;
  T Di = 0;
  if (Dc) {  // the cell's own D / 2A_i
    Di = Dc[cell];
    const T Ae = Ac ? Ai : a.Agrp;
    kbc = Ae > T(0) ? T(0.5) * Di / Ae : T(0);
  }
  T curl[3] = {0, 0, 0};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (a.nax[ax] == 1) continue;
    const int n = a.nax[ax];
    T mm[3], mp[3];
    // ghost offset D_a x (edge-condition derivative): (D/2A)(z x n) x m on
    // x and y, plus (Db/2A) e_ax x m
    T ev[3] = {0, 0, 0};
    if (ax == 0) { ev[0] = mc[2]; ev[2] = -mc[0]; }
    if (ax == 1) { ev[1] = mc[2]; ev[2] = -mc[1]; }
    const T g = (ax < 2) ? a.hd[ax] * kbc : T(0);
    T gv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) gv[c] = g * ev[c];
    if (EXT && kbb != T(0)) {
      const T gb = a.hd[ax] * kbb;
      if (ax == 0) { gv[1] -= gb * mc[2]; gv[2] += gb * mc[1]; }
      if (ax == 1) { gv[0] += gb * mc[2]; gv[2] -= gb * mc[0]; }
      if (ax == 2) { gv[0] -= gb * mc[1]; gv[1] += gb * mc[0]; }
    }
    // neighbour cells (jm, jp); a ghost keeps the cell's own index
    unsigned jm = cell, jp = cell;
    if (coord[ax] > 0) { jm = cell - stride[ax]; ld3<T, O32>(mr, N, jm, mm); }
    else if (a.pbc[ax]) { jm = cell + (unsigned)(n - 1) * stride[ax]; ld3<T, O32>(mr, N, jm, mm); }
    else { for (int c = 0; c < 3; ++c) mm[c] = mc[c] - gv[c]; }
    if (coord[ax] < n - 1) { jp = cell + stride[ax]; ld3<T, O32>(mr, N, jp, mp); }
    else if (a.pbc[ax]) { jp = cell - (unsigned)(n - 1) * stride[ax]; ld3<T, O32>(mr, N, jp, mp); }
    else { for (int c = 0; c < 3; ++c) mp[c] = mc[c] + gv[c]; }
    if (a.terms & T_EXCH) {
      if (EXT && Ac) {
        // harmonic mean of the pair's stiffness (a ghost takes the cell's own)
        const T Am = Ac[jm], Ap = Ac[jp];
        const T wm = (Ai + Am > T(0)) ? T(2) * Ai * Am / (Ai + Am) : T(0);
        const T wp = (Ai + Ap > T(0)) ? T(2) * Ai * Ap / (Ai + Ap) : T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
          Hex[c] += a.exs * a.idd2[ax] * (wm * (mm[c] - mc[c]) + wp * (mp[c] - mc[c]));
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) Hex[c] += a.cex * a.idd2[ax] * (mm[c] + mp[c] - T(2) * mc[c]);
      }
    }
    if ((a.terms & T_DMI) && ax < 2) {
      if (EXT && Dc) {
        // pair couplings (D_i + D_j) / 2 of the per-cell energy density (a
        // ghost takes the cell's own D)
        const T wm = T(0.5) * (Di + Dc[jm]), wp = T(0.5) * (Di + Dc[jp]);
        const T f = a.c2ms * a.ih2[ax];
        Hdm[ax] += f * (wp * mp[2] - wm * mm[2]);
        Hdm[2] -= f * (wp * mp[ax] - wm * mm[ax]);
      } else {
        const T d_ax = (mp[ax] - mm[ax]) * a.ih2[ax];
        const T d_z = (mp[2] - mm[2]) * a.ih2[ax];
        Hdm[ax] += a.cdmi * d_z;
        Hdm[2] -= a.cdmi * d_ax;
      }
    }
    if (bulk) {
      T d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) d[c] = (mp[c] - mm[c]) * a.ih2[ax];
      if (ax == 0) { curl[1] -= d[2]; curl[2] += d[1]; }
      if (ax == 1) { curl[0] += d[2]; curl[2] -= d[0]; }
      if (ax == 2) { curl[0] -= d[1]; curl[1] += d[0]; }
    }
  }
  if (bulk) {
#pragma unroll
    for (int c = 0; c < 3; ++c) Hdm[c] += a.cbulk * curl[c];
  }
  if (a.terms & T_ANIS) {
    const T mu = mc[0] * a.u[0] + mc[1] * a.u[1] + mc[2] * a.u[2];
    const T can = (EXT && a.kuc) ? a.kuc[cell] : a.can;
#pragma unroll
    for (int c = 0; c < 3; ++c) Han[c] = can * mu * a.u[c];
  }
  if (EXT && (a.terms & T_CUBIC)) {
    T Hc[3], dens;
    cubic_terms(a, mc, Hc, dens);
#pragma unroll
    for (int c = 0; c < 3; ++c) Han[c] += Hc[c];
  }
  if (EXT && (a.terms & T_RKKY) && (z == a.rkz0 || z == a.rkz1)) {
    const int zp = (z == a.rkz0) ? a.rkz1 : a.rkz0;
    T mo[3];
    ld3<T, O32>(mr, N, (unsigned)((int)cell + (zp - z) * (int)stride[2]), mo);
#pragma unroll
    for (int c = 0; c < 3; ++c) Hex[c] += a.crkky * mo[c];
  }
  if (EXT && a.mgi) {  // every local term carries 1 / (mu0 Ms_i)
    const T g = a.mgi[cell];
#pragma unroll
    for (int c = 0; c < 3; ++c) { Hex[c] *= g; Hdm[c] *= g; Han[c] *= g; }
  }
  if (a.terms & T_ZEEMAN) { Hz[0] = a.hz[0]; Hz[1] = a.hz[1]; Hz[2] = a.hz[2]; }
}

// LLG torque -gamma' mu0 [m x H + alpha m x (m x H)]
template <typename T>
__device__ inline void llg_torque(const T mc[3], const T H[3], T gpm, T alpha, T k[3]) {
  const T cx = mc[1] * H[2] - mc[2] * H[1];
  const T cy = mc[2] * H[0] - mc[0] * H[2];
  const T cz = mc[0] * H[1] - mc[1] * H[0];
  const T dx = mc[1] * cz - mc[2] * cy;
  const T dy = mc[2] * cx - mc[0] * cz;
  const T dz = mc[0] * cy - mc[1] * cx;
  k[0] = -gpm * (cx + alpha * dx);
  k[1] = -gpm * (cy + alpha * dy);
  k[2] = -gpm * (cz + alpha * dz);
}

// Slonczewski spin-transfer torque in the Landau-Lifshitz form of the LLG
// equation (Methods, "Physics and discretization": spin torques are added per
// integrator stage): the Gilbert-form torque gamma0 mu0 b_J [eps m x (m x p)
// - eps' m x p] becomes
//   tau = gamma' mu0 b_J [(eps - alpha eps') m x (m x p) - (eps' + alpha eps) m x p],
//   eps = P Lambda^2 / ((Lambda^2 + 1) + (Lambda^2 - 1) m.p).
template <typename T>
__device__ inline void stt_tau(const FArgs<T>& a, T gpm, T alpha, T bJ, const T m[3], T tau[3]) {
  const T* p = a.sttp;
  const T mp = m[0] * p[0] + m[1] * p[1] + m[2] * p[2];
  const T eps = a.stt_P * a.stt_L2 / ((a.stt_L2 + T(1)) + (a.stt_L2 - T(1)) * mp);
  const T x[3] = {m[1] * p[2] - m[2] * p[1], m[2] * p[0] - m[0] * p[2], m[0] * p[1] - m[1] * p[0]};
  const T xx[3] = {m[1] * x[2] - m[2] * x[1], m[2] * x[0] - m[0] * x[2], m[0] * x[1] - m[1] * x[0]};
  const T c1 = gpm * bJ * (eps - alpha * a.stt_e2);
  const T c2 = gpm * bJ * (a.stt_e2 + alpha * eps);
#pragma unroll
  for (int c = 0; c < 3; ++c) tau[c] = c1 * xx[c] - c2 * x[c];
}

// b_J of replica r (0 without the spin-transfer term)
template <typename T>
__device__ inline T stt_bj(const FArgs<T>& a, int r) {
  return (a.terms & T_STT) ? (T)(a.stt_c * a.Jrep[r]) : T(0);
}

// Torque of the cell with the spin-transfer term added; tau receives that
// term alone (zero without it) for the rotation scheme.
template <typename T>
__device__ inline void cell_torque(const FArgs<T>& a, T gpm, T alpha, T bJ, const T mc[3],
                                   const T H[3], T k[3], T tau[3]) {
  llg_torque(mc, H, gpm, alpha, k);
  if (a.noprec) {
    // damping-only dynamics: -gamma' mu0 alpha m x (m x H)
    const T cx = mc[1] * H[2] - mc[2] * H[1];
    const T cy = mc[2] * H[0] - mc[0] * H[2];
    const T cz = mc[0] * H[1] - mc[1] * H[0];
    k[0] = -gpm * (alpha * (mc[1] * cz - mc[2] * cy));
    k[1] = -gpm * (alpha * (mc[2] * cx - mc[0] * cz));
    k[2] = -gpm * (alpha * (mc[0] * cy - mc[1] * cx));
  }
  tau[0] = tau[1] = tau[2] = T(0);
  if (bJ != T(0)) {
    stt_tau(a, gpm, alpha, bJ, mc, tau);
#pragma unroll
    for (int c = 0; c < 3; ++c) k[c] += tau[c];
  }
}

// the group's uniform damping
template <typename T>
__device__ inline void cell_torque(const FArgs<T>& a, T bJ, const T mc[3], const T H[3], T k[3],
                                   T tau[3]) {
  cell_torque(a, a.gpm, a.alpha, bJ, mc, H, k, tau);
}

// The LLG equation as a rotation, dm/dt = Omega x m with Omega =
// gamma' mu0 (H + alpha m x H) (Results, replica-batched engine: norm-exact
// Depondt-Mertens rotation scheme).
template <typename T>
__device__ inline void llg_omega(const T mc[3], const T H[3], T gpm, T alpha, T o[3]) {
  const T cx = mc[1] * H[2] - mc[2] * H[1];
  const T cy = mc[2] * H[0] - mc[0] * H[2];
  const T cz = mc[0] * H[1] - mc[1] * H[0];
  o[0] = gpm * (H[0] + alpha * cx);
  o[1] = gpm * (H[1] + alpha * cy);
  o[2] = gpm * (H[2] + alpha * cz);
}

// Rodrigues rotation of v about w by the angle |w|:
// v cos|w| + (w x v) sin|w|/|w| + w (w.v) (1 - cos|w|)/|w|^2, with
// 1 - cos|w| = 2 sin^2(|w|/2) (no cancellation) and Taylor series of both
// ratios below |w| = 1e-3.
template <typename T>
__device__ inline void rodrigues(const T v[3], const T w[3], T out[3]) {
  const T t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  T s1, s2;  // sin|w| / |w|, (1 - cos|w|) / |w|^2
  if (t2 < T(1e-6)) {
    s1 = T(1) - t2 * (T(1) / T(6) - t2 * (T(1) / T(120)));
    s2 = T(0.5) - t2 * (T(1) / T(24) - t2 * (T(1) / T(720)));
  } else {
    const T t = sqrt(t2);
    const T sh = sin(T(0.5) * t);
    s1 = sin(t) / t;
    s2 = T(2) * sh * sh / t2;
  }
  const T c = T(1) - t2 * s2;  // cos|w|
  const T wv = w[0] * v[0] + w[1] * v[1] + w[2] * v[2];
  out[0] = c * v[0] + s1 * (w[1] * v[2] - w[2] * v[1]) + s2 * wv * w[0];
  out[1] = c * v[1] + s1 * (w[2] * v[0] - w[0] * v[2]) + s2 * wv * w[1];
  out[2] = c * v[2] + s1 * (w[0] * v[1] - w[1] * v[0]) + s2 * wv * w[2];
}

// o += m x t
template <typename T>
__device__ inline void add_cross(const T m[3], const T t[3], T o[3]) {
  o[0] += m[1] * t[2] - m[2] * t[1];
  o[1] += m[2] * t[0] - m[0] * t[2];
  o[2] += m[0] * t[1] - m[1] * t[0];
}

// m_z of a corrected state for the per-workgroup sums of the switching
// check, made non-finite when any component of the state is (x - x is 0 for
// every finite x and NaN otherwise), so that the workgroup sum tells whether
// the new state is finite without a separate reduction
template <typename T>
__device__ inline double mz_checked(const T mn[3]) {
  return (double)(mn[2] + ((mn[0] - mn[0]) + (mn[1] - mn[1])));
}

// Heun-stage epilogues shared by the field kernels.  Predictor: m~ = m + dt k
// (Heun; the slope is not kept) or k1 <- Omega, m~ = rotation of m by
// dt Omega.  Corrector at m~ (mc) from the saved state mo: Heun's
// m + dt/2 (k1 + k) written as (mo + m~)/2 + dt/2 k (m~ = mo + dt k1, so no
// slope has to be stored), normalised; or the rotation of mo by
// dt/2 (Omega_1 + Omega_2), which keeps |m| = 1 in exact arithmetic.  In FP32
// the rounding of cos|w| near 1 repeats step after step when the rotation
// barely changes (a macrospin at rest near its easy axis drifted by 1e-3 in
// |m| over 2e5 steps), so the FP32 rotation is renormalised; FP64 is not.
// tau: spin-transfer torque at (mc), entering Omega as mc x tau
template <typename T>
__device__ inline void heun_predict(T gpm, T alpha, bool rot, const T mc[3], const T H[3],
                                    const T k[3], const T tau[3], T dt, T k1v[3], T mn[3]) {
  if (rot) {
    T w[3];
    llg_omega(mc, H, gpm, alpha, k1v);
    add_cross(mc, tau, k1v);
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = dt * k1v[c];
    rodrigues(mc, w, mn);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      k1v[c] = k[c];
      mn[c] = mc[c] + dt * k[c];
    }
  }
}

template <typename T>
__device__ inline void heun_correct(T gpm, T alpha, bool rot, const T mc[3], const T H[3],
                                    const T k[3], const T tau[3], const T mo[3], const T k1v[3],
                                    T dt, T mn[3]) {
  if (rot) {
    T o[3], w[3];
    llg_omega(mc, H, gpm, alpha, o);
    add_cross(mc, tau, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = T(0.5) * dt * (k1v[c] + o[c]);
    rodrigues(mo, w, mn);
    if constexpr (sizeof(T) == sizeof(float)) {
      const T inv = T(1) / sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) mn[c] *= inv;
    }
  } else {
    T u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = T(0.5) * (mo[c] + mc[c]) + T(0.5) * dt * k[c];
    const T inv = T(1) / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) mn[c] = u[c] * inv;
  }
}

// with the group's uniform damping
template <typename T>
__device__ inline void heun_predict(const FArgs<T>& a, bool rot, const T mc[3], const T H[3],
                                    const T k[3], const T tau[3], T dt, T k1v[3], T mn[3]) {
  heun_predict(a.gpm, a.alpha, rot, mc, H, k, tau, dt, k1v, mn);
}
template <typename T>
__device__ inline void heun_correct(const FArgs<T>& a, bool rot, const T mc[3], const T H[3],
                                    const T k[3], const T tau[3], const T mo[3], const T k1v[3],
                                    T dt, T mn[3]) {
  heun_correct(a.gpm, a.alpha, rot, mc, H, k, tau, mo, k1v, dt, mn);
}

// Step index and trial generation of the thermal noise of replica r.
template <typename T>
__device__ inline uint64_t noise_step(const FArgs<T>& a, int r, uint64_t step_now, uint32_t& gen) {
  gen = 0;
  if (!a.tgen) return step_now;
  gen = (uint32_t)a.tgen[r];
  return step_now - a.tstart[r];
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_fields(FArgs<T> a) {
  if (MODE != FM_ENERGY && a.done && *a.done) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
  const int hx = a.hx, L = a.L, nl = 3 * L;
  cpx<T>* Bf = A + nl * hx;
  __shared__ double red[kBlock * (MODE == FM_ENERGY ? 5 : 1)];
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, z = by, y0 = bx * L;
  const size_t rb = (size_t)r * 3 * a.N;
  const bool demag = (a.terms & T_DEMAG) != 0;
  const T* Hd = nullptr;  // real view of the inverse transform, line stride 2 hx
  cpx<T>* Hbuf = nullptr;
  const cpx<T>* tw_lds = nullptr;
  if (demag) {
    const cpx<T>* tw = stage_table(Bf + nl * hx, a.tw, hx);
    tw_lds = tw;
    const int Kx = a.Kx;
    batched_move<cpx<T>>(
        nl * hx,
        [&](int t) {
          const int line = udiv(t, hx), k = t - line * hx;
          const int c = udiv(line, L), l = line - c * L, y = y0 + l;
          cpx<T> Z = {0, 0};
          if (y < a.ny) {
            const cpx<T>* row = a.S + ((((size_t)r * 3 + c) * a.nz + z) * a.Sy + y) * Kx;
            if (a.xone) {
              Z = {row[0].re, T(0)};
            } else {
              const cpx<T> Xk = row[k];
              cpx<T> Xc = row[hx - k];
              Xc.im = -Xc.im;
              const cpx<T> E = cadd(Xk, Xc);
              const cpx<T> D = csub(Xk, Xc);
              const cpx<T> w = a.wpost[k];
              const cpx<T> O = cmulc(D, w);  // D * conj(W^k)
              Z = {E.re - O.im, E.im + O.re};
            }
          }
          return Z;
        },
        [&](int t, cpx<T> Z) { A[t] = Z; });
    __syncthreads();
    Hbuf = lds_fft<T, true>(A, Bf, nl, a.plan, tw);
    Hd = reinterpret_cast<const T*>(Hbuf);
  }
  // Heun epilogues with `fwd`: the new state of the block's rows is packed
  // into the free LDS buffer (real view, line c L + l) and x-transformed
  // after the cell loop, so the next field evaluation needs no k_xfwd pass
  constexpr bool kFwdMode = (MODE == FM_HEUN1 || MODE == FM_HEUN2 || MODE == FM_RKK);
  const bool fwd = kFwdMode && demag && a.fwd;
  T* F = fwd ? reinterpret_cast<T*>(Hbuf == A ? Bf : A) : nullptr;
  if (fwd && !a.plan_f.prune) {
    const int tail = 2 * hx - a.nx;  // zero input beyond the last cell
    for (int t = threadIdx.x; t < nl * tail; t += blockDim.x) {
      const int line = t / tail;
      F[line * 2 * hx + a.nx + (t - line * tail)] = T(0);
    }
  }
  const int ncell_blk = L * a.nx;
  const double dt_state = a.dtdev ? *a.dtdev : a.dth;
  const T dt = (T)dt_state;
  T sigma = 0;
  if ((a.terms & T_THERMAL) && a.Trep) {
    const double Tr = a.Trep[r];
    // per-cell damping or Ms: sigma_i = sqrt(sigunit T / dt) sqrt(alpha_i Ms / Ms_i)
    if (Tr > 0) sigma = (T)sqrt((a.sgc ? a.sigunit : a.sig2pref) * Tr / a.dt_th);
  }
  const T kbc = a.kbc;  // free-edge condition of the material's D (0 when D = 0)
  const unsigned N = (unsigned)a.N;
  const T* __restrict__ mr = a.m + rb;  // replica bases (uniform per workgroup)
  T* out_r = a.out ? a.out + rb : nullptr;
  T* mout_r = a.mout ? a.mout + rb : nullptr;
  T* k1_r = a.k1 ? a.k1 + rb : nullptr;
  const uint64_t step_now = (a.stepdev ? *a.stepdev : 0ull) + a.step;
  const T bJ = stt_bj(a, r);
  double acc[5] = {0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < ncell_blk; t += blockDim.x) {
    const int l = udiv(t, a.nx), x = t - l * a.nx, y = y0 + l;
    if (y >= a.ny) continue;
    const unsigned cell = (unsigned)x + (unsigned)a.nx * (unsigned)(y + a.ny * z);
    // the epilogue's own inputs (the step's base state and the earlier
    // slopes) are loaded before the field is computed, so their latencies
    // overlap it instead of following it one load at a time
    constexpr bool kPre = (MODE == FM_RKK || MODE == FM_RK7 || MODE == FM_HEUN2);
    T pm0[kPre ? 3 : 1], pk[kPre ? 6 : 1][3];
    if constexpr (MODE == FM_RKK) {
      if (fwd) {
        ld3(a.m0 + rb, N, cell, pm0);
#pragma unroll
        for (int j = 0; j < 6; ++j)
          if (a.cn[j] != T(0) && j != a.cstage) ld3(a.kk[j] + rb, N, cell, pk[j]);
      }
    } else if constexpr (MODE == FM_RK7) {
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (a.e[j] != 0.0) ld3(a.kk[j] + rb, N, cell, pk[j]);
    } else if constexpr (MODE == FM_HEUN2) {
      ld3(a.m0 + rb, N, cell, pm0);
      if (a.rot) ld3(k1_r, N, cell, pk[0]);
    }
    T mc[3];
    ld3(mr, N, cell, mc);
    T Hex[3], Hdm[3], Han[3], Hz[3];
    local_terms(a, mr, cell, x, y, z, mc, kbc, Hex, Hdm, Han, Hz);
    T Hdd[3] = {0, 0, 0};
    if (demag) {
#pragma unroll
      for (int c = 0; c < 3; ++c) Hdd[c] = Hd[(c * L + l) * 2 * hx + x];
      if (a.hd_out) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.hd_out[rb + c * N + cell] = Hdd[c];
      }
    } else if (a.hext) {
#pragma unroll
      for (int c = 0; c < 3; ++c) Hdd[c] = a.hext_scale * (T)a.hext[rb + c * N + cell];
      Hdd[2] += a.hext_mz * mc[2];
    }
    if (MODE == FM_ENERGY) {
      // per-cell Ms weighs each cell's -mu0 Ms_i m.H / 2 against the group's Ms
      const double w = a.msr ? (double)a.msr[cell] : 1.0;
      acc[0] += w * (double)(mc[0] * Hex[0] + mc[1] * Hex[1] + mc[2] * Hex[2]);
      acc[1] += w * (double)(mc[0] * Hdm[0] + mc[1] * Hdm[1] + mc[2] * Hdm[2]);
      acc[2] += w * (double)(mc[0] * Hdd[0] + mc[1] * Hdd[1] + mc[2] * Hdd[2]);
      acc[3] += w * (double)(mc[0] * Han[0] + mc[1] * Han[1] + mc[2] * Han[2]);
      if (a.terms & T_CUBIC) {
        // the quartic cubic term enters by its energy density, not -m.H/2
        T Hc[3], dens;
        cubic_terms(a, mc, Hc, dens);
        const double gi = a.mgi ? (double)a.mgi[cell] : 1.0;
        acc[3] += a.ecub * (double)dens -
                  w * gi * (double)(mc[0] * Hc[0] + mc[1] * Hc[1] + mc[2] * Hc[2]);
      }
      acc[4] += w * (double)(mc[0] * Hz[0] + mc[1] * Hz[1] + mc[2] * Hz[2]);
      continue;
    }
    T H[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) H[c] = Hex[c] + Hdm[c] + Han[c] + Hz[c] + Hdd[c];
    if (sigma != T(0)) {
      T eta[3];
      uint32_t gen;
      const uint64_t sn = noise_step(a, r, step_now, gen);
      thermal_eta<T>(a.seeds[r], (uint32_t)cell, sn, eta, gen);
      const T sg = a.sgc ? sigma * a.sgc[cell] : sigma;
#pragma unroll
      for (int c = 0; c < 3; ++c) H[c] += sg * eta[c];
    }
    if (MODE == FM_FIELD) {
#pragma unroll
      for (int c = 0; c < 3; ++c) out_r[c * N + cell] = H[c];
      continue;
    }
    // the cell's damping and spin-transfer strength (per-cell materials)
    const T gpm = a.gpc ? a.gpc[cell] : a.gpm;
    const T alpha = a.alc ? a.alc[cell] : a.alpha;
    const T bJc = a.mgi ? bJ * a.mgi[cell] : bJ;
    T k[3], tau[3];
    cell_torque(a, gpm, alpha, bJc, mc, H, k, tau);
    if (MODE == FM_TORQUE || MODE == FM_RKK) {
#pragma unroll
      for (int c = 0; c < 3; ++c) out_r[c * N + cell] = k[c];
      if (MODE == FM_RKK && fwd) {
        // the next stage's combined state, in the order of the combine pass
        T mv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T sv = pm0[c];
#pragma unroll
          for (int j = 0; j < 6; ++j) {
            if (a.cn[j] == T(0)) continue;
            const T kj = (j == a.cstage) ? k[c] : pk[j][c];
            sv += dt * a.cn[j] * kj;
          }
          mv[c] = sv;
        }
        if (a.cnext == 2) {
          const T inv = T(1) / sqrt(mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2]);
          mv[0] *= inv; mv[1] *= inv; mv[2] *= inv;
        }
        const T ws = a.msr ? a.msr[cell] : T(1);  // transform input M = Ms_i m
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          a.mnext[rb + c * N + cell] = mv[c];
          F[(c * L + l) * 2 * hx + x] = a.msr ? ws * mv[c] : mv[c];
        }
      }
    } else if (MODE == FM_HEUN1) {
      T k1v[3], mn[3];
      heun_predict(gpm, alpha, a.rot != 0, mc, H, k, tau, dt, k1v, mn);
      const T ws = a.msr ? a.msr[cell] : T(1);  // transform input M = Ms_i m
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (a.rot) k1_r[c * N + cell] = k1v[c];
        mout_r[c * N + cell] = mn[c];
        if (fwd) F[(c * L + l) * 2 * hx + x] = a.msr ? ws * mn[c] : mn[c];
      }
    } else if (MODE == FM_HEUN2) {
      T k1v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) k1v[c] = a.rot ? pk[0][c] : T(0);
      T mn[3];
      heun_correct(gpm, alpha, a.rot != 0, mc, H, k, tau, pm0, k1v, dt, mn);
      const T ws = a.msr ? a.msr[cell] : T(1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mout_r[c * N + cell] = mn[c];
        if (fwd) F[(c * L + l) * 2 * hx + x] = a.msr ? ws * mn[c] : mn[c];
      }
      acc[0] += mz_checked(mn);
    } else if (MODE == FM_RK7) {
#pragma unroll
      for (int c = 0; c < 3; ++c) out_r[c * N + cell] = k[c];
      double d2 = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double s = a.e[6] * (double)k[c];
#pragma unroll
        for (int j = 0; j < 6; ++j)
          if (a.e[j] != 0.0) s += a.e[j] * (double)pk[j][c];
        s *= dt_state;
        d2 += s * s;
      }
      const double en = sqrt(d2);
      acc[0] = (en != en) ? __builtin_inf() : fmax(acc[0], en);
    }
  }
  if (fwd) {
    __syncthreads();
    const cpx<T>* X =
        lds_fft<T, false>(reinterpret_cast<cpx<T>*>(F), Hbuf, nl, a.plan_f, tw_lds);
    xfwd_store(X, a.wpost, a.S, r, z, y0, L, hx, a.Kx, a.ny, a.nz, a.Sy,
               a.xone);
  }
  // workgroup reductions
  if (MODE == FM_HEUN2 || MODE == FM_ENERGY || MODE == FM_RK7) {
    const int nv = (MODE == FM_ENERGY) ? 5 : 1;
    for (int v = 0; v < nv; ++v) red[v * kBlock + threadIdx.x] = acc[v];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        for (int v = 0; v < nv; ++v) {
          const double o = red[v * kBlock + threadIdx.x + s];
          double& me = red[v * kBlock + threadIdx.x];
          me = (MODE == FM_RK7) ? fmax(me, o) : me + o;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const size_t blk = (size_t)by * gridDim.x + bx;
      const size_t nblk = (size_t)gridDim.x * gridDim.y;
      if (MODE == FM_RK7) {
        const double e = red[0];
        if (!(e <= 1.7976931348623157e308)) {
          a.st->nonfinite = 1;
        } else {
          atomicMax(&a.st->err_bits, (unsigned long long)__double_as_longlong(e));
        }
      } else {
        for (int v = 0; v < nv; ++v) a.partial[((size_t)r * nblk + blk) * nv + v] = red[v * kBlock];
        if (MODE == FM_HEUN2 && a.nblk_out && blk == 0 && r == 0) *a.nblk_out = (int)nblk;
        if (MODE == FM_HEUN2 && a.nonfinite && !(fabs(red[0]) <= 1.7976931348623157e308))
          *a.nonfinite = 1;
      }
    }
  }
}

}  // namespace mmx
