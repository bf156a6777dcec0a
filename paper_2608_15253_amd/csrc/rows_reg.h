// Row pass of the stochastic Heun stages (ROT: of the rotation scheme; STT:
// with the spin-transfer torque) with
// the rows' transforms in registers (device code): inverse x transform of the
// demag spectrum, local fields, torque, predictor or corrector update, and the
// forward x transform
// of the state just written, for films whose half-length x transform has
// hx = N1 * N2 points (4 x 4, 4 x 8, 8 x 8, 8 x 12, 8 x 16, 16 x 16).
//
// One wave holds RPW = 64 / N1 grid rows, N1 lanes per row.  A transform of
// a row, X[c + N1 d] = sum_k x[k] w^(+-k (c + N1 d)), splits k = a + N2 b:
// lane q takes the N1-point DFTs over b for a = q, q + N1, ... in registers,
// multiplies by w^(+-a c), the values are transposed through LDS so that lane
// c holds all a, and an N2-point DFT over a leaves lane c the outputs
// c + N1 d.  Each spectrum row is read once in coalesced order and paired
// (S[k] with S[hx - k]) through LDS for the complex-to-real combination.  The
// inverse transform's output (the demag field of the row) is staged in LDS,
// the lanes take the row's cells in coalesced order (x = q + N1 j) and
// overwrite each cell's field with its new state, which then leaves for HBM
// in 16-byte pieces and is read back in the input order of the forward
// transform; one more LDS exchange pairs X[k] with X[hx - k] for the
// real-to-complex split.  A row thus crosses LDS a fixed handful of times
// instead of once per radix pass.
// The cell arithmetic is the one of k_fields; only the butterfly order of
// the transforms differs.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "philox.h"
#include "yconv_reg.h"

namespace mmx {

// Split of a line of hx = N1 N2 points over N1 lanes: lane q holds the a =
// q + N1 s < N2 (s < S2); when N1 does not divide N2 the lanes with q >=
// N2 - N1 (S2 - 1) have one value slot less, and NV = S2 N1 >= N2 slots per
// component hold a line.
template <int N1, int N2>
struct RowSplit {
  static constexpr int S2 = (N2 + N1 - 1) / N1, NV = S2 * N1, n = N1 * N2;
  static constexpr bool even = N2 % N1 == 0;
  // whether lane q holds a = q + N1 s
  static __device__ inline bool has(int q, int s) { return even || q + N1 * s < N2; }
  // table index of w^(a c) (a c < n); powers of two keep their mask form
  static __device__ inline int tw(int ac) { return ((n & (n - 1)) == 0) ? (ac & (n - 1)) : ac; }
};

// One N1 x N2 transform of a line held by N1 lanes: in, v[s N1 + b] =
// x[q + N1 s + N2 b] (s < S2 with q + N1 s < N2, b < N1); out, v[d] =
// X[q + N1 d] (d < N2).  E: N1 (N2 + 1) LDS slots of this line (one-wave
// workgroup, wavefront-scope synchronisation).
template <typename T, int N1, int N2, bool INV, int NV>
__device__ inline void line_transform(cpx<T> (&v)[NV], cpx<T>* E, int q,
                                      const cpx<T>* __restrict__ tw) {
  using RS = RowSplit<N1, N2>;
  static_assert(NV == RS::NV, "line storage");
  constexpr int S2 = RS::S2, STR = N2 + 1;
#pragma unroll
  for (int s = 0; s < S2; ++s) {
    const int av = q + N1 * s;
    if (!RS::has(q, s)) continue;
    dft_reg<T, INV, N1>(&v[s * N1]);
    E[av] = v[s * N1];
#pragma unroll
    for (int cc = 1; cc < N1; ++cc) {
      const cpx<T> w = tw[RS::tw(av * cc)];
      E[cc * STR + av] = INV ? cmulc(v[s * N1 + cc], w) : cmul(v[s * N1 + cc], w);
    }
  }
  wave_sync();
#pragma unroll
  for (int av = 0; av < N2; ++av) v[av] = E[q * STR + av];
  wave_sync();
  dft_reg<T, INV, N2>(v);
}

// Real-to-complex split S[kx] = E + conj(W^kx) O of a row whose half-length
// transform X sits in the lanes as v[c][d] = X[q + N1 d]: lane q stores
// kx = q + N1 d and (lane 0) kx = hx; the partner X[hx - kx] comes through
// LDS, one component at a time (hx slots of E).  Followed by no
// synchronisation: E is reused only after the next one.
template <typename T, int N1, int N2, int NV>
__device__ inline void rows_store_spectrum(const cpx<T> (&v)[3][NV], cpx<T>* E, int q, bool live,
                                           cpx<T>* __restrict__ Srow, size_t cstride,
                                           const cpx<T>* __restrict__ wpost) {
  constexpr int hx = N1 * N2;
  auto split = [&](int kx) -> cpx<T> {
    const cpx<T> Zk = E[kx == hx ? 0 : kx];
    cpx<T> Zc = E[kx == 0 ? 0 : hx - kx];
    Zc.im = -Zc.im;
    const cpx<T> Ev = {T(0.5) * (Zk.re + Zc.re), T(0.5) * (Zk.im + Zc.im)};
    const cpx<T> O = {T(0.5) * (Zk.re - Zc.re), T(0.5) * (Zk.im - Zc.im)};
    const cpx<T> w = wpost[kx];
    return {Ev.re + (w.re * O.im + w.im * O.re), Ev.im - (w.re * O.re - w.im * O.im)};
  };
  // each lane stores two adjacent columns per instruction (a row's N1 lanes
  // cover 2 N1 consecutive columns), lane 0 also the last column kx = hx
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c > 0) wave_sync();  // the previous component's reads are done
#pragma unroll
    for (int d = 0; d < N2; ++d) E[q + N1 * d] = v[c][d];
    wave_sync();
    if (live) {
#pragma unroll
      for (int d = 0; d < N2 / 2; ++d) {
        const int kx = 2 * q + 2 * N1 * d;
        const cpx<T> s0 = split(kx), s1 = split(kx + 1);
        cpx<T>* dst = Srow + c * cstride + kx;
        dst[0] = s0;
        dst[1] = s1;
      }
      if (q == 0) Srow[c * cstride + hx] = split(hx);
    }
  }
}

// The half spectrum of state m for the films of k_rows_reg, with the same
// transform arithmetic as its forward part: a Heun run can then start (or
// resume) from a state in global memory and take bit for bit the steps that
// an uninterrupted run takes.
template <typename T, int N1, int N2>
__global__ void __launch_bounds__(64) k_rows_fwd(FArgs<T> a) {
  static_assert(N2 >= N1 && 64 % N1 == 0, "row split");
  using SP = RowSplit<N1, N2>;
  constexpr int hx = N1 * N2, RPW = 64 / N1, S2 = SP::S2;
  constexpr int RS = hx + N1;  // transpose slots N1 (N2 + 1); split slots hx
  __shared__ cpx<T> Es[RPW * RS];
  const int lane = threadIdx.x, row = lane / N1, q = lane - row * N1;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, z = by, y = bx * RPW + row;
  const bool live = y < a.ny;
  cpx<T>* E = Es + row * RS;
  const size_t rb = (size_t)r * 3 * a.N;
  const unsigned N = (unsigned)a.N;
  const int Kx = a.Kx;
  cpx<T>* Srow = a.S + (((size_t)r * 3 * a.nz + z) * a.Sy + (live ? y : 0)) * Kx;
  const size_t cstride = (size_t)a.nz * a.Sy * Kx;
  __shared__ cpx<T> twl[hx], wpl[hx + 1];  // transform and split tables
  for (int i = lane; i <= hx; i += 64) {
    if (i < hx) twl[i] = a.tw[i];
    wpl[i] = a.wpost[i];
  }
  wave_sync();
  const T* __restrict__ mr = a.m + rb;
  const unsigned row0 = (unsigned)a.nx * (unsigned)(y + a.ny * z);
  cpx<T> v[3][SP::NV];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        const int k = q + N1 * s + N2 * b;
        const int x = 2 * k;
        cpx<T> p = {0, 0};
        if (SP::has(q, s) && live && x < a.nx) p.re = mr[c * N + row0 + x];
        if (SP::has(q, s) && live && x + 1 < a.nx) p.im = mr[c * N + row0 + x + 1];
        v[c][s * N1 + b] = p;
      }
#pragma unroll
  for (int c = 0; c < 3; ++c) line_transform<T, N1, N2, false>(v[c], E, q, twl);
  rows_store_spectrum<T, N1, N2>(v, E, q, live, Srow, cstride, wpl);
}

// LDS row stride of k_rows_reg (complex slots): at least the row's field (3
// components of nx reals; nx = hx for an open x axis, 2 hx periodic), which
// covers the transpose slots N1 (N2 + 1) and the split slots hx, rounded to
// 8 mod 16 slots so that the 8-byte accesses of two neighbouring rows fall
// into complementary halves of the LDS banks
__host__ __device__ constexpr int rows_lds_stride(int nx) {
  return ((3 * nx / 2 + 7) & ~15) + 8;
}

template <typename T, int N1, int N2, int MODE, bool ROT, bool STT>
__global__ void __launch_bounds__(64) k_rows_reg(FArgs<T> a) {
  static_assert(MODE == FM_HEUN1 || MODE == FM_HEUN2, "Heun stages only");
  static_assert(sizeof(T) == sizeof(float), "FP32 row kernels");
  static_assert(N2 >= N1 && 64 % N1 == 0, "row split");
  using SP = RowSplit<N1, N2>;
  constexpr int hx = N1 * N2, RPW = 64 / N1, S2 = SP::S2;
  const int nx = a.nx, RS = rows_lds_stride(nx);  // LDS per row (dynamic)
  extern __shared__ unsigned char smem_raw[];
  // dynamic LDS starts 16-byte aligned and rows are whole complex slots: with
  // the alignment stated, complex LDS accesses are single 8-byte operations
  // (not pairs of 4-byte ones)
  cpx<T>* Es = static_cast<cpx<T>*>(__builtin_assume_aligned(smem_raw, 16));
  __shared__ double red[64];
  const int lane = threadIdx.x, row = lane / N1, q = lane - row * N1;
  int bx, by, bz;
  xcd_block(bx, by, bz);
  const int r = bz, z = by, y = bx * RPW + row;
  const bool live = y < a.ny;
  cpx<T>* E = static_cast<cpx<T>*>(__builtin_assume_aligned(Es + row * RS, 8));
  T* Hs = reinterpret_cast<T*>(E);  // real view [c][x], x < nx
  const size_t rb = (size_t)r * 3 * a.N;
  const unsigned N = (unsigned)a.N;
  const int Kx = a.Kx;
  // spectrum row of component c: S[(((r 3 + c) nz + z) Sy + y) Kx + kx]
  cpx<T>* Srow = a.S + (((size_t)r * 3 * a.nz + z) * a.Sy + (live ? y : 0)) * Kx;
  const size_t cstride = (size_t)a.nz * a.Sy * Kx;
  // spectrum row loads are unconditional, so that no branch splits the batch
  // and the waits for it count exactly: a row past the last reads row 0, and
  // what it computes from it is never stored (every store of the kernel is
  // guarded by `live`, and lanes exchange data only within their row)
  auto sload = [&](int c, int i) { return Srow[c * cstride + q + N1 * i]; };
  auto slast_load = [&](int c) { return Srow[c * cstride + hx]; };
  // transform and split tables staged in LDS: their loads go out first and
  // the spectrum loads of the up-front case (step 1) right after them, so the
  // two global latencies overlap
  __shared__ cpx<T> twl[hx], wpl[hx + 1];
  constexpr int TWL = (hx + 1 + 63) / 64;
  cpx<T> twv[TWL], wpv[TWL];
#pragma unroll
  for (int j = 0; j < TWL; ++j) {
    const int i = lane + 64 * j;
    if (i < hx) twv[j] = a.tw[i];
    if (i <= hx) wpv[j] = a.wpost[i];
  }
  constexpr bool kUpFront = N2 < 12;
  cpx<T> sv[kUpFront ? 3 : 1][N2], slast[kUpFront ? 3 : 1];
  if constexpr (kUpFront) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int i = 0; i < N2; ++i)
        sv[c][i] = sload(c, i);
      slast[c] = slast_load(c);
    }
  }
#pragma unroll
  for (int j = 0; j < TWL; ++j) {
    const int i = lane + 64 * j;
    if (i < hx) twl[i] = twv[j];
    if (i <= hx) wpl[i] = wpv[j];
  }
  wave_sync();
  const cpx<T>* tw = twl;  // exp(-2 pi i k / hx), k < hx
  // 1. inverse x transform of the demag spectrum: inputs Z[k] at k = q + N1 s
  //    + N2 b (complex-to-real combination of S[k] and S[hx - k]).  Each
  //    spectrum row is read once, in coalesced order (columns q + N1 i, lane
  //    0 also hx; all loads issued up front), and staged in LDS, where each
  //    lane picks its pairs
  //    Rows of up to 64 points load all three components up front; longer
  //    rows (N2 >= 12) load one component at a time, which keeps their
  //    register count down (16 x 16: 195 -> 170 VGPRs; measured faster there
  //    and slower on the 8 x 8 rows); the up-front loads are issued above
  cpx<T> v[3][SP::NV];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (kUpFront) {
#pragma unroll
      for (int i = 0; i < N2; ++i) E[q + N1 * i] = sv[c][i];
      if (q == 0) E[hx] = slast[c];
    } else {
#pragma unroll
      for (int i = 0; i < N2; ++i)
        sv[0][i] = sload(c, i);
      slast[0] = slast_load(c);
#pragma unroll
      for (int i = 0; i < N2; ++i) E[q + N1 * i] = sv[0][i];
      if (q == 0) E[hx] = slast[0];
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        if (!SP::has(q, s)) {
          v[c][s * N1 + b] = cpx<T>{0, 0};
          continue;
        }
        const int k = q + N1 * s + N2 * b;
        const cpx<T> Xk = E[k];
        cpx<T> Xc = E[hx - k];
        Xc.im = -Xc.im;
        const cpx<T> Ev = cadd(Xk, Xc);
        const cpx<T> D = csub(Xk, Xc);
        const cpx<T> O = cmulc(D, wpl[k]);  // D * conj(W^k)
        v[c][s * N1 + b] = live ? cpx<T>{Ev.re - O.im, Ev.im + O.re} : cpx<T>{0, 0};
      }
    wave_sync();
    line_transform<T, N1, N2, true>(v[c], E, q, tw);
  }
  // lane q holds z[q + N1 d] = H_demag at cells x = 2 (q + N1 d) + {0, 1};
  // stage the row's field in LDS (cells x < nx; nx is even)
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < N2; ++d) {
      const int x = 2 * (q + N1 * d);
      if (x < nx) {
        Hs[c * nx + x] = v[c][d].re;
        Hs[c * nx + x + 1] = v[c][d].im;
      }
    }
  wave_sync();
  const T dt = (T)a.dth;
  T sigma = 0;
  if ((a.terms & T_THERMAL) && a.Trep) {
    const double Tr = a.Trep[r];
    if (Tr > 0) sigma = (T)sqrt(a.sig2pref * Tr / a.dt_th);
  }
  const uint64_t step_now = (a.stepdev ? *a.stepdev : 0ull) + a.step;
  const T bJ = STT ? stt_bj(a, r) : T(0);
  const T* __restrict__ mr = a.m + rb;
  T* mout_r = a.mout + rb;
  T* k1_r = a.k1 + rb;
  double acc = 0;
#pragma unroll 2
  for (int j = 0; j < 2 * N2; ++j) {
    const int x = q + N1 * j;
    T mn_out[3] = {0, 0, 0};
    if (x >= nx) break;  // x grows with j
    if (live) {
      const unsigned cell = (unsigned)x + (unsigned)nx * (unsigned)(y + a.ny * z);
      T mc[3];
      ld3<T, true>(mr, N, cell, mc);
      T Hex[3], Hdm[3], Han[3], Hz[3];
      local_terms<T, false, true>(a, mr, cell, x, y, z, mc, a.kbc, Hex, Hdm, Han, Hz);
      T H[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) H[c] = Hex[c] + Hdm[c] + Han[c] + Hz[c] + Hs[c * nx + x];
      if (sigma != T(0)) {
        T eta[3];
        uint32_t gen;
        const uint64_t sn = noise_step(a, r, step_now, gen);
        thermal_eta<T>(a.seeds[r], (uint32_t)cell, sn, eta, gen);
#pragma unroll
        for (int c = 0; c < 3; ++c) H[c] += sigma * eta[c];
      }
      T kv[3], tau[3] = {0, 0, 0};
      if (STT) cell_torque(a, bJ, mc, H, kv, tau);
      else llg_torque(mc, H, a.gpm, a.alpha, kv);
      if (MODE == FM_HEUN1) {
        T k1v[3];
        heun_predict(a, ROT, mc, H, kv, tau, dt, k1v, mn_out);
        if (ROT) {
#pragma unroll
          for (int c = 0; c < 3; ++c) k1_r[c * N + cell] = k1v[c];
        }
      } else {
        T mo[3], k1v[3];
        ld3<T, true>(a.m0 + rb, N, cell, mo);
        if (ROT) ld3<T, true>(k1_r, N, cell, k1v);
        else k1v[0] = k1v[1] = k1v[2] = T(0);
        heun_correct(a, ROT, mc, H, kv, tau, mo, k1v, dt, mn_out);
        acc += mz_checked(mn_out);
      }
    }
    // the new state is the forward transform's input; it replaces the field
    // value of the same cell
#pragma unroll
    for (int c = 0; c < 3; ++c) Hs[c * nx + x] = mn_out[c];
  }
  wave_sync();
  // the row's new state goes out from LDS in 16-byte pieces (the N1 lanes of
  // a row write 16 N1 consecutive bytes per instruction), or cell by cell
  // when the state of this replica group is not 16-byte aligned
  if (live) {
    const unsigned row0 = (unsigned)nx * (unsigned)(y + a.ny * z);
    if ((((uintptr_t)mout_r) & 15) == 0 && (N & 3) == 0) {
      const int nq = nx / 4;
      for (int i = q; i < 3 * nq; i += N1) {
        const int c = i / nq, x4 = 4 * (i - c * nq);
        const T* h = Hs + c * nx + x4;
        *reinterpret_cast<float4*>(mout_r + c * N + row0 + x4) = float4{h[0], h[1], h[2], h[3]};
      }
    } else {
      for (int i = q; i < 3 * nx; i += N1) {
        const int c = i / nx, x = i - c * nx;
        mout_r[c * N + row0 + x] = Hs[c * nx + x];
      }
    }
  }
  // 2. forward x transform of the new state, inputs at k = q + N1 s + N2 b
  //    (zero beyond the last cell)
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int s = 0; s < S2; ++s)
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        const int k = q + N1 * s + N2 * b;
        v[c][s * N1 + b] = (SP::has(q, s) && 2 * k < nx)
                               ? cpx<T>{Hs[c * nx + 2 * k], Hs[c * nx + 2 * k + 1]}
                               : cpx<T>{0, 0};
      }
  wave_sync();
#pragma unroll
  for (int c = 0; c < 3; ++c) line_transform<T, N1, N2, false>(v[c], E, q, tw);
  // 3. the half spectrum of the new state
  rows_store_spectrum<T, N1, N2>(v, E, q, live, Srow, cstride, wpl);
  if (MODE == FM_HEUN2) {
    // per-workgroup sum of m_z (fixed order) for the switching detector
    red[lane] = acc;
    wave_sync();
    for (int s = 32; s > 0; s >>= 1) {
      if (lane < s) red[lane] += red[lane + s];
      wave_sync();
    }
    if (lane == 0) {
      const size_t blk = (size_t)by * gridDim.x + bx;
      const size_t nblk = (size_t)gridDim.x * gridDim.y;
      a.partial[(size_t)r * nblk + blk] = red[0];
      if (a.nblk_out && blk == 0 && r == 0) *a.nblk_out = (int)nblk;
      if (a.nonfinite && !(fabs(red[0]) <= 1.7976931348623157e308)) *a.nonfinite = 1;
    }
  }
}

}  // namespace mmx
