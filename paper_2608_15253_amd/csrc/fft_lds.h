// Workgroup-cooperative Stockham FFT staged in LDS (device code).
//
// A workgroup transforms `nlines` independent lines of length n held
// contiguously in LDS ([line][n], complex).  Each pass of radix R reads the R
// inputs of a butterfly at stride n/R, applies the Stockham twiddles
// exp(-+2 pi i r (j mod Ns) / (Ns R)), transforms them with a small DFT and
// writes them to the autosorted position (j / Ns) Ns R + (j mod Ns) + r Ns of
// the other buffer; Ns grows by R per pass, so mixed radices 2, 3, 4, 5, 8 and
// 16 combine in any order and the output is in natural order.  A pruned first
// pass (radix 2, input zero beyond n/2, as in the zero-padded demag
// convolution) reduces to duplicating its input.  Transforms are unnormalised.
#pragma once
#include "common.h"

namespace mmx {

// a / d and a % d with shifts when the (uniform) divisor is a power of two
__device__ inline int udiv(int a, int d) {
  return ((d & (d - 1)) == 0) ? (a >> __builtin_ctz(d)) : a / d;
}
__device__ inline int umod(int a, int d) {
  return ((d & (d - 1)) == 0) ? (a & (d - 1)) : a % d;
}

template <typename T, bool INV>
struct Dft {
  static __device__ inline void r2(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
  // multiply by -i (forward) or +i (inverse)
  static __device__ inline cpx<T> rot(cpx<T> a) {
    return INV ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
  }
  static __device__ inline void r4(cpx<T>* v) {
    cpx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cpx<T> s13 = cadd(v[1], v[3]), d13 = rot(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
  static __device__ inline void r3(cpx<T>* v) {
    const T c = T(-0.5);
    const T s = INV ? T(0.86602540378443864676) : T(-0.86602540378443864676);
    cpx<T> a = v[0], b = v[1], d = v[2];
    cpx<T> t = cadd(b, d);
    cpx<T> u = csub(b, d);
    cpx<T> m = {a.re + c * t.re, a.im + c * t.im};
    // s * i * u
    cpx<T> su = {-s * u.im, s * u.re};
    v[0] = cadd(a, t);
    v[1] = cadd(m, su);
    v[2] = csub(m, su);
  }
  static __device__ inline void r5(cpx<T>* v) {
    const T c1 = T(0.30901699437494742410);   // cos(2pi/5)
    const T c2 = T(-0.80901699437494742410);  // cos(4pi/5)
    const T s1 = INV ? T(0.95105651629515357212) : T(-0.95105651629515357212);
    const T s2 = INV ? T(0.58778525229247312917) : T(-0.58778525229247312917);
    cpx<T> a = v[0];
    cpx<T> t1 = cadd(v[1], v[4]), u1 = csub(v[1], v[4]);
    cpx<T> t2 = cadd(v[2], v[3]), u2 = csub(v[2], v[3]);
    cpx<T> m1 = {a.re + c1 * t1.re + c2 * t2.re, a.im + c1 * t1.im + c2 * t2.im};
    cpx<T> m2 = {a.re + c2 * t1.re + c1 * t2.re, a.im + c2 * t1.im + c1 * t2.im};
    // i*(s1 u1 + s2 u2) and i*(s2 u1 - s1 u2)
    cpx<T> n1 = {-(s1 * u1.im + s2 * u2.im), s1 * u1.re + s2 * u2.re};
    cpx<T> n2 = {-(s2 * u1.im - s1 * u2.im), s2 * u1.re - s1 * u2.re};
    v[0] = cadd(a, cadd(t1, t2));
    v[1] = cadd(m1, n1);
    v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2);
    v[3] = csub(m2, n2);
  }
  static __device__ inline void r8(cpx<T>* v) {
    const T h = T(0.70710678118654752440);
    // radix-2 first stage: pairs (k, k+4)
    cpx<T> a[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = cadd(v[k], v[k + 4]);
      a[k + 4] = csub(v[k], v[k + 4]);
    }
    // twiddles w8^k on the odd half (w8 = exp(-+ i pi / 4))
    {
      cpx<T> x = a[5];
      a[5] = INV ? cpx<T>{h * (x.re - x.im), h * (x.re + x.im)}
                 : cpx<T>{h * (x.re + x.im), h * (x.im - x.re)};
      a[6] = rot(a[6]);
      x = a[7];
      a[7] = INV ? cpx<T>{-h * (x.re + x.im), h * (x.re - x.im)}
                 : cpx<T>{h * (x.im - x.re), -h * (x.re + x.im)};
    }
    cpx<T> e[4] = {a[0], a[1], a[2], a[3]};
    cpx<T> o[4] = {a[4], a[5], a[6], a[7]};
    r4(e);
    r4(o);
    v[0] = e[0]; v[2] = e[1]; v[4] = e[2]; v[6] = e[3];
    v[1] = o[0]; v[3] = o[1]; v[5] = o[2]; v[7] = o[3];
  }
  // 12-point DFT as 3 x 4: DFT3 over n1 of x[4 n1 + n2], twiddle w12^(n2 k1),
  // DFT4 over n2; output index k1 + 3 k2.
  static __device__ inline void r12(cpx<T>* v) {
    const T h = T(0.86602540378443864676);
    // w12^j = cos(2 pi j / 12) -/+ i sin(2 pi j / 12) for j = 0..6
    const T wc[7] = {T(1), h, T(0.5), T(0), T(-0.5), -h, T(-1)};
    const T ws[7] = {T(0), T(0.5), h, T(1), h, T(0.5), T(0)};
    cpx<T> a[4][3];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cpx<T> t[3] = {v[n2], v[4 + n2], v[8 + n2]};
      r3(t);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) {
        const int j = n2 * k1;
        const cpx<T> w = {wc[j], INV ? ws[j] : -ws[j]};
        a[n2][k1] = (j == 0) ? t[k1] : cmul(t[k1], w);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cpx<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      r4(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 3 * k2] = t[k2];
    }
  }
  // A B-point DFT as A x B: DFT_A over n1 of x[B n1 + n2], twiddle
  // w^(n2 k1) from the tables (cos, sin of 2 pi j / (A B)), DFT_B over n2;
  // output index k1 + A k2.
  template <int A, int B>
  static __device__ inline void split(cpx<T>* v, const T* wc, const T* ws) {
    cpx<T> a[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      cpx<T> t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
      if constexpr (A == 3) r3(t);
      if constexpr (A == 4) r4(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int j = n2 * k1;
        const cpx<T> w = {wc[j], INV ? ws[j] : -ws[j]};
        a[n2][k1] = (j == 0) ? t[k1] : cmul(t[k1], w);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cpx<T> t[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) t[n2] = a[n2][k1];
      if constexpr (B == 8) r8(t);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = t[k2];
    }
  }
  // 24-point DFT as 3 x 8
  static __device__ inline void r24(cpx<T>* v) {
    const T wc[15] = {T(1.0), T(0.9659258262890683), T(0.8660254037844386), T(0.7071067811865476), T(0.5), T(0.25881904510252074), T(0.0), T(-0.25881904510252074), T(-0.5), T(-0.7071067811865476), T(-0.8660254037844386), T(-0.9659258262890683), T(-1.0), T(-0.9659258262890683), T(-0.8660254037844386)};
    const T ws[15] = {T(0.0), T(0.25881904510252074), T(0.5), T(0.7071067811865476), T(0.8660254037844386), T(0.9659258262890683), T(1.0), T(0.9659258262890683), T(0.8660254037844386), T(0.7071067811865476), T(0.5), T(0.25881904510252074), T(0.0), T(-0.25881904510252074), T(-0.5)};
    split<3, 8>(v, wc, ws);
  }
  // 32-point DFT as 4 x 8
  static __device__ inline void r32(cpx<T>* v) {
    const T wc[22] = {T(1.0), T(0.9807852804032304), T(0.9238795325112867), T(0.8314696123025452), T(0.7071067811865476), T(0.5555702330196022), T(0.3826834323650898), T(0.19509032201612828), T(0.0), T(-0.19509032201612828), T(-0.3826834323650898), T(-0.5555702330196022), T(-0.7071067811865476), T(-0.8314696123025452), T(-0.9238795325112867), T(-0.9807852804032304), T(-1.0), T(-0.9807852804032304), T(-0.9238795325112867), T(-0.8314696123025452), T(-0.7071067811865476), T(-0.5555702330196022)};
    const T ws[22] = {T(0.0), T(0.19509032201612828), T(0.3826834323650898), T(0.5555702330196022), T(0.7071067811865476), T(0.8314696123025452), T(0.9238795325112867), T(0.9807852804032304), T(1.0), T(0.9807852804032304), T(0.9238795325112867), T(0.8314696123025452), T(0.7071067811865476), T(0.5555702330196022), T(0.3826834323650898), T(0.19509032201612828), T(0.0), T(-0.19509032201612828), T(-0.3826834323650898), T(-0.5555702330196022), T(-0.7071067811865476), T(-0.8314696123025452)};
    split<4, 8>(v, wc, ws);
  }
  // 16-point DFT as 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle w16^(n2 k1),
  // DFT4 over n2; output index k1 + 4 k2.
  static __device__ inline void r16(cpx<T>* v) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T h = T(0.70710678118654752440);
    // w16^j = cos(2 pi j / 16) -/+ i sin(2 pi j / 16) for j = 0..9
    const T wc[10] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1};
    const T ws[10] = {T(0), s1, h, c1, T(1), c1, h, s1, T(0), -s1};
    cpx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cpx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      r4(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) {
        const int j = n2 * k1;
        const cpx<T> w = {wc[j], INV ? ws[j] : -ws[j]};
        a[n2][k1] = (j == 0) ? t[k1] : cmul(t[k1], w);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      r4(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

template <typename T, bool INV, int R>
__device__ inline void stockham_pass(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                     int n, int Ns, int nlines, const cpx<T>* __restrict__ tw,
                                     int tid, int nthr, int ld) {
  const int nb = n / R;
  const int total = nb * nlines;
  const int twscale = n / (Ns * R);
  // power-of-two extents (the common case) index with shifts and masks
  const bool p2 = ((nb & (nb - 1)) == 0) && ((Ns & (Ns - 1)) == 0);
  const int lnb = __builtin_ctz(nb), lns = __builtin_ctz(Ns);
  for (int t = tid; t < total; t += nthr) {
    const int line = p2 ? (t >> lnb) : t / nb;
    const int j = t - line * nb;
    const cpx<T>* s = src + line * ld;
    cpx<T>* d = dst + line * ld;
    const int jq = p2 ? (j >> lns) : j / Ns;
    const int jm = j - jq * Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    if (jm != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cpx<T> w = tw[r * jm * twscale];
        v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    if constexpr (R == 2) Dft<T, INV>::r2(v);
    if constexpr (R == 3) Dft<T, INV>::r3(v);
    if constexpr (R == 4) Dft<T, INV>::r4(v);
    if constexpr (R == 5) Dft<T, INV>::r5(v);
    if constexpr (R == 8) Dft<T, INV>::r8(v);
    if constexpr (R == 16) Dft<T, INV>::r16(v);
    const int idxD = jq * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) d[idxD + r * Ns] = v[r];
  }
}

// Transforms nlines lines in `a` (scratch `b`), returns the buffer holding the
// result.  `tw` is the table exp(-2 pi i k / n), k < n.  Lines start every
// `ld` slots (0: every n, contiguous).  Must be called by the whole
// workgroup; ends with a barrier.
template <typename T, bool INV>
__device__ cpx<T>* lds_fft(cpx<T>* a, cpx<T>* b, int nlines, const FftPlan& p,
                           const cpx<T>* __restrict__ tw, int ld = 0) {
  const int n = p.n;
  if (ld == 0) ld = n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  int Ns = 1;
  for (int ps = 0; ps < p.npass; ++ps) {
    const int R = p.radix[ps];
    if (ps == 0 && p.prune) {
      const int half = n / 2;
      const int total = half * nlines;
      for (int t = tid; t < total; t += nthr) {
        const int line = udiv(t, half);
        const int j = t - line * half;
        const cpx<T> v = a[line * ld + j];
        b[line * ld + 2 * j] = v;
        b[line * ld + 2 * j + 1] = v;
      }
    } else {
      switch (R) {
        case 2: stockham_pass<T, INV, 2>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
        case 3: stockham_pass<T, INV, 3>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
        case 4: stockham_pass<T, INV, 4>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
        case 5: stockham_pass<T, INV, 5>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
        case 8: stockham_pass<T, INV, 8>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
        default: stockham_pass<T, INV, 16>(a, b, n, Ns, nlines, tw, tid, nthr, ld); break;
      }
    }
    __syncthreads();
    cpx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

}  // namespace mmx
