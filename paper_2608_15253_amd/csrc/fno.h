// Learned demag surrogate: Fourier neural operator forward, backward and Adam
// kernels (device code).
//
// Activations are FP32, [b][channel][pixel] with x fastest.  The pointwise
// (1x1) channel maps are GEMMs over channels for every pixel and run on the
// matrix cores: v_mfma_f32_16x16x32_bf16 with BF16 operands staged in LDS and
// FP32 accumulation (a VALU FP32 variant of the same kernel serves parity
// checks).  The truncated Fourier transforms (M1 x-modes, 2 M2 y-modes), the
// per-mode complex channel mixing and the weight gradients run as FP32
// matrix-core products (fno_mfma.h); the VALU kernels below serve shapes
// outside those kernels' limits, the loss and Adam.
#pragma once
#include "common.h"

namespace mmx {

constexpr int kFnoBlock = 256;
constexpr int kFnoPixTile = 64;   // pixels per VALU 1x1-map workgroup
constexpr int kConvPixMfma = 64;  // pixels per matrix-core 1x1-map workgroup (a multiple of 64)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum ConvEpi { CE_STORE = 0, CE_GELU = 1, CE_GELU_GRAD = 2, CE_ACCUM = 3 };

struct ConvArgs {
  const float* X;      // [B][K][P]
  const float* Wt;     // [M][K] (or [K][M] when trans)
  const float* bias;   // [M] or null
  float* Y;            // [B][M][P]: result (pre-activation / product / sum)
  float* A;            // [B][M][P]: gelu(Y) when CE_GELU
  const float* S;      // [B][M][P]: saved pre-activation for CE_GELU_GRAD
  int M, K, P, trans, epi;
};

// Y[b][m][p] = sum_k W[m][k] X[b][k][p] + bias[m], then the epilogue.
// Workgroup: sample blockIdx.y, pixels [PT blockIdx.x, +PT); on the matrix
// cores wave w owns PT / 64 tiles of 16 pixels and every 16-row tile of the
// output channels (64-pixel workgroups measured faster than 128).
template <bool MFMA>
__global__ void __launch_bounds__(kFnoBlock) k_conv1x1(ConvArgs a) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int PT = MFMA ? kConvPixMfma : kFnoPixTile;
  const int b = blockIdx.y, p0 = blockIdx.x * PT;
  const int Mp = (a.M + 15) & ~15, Kp = (a.K + 31) & ~31;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* Xb = a.X + (size_t)b * a.K * a.P;
  if (MFMA) {
    // both operands k-contiguous in LDS, rows padded by 8 elements, so that a
    // lane's 8 reduction values are one 16-byte read
    const int KS = Kp + 8;
    __bf16* Ws = reinterpret_cast<__bf16*>(smem_raw);   // [Mp][KS]
    __bf16* Xs = Ws + (size_t)Mp * KS;                  // [PT pixels][KS]
    // weights, then pixels: four global loads in flight per thread before the
    // converted values go to LDS
    const int nw = Mp * Kp;
    for (int i0 = threadIdx.x; i0 < nw; i0 += 4 * kFnoBlock) {
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kFnoBlock, m = i / Kp, k = i - m * Kp;
        v[u] = 0.f;
        if (i < nw && m < a.M && k < a.K)
          v[u] = a.trans ? a.Wt[(size_t)k * a.M + m] : a.Wt[(size_t)m * a.K + k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kFnoBlock, m = i / Kp, k = i - m * Kp;
        if (i < nw) Ws[(size_t)m * KS + k] = (__bf16)v[u];
      }
    }
    if (a.P % 4 == 0) {
      // 16-byte loads of four pixels of one channel
      constexpr int QX = PT / 4;  // 16-byte pieces per channel row
      const int nx = Kp * QX;
      for (int i0 = threadIdx.x; i0 < nx; i0 += 4 * kFnoBlock) {
        f32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * kFnoBlock, k = i / QX, px = p0 + 4 * (i % QX);
          v[u] = f32x4{0.f, 0.f, 0.f, 0.f};
          if (i < nx && k < a.K && px < a.P)
            v[u] = *reinterpret_cast<const f32x4*>(Xb + (size_t)k * a.P + px);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * kFnoBlock, k = i / QX, q = 4 * (i % QX);
          if (i < nx) {
#pragma unroll
            for (int e = 0; e < 4; ++e) Xs[(size_t)(q + e) * KS + k] = (__bf16)v[u][e];
          }
        }
      }
    } else {
      for (int i = threadIdx.x; i < Kp * PT; i += blockDim.x) {
        const int k = i / PT, px = i - k * PT;
        float v = 0.f;
        if (k < a.K && p0 + px < a.P) v = Xb[(size_t)k * a.P + p0 + px];
        Xs[(size_t)px * KS + k] = (__bf16)v;
      }
    }
    __syncthreads();
    const int col = lane & 15, grp = lane >> 4, nkt = Kp / 32;
    for (int pt = 0; pt < PT / 64; ++pt) {
      const int px = wave * (PT / 4) + pt * 16 + col;  // this lane's pixel column
      // B operands of every reduction step (Kp <= 128)
      bf16x8 bv[4];
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        if (kt < nkt) bv[kt] = *reinterpret_cast<const bf16x8*>(Xs + (size_t)px * KS + kt * 32 + 8 * grp);
      for (int mt = 0; mt < Mp / 16; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const __bf16* wrow = Ws + (size_t)(mt * 16 + col) * KS + 8 * grp;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
          if (kt < nkt)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                *reinterpret_cast<const bf16x8*>(wrow + kt * 32), bv[kt], acc, 0, 0, 0);
        const int p = p0 + px;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int m = mt * 16 + 4 * grp + j;
          if (m < a.M && p < a.P) {
            const size_t o = ((size_t)b * a.M + m) * a.P + p;
            float y = acc[j] + (a.bias ? a.bias[m] : 0.f);
            if (a.epi == CE_ACCUM) y += a.Y[o];
            if (a.epi == CE_GELU_GRAD) y *= gelu_grad_f(a.S[o]);
            a.Y[o] = y;
            if (a.epi == CE_GELU) a.A[o] = gelu_f(y);
          }
        }
      }
    }
  } else {
    float* Ws = reinterpret_cast<float*>(smem_raw);     // [M][K]
    float* Xs = Ws + (size_t)a.M * a.K;                  // [K][64]
    for (int i = threadIdx.x; i < a.M * a.K; i += blockDim.x) {
      const int m = i / a.K, k = i - m * a.K;
      Ws[i] = a.trans ? a.Wt[(size_t)k * a.M + m] : a.Wt[(size_t)m * a.K + k];
    }
    for (int i = threadIdx.x; i < a.K * kFnoPixTile; i += blockDim.x) {
      const int k = i / kFnoPixTile, px = i - k * kFnoPixTile;
      Xs[i] = (p0 + px < a.P) ? Xb[(size_t)k * a.P + p0 + px] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.M * kFnoPixTile; i += blockDim.x) {
      const int m = i / kFnoPixTile, px = i - m * kFnoPixTile, p = p0 + px;
      if (p >= a.P) continue;
      float y = 0.f;
      for (int k = 0; k < a.K; ++k) y += Ws[(size_t)m * a.K + k] * Xs[(size_t)k * kFnoPixTile + px];
      y += a.bias ? a.bias[m] : 0.f;
      const size_t o = ((size_t)b * a.M + m) * a.P + p;
      if (a.epi == CE_ACCUM) y += a.Y[o];
      if (a.epi == CE_GELU_GRAD) y *= gelu_grad_f(a.S[o]);
      a.Y[o] = y;
      if (a.epi == CE_GELU) a.A[o] = gelu_f(y);
    }
  }
}

// Truncated forward transform of every (b, channel) plane:
// Vh[b][c][kx][j] = scale[kx] sum_{y,x} V[b][c][y][x] Fx[kx][x] Fy[j][y].
struct SpecArgs {
  const float* in;           // spec_fwd: real planes; spec_inv: complex modes
  float* out;
  const cpx<float>* Fx;      // [M1][W]  exp(-2 pi i kx x / W)
  const cpx<float>* Fy;      // [J][H]   exp(-2 pi i ky_j y / H)
  const float* coef;         // [M1] per-kx scale
  const float* add;          // spec_inv: added field (may alias out) or null
  float* act;                // spec_inv: gelu(out) or null
  int H, W, M1, J;
};

__global__ void __launch_bounds__(kFnoBlock) k_spec_fwd(SpecArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cpx<float>* Fxs = reinterpret_cast<cpx<float>*>(smem_raw);  // [M1][W]
  cpx<float>* Fys = Fxs + a.M1 * a.W;                          // [J][H]
  cpx<float>* Ax = Fys + a.J * a.H;                            // [H][M1]
  const int plane = blockIdx.x;
  const float* V = a.in + (size_t)plane * a.H * a.W;
  for (int i = threadIdx.x; i < a.M1 * a.W; i += blockDim.x) Fxs[i] = a.Fx[i];
  for (int i = threadIdx.x; i < a.J * a.H; i += blockDim.x) Fys[i] = a.Fy[i];
  __syncthreads();
  for (int i = threadIdx.x; i < a.H * a.M1; i += blockDim.x) {
    const int y = i / a.M1, kx = i - y * a.M1;
    const float* row = V + (size_t)y * a.W;
    float re = 0.f, im = 0.f;
    for (int x = 0; x < a.W; ++x) {
      const float v = row[x];
      re += v * Fxs[kx * a.W + x].re;
      im += v * Fxs[kx * a.W + x].im;
    }
    Ax[i] = {re, im};
  }
  __syncthreads();
  cpx<float>* out = reinterpret_cast<cpx<float>*>(a.out) + (size_t)plane * a.M1 * a.J;
  for (int i = threadIdx.x; i < a.M1 * a.J; i += blockDim.x) {
    const int kx = i / a.J, j = i - kx * a.J;
    float re = 0.f, im = 0.f;
    for (int y = 0; y < a.H; ++y) {
      const cpx<float> u = Ax[y * a.M1 + kx], f = Fys[j * a.H + y];
      re += u.re * f.re - u.im * f.im;
      im += u.re * f.im + u.im * f.re;
    }
    const float s = a.coef ? a.coef[kx] : 1.f;
    out[i] = {s * re, s * im};
  }
}

// Inverse of the truncated modes of every (b, channel) plane:
// U[y][x] = sum_kx coef[kx] Re(sum_j Uh[kx][j] conj(Fy[j][y]) conj(Fx[kx][x]));
// out = U + add (add may alias out), act = gelu(out) when requested.
__global__ void __launch_bounds__(kFnoBlock) k_spec_inv(SpecArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cpx<float>* Fxs = reinterpret_cast<cpx<float>*>(smem_raw);  // [M1][W]
  cpx<float>* Fys = Fxs + a.M1 * a.W;                          // [J][H]
  cpx<float>* Ay = Fys + a.J * a.H;                            // [M1][H]
  cpx<float>* Us = Ay + a.M1 * a.H;                            // [M1][J]
  const int plane = blockIdx.x;
  const cpx<float>* Uh = reinterpret_cast<const cpx<float>*>(a.in) + (size_t)plane * a.M1 * a.J;
  for (int i = threadIdx.x; i < a.M1 * a.W; i += blockDim.x) Fxs[i] = a.Fx[i];
  for (int i = threadIdx.x; i < a.J * a.H; i += blockDim.x) Fys[i] = a.Fy[i];
  for (int i = threadIdx.x; i < a.M1 * a.J; i += blockDim.x) Us[i] = Uh[i];
  __syncthreads();
  for (int i = threadIdx.x; i < a.M1 * a.H; i += blockDim.x) {
    const int kx = i / a.H, y = i - kx * a.H;
    float re = 0.f, im = 0.f;
    for (int j = 0; j < a.J; ++j) {
      const cpx<float> u = Us[kx * a.J + j], f = Fys[j * a.H + y];  // u * conj(f)
      re += u.re * f.re + u.im * f.im;
      im += u.im * f.re - u.re * f.im;
    }
    const float c = a.coef[kx];
    Ay[i] = {c * re, c * im};
  }
  __syncthreads();
  float* out = a.out + (size_t)plane * a.H * a.W;
  const float* add = a.add ? a.add + (size_t)plane * a.H * a.W : nullptr;
  float* act = a.act ? a.act + (size_t)plane * a.H * a.W : nullptr;
  for (int i = threadIdx.x; i < a.H * a.W; i += blockDim.x) {
    const int y = i / a.W, x = i - y * a.W;
    float s = 0.f;
    for (int kx = 0; kx < a.M1; ++kx) {
      const cpx<float> u = Ay[kx * a.H + y], f = Fxs[kx * a.W + x];  // Re(u conj(f))
      s += u.re * f.re + u.im * f.im;
    }
    if (add) s += add[i];
    out[i] = s;
    if (act) act[i] = gelu_f(s);
  }
}

// Input features [m_x, m_y, m_z, x/W - 1/2, y/H - 1/2] per pixel.
__global__ void k_fno_features(const float* m, float* X0, int B, int H, int W) {
  const long P = (long)H * W;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * P) return;
  const long b = i / P, p = i - b * P;
  const int y = p / W, x = p - (long)y * W;
  float* o = X0 + (size_t)b * 5 * P + p;
  const float* mi = m + (size_t)b * 3 * P + p;
  o[0] = mi[0];
  o[P] = mi[P];
  o[2 * P] = mi[2 * P];
  o[3 * P] = (x + 0.5f) / W - 0.5f;
  o[4 * P] = (y + 0.5f) / H - 0.5f;
}

// Relative squared error per sample: num/den in FP64 partials, then
// dh = 2 (h - t) / den / B and the batch-mean loss.
__global__ void __launch_bounds__(kFnoBlock) k_fno_loss_partial(const float* h, const float* t,
                                                                long n_per, double* part) {
  __shared__ double rn[kFnoBlock], rd[kFnoBlock];
  const int b = blockIdx.y;
  double sn = 0, sd = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n_per;
       i += (long)gridDim.x * blockDim.x) {
    const double d = (double)h[b * n_per + i] - (double)t[b * n_per + i];
    const double tv = t[b * n_per + i];
    sn += d * d;
    sd += tv * tv;
  }
  rn[threadIdx.x] = sn;
  rd[threadIdx.x] = sd;
  __syncthreads();
  for (int s = kFnoBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      rn[threadIdx.x] += rn[threadIdx.x + s];
      rd[threadIdx.x] += rd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2] = rn[0];
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = rd[0];
  }
}

// Per-sample sums of the partials (one wave per sample, fixed-order tree),
// then the batch-mean loss from one wave.
__global__ void __launch_bounds__(64) k_fno_loss_sample(const double* part, int nblk,
                                                        double* per_sample) {
  const int b = blockIdx.x, k = threadIdx.x;
  double n = 0, d = 0;
  for (int i = k; i < nblk; i += 64) {
    n += part[((size_t)b * nblk + i) * 2];
    d += part[((size_t)b * nblk + i) * 2 + 1];
  }
  for (int s = 32; s > 0; s >>= 1) {
    n += __shfl_xor(n, s);
    d += __shfl_xor(d, s);
  }
  if (k == 0) {
    per_sample[2 * b] = n;
    per_sample[2 * b + 1] = d;
  }
}

__global__ void __launch_bounds__(64) k_fno_loss_mean(const double* per_sample, int B,
                                                      double* loss) {
  const int k = threadIdx.x;
  double L = 0;
  for (int b = k; b < B; b += 64) L += per_sample[2 * b] / per_sample[2 * b + 1];
  for (int s = 32; s > 0; s >>= 1) L += __shfl_xor(L, s);
  if (k == 0) *loss = L / B;
}

__global__ void k_fno_dh(const float* h, const float* t, const double* per_sample, long n_per,
                         int B, float* dh) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * n_per) return;
  const long b = i / n_per;
  dh[i] = (float)(2.0 * ((double)h[i] - (double)t[i]) / per_sample[2 * b + 1] / B);
}

// Adam (Kingma & Ba 2015) on every real parameter component.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace mmx
