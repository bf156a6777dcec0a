// Learned demag surrogate: Fourier neural operator forward, backward and Adam
// kernels (device code).
//
// Activations are FP32, [b][channel][pixel] with x fastest.  The pointwise
// (1x1) channel maps are GEMMs over channels for every pixel and run on the
// matrix cores: v_mfma_f32_16x16x32_bf16 with BF16 operands staged in LDS and
// FP32 accumulation (a VALU FP32 variant of the same kernel serves parity
// checks).  The truncated Fourier transforms (M1 x-modes, 2 M2 y-modes), the
// per-mode complex channel mixing and all reductions are FP32 on the VALU.
#pragma once
#include "common.h"

namespace mmx {

constexpr int kFnoBlock = 256;
constexpr int kFnoPixTile = 64;  // pixels per GEMM workgroup (16 per wave)

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
// Workgroup: sample blockIdx.y, pixels [64 blockIdx.x, +64); wave w owns 16
// pixels and every 16-row tile of the output channels.
template <bool MFMA>
__global__ void __launch_bounds__(kFnoBlock) k_conv1x1(ConvArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int b = blockIdx.y, p0 = blockIdx.x * kFnoPixTile;
  const int Mp = (a.M + 15) & ~15, Kp = (a.K + 31) & ~31;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* Xb = a.X + (size_t)b * a.K * a.P;
  if (MFMA) {
    __bf16* Ws = reinterpret_cast<__bf16*>(smem_raw);   // [Mp][Kp]
    __bf16* Xs = Ws + (size_t)Mp * Kp;                  // [Kp][64]
    for (int i = threadIdx.x; i < Mp * Kp; i += blockDim.x) {
      const int m = i / Kp, k = i - m * Kp;
      float v = 0.f;
      if (m < a.M && k < a.K) v = a.trans ? a.Wt[(size_t)k * a.M + m] : a.Wt[(size_t)m * a.K + k];
      Ws[i] = (__bf16)v;
    }
    for (int i = threadIdx.x; i < Kp * kFnoPixTile; i += blockDim.x) {
      const int k = i / kFnoPixTile, px = i - k * kFnoPixTile;
      float v = 0.f;
      if (k < a.K && p0 + px < a.P) v = Xb[(size_t)k * a.P + p0 + px];
      Xs[i] = (__bf16)v;
    }
    __syncthreads();
    const int col = lane & 15, grp = lane >> 4;
    for (int mt = 0; mt < Mp / 16; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kt = 0; kt < Kp / 32; ++kt) {
        bf16x8 av, bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = kt * 32 + 8 * grp + j;
          av[j] = Ws[(size_t)(mt * 16 + col) * Kp + k];
          bv[j] = Xs[(size_t)k * kFnoPixTile + wave * 16 + col];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = mt * 16 + 4 * grp + j;
        const int p = p0 + wave * 16 + col;
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

// Partial weight gradients of a channel map: for pixel chunk blockIdx.x,
// part[chunk][m][k] = sum dY[b][m][p] X[b][k][p], part[chunk][M][... ] bias
// row: part[chunk][M*K + m] = sum dY[b][m][p].  Chunks span 1024 pixels of the
// flattened (b, p) range.
constexpr int kDwChunk = 1024;
constexpr int kDwTile = 32;

__global__ void __launch_bounds__(kFnoBlock) k_dw_partial(const float* dY, const float* X, int M,
                                                          int K, int P, int B, float* part) {
  extern __shared__ unsigned char smem_raw[];
  float* Ys = reinterpret_cast<float*>(smem_raw);   // [M][tile]
  float* Xs = Ys + (size_t)M * kDwTile;              // [K][tile]
  const long total = (long)B * P;
  const long q0 = (long)blockIdx.x * kDwChunk;
  const int npair = M * K + M;
  float acc[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = 0.f;
  for (long t0 = q0; t0 < q0 + kDwChunk && t0 < total; t0 += kDwTile) {
    __syncthreads();
    for (int i = threadIdx.x; i < (M + K) * kDwTile; i += blockDim.x) {
      const int row = i / kDwTile, px = i - row * kDwTile;
      const long q = t0 + px;
      float v = 0.f;
      if (q < total) {
        const long b = q / P, p = q - b * P;
        v = (row < M) ? dY[((size_t)b * M + row) * P + p] : X[((size_t)b * K + row - M) * P + p];
      }
      Ys[i] = v;  // rows >= M land in Xs (contiguous)
    }
    __syncthreads();
    int slot = 0;
    for (int pr = threadIdx.x; pr < npair; pr += blockDim.x, ++slot) {
      float s = 0.f;
      if (pr < M * K) {
        const int m = pr / K, k = pr - m * K;
        for (int px = 0; px < kDwTile; ++px) s += Ys[m * kDwTile + px] * Xs[k * kDwTile + px];
      } else {
        const int m = pr - M * K;
        for (int px = 0; px < kDwTile; ++px) s += Ys[m * kDwTile + px];
      }
      acc[slot] += s;
    }
  }
  int slot = 0;
  for (int pr = threadIdx.x; pr < npair; pr += blockDim.x, ++slot)
    part[(size_t)blockIdx.x * npair + pr] = acc[slot];
}

// out[i] (+)= sum over chunks of part[chunk][i], fixed order
__global__ void k_sum_chunks(const float* part, int nchunk, int n, float* out, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * n + i];
  out[i] = accumulate ? out[i] + s : s;
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

// Per-mode complex channel mixing.  Forward: out[b][o][mode] =
// sum_i R[mode][i][o] in[b][i][mode]; adjoint: out[b][i][mode] =
// sum_o conj(R[mode][i][o]) in[b][o][mode].  Modes are (kx, j), J fastest.
__global__ void __launch_bounds__(kFnoBlock) k_mix(const cpx<float>* in, const cpx<float>* R,
                                                   cpx<float>* out, int B, int C, int nmode,
                                                   int adjoint) {
  extern __shared__ unsigned char smem_raw[];
  cpx<float>* Rs = reinterpret_cast<cpx<float>*>(smem_raw);  // [C][C]
  cpx<float>* Vs = Rs + C * C;                               // [B][C]
  const int mode = blockIdx.x;
  for (int i = threadIdx.x; i < C * C; i += blockDim.x) Rs[i] = R[(size_t)mode * C * C + i];
  for (int i = threadIdx.x; i < B * C; i += blockDim.x) Vs[i] = in[(size_t)i * nmode + mode];
  __syncthreads();
  for (int i = threadIdx.x; i < B * C; i += blockDim.x) {
    const int b = i / C, q = i - b * C;
    float re = 0.f, im = 0.f;
    for (int s = 0; s < C; ++s) {
      const cpx<float> v = Vs[b * C + s];
      if (!adjoint) {
        const cpx<float> r = Rs[s * C + q];           // R[i = s][o = q]
        re += r.re * v.re - r.im * v.im;
        im += r.re * v.im + r.im * v.re;
      } else {
        const cpx<float> r = Rs[q * C + s];           // conj(R[i = q][o = s])
        re += r.re * v.re + r.im * v.im;
        im += r.re * v.im - r.im * v.re;
      }
    }
    out[(size_t)i * nmode + mode] = {re, im};
  }
}

// dR[mode][i][o] = sum_b conj(Vh[b][i][mode]) dUh[b][o][mode]
__global__ void __launch_bounds__(kFnoBlock) k_mix_grad(const cpx<float>* Vh, const cpx<float>* dUh,
                                                        cpx<float>* dR, int B, int C, int nmode) {
  const int mode = blockIdx.x;
  for (int i = threadIdx.x; i < C * C; i += blockDim.x) {
    const int ci = i / C, co = i - ci * C;
    float re = 0.f, im = 0.f;
    for (int b = 0; b < B; ++b) {
      const cpx<float> v = Vh[((size_t)b * C + ci) * nmode + mode];
      const cpx<float> d = dUh[((size_t)b * C + co) * nmode + mode];
      re += v.re * d.re + v.im * d.im;
      im += v.re * d.im - v.im * d.re;
    }
    dR[(size_t)mode * C * C + i] = {re, im};
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

__global__ void k_fno_loss_final(const double* part, int nblk, int B, double* per_sample,
                                 double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double L = 0;
  for (int b = 0; b < B; ++b) {
    double n = 0, d = 0;
    for (int k = 0; k < nblk; ++k) {
      n += part[((size_t)b * nblk + k) * 2];
      d += part[((size_t)b * nblk + k) * 2 + 1];
    }
    per_sample[2 * b] = n;
    per_sample[2 * b + 1] = d;
    L += n / d;
  }
  *loss = L / B;
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
