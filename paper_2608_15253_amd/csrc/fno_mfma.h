// Matrix-core kernels of the learned demag surrogate (device code): the
// truncated Fourier transforms, the per-mode channel mixing and its gradient,
// and the weight gradients of the 1x1 channel maps.
//
// All are FP32 products with FP32 accumulation on v_mfma_f32_16x16x4_f32
// (a 16 x 16 result tile, a reduction of 4 per instruction), so they keep the
// precision of the VALU kernels they replace.  Operand layout of one
// instruction for lane l = 16 g + r:  A[i = r][k = g] and B[k = g][j = r] in,
// D[i = 4 g + t][j = r] in component t of the accumulator.  A result tile
// whose row index runs over 4 g + t is therefore directly the operand of a
// next product that reduces over those rows (reduction index g, one
// instruction per t): both stages of a transform stay in registers.
//
// LDS tables read with the reduction index g on the row have row strides
// chosen so that the four g groups of a wave land 16 banks apart.
#pragma once
#include "common.h"
#include "fno.h"

namespace mmx {

__device__ inline f32x4 mma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS table fill by a 256-thread workgroup: element i = tid + 256 u, four
// global loads in flight per thread before the stores
template <typename Load, typename Store>
__device__ inline void stage_table(int n, int tid, Load load, Store store) {
  for (int i0 = tid; i0 < n; i0 += 4 * 256) {
    cpx<float> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 256 * u < n) v[u] = load(i0 + 256 * u);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 256 * u < n) store(i0 + 256 * u, v[u]);
  }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of a channel map Y = W X + bias:
//   part[c][m K + k] = sum_p dY[b][m][p] X[b][k][p],  part[c][M K + m] = sum_p dY[b][m][p]
// over the pixels [chunk blockIdx.x, +chunk) of sample b = blockIdx.y, partial
// row c = blockIdx.y gridDim.x + blockIdx.x; blockIdx.z selects a group of
// MT x KT output tiles.  One wave per workgroup.  Lane (g, r) reads four
// consecutive pixels of channel rows r: instruction t reduces pixel 4 g + t of
// each 16-pixel step.  VEC: 16-byte loads (P a multiple of 4).
constexpr int kDwRows = 1024;  // partial rows aimed at (pixel chunks x samples)

template <int MT, int KT, bool VEC>
__global__ void __launch_bounds__(64) k_dw_mfma(const float* __restrict__ dY,
                                                const float* __restrict__ X, int M, int K, int P,
                                                int chunk, int kgroups, float* __restrict__ part) {
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int b = blockIdx.y;
  const int gm = blockIdx.z / kgroups, gk = blockIdx.z - gm * kgroups;
  const int m0 = gm * MT * 16, k0 = gk * KT * 16;
  const int p0 = blockIdx.x * chunk, p1 = min(p0 + chunk, P);
  const float* yrow[MT];
  const float* xrow[KT];
  bool yok[MT], xok[KT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int m = m0 + i * 16 + r;
    yok[i] = m < M;
    yrow[i] = dY + ((size_t)b * M + (yok[i] ? m : 0)) * P;
  }
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    const int k = k0 + i * 16 + r;
    xok[i] = k < K;
    xrow[i] = X + ((size_t)b * K + (xok[i] ? k : 0)) * P;
  }
  f32x4 acc[MT][KT];
  float bsum[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    bsum[i] = 0.f;
#pragma unroll
    for (int j = 0; j < KT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  auto load = [&](const float* row, bool ok, int p) -> f32x4 {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (VEC) {
      if (ok && p < p1) v = *reinterpret_cast<const f32x4*>(row + p);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = (ok && p + t < p1) ? row[p + t] : 0.f;
    }
    return v;
  };
  for (int pb = p0; pb < p1; pb += 16) {
    const int p = pb + 4 * g;
    f32x4 av[MT], bv[KT];
#pragma unroll
    for (int i = 0; i < MT; ++i) av[i] = load(yrow[i], yok[i], p);
#pragma unroll
    for (int j = 0; j < KT; ++j) bv[j] = load(xrow[j], xok[j], p);
#pragma unroll
    for (int i = 0; i < MT; ++i) bsum[i] += (av[i][0] + av[i][1]) + (av[i][2] + av[i][3]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < KT; ++j) acc[i][j] = mma4(av[i][t], bv[j][t], acc[i][j]);
  }
  const int npair = M * K + M;
  float* out = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * npair;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < KT; ++j) {
      const int k = k0 + j * 16 + r;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + i * 16 + 4 * g + t;
        if (m < M && k < K) out[(size_t)m * K + k] = acc[i][j][t];
      }
    }
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    float s = bsum[i];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    const int m = m0 + i * 16 + r;
    if (gk == 0 && g == 0 && m < M) out[(size_t)M * K + m] = s;
  }
}

// out[i] = sum over rows of part[row][i] in a fixed order: 64 columns per
// workgroup, 16 row phases with 8 loads in flight each, the phases summed in
// phase order.
__global__ void __launch_bounds__(1024) k_sum_rows(const float* __restrict__ part, int rows, int n,
                                                   float* __restrict__ out) {
  __shared__ float red[16][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + c;
  float s = 0.f;
  if (i < n) {
    int row = ph;
    for (; row + 7 * 16 < rows; row += 8 * 16) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(row + 16 * u) * n + i];
      s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; row < rows; row += 16) s += part[(size_t)row * n + i];
  }
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && i < n) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][c];
    out[i] = t;
  }
}

// ---------------------------------------------------------------------------
// Truncated forward transform of one (b, channel) plane per workgroup of four
// waves (M1 <= 16 x-modes, J <= 32 y-modes):
//   stage 1  A[y][kx] = sum_x V[y][x] Fx[kx][x]      (Re and Im of A as two
//            16-column tiles; reduction over x in steps of 16)
//   stage 2  Out[kx][j] = s[kx] sum_y A[y][kx] Fy[j][y]  (Out transposed:
//            rows j, columns kx; the stage-1 tiles are the B operand)
// Wave w takes the 16-row y tiles w, w + 4, ...; the four waves' stage-2
// tiles are summed in LDS in wave order.  VEC: 16-byte row loads (W % 4 == 0).
constexpr int kSpecStride = 36;  // row stride of the x- and y-tables (floats)

__host__ __device__ inline int spec_fwd_lds_floats(int H, int W) {
  const int Wp = (W + 15) & ~15, Hp = (H + 15) & ~15;
  const int tables = (Wp + 2 * Hp) * kSpecStride;
  return tables > 4096 ? tables : 4096;  // the reduction reuses the tables
}

template <bool VEC>
__global__ void __launch_bounds__(256) k_spec_fwd_mfma(SpecArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int Wp = (a.W + 15) & ~15, Hp = (a.H + 15) & ~15;
  float* Gx = reinterpret_cast<float*>(smem_raw);  // [Wp][36]: Re Fx[kx][x] at [x][kx], Im at [x][16 + kx]
  float* FyR = Gx + (size_t)Wp * kSpecStride;      // [Hp][36]: Re Fy[j][y] at [y][j], j < 32
  float* FyI = FyR + (size_t)Hp * kSpecStride;
  const int tid = threadIdx.x, plane = blockIdx.x;
  // table fills: four loads in flight per thread before the LDS stores
  stage_table(16 * Wp, tid, [&](int i) {
    const int kx = i / Wp, x = i - kx * Wp;
    return (kx < a.M1 && x < a.W) ? a.Fx[(size_t)kx * a.W + x] : cpx<float>{0.f, 0.f};
  }, [&](int i, cpx<float> f) {
    const int kx = i / Wp, x = i - kx * Wp;
    Gx[x * kSpecStride + kx] = f.re;
    Gx[x * kSpecStride + 16 + kx] = f.im;
  });
  stage_table(32 * Hp, tid, [&](int i) {
    const int j = i / Hp, y = i - j * Hp;
    return (j < a.J && y < a.H) ? a.Fy[(size_t)j * a.H + y] : cpx<float>{0.f, 0.f};
  }, [&](int i, cpx<float> f) {
    const int j = i / Hp, y = i - j * Hp;
    FyR[y * kSpecStride + j] = f.re;
    FyI[y * kSpecStride + j] = f.im;
  });
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
  const float* V = a.in + (size_t)plane * a.H * a.W;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 oR0 = z4, oI0 = z4, oR1 = z4, oI1 = z4;  // stage 2, j tiles 0 and 1
  for (int ty = w; ty < Hp / 16; ty += 4) {
    const int y = ty * 16 + r;
    const bool yin = y < a.H;
    const float* row = V + (size_t)(yin ? y : 0) * a.W;
    f32x4 cR = z4, cI = z4;  // stage 1: Re and Im of A[y][kx]
    for (int xb0 = 0; xb0 < Wp; xb0 += 128) {
      // the row's next 128 x values: all loads issued before the products
      f32x4 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int x = xb0 + 16 * q + 4 * g;
        v[q] = z4;
        if (VEC) {
          if (yin && x < a.W) v[q] = *reinterpret_cast<const f32x4*>(row + x);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) v[q][t] = (yin && x + t < a.W) ? row[x + t] : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (xb0 + 16 * q >= Wp) break;  // uniform
        const float* gx = Gx + (size_t)(xb0 + 16 * q + 4 * g) * kSpecStride + r;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          cR = mma4(v[q][t], gx[t * kSpecStride], cR);
          cI = mma4(v[q][t], gx[t * kSpecStride + 16], cI);
        }
      }
    }
    // cR[t], cI[t] hold A[y = 16 ty + 4 g + t][kx = r]: reduction index g
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int yy = ty * 16 + 4 * g + t;
      const float r0 = FyR[yy * kSpecStride + r], r1 = FyR[yy * kSpecStride + 16 + r];
      const float i0 = FyI[yy * kSpecStride + r], i1 = FyI[yy * kSpecStride + 16 + r];
      oR0 = mma4(r0, cR[t], oR0);
      oR0 = mma4(-i0, cI[t], oR0);
      oI0 = mma4(i0, cR[t], oI0);
      oI0 = mma4(r0, cI[t], oI0);
      oR1 = mma4(r1, cR[t], oR1);
      oR1 = mma4(-i1, cI[t], oR1);
      oI1 = mma4(i1, cR[t], oI1);
      oI1 = mma4(r1, cI[t], oI1);
    }
  }
  __syncthreads();  // tables no longer read: reuse them for the reduction
  f32x4* red = reinterpret_cast<f32x4*>(smem_raw);  // [wave][tile][lane]
  red[(w * 4 + 0) * 64 + lane] = oR0;
  red[(w * 4 + 1) * 64 + lane] = oI0;
  red[(w * 4 + 2) * 64 + lane] = oR1;
  red[(w * 4 + 3) * 64 + lane] = oI1;
  __syncthreads();
  // wave w finishes tile w: j tile w / 2, real (even w) or imaginary part
  const f32x4 s = ((red[(0 * 4 + w) * 64 + lane] + red[(1 * 4 + w) * 64 + lane]) +
                   red[(2 * 4 + w) * 64 + lane]) + red[(3 * 4 + w) * 64 + lane];
  const int kx = r, jt = w >> 1, part = w & 1;
  if (kx < a.M1) {
    const float sc = a.coef ? a.coef[kx] : 1.f;
    float* out = a.out + 2 * ((size_t)plane * a.M1 + kx) * a.J;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = jt * 16 + 4 * g + t;
      if (j < a.J) out[2 * j + part] = sc * s[t];
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse of the truncated modes of one (b, channel) plane per workgroup of
// four waves (M1 <= 16, J <= 32):
//   stage 1  D[kx][y] = c[kx] sum_j Uh[kx][j] conj(Fy[j][y])   (Re and Im
//            tiles, rows kx, columns y; reduction over j)
//   stage 2  U[y][x] = sum_kx Re(D[kx][y] conj(Fx[kx][x]))      (the stage-1
//            tiles are the A operand: reduction over kx = 4 g + t)
// then out = U + add (add may alias out) and act = gelu(out).  The plane's
// y tiles are dealt to the waves of gridDim.y workgroups (wave w of
// workgroup s: tiles 4 s + w, + 4 gridDim.y, ...), each with all x tiles.
__host__ __device__ inline int spec_inv_lds_floats(int H, int W, int J) {
  const int Wp = (W + 15) & ~15, Hp = (H + 15) & ~15, Jp = (J + 3) & ~3;
  const int SY = ((Hp + 63) & ~63) + 16, SX = Wp + 4;
  return 2 * Jp * 16 + 2 * Jp * SY + 2 * 16 * SX;
}

__global__ void __launch_bounds__(256) k_spec_inv_mfma(SpecArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int Wp = (a.W + 15) & ~15, Hp = (a.H + 15) & ~15, Jp = (a.J + 3) & ~3;
  const int SY = ((Hp + 63) & ~63) + 16, SX = Wp + 4;
  float* UR = reinterpret_cast<float*>(smem_raw);  // [Jp][16]: c[kx] Re Uh[kx][j] at [j][kx]
  float* UI = UR + Jp * 16;
  float* FR = UI + Jp * 16;                        // [Jp][SY]: Re Fy[j][y]
  float* FI = FR + (size_t)Jp * SY;
  float* XR = FI + (size_t)Jp * SY;                // [16][SX]: Re Fx[kx][x]
  float* XI = XR + 16 * SX;
  const int tid = threadIdx.x, plane = blockIdx.x;
  const cpx<float>* Uh = reinterpret_cast<const cpx<float>*>(a.in) + (size_t)plane * a.M1 * a.J;
  stage_table(16 * Jp, tid, [&](int i) {
    const int kx = i / Jp, j = i - kx * Jp;
    if (kx >= a.M1 || j >= a.J) return cpx<float>{0.f, 0.f};
    const float c = a.coef ? a.coef[kx] : 1.f;
    const cpx<float> u = Uh[(size_t)kx * a.J + j];
    return cpx<float>{c * u.re, c * u.im};
  }, [&](int i, cpx<float> u) {
    const int kx = i / Jp, j = i - kx * Jp;
    UR[j * 16 + kx] = u.re;
    UI[j * 16 + kx] = u.im;
  });
  stage_table(Jp * Hp, tid, [&](int i) {
    const int j = i / Hp, y = i - j * Hp;
    return (j < a.J && y < a.H) ? a.Fy[(size_t)j * a.H + y] : cpx<float>{0.f, 0.f};
  }, [&](int i, cpx<float> f) {
    const int j = i / Hp, y = i - j * Hp;
    FR[j * SY + y] = f.re;
    FI[j * SY + y] = f.im;
  });
  stage_table(16 * Wp, tid, [&](int i) {
    const int kx = i / Wp, x = i - kx * Wp;
    return (kx < a.M1 && x < a.W) ? a.Fx[(size_t)kx * a.W + x] : cpx<float>{0.f, 0.f};
  }, [&](int i, cpx<float> f) {
    const int kx = i / Wp, x = i - kx * Wp;
    XR[kx * SX + x] = f.re;
    XI[kx * SX + x] = f.im;
  });
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
  const size_t base = (size_t)plane * a.H * a.W;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  const int ntx = Wp / 16, nsplit = gridDim.y;
  for (int ty = 4 * blockIdx.y + w; ty < Hp / 16; ty += 4 * nsplit) {
    // added field of 8 x tiles of these rows, fetched ahead of the products
    float av[8][4];
    auto fetch = [&](int tx0) {
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int y = ty * 16 + 4 * g + t, x = (tx0 + q) * 16 + r;
          av[q][t] = (a.add && y < a.H && x < a.W) ? a.add[base + (size_t)y * a.W + x] : 0.f;
        }
    };
    fetch(0);
    f32x4 dR = z4, dI = z4;
    for (int jb = 0; jb < Jp; jb += 4) {
      const int j = jb + g;
      const float ur = UR[j * 16 + r], ui = UI[j * 16 + r];
      const float fr = FR[j * SY + ty * 16 + r], fi = FI[j * SY + ty * 16 + r];
      dR = mma4(ur, fr, dR);   // Re(u conj f) = ur fr + ui fi
      dR = mma4(ui, fi, dR);
      dI = mma4(ui, fr, dI);   // Im(u conj f) = ui fr - ur fi
      dI = mma4(-ur, fi, dI);
    }
    // dR[t], dI[t] hold D[kx = 4 g + t][y = 16 ty + r]
    for (int tx0 = 0; tx0 < ntx; tx0 += 8) {
      if (tx0) fetch(tx0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int tx = tx0 + q;
        if (tx >= ntx) break;  // uniform
        f32x4 o = z4;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int k = 4 * g + t;
          o = mma4(dR[t], XR[k * SX + tx * 16 + r], o);
          o = mma4(dI[t], XI[k * SX + tx * 16 + r], o);
        }
        const int x = tx * 16 + r;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int y = ty * 16 + 4 * g + t;
          if (y < a.H && x < a.W) {
            const size_t i = base + (size_t)y * a.W + x;
            const float v = o[t] + av[q][t];
            a.out[i] = v;
            if (a.act) a.act[i] = gelu_f(v);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-mode complex channel mixing, one (mode, batch tile, channel tile) per
// wave.  Forward out[b][o] = sum_i in[b][i] R[i][o]; adjoint
// out[b][i] = sum_o in[b][o] conj(R[i][o]).  Rows b, columns the output
// channel, reduction over the input channel; each complex product is four
// real ones.  Modes are (kx, j), J fastest; in/out are [b][channel][mode].
__global__ void __launch_bounds__(256) k_mix_mfma(const cpx<float>* __restrict__ in,
                                                  const cpx<float>* __restrict__ R,
                                                  cpx<float>* __restrict__ out, int B, int C,
                                                  int nmode, int adjoint) {
  const int Bt = (B + 15) >> 4, Ct = (C + 15) >> 4, Cq = (C + 3) & ~3;
  const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= (long)nmode * Bt * Ct) return;  // whole waves
  const int mode = (int)(wid / (Bt * Ct));
  const int rem = (int)(wid - (long)mode * Bt * Ct), bt = rem / Ct, ot = rem - bt * Ct;
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const cpx<float>* Rm = R + (size_t)mode * C * C;
  const int b = bt * 16 + r, o = ot * 16 + r;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 re = z4, im = z4;
  for (int kb = 0; kb < Cq; kb += 4) {
    const int k = kb + g;
    cpx<float> v = {0.f, 0.f}, q = {0.f, 0.f};
    if (b < B && k < C) v = in[((size_t)b * C + k) * nmode + mode];
    if (o < C && k < C) q = adjoint ? Rm[(size_t)o * C + k] : Rm[(size_t)k * C + o];
    if (!adjoint) {  // v q
      re = mma4(v.re, q.re, re);
      re = mma4(-v.im, q.im, re);
      im = mma4(v.re, q.im, im);
      im = mma4(v.im, q.re, im);
    } else {  // v conj(q)
      re = mma4(v.re, q.re, re);
      re = mma4(v.im, q.im, re);
      im = mma4(v.im, q.re, im);
      im = mma4(-v.re, q.im, im);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int bb = bt * 16 + 4 * g + t;
    if (bb < B && o < C) out[((size_t)bb * C + o) * nmode + mode] = {re[t], im[t]};
  }
}

// dR[mode][i][o] = sum_b conj(Vh[b][i][mode]) dUh[b][o][mode], one (mode,
// i tile, o tile) per wave; reduction over the batch.
__global__ void __launch_bounds__(256) k_mix_grad_mfma(const cpx<float>* __restrict__ Vh,
                                                       const cpx<float>* __restrict__ dUh,
                                                       cpx<float>* __restrict__ dR, int B, int C,
                                                       int nmode) {
  const int Ct = (C + 15) >> 4, Bq = (B + 3) & ~3;
  const long wid = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= (long)nmode * Ct * Ct) return;  // whole waves
  const int mode = (int)(wid / (Ct * Ct));
  const int rem = (int)(wid - (long)mode * Ct * Ct), it = rem / Ct, ot = rem - it * Ct;
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const int i = it * 16 + r, o = ot * 16 + r;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 re = z4, im = z4;
  for (int kb = 0; kb < Bq; kb += 4) {
    const int b = kb + g;
    cpx<float> v = {0.f, 0.f}, d = {0.f, 0.f};
    if (b < B && i < C) v = Vh[((size_t)b * C + i) * nmode + mode];
    if (b < B && o < C) d = dUh[((size_t)b * C + o) * nmode + mode];
    re = mma4(v.re, d.re, re);  // conj(v) d
    re = mma4(v.im, d.im, re);
    im = mma4(v.re, d.im, im);
    im = mma4(-v.im, d.re, im);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ii = it * 16 + 4 * g + t;
    if (ii < C && o < C) dR[((size_t)mode * C + ii) * C + o] = {re[t], im[t]};
  }
}

}  // namespace mmx
