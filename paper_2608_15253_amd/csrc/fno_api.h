// Host side of the learned demag surrogate: buffers, forward, backward, Adam,
// parameter layout (see include/mmx.h).  Included by mmx.hip.
#pragma once
#include "fno.h"
#include "fno_mfma.h"

struct mmx_fno {
  int H = 0, W = 0, C = 0, M1 = 0, M2 = 0, J = 0, L = 0, Cp = 0, Bmax = 0, mfma = 1;
  long P = 0;
  hipStream_t stream = nullptr;
  // parameter offsets (floats)
  long oP = 0, op = 0, oQ1 = 0, oq1 = 0, oQ2 = 0, oq2 = 0, nparam = 0;
  std::vector<long> oR, oW, ob;
  // tables and activations
  DevBuf Fx, Fy, cinv, cone, X0, Y1, A1, dh, dA, dV, dV2, dZ, Uh, dUh, dVh, part, lpart, lsum,
      loss;
  std::vector<DevBuf> V, Z, Vh;
  int batch = 0;  // batch of the cached forward
};

namespace {

using namespace mmx;

mmx_status fno_conv(mmx_fno* f, const float* X, const float* Wt, const float* bias, float* Y,
                    float* A, const float* S, int M, int K, int trans, int epi, int B) {
  ConvArgs a{X, Wt, bias, Y, A, S, M, K, (int)f->P, trans, epi};
  if (f->mfma) {
    const dim3 grid((unsigned)((f->P + kConvPixMfma - 1) / kConvPixMfma), B);
    const int Mp = (M + 15) & ~15, KS = ((K + 31) & ~31) + 8;
    const size_t lds = ((size_t)Mp * KS + (size_t)kConvPixMfma * KS) * sizeof(__bf16);
    k_conv1x1<true><<<grid, kFnoBlock, lds, f->stream>>>(a);
  } else {
    const dim3 grid((unsigned)((f->P + kFnoPixTile - 1) / kFnoPixTile), B);
    const size_t lds = ((size_t)M * K + (size_t)K * kFnoPixTile) * sizeof(float);
    k_conv1x1<false><<<grid, kFnoBlock, lds, f->stream>>>(a);
  }
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

template <int MT, int KT>
void launch_dw(dim3 grid, hipStream_t st, bool vec, const float* dY, const float* X, int M, int K,
               int P, int chunk, int kgroups, float* part) {
  if (vec)
    k_dw_mfma<MT, KT, true><<<grid, 64, 0, st>>>(dY, X, M, K, P, chunk, kgroups, part);
  else
    k_dw_mfma<MT, KT, false><<<grid, 64, 0, st>>>(dY, X, M, K, P, chunk, kgroups, part);
}

// pixel chunk of the weight-gradient partials: about kDwRows partial rows
// (chunks x samples) per map, at least 64 pixels, a multiple of 16
long dw_chunk(long P, int B) {
  const long chunk = ((long)B * P + kDwRows - 1) / kDwRows;
  return std::max(64L, (chunk + 15) / 16 * 16);
}

long dw_rows(long P, int B) { return (P + dw_chunk(P, B) - 1) / dw_chunk(P, B) * B; }

// grads[0 .. M K + M) = weight and bias gradients of a channel map: partial
// sums per pixel chunk on the matrix cores, then a fixed-order sum of the
// chunks.  The partial buffer is sized at creation for every batch up to the
// maximum, so the backward pass allocates nothing.
mmx_status fno_dw(mmx_fno* f, const float* dY, const float* X, int M, int K, int B, float* out) {
  const int npair = M * K + M;
  const long P = f->P;
  const long chunk = dw_chunk(P, B);
  const int nch = (int)((P + chunk - 1) / chunk);
  const int rows = nch * B;
  if (f->part.bytes < (size_t)rows * npair * sizeof(float))
    return fail(MMX_ESTATE, "weight-gradient partial buffer too small");
  // output tiles in groups of at most 4 x 4
  auto group = [](int tiles) { return tiles >= 3 ? 4 : tiles; };
  const int mt = (M + 15) / 16, kt = (K + 15) / 16, MT = group(mt), KT = group(kt);
  const int gm = (mt + MT - 1) / MT, gk = (kt + KT - 1) / KT;
  const dim3 grid((unsigned)nch, (unsigned)B, (unsigned)(gm * gk));
  const bool vec = P % 4 == 0;
  float* part = f->part.as<float>();
  const int c = (int)chunk;
  switch (MT * 8 + KT) {
    case 1 * 8 + 1: launch_dw<1, 1>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 1 * 8 + 2: launch_dw<1, 2>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 1 * 8 + 4: launch_dw<1, 4>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 2 * 8 + 1: launch_dw<2, 1>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 2 * 8 + 2: launch_dw<2, 2>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 2 * 8 + 4: launch_dw<2, 4>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 4 * 8 + 1: launch_dw<4, 1>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    case 4 * 8 + 2: launch_dw<4, 2>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
    default: launch_dw<4, 4>(grid, f->stream, vec, dY, X, M, K, (int)P, c, gk, part); break;
  }
  HIP_TRY(hipGetLastError());
  k_sum_rows<<<(npair + 63) / 64, 1024, 0, f->stream>>>(part, rows, npair, out);
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

// the matrix-core transforms take up to 16 x-modes and 32 y-modes
bool spec_mfma_fits(const mmx_fno* f, size_t lds_bytes) {
  return f->M1 <= 16 && f->J <= 32 && lds_bytes <= 65536;
}

mmx_status fno_spec_fwd(mmx_fno* f, const float* in, float* out, const float* coef, int planes) {
  SpecArgs a{in, out, f->Fx.as<cpx<float>>(), f->Fy.as<cpx<float>>(), coef, nullptr, nullptr,
             f->H, f->W, f->M1, f->J};
  const size_t mlds = (size_t)spec_fwd_lds_floats(f->H, f->W) * sizeof(float);
  if (spec_mfma_fits(f, mlds)) {
    if (f->W % 4 == 0)
      k_spec_fwd_mfma<true><<<planes, kFnoBlock, mlds, f->stream>>>(a);
    else
      k_spec_fwd_mfma<false><<<planes, kFnoBlock, mlds, f->stream>>>(a);
  } else {
    const size_t lds = ((size_t)f->M1 * f->W + (size_t)f->J * f->H + (size_t)f->H * f->M1) *
                       sizeof(cpx<float>);
    k_spec_fwd<<<planes, kFnoBlock, lds, f->stream>>>(a);
  }
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

mmx_status fno_spec_inv(mmx_fno* f, const float* in, float* out, const float* coef,
                        const float* add, float* act, int planes) {
  SpecArgs a{in, out, f->Fx.as<cpx<float>>(), f->Fy.as<cpx<float>>(), coef, add, act,
             f->H, f->W, f->M1, f->J};
  const size_t mlds = (size_t)spec_inv_lds_floats(f->H, f->W, f->J) * sizeof(float);
  if (spec_mfma_fits(f, mlds)) {
    // two workgroups per plane once each wave still has a y tile
    const int split = ((f->H + 15) / 16 >= 8) ? 2 : 1;
    k_spec_inv_mfma<<<dim3(planes, split), kFnoBlock, mlds, f->stream>>>(a);
  } else {
    const size_t lds = ((size_t)f->M1 * f->W + (size_t)f->J * f->H + (size_t)f->M1 * f->H +
                        (size_t)f->M1 * f->J) * sizeof(cpx<float>);
    k_spec_inv<<<planes, kFnoBlock, lds, f->stream>>>(a);
  }
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

mmx_status fno_mix(mmx_fno* f, const float* in, const float* R, float* out, int B, int adjoint) {
  const int nmode = f->M1 * f->J, ct = (f->C + 15) / 16, bt = (B + 15) / 16;
  const long waves = (long)nmode * bt * ct;
  k_mix_mfma<<<(unsigned)((waves + 3) / 4), kFnoBlock, 0, f->stream>>>(
      reinterpret_cast<const cpx<float>*>(in), reinterpret_cast<const cpx<float>*>(R),
      reinterpret_cast<cpx<float>*>(out), B, f->C, nmode, adjoint);
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

__global__ void k_mul_gelu_grad(const float* d, const float* z, float* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = d[i] * gelu_grad_f(z[i]);
}

mmx_status fno_forward_impl(mmx_fno* f, const float* prm, const float* m, float* h, int B) {
  const long nC = (long)B * f->C * f->P;
  (void)nC;
  k_fno_features<<<(unsigned)((B * f->P + 255) / 256), 256, 0, f->stream>>>(m, f->X0.as<float>(),
                                                                           B, f->H, f->W);
  HIP_TRY(hipGetLastError());
  MMX_TRY(fno_conv(f, f->X0.as<float>(), prm + f->oP, prm + f->op, f->V[0].as<float>(), nullptr,
                   nullptr, f->C, 5, 0, CE_STORE, B));
  for (int l = 0; l < f->L; ++l) {
    const float* Vl = f->V[l].as<float>();
    MMX_TRY(fno_spec_fwd(f, Vl, f->Vh[l].as<float>(), nullptr, B * f->C));
    MMX_TRY(fno_mix(f, f->Vh[l].as<float>(), prm + f->oR[l], f->Uh.as<float>(), B, 0));
    float* Zl = f->Z[l].as<float>();
    MMX_TRY(fno_conv(f, Vl, prm + f->oW[l], prm + f->ob[l], Zl, nullptr, nullptr, f->C, f->C, 0,
                     CE_STORE, B));
    float* act = (l < f->L - 1) ? f->V[l + 1].as<float>() : nullptr;
    MMX_TRY(fno_spec_inv(f, f->Uh.as<float>(), Zl, f->cinv.as<float>(), Zl, act, B * f->C));
  }
  const float* VL = f->Z[f->L - 1].as<float>();
  MMX_TRY(fno_conv(f, VL, prm + f->oQ1, prm + f->oq1, f->Y1.as<float>(), f->A1.as<float>(),
                   nullptr, f->Cp, f->C, 0, CE_GELU, B));
  MMX_TRY(fno_conv(f, f->A1.as<float>(), prm + f->oQ2, prm + f->oq2, h, nullptr, nullptr, 3,
                   f->Cp, 0, CE_STORE, B));
  f->batch = B;
  return MMX_OK;
}

mmx_status fno_backward_impl(mmx_fno* f, const float* prm, const float* h, const float* t,
                             float* g, double* loss_host) {
  const int B = f->batch;
  const long n_per = 3 * f->P;
  const int nblk = 64;
  k_fno_loss_partial<<<dim3(nblk, B), kFnoBlock, 0, f->stream>>>(h, t, n_per,
                                                                 f->lpart.as<double>());
  HIP_TRY(hipGetLastError());
  k_fno_loss_sample<<<B, 64, 0, f->stream>>>(f->lpart.as<double>(), nblk, f->lsum.as<double>());
  HIP_TRY(hipGetLastError());
  k_fno_loss_mean<<<1, 64, 0, f->stream>>>(f->lsum.as<double>(), B, f->loss.as<double>());
  HIP_TRY(hipGetLastError());
  k_fno_dh<<<(unsigned)((B * n_per + 255) / 256), 256, 0, f->stream>>>(
      h, t, f->lsum.as<double>(), n_per, B, f->dh.as<float>());
  HIP_TRY(hipGetLastError());
  // projection
  MMX_TRY(fno_dw(f, f->dh.as<float>(), f->A1.as<float>(), 3, f->Cp, B, g + f->oQ2));
  MMX_TRY(fno_conv(f, f->dh.as<float>(), prm + f->oQ2, nullptr, f->dA.as<float>(), nullptr,
                   f->Y1.as<float>(), f->Cp, 3, 1, CE_GELU_GRAD, B));
  const float* VL = f->Z[f->L - 1].as<float>();
  MMX_TRY(fno_dw(f, f->dA.as<float>(), VL, f->Cp, f->C, B, g + f->oQ1));
  float* dV = f->dV.as<float>();
  float* dV2 = f->dV2.as<float>();
  MMX_TRY(fno_conv(f, f->dA.as<float>(), prm + f->oQ1, nullptr, dV, nullptr, nullptr, f->C,
                   f->Cp, 1, CE_STORE, B));
  const long nC = (long)B * f->C * f->P;
  for (int l = f->L - 1; l >= 0; --l) {
    const float* dZ = dV;
    if (l < f->L - 1) {
      k_mul_gelu_grad<<<(unsigned)((nC + 255) / 256), 256, 0, f->stream>>>(
          dV, f->Z[l].as<float>(), f->dZ.as<float>(), nC);
      HIP_TRY(hipGetLastError());
      dZ = f->dZ.as<float>();
    }
    const float* Vl = f->V[l].as<float>();
    MMX_TRY(fno_dw(f, dZ, Vl, f->C, f->C, B, g + f->oW[l]));
    MMX_TRY(fno_conv(f, dZ, prm + f->oW[l], nullptr, dV2, nullptr, nullptr, f->C, f->C, 1,
                     CE_STORE, B));
    MMX_TRY(fno_spec_fwd(f, dZ, f->dUh.as<float>(), f->cinv.as<float>(), B * f->C));
    const int nmode = f->M1 * f->J, ct = (f->C + 15) / 16;
    k_mix_grad_mfma<<<(unsigned)(((long)nmode * ct * ct + 3) / 4), kFnoBlock, 0, f->stream>>>(
        reinterpret_cast<const cpx<float>*>(f->Vh[l].as<float>()),
        reinterpret_cast<const cpx<float>*>(f->dUh.as<float>()),
        reinterpret_cast<cpx<float>*>(g + f->oR[l]), B, f->C, nmode);
    HIP_TRY(hipGetLastError());
    MMX_TRY(fno_mix(f, f->dUh.as<float>(), prm + f->oR[l], f->dVh.as<float>(), B, 1));
    MMX_TRY(fno_spec_inv(f, f->dVh.as<float>(), dV2, f->cone.as<float>(), dV2, nullptr, B * f->C));
    std::swap(dV, dV2);
  }
  MMX_TRY(fno_dw(f, dV, f->X0.as<float>(), f->C, 5, B, g + f->oP));
  if (loss_host) {
    HIP_TRY(hipMemcpyAsync(loss_host, f->loss.p, sizeof(double), hipMemcpyDeviceToHost, f->stream));
    HIP_TRY(hipStreamSynchronize(f->stream));
  }
  return MMX_OK;
}

// deterministic normals for the initial weights (SplitMix64 + Box-Muller)
struct InitRng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u = uniform(), v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(2.0 * kPi * v);
  }
};

}  // namespace

extern "C" {

mmx_status mmx_fno_create(int32_t H, int32_t W, int32_t C, int32_t M1, int32_t M2, int32_t L,
                          int32_t Cp, int32_t batch_max, int32_t use_mfma, mmx_fno** out) {
  if (!out) return fail(MMX_EINVAL, "out is null");
  *out = nullptr;
  if (H < 2 || W < 2 || C < 1 || L < 1 || Cp < 1 || batch_max < 1 || M1 < 1 || M2 < 1)
    return fail(MMX_EINVAL, "FNO sizes must be positive");
  if (2 * M1 >= W || 2 * M2 > H) return fail(MMX_EINVAL, "too many modes for the grid");
  if (C > 128 || Cp > 128 || batch_max > 64)
    return fail(MMX_EUNSUP, "FNO width, projection width <= 128 and batch <= 64 supported");
  auto f = std::make_unique<mmx_fno>();
  f->H = H; f->W = W; f->C = C; f->M1 = M1; f->M2 = M2; f->J = 2 * M2; f->L = L; f->Cp = Cp;
  f->Bmax = batch_max; f->mfma = use_mfma ? 1 : 0;
  f->P = (long)H * W;
  long o = 0;
  f->oP = o; o += (long)C * 5;
  f->op = o; o += C;
  for (int l = 0; l < L; ++l) {
    f->oR.push_back(o); o += (long)M1 * f->J * C * C * 2;
    f->oW.push_back(o); o += (long)C * C;
    f->ob.push_back(o); o += C;
  }
  f->oQ1 = o; o += (long)Cp * C;
  f->oq1 = o; o += Cp;
  f->oQ2 = o; o += 3L * Cp;
  f->oq2 = o; o += 3;
  f->nparam = o;
  // DFT tables in FP64 rounded to FP32
  std::vector<cpx<float>> fx((size_t)M1 * W), fy((size_t)f->J * H);
  for (int k = 0; k < M1; ++k)
    for (int x = 0; x < W; ++x) {
      const double a = -2.0 * kPi * (double)((long)k * x % W) / W;
      fx[(size_t)k * W + x] = {(float)std::cos(a), (float)std::sin(a)};
    }
  for (int j = 0; j < f->J; ++j) {
    const long ky = j < M2 ? j : H - f->J + j;
    for (int y = 0; y < H; ++y) {
      const double a = -2.0 * kPi * (double)(ky * y % H) / H;
      fy[(size_t)j * H + y] = {(float)std::cos(a), (float)std::sin(a)};
    }
  }
  std::vector<float> ci(M1), c1(M1, 1.0f);
  for (int k = 0; k < M1; ++k) ci[k] = (float)((k == 0 ? 1.0 : 2.0) / ((double)H * W));
  auto up = [&](DevBuf& b, const void* src, size_t bytes) -> mmx_status {
    HIP_TRY(b.alloc(bytes));
    HIP_TRY(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
    return MMX_OK;
  };
  MMX_TRY(up(f->Fx, fx.data(), fx.size() * sizeof(cpx<float>)));
  MMX_TRY(up(f->Fy, fy.data(), fy.size() * sizeof(cpx<float>)));
  MMX_TRY(up(f->cinv, ci.data(), M1 * sizeof(float)));
  MMX_TRY(up(f->cone, c1.data(), M1 * sizeof(float)));
  const size_t act = (size_t)batch_max * C * f->P * sizeof(float);
  const size_t spec = (size_t)batch_max * C * M1 * f->J * sizeof(cpx<float>);
  f->V.resize(L);
  f->Z.resize(L);
  f->Vh.resize(L);
  for (int l = 0; l < L; ++l) {
    HIP_TRY(f->V[l].alloc(act));
    HIP_TRY(f->Z[l].alloc(act));
    HIP_TRY(f->Vh[l].alloc(spec));
  }
  HIP_TRY(f->X0.alloc((size_t)batch_max * 5 * f->P * sizeof(float)));
  HIP_TRY(f->Y1.alloc((size_t)batch_max * Cp * f->P * sizeof(float)));
  HIP_TRY(f->A1.alloc((size_t)batch_max * Cp * f->P * sizeof(float)));
  HIP_TRY(f->dA.alloc((size_t)batch_max * Cp * f->P * sizeof(float)));
  HIP_TRY(f->dh.alloc((size_t)batch_max * 3 * f->P * sizeof(float)));
  HIP_TRY(f->dV.alloc(act));
  HIP_TRY(f->dV2.alloc(act));
  HIP_TRY(f->dZ.alloc(act));
  HIP_TRY(f->Uh.alloc(spec));
  HIP_TRY(f->dUh.alloc(spec));
  HIP_TRY(f->dVh.alloc(spec));
  // weight-gradient partials: largest map (lift, C x C, projections) at the
  // largest row count over batches 1 .. batch_max
  long rows_max = 0;
  for (int b = 1; b <= batch_max; ++b) rows_max = std::max(rows_max, dw_rows(f->P, b));
  const long npair_max =
      std::max(std::max((long)C * 5 + C, (long)C * C + C), std::max((long)Cp * C + Cp, 3L * Cp + 3));
  HIP_TRY(f->part.alloc((size_t)rows_max * npair_max * sizeof(float)));
  HIP_TRY(f->lpart.alloc((size_t)batch_max * 64 * 2 * sizeof(double)));
  HIP_TRY(f->lsum.alloc((size_t)batch_max * 2 * sizeof(double)));
  HIP_TRY(f->loss.alloc(sizeof(double)));
  *out = f.release();
  return MMX_OK;
}

void mmx_fno_destroy(mmx_fno* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->stream);
  delete f;
}

mmx_status mmx_fno_set_stream(mmx_fno* f, void* stream) {
  if (!f) return fail(MMX_EINVAL, "null FNO");
  f->stream = reinterpret_cast<hipStream_t>(stream);
  return MMX_OK;
}

mmx_status mmx_fno_param_count(const mmx_fno* f, int64_t* n) {
  if (!f || !n) return fail(MMX_EINVAL, "null argument");
  *n = f->nparam;
  return MMX_OK;
}

mmx_status mmx_fno_init(mmx_fno* f, float* params, uint64_t seed) {
  if (!f || !params) return fail(MMX_EINVAL, "null argument");
  std::vector<float> h(f->nparam, 0.0f);
  InitRng rng{seed};
  auto fill = [&](long off, long n, double scale) {
    for (long i = 0; i < n; ++i) h[off + i] = (float)(scale * rng.normal());
  };
  fill(f->oP, (long)f->C * 5, 1.0 / std::sqrt(5.0));
  const double rs = 1.0 / ((double)f->C * f->C);
  for (int l = 0; l < f->L; ++l) {
    const long n = (long)f->M1 * f->J * f->C * f->C * 2;
    for (long i = 0; i < n; ++i) h[f->oR[l] + i] = (float)(rs * rng.uniform());
    fill(f->oW[l], (long)f->C * f->C, 1.0 / std::sqrt((double)f->C));
  }
  fill(f->oQ1, (long)f->Cp * f->C, 1.0 / std::sqrt((double)f->C));
  fill(f->oQ2, 3L * f->Cp, 1.0 / std::sqrt((double)f->Cp));
  HIP_TRY(hipMemcpy(params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  return MMX_OK;
}

mmx_status mmx_fno_forward(mmx_fno* f, const float* params, const float* m, float* h,
                           int32_t batch) {
  if (!f || !params || !m || !h) return fail(MMX_EINVAL, "null argument");
  if (batch < 1 || batch > f->Bmax) return fail(MMX_EINVAL, "batch out of range");
  return fno_forward_impl(f, params, m, h, batch);
}

mmx_status mmx_fno_backward(mmx_fno* f, const float* params, const float* h, const float* target,
                            float* grads, double* loss) {
  if (!f || !params || !h || !target || !grads) return fail(MMX_EINVAL, "null argument");
  if (f->batch < 1) return fail(MMX_ESTATE, "no forward pass to differentiate");
  return fno_backward_impl(f, params, h, target, grads, loss);
}

mmx_status mmx_fno_adam(mmx_fno* f, float* params, const float* grads, float* moments, double lr,
                        int64_t t) {
  if (!f || !params || !grads || !moments) return fail(MMX_EINVAL, "null argument");
  if (t < 1) return fail(MMX_EINVAL, "Adam step count starts at 1");
  const long n = f->nparam;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)t));
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, f->stream>>>(params, grads, moments, moments + n, n,
                                                            (float)lr, 0.9f, 0.999f, 1e-8f, c1, c2);
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

}  // extern "C"
