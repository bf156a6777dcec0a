// Dormand-Prince RK45 whose intermediate stages take the demagnetising field
// from the learned operator (mmx_fno), checked at every accepted step against
// the exact convolution.  Included by mmx.hip after the network's host code.
#pragma once

namespace {

using namespace mmx;

// per-replica partial sums of |scale h + (0, 0, mz m_z) - hd|^2 and |hd|^2
__global__ void __launch_bounds__(256) k_gate_partial(const float* __restrict__ h,
                                                      const float* __restrict__ hd,
                                                      const float* __restrict__ m, double scale,
                                                      double mz, int N, double* part) {
  __shared__ double red[2][256];
  const int r = blockIdx.y, nb = gridDim.x;
  const size_t base = (size_t)r * 3 * N;
  double num = 0, den = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += nb * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t o = base + (size_t)c * N + i;
      double v = scale * (double)h[o];
      if (c == 2) v += mz * (double)m[o];
      const double x = (double)hd[o];
      num += (v - x) * (v - x);
      den += x * x;
    }
  }
  red[0][threadIdx.x] = num;
  red[1][threadIdx.x] = den;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((size_t)r * nb + blockIdx.x) * 2 + 0] = red[0][0];
    part[((size_t)r * nb + blockIdx.x) * 2 + 1] = red[1][0];
  }
}

// relative L2 error of each replica's film (fixed summation order)
__global__ void k_gate_final(const double* part, int nb, int R, double* err) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double num = 0, den = 0;
  for (int b = 0; b < nb; ++b) {
    num += part[((size_t)r * nb + b) * 2 + 0];
    den += part[((size_t)r * nb + b) * 2 + 1];
  }
  err[r] = den > 0 ? sqrt(num / den) : (num > 0 ? __builtin_inf() : 0.0);
}

struct FnoHook : StageHook {
  mmx_fno* f = nullptr;
  const float* prm = nullptr;
  int R = 0;
  mmx_status field(mmx_ctx* ctx, Group& G, const float* m) const override {
    (void)G;
    ProfScope ps(ctx->prof, "fno_forward", ctx->stream);
    return fno_forward_impl(f, prm, m, h, R);
  }
};

struct FnoStreamGuard {
  mmx_fno* f;
  hipStream_t saved;
  FnoStreamGuard(mmx_fno* f_, hipStream_t s) : f(f_), saved(f_->stream) { f->stream = s; }
  ~FnoStreamGuard() { f->stream = saved; }
};

constexpr int kGateBlocks = 64;

mmx_status rk45_surrogate_impl(mmx_ctx* ctx, mmx_fno* f, const float* prm, void* m, double t0,
                               double t_end, double tol, double dt0, double gate_tol,
                               int residual_mz, int exact_after_fail, double* gate_log,
                               int64_t gate_cap, mmx_surrogate_stats* stats) {
  if (ctx->prec != MMX_F32) return fail(MMX_EUNSUP, "learned demag stages need an FP32 context");
  if (ctx->groups.size() != 1) return fail(MMX_EUNSUP, "learned demag stages need one group");
  if (!(ctx->terms & MMX_DEMAG)) return fail(MMX_ESTATE, "demag term is off");
  Group& G = *ctx->groups[0];
  if (G.nz != 1 || G.nx != f->W || G.ny != f->H)
    return fail(MMX_ESHAPE, "network grid differs from the film");
  if (G.R > f->Bmax) return fail(MMX_ESHAPE, "more replicas than the network's batch_max");
  if (G.cells_on) return fail(MMX_EUNSUP, "learned demag stages with per-cell materials");
  if (!(gate_tol >= 0)) return fail(MMX_EINVAL, "gate_tol must be >= 0");
  if (exact_after_fail < 0) return fail(MMX_EINVAL, "exact_after_fail must be >= 0");
  if (gate_cap > 0 && !gate_log) return fail(MMX_EINVAL, "gate_log is null");
  ctx->rk_valid = 0;  // the learned-stage run reuses the stage buffers
  RkState h;
  MMX_TRY(rk_begin<float>(ctx, t0, t_end, tol, dt0, nullptr, 0, h));
  const size_t nel = (size_t)G.R * 3 * G.N;
  const size_t npart = (size_t)G.R * kGateBlocks * 2 * sizeof(double);
  // the arena of an FP32 one-film context holds these buffers
  if (ctx->sg_h.bytes < nel * sizeof(float) || ctx->sg_hd.bytes < nel * sizeof(float) ||
      ctx->sg_part.bytes < npart || ctx->sg_err.bytes < G.R * sizeof(double))
    return fail(MMX_ESTATE, "learned-stage buffers missing from the context");
  hipStream_t s = ctx->stream;
  FnoStreamGuard guard(f, s);
  FnoHook hook;
  hook.f = f;
  hook.prm = prm;
  hook.R = G.R;
  hook.h = ctx->sg_h.as<float>();
  hook.scale = G.mat.Ms;
  hook.mz = residual_mz ? -G.mat.Ms : 0.0;
  hook.hd = ctx->sg_hd.p;
  float* mb = reinterpret_cast<float*>(m);
  double e[7];
  for (int j = 0; j < 7; ++j) e[j] = (j < 6 ? DP_A[6][j] : 0.0) - DP_B4[j];
  std::vector<double> err(G.R);
  mmx_surrogate_stats S{};
  auto read_state = [&]() -> mmx_status {
    HIP_TRY(hipMemcpyAsync(&h, ctx->st.p, sizeof(RkState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MMX_OK;
  };
  MMX_TRY(rk_first_stage<float>(ctx, mb));  // k1 with the exact field
  int exact_left = 0;
  while (!h.done) {
    const RkState before = h;
    const bool try_net = exact_left == 0;
    if (try_net) {
      MMX_TRY(rk_stages<float>(ctx, G, mb, e, &hook));
      {
        ProfScope psc(ctx->prof, "k_rk_controller", s);
        k_rk_controller<<<1, 1, 0, s>>>(ctx->st.as<RkState>(), nullptr, ctx->dts.as<double>(),
                                        ctx->dts_cap);
        HIP_TRY(hipGetLastError());
      }
      MMX_TRY(read_state());
      bool keep = false;
      if (h.accepted_flag) {
        // gate at the accepted point: network field of m7 against the exact
        // stage-7 field stored by the last evaluation
        MMX_TRY(hook.field(ctx, G, G.m7.as<float>()));
        {
          ProfScope ps(ctx->prof, "k_gate", s);
          k_gate_partial<<<dim3(kGateBlocks, G.R), 256, 0, s>>>(
              hook.h, ctx->sg_hd.as<float>(), G.m7.as<float>(), hook.scale, hook.mz, G.N,
              ctx->sg_part.as<double>());
          HIP_TRY(hipGetLastError());
          k_gate_final<<<(G.R + 63) / 64, 64, 0, s>>>(ctx->sg_part.as<double>(), kGateBlocks,
                                                       G.R, ctx->sg_err.as<double>());
          HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipMemcpyAsync(err.data(), ctx->sg_err.p, G.R * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double gmax = 0;
        for (double v : err) gmax = (v != v || v > gmax) ? v : gmax;  // NaN propagates
        if (S.gate_checks < gate_cap) gate_log[S.gate_checks] = gmax;
        S.gate_checks += 1;
        keep = gmax <= gate_tol;
        if (keep) {
          S.gate_max_passed = std::max(S.gate_max_passed, gmax);
        } else {
          S.gate_failures += 1;
          exact_left = exact_after_fail;
        }
      } else {
        S.surrogate_rejected += 1;
      }
      if (keep) {
        const unsigned nb = (unsigned)std::min<size_t>((nel + 255) / 256, 4096);
        ProfScope ps(ctx->prof, "k_rk_commit", s);
        k_rk_commit<float><<<nb, 256, 0, s>>>(ctx->st.as<RkState>(), mb, G.m7.as<float>(),
                                              G.k[0].as<float>(), G.k[6].as<float>(), nel);
        HIP_TRY(hipGetLastError());
        S.surrogate_steps += 1;
        continue;
      }
      // discard the attempt: restore the controller and repeat it exactly
      h = before;
      HIP_TRY(hipMemcpyAsync(ctx->st.p, &h, sizeof(RkState), hipMemcpyHostToDevice, s));
    }
    MMX_TRY(rk_stages<float>(ctx, G, mb, e, nullptr));
    MMX_TRY(rk_finish<float>(ctx, mb, nullptr));
    MMX_TRY(read_state());
    if (h.accepted_flag) {
      S.exact_steps += 1;
      if (!try_net && exact_left > 0) exact_left -= 1;
    }
  }
  if (stats) {
    S.t = h.t;
    S.dt = h.dt;
    S.err = h.last_err;
    S.accepted = h.accepted;
    S.rejected = h.rejected;
    *stats = S;
  }
  ctx->last_accepted = h.accepted;
  if (h.dtmin_hit) return fail(MMX_EDTMIN, "step size fell below dt_min");
  return MMX_OK;
}

}  // namespace

extern "C" {

mmx_status mmx_rk45_surrogate(mmx_ctx* ctx, mmx_fno* net, const float* params, void* m, double t0,
                              double t_end, double tol, double dt0, double gate_tol,
                              int32_t residual_mz, int32_t exact_after_fail, double* gate_log,
                              int64_t gate_cap, mmx_surrogate_stats* stats) {
  if (!ctx || !net || !params || !m) return fail(MMX_EINVAL, "null argument");
  if (!(t_end > t0)) return fail(MMX_EINVAL, "t_end must exceed t0");
  if (!(tol > 0)) return fail(MMX_EINVAL, "tol must be > 0");
  if (!(dt0 > 0)) return fail(MMX_EINVAL, "dt0 must be > 0");
  if (ctx->terms & MMX_THERMAL) return fail(MMX_EUNSUP, "thermal field with RK45");
  return rk45_surrogate_impl(ctx, net, params, m, t0, t_end, tol, dt0, gate_tol, residual_mz,
                             exact_after_fail, gate_log, gate_cap, stats);
}

}  // extern "C"
