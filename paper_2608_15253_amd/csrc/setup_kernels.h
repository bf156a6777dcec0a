// One-off setup kernels: Newell kernel in FP64 on the padded grid, FP64 line
// FFTs of the kernel and parity compression of its (real) spectrum; plus the
// small integrator bookkeeping kernels.
#pragma once
#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "newell.h"

namespace mmx {

struct AxisMap {   // per axis of the padded grid
  int n, P, periodic, images;
};

// For FFT index k on one axis: number of representative offsets (1 or 2) and
// their values.  Open axis of size 2n: k < n -> k, k > n -> k - 2n, k == n
// (Nyquist) -> none.  Periodic: minimum image; for even n the offset n/2 is
// averaged with -n/2.
__device__ inline int axis_reps(const AxisMap& m, int k, long o[2]) {
  if (m.n == 1) { o[0] = 0; return 1; }
  if (m.periodic) {
    const long v = (k < m.n - k) ? k : (long)k - m.n;
    o[0] = v;
    if (m.n % 2 == 0 && (v == m.n / 2 || v == -m.n / 2)) { o[1] = -v; return 2; }
    return 1;
  }
  if (k < m.n) { o[0] = k; return 1; }
  if (k > m.n) { o[0] = (long)k - 2 * m.n; return 1; }
  return 0;
}

// K (complex FP64, [6][Pz][Py][Px], imaginary part 0): real-space kernel.
__global__ void k_newell_kernel(cpx<double>* K, AxisMap ax, AxisMap ay, AxisMap az, double dx,
                                double dy, double dz, GaussRules rules) {
  const long total = (long)ax.P * ay.P * az.P;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int kx = id % ax.P;
  const int ky = (id / ax.P) % ay.P;
  const int kz = id / ((long)ax.P * ay.P);
  long ox[2], oy[2], oz[2];
  const int nxr = axis_reps(ax, kx, ox), nyr = axis_reps(ay, ky, oy), nzr = axis_reps(az, kz, oz);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (nxr && nyr && nzr) {
    const double w = 1.0 / (nxr * nyr * nzr);
    const int px = (ax.periodic && ax.n > 1) ? ax.images : 0;
    const int py = (ay.periodic && ay.n > 1) ? ay.images : 0;
    const int pz = (az.periodic && az.n > 1) ? az.images : 0;
    for (int a = 0; a < nxr; ++a)
      for (int b = 0; b < nyr; ++b)
        for (int c = 0; c < nzr; ++c)
          for (int iz = -pz; iz <= pz; ++iz)
            for (int iy = -py; iy <= py; ++iy)
              for (int ix = -px; ix <= px; ++ix)
                tensor_add(ox[a] + (long)ix * ax.n, oy[b] + (long)iy * ay.n,
                           oz[c] + (long)iz * az.n, dx, dy, dz, rules, w, acc);
  }
  for (int c = 0; c < 6; ++c) K[(size_t)c * total + id] = {acc[c], 0.0};
}

// In-place FP64 FFT of lines: element k of line (o, i) at o*os + i*is + k*stride.
__global__ void k_line_fft(cpx<double>* data, long os, long is, long stride, FftPlan plan,
                           const cpx<double>* tw) {
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* A = reinterpret_cast<cpx<double>*>(smem_raw);
  cpx<double>* Bf = A + plan.n;
  const long base = (long)blockIdx.y * os + (long)blockIdx.x * is;
  for (int k = threadIdx.x; k < plan.n; k += blockDim.x) A[k] = data[base + k * stride];
  __syncthreads();
  const cpx<double>* X = lds_fft<double, false>(A, Bf, 1, plan, tw);
  for (int k = threadIdx.x; k < plan.n; k += blockDim.x) data[base + k * stride] = X[k];
}

// Nt[((tz Ty + ty) Kx + kx) 8 + c] = scale * Re Khat[c][tz][ty][kx] for
// kx <= Px/2, ty <= Py/2, tz <= Pz/2: the six components of one frequency are
// adjacent (slots 6, 7 unused), one aligned vector load per frequency.
template <typename T>
__global__ void k_compress(T* Nt, const cpx<double>* K, int Px, int Py, int Pz, int Kx, int Ty,
                           int Tz, double scale) {
  const long tot = (long)6 * Tz * Ty * Kx;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int kx = id % Kx;
  const int ty = (id / Kx) % Ty;
  const int tz = (id / ((long)Kx * Ty)) % Tz;
  const int c = id / ((long)Kx * Ty * Tz);
  const long full = (long)Px * Py * Pz;
  const long f = ((long)tz * Ty + ty) * Kx + kx;
  Nt[f * kTensorStride + c] = (T)(scale * K[(size_t)c * full + ((long)tz * Py + ty) * Px + kx].re);
}

// ---------------------------------------------------------------------------
// integrator bookkeeping
// ---------------------------------------------------------------------------
__global__ void k_rk_controller(RkState* st, const double* replay, double* dts, long long dts_cap) {
  if (st->done) return;
  double err = __longlong_as_double((long long)st->err_bits);
  if (st->nonfinite) err = __builtin_nan("");
  st->err_bits = 0ull;
  st->nonfinite = 0;
  st->last_err = err;
  const double dt = st->dt;
  bool accept;
  double next;
  if (replay) {
    accept = true;
    st->replay_idx += 1;
    next = (st->replay_idx < st->n_replay) ? replay[st->replay_idx] : 0.0;
  } else {
    double fac;
    if (!(err == err)) { fac = 0.2; accept = false; }
    else {
      accept = err <= st->tol;
      fac = (err == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(st->tol / err, 0.2)));
    }
    next = fmin(dt * fac, st->dt_max);
  }
  if (accept) {
    if (st->accepted < dts_cap) dts[st->accepted] = dt;
    st->accepted += 1;
    st->t = (st->final_flag && !replay) ? st->t_end : st->t + dt;
  } else {
    st->rejected += 1;
  }
  st->accepted_flag = accept ? 1 : 0;
  if (replay) {
    st->dt = next;
    if (st->replay_idx >= st->n_replay) st->done = 1;
    return;
  }
  st->dt_prop = next;
  st->final_flag = (st->t + next >= st->t_end) ? 1 : 0;
  if (st->final_flag) next = st->t_end - st->t;
  st->dt = next;
  if (st->t >= st->t_end) st->done = 1;
  else if (next < st->dt_min) { st->done = 1; st->dtmin_hit = 1; }
}

template <typename T>
__global__ void k_rk_commit(const RkState* st, T* m, const T* m7, T* k1, const T* k7, size_t n) {
  if (!st->accepted_flag) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    m[i] = m7[i];
    k1[i] = k7[i];
  }
}

// per-replica fixed-order sums of workgroup partials; the check's time is
// step_after dt, step_after = (*stepdev if set) + the given count
__global__ void k_switch_reduce(const double* partial, int nblk, int R, int N, double* tsw,
                                unsigned long long step_after, const unsigned long long* stepdev,
                                double dt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const unsigned long long st = (stepdev ? *stepdev : 0ull) + step_after;
  switch_check(partial, tsw, nblk, N, r, (double)st * dt);
}

// Retire/refill bookkeeping after a step (one thread per replica): a replica
// whose mean m_z is negative ends its trial, records the trial's duration
// (while fewer than cap are recorded), starts trial g + 1 at the next step and
// is flagged for a reset to its initial state.
__global__ void k_refill_check(const double* partial, int nblk, int R, int N, int* tgen,
                               unsigned long long* tstart, int* flag, int* counts, double* times,
                               int cap, unsigned long long step_host,
                               const unsigned long long* stepdev, double dt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)r * nblk + b];
  const unsigned long long step = (stepdev ? *stepdev : 0ull) + step_host;
  int f = 0;
  if (s / N < 0) {
    const int c = counts[r];
    if (c < cap) times[(size_t)r * cap + c] = (double)(step + 1 - tstart[r]) * dt;
    counts[r] = c + 1;
    tgen[r] += 1;
    tstart[r] = step + 1;
    f = 1;
  }
  flag[r] = f;
}

// Reset of flagged replicas: state (n per replica) and, if present, its half
// spectrum (ns per replica) from the saved initial copies.  Grid (x, R).
template <typename T>
__global__ void k_refill_copy(const int* flag, T* m, const T* m_init, size_t n, cpx<T>* S,
                              const cpx<T>* S_init, size_t ns) {
  const int r = blockIdx.y;
  if (!flag[r]) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    m[(size_t)r * n + i] = m_init[(size_t)r * n + i];
  if (S)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += stride)
      S[(size_t)r * ns + i] = S_init[(size_t)r * ns + i];
}

__global__ void k_fill_i32(int* p, size_t n, int v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// max over cells of |v| for vectors stored component-major per replica
// (n cells per replica, R replicas): per-workgroup maxima, then one workgroup
// folds them (part: gridDim.x doubles).
template <typename T>
__global__ void k_norm_max(const T* v, size_t n, int R, double* part) {
  __shared__ double red[256];
  double mx = 0;
  const size_t total = n * (size_t)R;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t r = i / n, c = i - r * n;
    const T* b = v + r * 3 * n + c;
    const double x = (double)b[0], y = (double)b[n], z = (double)b[2 * n];
    mx = fmax(mx, sqrt(x * x + y * y + z * z));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_max_fold(double* part, int n) {
  __shared__ double red[256];
  double mx = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, part[i]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[n] = red[0];
}

// step counter of captured graphs: set before a replay, advanced inside it
__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }
__global__ void k_inc_u64(unsigned long long* p, unsigned long long d) { *p += d; }

__global__ void k_energy_reduce(const double* partial, int nblk, int R, double cq, double cz,
                                double* E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < nblk; ++b)
    for (int v = 0; v < 5; ++v) s[v] += partial[((size_t)r * nblk + b) * 5 + v];
  double tot = 0;
  for (int v = 0; v < 5; ++v) {
    const double e = (v == 4 ? cz : cq) * s[v];
    E[(size_t)r * 6 + v] = e;
    tot += e;
  }
  E[(size_t)r * 6 + 5] = tot;
}

// trace[accepted] = sum over replicas of E[.][5] when the last attempt was accepted
__global__ void k_trace_store(const RkState* st, const double* E, int R, double* trace,
                              long long cap, int force0) {
  if (!force0 && !st->accepted_flag) return;
  const long long idx = force0 ? 0 : st->accepted;
  if (idx >= cap) return;
  double s = 0;
  for (int r = 0; r < R; ++r) s += E[(size_t)r * 6 + 5];
  trace[idx] = s;
}

template <typename T>
__global__ void k_topo(const T* m, int nx, int ny, int N, int pbcx, int pbcy, double i2dx,
                       double i2dy, double* partial, int nblk) {
  __shared__ double red[kBlock];
  const int r = blockIdx.y;
  const size_t rb = (size_t)r * 3 * N;
  double acc = 0;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < nx * ny;
       cell += gridDim.x * blockDim.x) {
    const int x = cell % nx, y = cell / nx;
    double mc[3], xm[3], xp[3], ym[3], yp[3];
    for (int c = 0; c < 3; ++c) mc[c] = m[rb + (size_t)c * N + cell];
    auto get = [&](int xx, int yy, double v[3]) {
      for (int c = 0; c < 3; ++c) v[c] = m[rb + (size_t)c * N + xx + (size_t)nx * yy];
    };
    if (nx > 1) {
      if (x > 0) get(x - 1, y, xm); else if (pbcx) get(nx - 1, y, xm); else get(x, y, xm);
      if (x < nx - 1) get(x + 1, y, xp); else if (pbcx) get(0, y, xp); else get(x, y, xp);
    } else { get(x, y, xm); get(x, y, xp); }
    if (ny > 1) {
      if (y > 0) get(x, y - 1, ym); else if (pbcy) get(x, ny - 1, ym); else get(x, y, ym);
      if (y < ny - 1) get(x, y + 1, yp); else if (pbcy) get(x, 0, yp); else get(x, y, yp);
    } else { get(x, y, ym); get(x, y, yp); }
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) { a[c] = (xp[c] - xm[c]) * i2dx; b[c] = (yp[c] - ym[c]) * i2dy; }
    acc += mc[0] * (a[1] * b[2] - a[2] * b[1]) + mc[1] * (a[2] * b[0] - a[0] * b[2]) +
           mc[2] * (a[0] * b[1] - a[1] * b[0]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)r * nblk + blockIdx.x] = red[0];
}

__global__ void k_topo_reduce(const double* partial, int nblk, int R, double scale, double* Q) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += partial[(size_t)r * nblk + b];
  Q[r] = s * scale;
}

}  // namespace mmx
