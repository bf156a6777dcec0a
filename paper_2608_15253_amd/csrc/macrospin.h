// Replica-resident steps of single-cell systems (device code).
//
// A one-cell grid without the demag term has only cell-local field terms
// (anisotropy, Zeeman, thermal; exchange and DMI vanish with one cell), so
// one thread can hold one replica in registers for a whole run of Heun or
// rotation steps: fields, torque with the spin-transfer term, predictor and
// corrector, and the switching time, with the per-cell arithmetic of the field
// kernels in the same order (results equal the staged path to round-off; the
// compiler may contract multiply-adds differently in the two kernels).  The
// thermal noise of a step is drawn once and used by both stages, as there.
// Retire/refill runs here too, with the trial bookkeeping in registers.
#pragma once
#include "common.h"
#include "kernels.h"
#include "philox.h"

namespace mmx {

template <typename T, bool ROT>
__device__ inline void macrospin_field(const FArgs<T>& a, const T mc[3], T sigma,
                                       const T eta[3], T H[3]) {
  T Hex[3], Hdm[3], Han[3], Hz[3];
  local_terms(a, mc, 0u, 0, 0, 0, mc, a.kbc, Hex, Hdm, Han, Hz);
  const T Hdd[3] = {0, 0, 0};
#pragma unroll
  for (int c = 0; c < 3; ++c) H[c] = Hex[c] + Hdm[c] + Han[c] + Hz[c] + Hdd[c];
  if (sigma != T(0)) {
#pragma unroll
    for (int c = 0; c < 3; ++c) H[c] += sigma * eta[c];
  }
}

// Retire/refill state of the replicas (null: plain run): initial states, the
// trial generation and first step of the running trial (carried between
// launches), finished-trial counts and the recorded trial lengths.
template <typename T>
struct MacroRefill {
  const T* m_init;
  int* tgen;
  unsigned long long* tstart;
  int* counts;
  double* times;
  int cap;
};

// m: replicas' states (3 values each, D1 layout with one cell); tsw: switching
// times or null.  One thread per replica.
template <typename T, bool ROT>
__global__ void __launch_bounds__(256) k_macrospin(FArgs<T> a, T* m, double dt_d, int nsteps,
                                                   uint64_t step0, double* tsw, int R,
                                                   MacroRefill<T> rf) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const bool refill = rf.tgen != nullptr;
  uint32_t gen = refill ? (uint32_t)rf.tgen[r] : 0u;
  unsigned long long start = refill ? rf.tstart[r] : 0ull;
  int count = refill ? rf.counts[r] : 0;
  const T dt = (T)dt_d;
  T sigma = 0;
  if ((a.terms & T_THERMAL) && a.Trep) {
    const double Tr = a.Trep[r];
    if (Tr > 0) sigma = (T)sqrt(a.sig2pref * Tr / a.dt_th);
  }
  const uint64_t seed = sigma != T(0) ? a.seeds[r] : 0;
  const T bJ = stt_bj(a, r);
  T mv[3] = {m[(size_t)r * 3], m[(size_t)r * 3 + 1], m[(size_t)r * 3 + 2]};
  double ts = tsw ? tsw[r] : 0.0;
  for (int s = 0; s < nsteps; ++s) {
    const uint64_t step = step0 + (uint64_t)s;
    T eta[3] = {0, 0, 0};
    if (sigma != T(0)) thermal_eta<T>(seed, 0u, refill ? step - start : step, eta, gen);
    T H[3], k[3], tau[3], k1v[3], mp[3];
    macrospin_field<T, ROT>(a, mv, sigma, eta, H);
    cell_torque(a, bJ, mv, H, k, tau);
    heun_predict(a, ROT, mv, H, k, tau, dt, k1v, mp);
    macrospin_field<T, ROT>(a, mp, sigma, eta, H);
    cell_torque(a, bJ, mp, H, k, tau);
    T mn[3];
    heun_correct(a, ROT, mp, H, k, tau, mv, k1v, dt, mn);
#pragma unroll
    for (int c = 0; c < 3; ++c) mv[c] = mn[c];
    if (tsw && ts < 0 && (double)mv[2] < 0) ts = (double)(step + 1) * dt_d;
    if (refill && (double)mv[2] < 0) {
      // the trial ends: record its length, restart from the initial state
      if (count < rf.cap) rf.times[(size_t)r * rf.cap + count] = (double)(step + 1 - start) * dt_d;
      ++count;
      ++gen;
      start = step + 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) mv[c] = rf.m_init[(size_t)r * 3 + c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) m[(size_t)r * 3 + c] = mv[c];
  // a non-finite state stays non-finite through later steps and resets
  if (a.nonfinite && !(fabs(mv[0]) + fabs(mv[1]) + fabs(mv[2]) <= T(3))) *a.nonfinite = 1;
  if (tsw) tsw[r] = ts;
  if (refill) {
    rf.tgen[r] = (int)gen;
    rf.tstart[r] = start;
    rf.counts[r] = count;
  }
}

}  // namespace mmx
