// libmmx: host runtime and C ABI (see include/mmx.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mmx.h"
#include "common.h"
#include "fused.h"
#include "macrospin.h"
#include "kernels.h"
#include "setup_kernels.h"
#include "yconv_reg.h"
#include "rows_reg.h"
#include "axis_reg.h"

using namespace mmx;

// Per-workgroup partial sums of mmx_topological_charge_noalloc live in this
// file-scope array: 1 MiB (131072 doubles) on every device the library runs
// on, held until the process ends.  Host code never passes its name to a
// kernel (on the host it is a stand-in, not a device address); it uses the
// device address taken once per device by scratch_init.
constexpr size_t kScratchDoubles = size_t(1) << 17;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

thread_local std::string g_err;

mmx_status fail(mmx_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(MMX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define MMX_TRY(expr)                 \
  do {                                \
    mmx_status s_ = (expr);           \
    if (s_ != MMX_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------
// FFT planning
// ---------------------------------------------------------------------------
bool make_plan(int n, bool prune, FftPlan& p) {
  std::memset(&p, 0, sizeof(p));
  p.n = n;
  if (n <= 1) return n == 1;
  int rest = n;
  if (prune) {
    if (n % 2) return false;
    p.radix[p.npass++] = 2;
    p.prune = 1;
    rest /= 2;
  }
  // radix 4 first: measured faster on gfx950 than 8/16 up to 256 points (the
  // wider butterflies leave threads idle and write LDS with larger strides);
  // from 512 points on, radix 8 first: fewer passes, and such lines are few
  // per workgroup, so each pass's latency dominates (512x512 film RK45: 5 %
  // faster in FP32, 6 % in FP64)
  while (n >= 512 && rest % 8 == 0 && p.npass < kMaxPass) { p.radix[p.npass++] = 8; rest /= 8; }
  while (rest % 4 == 0 && p.npass < kMaxPass) { p.radix[p.npass++] = 4; rest /= 4; }
  while (rest % 2 == 0 && p.npass < kMaxPass) { p.radix[p.npass++] = 2; rest /= 2; }
  while (rest % 3 == 0 && p.npass < kMaxPass) { p.radix[p.npass++] = 3; rest /= 3; }
  while (rest % 5 == 0 && p.npass < kMaxPass) { p.radix[p.npass++] = 5; rest /= 5; }
  return rest == 1;
}

bool fft_ok(int n) {
  FftPlan p;
  return make_plan(n, false, p);
}

// Gauss-Legendre nodes/weights by Newton iteration on the Legendre recurrence.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

template <typename T>
std::vector<cpx<T>> twiddles(int n, int len) {
  std::vector<cpx<T>> t(len);
  for (int k = 0; k < len; ++k) {
    const double a = -2.0 * kPi * (double)k / (double)n;
    t[k] = {(T)std::cos(a), (T)std::sin(a)};
  }
  return t;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) {
    if (p) { (void)hipFree(p); p = nullptr; }
    bytes = b;
    if (b == 0) return hipSuccess;
    return hipMalloc(&p, b);
  }
  hipError_t ensure(size_t b) { return (p && bytes == b) ? hipSuccess : alloc(b); }
  template <typename U> U* as() const { return reinterpret_cast<U*>(p); }
};

// A region of the context's device arena (not owned; see arena_layout).
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename U> U* as() const { return reinterpret_cast<U*>(p); }
};

struct Group {
  mmx_group g{};
  int nx = 1, ny = 1, nz = 1, N = 1, R = 1;
  int Px = 1, Py = 1, Pz = 1, Kx = 1, hx = 1, Ty = 1, Tz = 1, Sy = 1;
  int xone = 0, is3d = 0;
  int L = 1, Wy = 1, Wz = 1;  // Wz: columns per workgroup of the fused y-z pass when it applies
  size_t max_lds = 64 * 1024;  // dynamic LDS per workgroup on the device
  FftPlan plan_x{}, plan_xi{}, plan_yf{}, plan_yi{}, plan_zf{}, plan_zi{};
  mmx_material mat{};
  int mat_set = 0;
  double B[3] = {0, 0, 0};
  size_t off = 0;  // element offset of this group in caller arrays
  // device buffers (regions of the context's arena)
  Buf tw_x, wpost, tw_y, tw_z, Nt, S, ms, ms2, m7, k[7], Trep, seeds, partial, E;
  Buf tgen, tstart, tflag, S_init;  // retire/refill trials
  Buf Jrep;  // spin-transfer current density per replica (A/m^2)
  mmx_material_ext ext{};  // bulk DMI, cubic anisotropy, RKKY
  Buf Acell;               // per-cell exchange stiffness (T[N]), used if acell_on
  Buf nblk_dev;            // int: the last corrector's workgroups per replica
  Buf topo_part;           // per-workgroup partial sums of the topological charge
  int acell_on = 0, jrep_on = 0;
  // per-cell Ms, alpha, Ku, D (mmx_set_material_cells): host values (empty:
  // uniform) and the derived device arrays of FArgs (msr, mgi, gpc, alc, sgc,
  // kuc, dmc)
  std::vector<double> cMs, calpha, cKu, cD;
  Buf cell[7];
  int cells_on = 0;
  std::vector<std::vector<unsigned char>> tables;  // host twiddle tables (tw_x, wpost, tw_y, tw_z)
  double stt_p[3] = {0, 0, 1}, stt_P = 0, stt_lambda = 1, stt_eps2 = 0;
  int nblk = 1;       // k_fields workgroups per replica
  int nblk_last = 1;  // workgroups per replica of the last field-kernel launch
  int demag_built = 0;
  int fused_faster = 0;  // set by mmx_autotune when the replica-resident path timed faster
  // few-layer 3-D groups: 1 = separate register y passes around the z pass
  // instead of the fused y-z kernel (mmx_autotune times both)
  int yz_split = 1;
};

// Opt-in per-kernel timing with HIP events recorded on the bound stream
// around every launch (mmx_profile_enable / mmx_profile_get).
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<long long> cnt;
  hipStream_t stream = nullptr;
  int id_of(const char* n) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) return (int)i;
    names.emplace_back(n);
    ms.push_back(0.0);
    cnt.push_back(0);
    return (int)names.size() - 1;
  }
  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void flush() {
    if (recs.empty()) return;
    (void)hipStreamSynchronize(stream);
    for (auto& r : recs) {
      float t = 0.f;
      (void)hipEventElapsedTime(&t, r.a, r.b);
      ms[r.id] += t;
      cnt[r.id] += 1;
    }
    recs.clear();
    used = 0;
  }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ProfScope {
  Prof* p;
  int id = -1;
  hipEvent_t a = nullptr;
  ProfScope(Prof& pr, const char* name, hipStream_t s) : p(&pr) {
    if (!p->on) return;
    if (p->recs.size() >= 4096) p->flush();
    p->stream = s;
    id = p->id_of(name);
    a = p->ev();
    (void)hipEventRecord(a, s);
  }
  // the launch did not happen here (another scope records it)
  void cancel() { id = -1; }
  ~ProfScope() {
    if (id < 0) return;
    hipEvent_t b = p->ev();
    (void)hipEventRecord(b, p->stream);
    p->recs.push_back({id, a, b});
  }
};

}  // namespace

// Captured step sequences kept between calls: Heun / rotation runs of 2^i
// steps (i < kHeunGraphs) and chunks of RK45 attempts, each valid for the
// call signature it was captured with (the context's configuration epoch,
// which every setter advances, and the arrays and scalars the captured
// launches hold).
constexpr int kHeunGraphs = 6;  // 1, 2, 4, ..., 32 steps
struct GraphKey {
  uint64_t epoch = 0;
  const void* p[8] = {};
  double d = 0;
  long long i[4] = {};
  bool operator==(const GraphKey& o) const {
    if (epoch != o.epoch || d != o.d) return false;
    for (int j = 0; j < 8; ++j)
      if (p[j] != o.p[j]) return false;
    for (int j = 0; j < 4; ++j)
      if (i[j] != o.i[j]) return false;
    return true;
  }
};
struct GraphSet {
  GraphKey key;
  bool valid = false;
  std::vector<hipGraphExec_t> exec;
  std::vector<int> nblk;  // per group: workgroups per replica of its last corrector
  void clear() {
    for (auto& g : exec)
      if (g) (void)hipGraphExecDestroy(g);
    exec.clear();
    nblk.clear();
    valid = false;
  }
};

struct mmx_ctx {
  Prof prof;
  int prec = MMX_F32;
  int device = 0;              // HIP device the context was created on
  double* scratch = nullptr;   // device address of `scratch` on that device
  int path = MMX_PATH_AUTO;
  size_t max_lds = 64 * 1024;  // dynamic LDS per workgroup on this device
  // graph replay: library stream, fencing events, step counter, cached graphs
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_user = nullptr, ev_cap = nullptr;
  GraphSet heun_graphs, rk_graphs;
  uint64_t epoch = 1;  // configuration epoch: advanced by every setter
  Buf stepdev;
  const unsigned long long* cur_stepdev = nullptr;
  Buf nfflag;  // int: set by kernels that produced a non-finite state
  ~mmx_ctx() {
    if (cap_stream) (void)hipStreamSynchronize(cap_stream);
    heun_graphs.clear();
    rk_graphs.clear();
    if (ev_user) (void)hipEventDestroy(ev_user);
    if (ev_cap) (void)hipEventDestroy(ev_cap);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (arena && arena_owned) (void)hipFree(arena);
  }
  std::vector<std::unique_ptr<Group>> groups;
  uint32_t terms = MMX_EXCH | MMX_DMI_INTERFACIAL | MMX_ANIS_UNIAXIAL | MMX_ZEEMAN | MMX_DEMAG;
  hipStream_t stream = nullptr;
  size_t total_elems = 0;
  // every device buffer of the context is a region of one arena: allocated by
  // mmx_create (owned) or supplied by the caller through mmx_bind
  void* arena = nullptr;
  size_t arena_bytes = 0;
  bool arena_owned = false;
  Buf st;          // RkState
  Buf dts;         // accepted step sizes
  Buf replay;      // dt replay list
  long long dts_cap = 0;
  long long last_accepted = 0;
  Buf Etmp;        // per-replica energies for traces
  // learned-demag stages: network field input and exact-demag output of k_fields
  const float* hext = nullptr;
  double hext_scale = 0, hext_mz = 0;
  void* hd_out = nullptr;
  Buf sg_h, sg_hd, sg_part, sg_err;  // surrogate integrator buffers (FP32 one-film contexts)
  int noprec = 0;  // damping-only dynamics (mmx_set_precession(ctx, 0), mmx_relax)
  Buf maxbuf;      // max-reduction partials (mmx_relax)
  // controller state and FSAL slope (k[0] of every group) left by the last
  // adaptive run, valid for continuation while the configuration epoch is
  // unchanged and no other integrator has used the stage buffers
  RkState rk_last{};
  int rk_valid = 0;
  uint64_t rk_epoch = 0;
  int rot = 0;     // Heun epilogues take the rotation update (mmx_depondt*)
  int refill = 0;  // per-replica trial generation and start step (mmx_depondt_refill)
};

namespace {

size_t esize(const mmx_ctx* c) { return c->prec == MMX_F64 ? 8 : 4; }

mmx_status ensure_graph_stream(mmx_ctx* ctx);

// Captures the launches `body` queues on ctx->stream into an executable graph
// (*out), on the library's own stream (capture is not possible on the null
// stream); nothing runs.
template <typename F>
mmx_status capture_graph(mmx_ctx* ctx, F&& body, hipGraphExec_t* out) {
  hipStream_t user = ctx->stream, cs = ctx->cap_stream;
  ctx->stream = cs;
  hipGraph_t graph = nullptr;
  mmx_status cap = MMX_OK;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    cap = body();
    e = hipStreamEndCapture(cs, &graph);
  }
  ctx->stream = user;
  if (cap != MMX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return cap;
  }
  if (e != hipSuccess) return fail(MMX_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MMX_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return MMX_OK;
}

template <typename T>
size_t cpxb() { return sizeof(cpx<T>); }

// LDS of a y workgroup of W spectrum columns of length Py: all three
// components in 2-D (the tensor product needs them together), one component
// per workgroup for the 3-D y passes (lines of Py + 1 slots)
// LDS of a fused y-z workgroup of W spectrum columns (3 nz W lines of Py + 1
// slots, two buffers, the y twiddles)
template <typename T>
size_t lds_yz(const Group& G, int W) {
  return (2 * 3 * (size_t)G.nz * W * (G.Py + 1) + G.Py) * cpxb<T>();
}

// whether the 3-D group G takes its y and z passes in one fused kernel (few
// layers, and one column of the workgroup fits the device's LDS)
template <typename T>
bool yz_applies(const Group& G) {
  return G.is3d && G.nz <= 8 && lds_yz<T>(G, 1) <= G.max_lds;
}

// the fused y-z kernels may take up to the device's LDS per workgroup
// (beyond the default 64 KB); set once per process, to the device maximum,
// so that groups with different tiles never undercut each other
template <typename T>
mmx_status yz_attr(const Group& G) {
  const int b = (int)G.max_lds;
  HIP_TRY(hipFuncSetAttribute((const void*)&k_yzconv<T, 2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute((const void*)&k_yzconv<T, 4>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  HIP_TRY(hipFuncSetAttribute((const void*)&k_yzconv<T, 8>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, b));
  return MMX_OK;
}

// whether Wz columns fit one workgroup of the 3-D group's z (or fused y-z) pass
template <typename T>
bool wz_fits(const Group& G, int Wz) {
  constexpr size_t kDefaultLds = 64 * 1024;
  return yz_applies<T>(G) ? lds_yz<T>(G, Wz) <= G.max_lds
                          : (2 * 3 * (size_t)Wz * G.Pz + G.Pz) * cpxb<T>() <= kDefaultLds;
}

template <typename T>
size_t lds_ycols(bool is3d, int W, int Py) {
  if (is3d) return (2 * (size_t)W * (Py + 1) + Py) * cpxb<T>();
  return (2 * 3 * (size_t)W * Py + Py) * cpxb<T>();
}

mmx_status check_group(const mmx_group& g) {
  for (int a = 0; a < 3; ++a) {
    if (g.n[a] < 1) return fail(MMX_ESHAPE, "group: n must be >= 1");
    if (!(g.cell[a] > 0)) return fail(MMX_EINVAL, "group: cell sizes must be > 0");
    if (g.pbc[a] && g.pbc_images[a] < 0) return fail(MMX_EINVAL, "group: negative image count");
  }
  if (g.replicas < 1) return fail(MMX_ESHAPE, "group: replicas must be >= 1");
  if ((long long)g.n[0] * g.n[1] * g.n[2] > (1LL << 31))
    return fail(MMX_ESHAPE, "group: too many cells");
  return MMX_OK;
}

template <typename T>
mmx_status setup_group(mmx_ctx* ctx, Group& G) {
  const mmx_group& g = G.g;
  G.nx = g.n[0]; G.ny = g.n[1]; G.nz = g.n[2];
  G.N = G.nx * G.ny * G.nz;
  G.R = g.replicas;
  auto padded = [&](int a) { return g.n[a] == 1 ? 1 : (g.pbc[a] ? g.n[a] : 2 * g.n[a]); };
  G.Px = padded(0); G.Py = padded(1); G.Pz = padded(2);
  G.xone = (G.nx == 1);
  if (!G.xone && (G.Px % 2)) return fail(MMX_EUNSUP, "periodic x needs an even cell count");
  G.hx = G.xone ? 1 : G.Px / 2;
  G.Kx = G.xone ? 1 : G.hx + 1;
  G.Ty = G.Py / 2 + 1;
  G.Tz = G.Pz / 2 + 1;
  G.is3d = G.nz > 1;
  G.Sy = G.is3d ? G.Py : G.ny;
  // x: half-length complex transform; input zero beyond ceil(nx/2) -> pruned when nx even & open
  const bool px_prune = !G.xone && !g.pbc[0] && (G.nx % 2 == 0) && G.hx >= 2;
  if (!make_plan(G.hx, px_prune, G.plan_x) || !make_plan(G.hx, false, G.plan_xi))
    return fail(MMX_EUNSUP, "x length not 2^a 3^b 5^c");
  const bool py_prune = G.ny > 1 && !g.pbc[1];
  if (!make_plan(G.Py, py_prune, G.plan_yf) || !make_plan(G.Py, false, G.plan_yi))
    return fail(MMX_EUNSUP, "y length not 2^a 3^b 5^c");
  const bool pz_prune = G.nz > 1 && !g.pbc[2];
  if (!make_plan(G.Pz, pz_prune, G.plan_zf) || !make_plan(G.Pz, false, G.plan_zi))
    return fail(MMX_EUNSUP, "z length not 2^a 3^b 5^c");
  G.L = std::max(1, std::min(G.ny, kBlock / std::max(1, G.nx)));
  const size_t budget = 48 * 1024;
  G.Wy = (int)std::max<size_t>(
      1, std::min<size_t>(16, budget / ((G.is3d ? 2 : 6) * (size_t)G.Py * cpxb<T>())));
  G.Wy = std::min(G.Wy, G.Kx);
  G.Wz = (int)std::max<size_t>(1, std::min<size_t>(16, budget / (6 * (size_t)G.Pz * cpxb<T>())));
  G.Wz = std::min(G.Wz, G.Kx);
  // the smallest tiles must fit the LDS budget of one workgroup
  if ((2 * 3 * (size_t)G.hx + 2 * G.hx + 1) * cpxb<T>() > 64 * 1024 ||
      (2 * 3 * (size_t)G.Py + G.Py) * cpxb<T>() > 64 * 1024 ||
      (2 * 3 * (size_t)G.Pz + G.Pz) * cpxb<T>() > 64 * 1024)
    return fail(MMX_EUNSUP, "grid too long along one axis for this precision");
  while (G.L > 1 && (2 * 3 * (size_t)G.L * G.hx + 2 * G.hx + 1) * cpxb<T>() > 64 * 1024) G.L /= 2;
  while (G.Wy > 1 && lds_ycols<T>(G.is3d, G.Wy, G.Py) > 64 * 1024) G.Wy /= 2;
  while (G.Wz > 1 && (2 * 3 * (size_t)G.Wz * G.Pz + G.Pz) * cpxb<T>() > 64 * 1024) G.Wz /= 2;
  G.nblk = ((G.ny + G.L - 1) / G.L) * G.nz;
  G.max_lds = ctx->max_lds;
  if (yz_applies<T>(G)) {  // widest column tile with four workgroups per CU
    G.Wz = 1;
    for (int W : {16, 8, 4, 2})
      if (W <= G.Kx && lds_yz<T>(G, W) <= G.max_lds / 4) { G.Wz = W; break; }
    MMX_TRY(yz_attr<T>(G));
  }
  // twiddle tables, uploaded into the arena by arena_init
  auto keep = [&](const std::vector<cpx<T>>& t) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(t.data());
    G.tables.emplace_back(b, b + t.size() * sizeof(cpx<T>));
  };
  G.tables.clear();
  keep(twiddles<T>(G.hx, G.hx));
  keep(twiddles<T>(G.xone ? 1 : G.Px, G.hx + 1));
  keep(twiddles<T>(G.Py, G.Py));
  keep(twiddles<T>(G.Pz, G.Pz));
  return MMX_OK;
}

// ---------------------------------------------------------------------------
// device arena: every buffer of a context, laid out in one allocation
// ---------------------------------------------------------------------------
constexpr long long kDtsCap = 1 << 18;  // accepted-step and replay list capacity
constexpr size_t kArenaAlign = 256;

int topo_blocks(const Group& G);

// Walks every device buffer of the context in a fixed order, calling
// take(buf, bytes) for each; the offsets follow from the sizes alone.
template <typename F>
void arena_walk(mmx_ctx* ctx, F&& take) {
  const size_t w = esize(ctx), c = 2 * w;  // real and complex element sizes
  int R_total = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    R_total += G.R;
    const size_t st = (size_t)G.R * 3 * G.N * w;
    take(G.tw_x, (size_t)G.hx * c);
    take(G.wpost, (size_t)(G.hx + 1) * c);
    take(G.tw_y, (size_t)G.Py * c);
    take(G.tw_z, (size_t)G.Pz * c);
    take(G.Nt, (size_t)kTensorStride * G.Tz * G.Ty * G.Kx * w);
    take(G.S, (size_t)G.R * 3 * G.nz * G.Sy * G.Kx * c);
    take(G.ms, st);
    take(G.ms2, st);
    take(G.m7, st);
    for (int j = 0; j < 7; ++j) take(G.k[j], st);
    take(G.Trep, (size_t)G.R * sizeof(double));
    take(G.seeds, (size_t)G.R * sizeof(uint64_t));
    // sized for one grid row per workgroup, the finest split any field kernel uses
    take(G.partial, (size_t)G.R * G.ny * G.nz * 5 * sizeof(double));
    take(G.E, (size_t)G.R * 6 * sizeof(double));
    take(G.tgen, (size_t)G.R * sizeof(int));
    take(G.tflag, (size_t)G.R * sizeof(int));
    take(G.tstart, (size_t)G.R * sizeof(unsigned long long));
    take(G.S_init, (size_t)G.R * 3 * G.nz * G.Sy * G.Kx * c);
    take(G.Jrep, (size_t)G.R * sizeof(double));
    take(G.Acell, (size_t)G.N * w);
    for (int j = 0; j < 7; ++j) take(G.cell[j], (size_t)G.N * w);
    take(G.nblk_dev, sizeof(int));
    take(G.topo_part, (size_t)G.R * topo_blocks(G) * sizeof(double));
  }
  take(ctx->st, sizeof(RkState));
  take(ctx->dts, (size_t)kDtsCap * sizeof(double));
  take(ctx->replay, (size_t)kDtsCap * sizeof(double));
  take(ctx->Etmp, (size_t)R_total * 6 * sizeof(double));
  take(ctx->maxbuf, 257 * sizeof(double));
  take(ctx->stepdev, sizeof(unsigned long long));
  take(ctx->nfflag, sizeof(int));
  // learned demag stages (FP32 contexts of one film only)
  const bool sg = ctx->prec == MMX_F32 && ctx->groups.size() == 1 && ctx->groups[0]->nz == 1;
  const Group& G0 = *ctx->groups[0];
  const size_t nel = sg ? (size_t)G0.R * 3 * G0.N : 0;
  take(ctx->sg_h, nel * sizeof(float));
  take(ctx->sg_hd, nel * sizeof(float));
  take(ctx->sg_part, sg ? (size_t)G0.R * 64 * 2 * sizeof(double) : 0);
  take(ctx->sg_err, sg ? (size_t)G0.R * sizeof(double) : 0);
}

size_t arena_size(mmx_ctx* ctx) {
  size_t off = 0;
  arena_walk(ctx, [&](Buf& b, size_t bytes) {
    (void)b;
    off = (off + kArenaAlign - 1) / kArenaAlign * kArenaAlign + bytes;
  });
  return (off + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// Points every buffer into the arena at `base`.
void arena_assign(mmx_ctx* ctx, void* base) {
  size_t off = 0;
  arena_walk(ctx, [&](Buf& b, size_t bytes) {
    off = (off + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    b.p = bytes ? static_cast<unsigned char*>(base) + off : nullptr;
    b.bytes = bytes;
    off += bytes;
  });
  ctx->dts_cap = kDtsCap;
}

// Allocates the context's arena and fills its initial contents: twiddle
// tables, zero temperatures, keys and flags, a cleared controller state.
mmx_status arena_init(mmx_ctx* ctx) {
  ctx->arena_bytes = arena_size(ctx);
  HIP_TRY(hipMalloc(&ctx->arena, ctx->arena_bytes));
  ctx->arena_owned = true;
  HIP_TRY(hipMemset(ctx->arena, 0, ctx->arena_bytes));
  arena_assign(ctx, ctx->arena);
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    Buf* dst[4] = {&G.tw_x, &G.wpost, &G.tw_y, &G.tw_z};
    for (int i = 0; i < 4; ++i)
      HIP_TRY(hipMemcpy(dst[i]->p, G.tables[i].data(), G.tables[i].size(), hipMemcpyHostToDevice));
  }
  return MMX_OK;
}

template <typename T>
mmx_status ensure_rk_buffers(Group&) {
  return MMX_OK;  // stage buffers are part of the arena
}

// ---------------------------------------------------------------------------
// demag kernel build
// ---------------------------------------------------------------------------
template <typename T>
mmx_status build_demag_group(mmx_ctx* ctx, Group& G) {
  GaussRules rules{};
  const int ns[5] = {3, 4, 6, 8, 10};
  for (int i = 0; i < 5; ++i) gauss_legendre(ns[i], rules.x[i], rules.w[i]);
  AxisMap ax{G.nx, G.Px, G.g.pbc[0], G.g.pbc_images[0]};
  AxisMap ay{G.ny, G.Py, G.g.pbc[1], G.g.pbc_images[1]};
  AxisMap az{G.nz, G.Pz, G.g.pbc[2], G.g.pbc_images[2]};
  const long total = (long)G.Px * G.Py * G.Pz;
  DevBuf K;
  HIP_TRY(K.alloc((size_t)6 * total * sizeof(cpx<double>)));
  hipStream_t s = ctx->stream;
  k_newell_kernel<<<(unsigned)((total + 127) / 128), 128, 0, s>>>(
      K.as<cpx<double>>(), ax, ay, az, G.g.cell[0], G.g.cell[1], G.g.cell[2], rules);
  HIP_TRY(hipGetLastError());
  // FFT along x, y, z in FP64
  auto line_fft = [&](int n, long os, long is, long stride, unsigned ni, unsigned no) -> mmx_status {
    if (n == 1) return MMX_OK;
    FftPlan p;
    make_plan(n, false, p);
    auto tw = twiddles<double>(n, n);
    DevBuf tb;
    HIP_TRY(tb.alloc(n * sizeof(cpx<double>)));
    HIP_TRY(hipMemcpy(tb.p, tw.data(), n * sizeof(cpx<double>), hipMemcpyHostToDevice));
    for (unsigned o0 = 0; o0 < no; o0 += 65535u) {
      const unsigned nob = std::min(65535u, no - o0);
      dim3 grid(ni, nob);
      k_line_fft<<<grid, 128, 2 * n * sizeof(cpx<double>), s>>>(
          K.as<cpx<double>>() + (long)o0 * os, os, is, stride, p, tb.as<cpx<double>>());
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    return MMX_OK;
  };
  const long Px = G.Px, Py = G.Py, Pz = G.Pz;
  MMX_TRY(line_fft(G.Px, Px, 0, 1, 1u, (unsigned)(6 * Pz * Py)));                 // rows
  MMX_TRY(line_fft(G.Py, Py * Px, 1, Px, (unsigned)Px, (unsigned)(6 * Pz)));     // columns
  MMX_TRY(line_fft(G.Pz, Pz * Py * Px, 1, Py * Px, (unsigned)(Py * Px), 6u));    // pillars
  const double scale = -G.mat.Ms / ((double)G.Px * G.Py * G.Pz);
  const long tot = (long)6 * G.Tz * G.Ty * G.Kx;
  k_compress<T><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(G.Nt.as<T>(), K.as<cpx<double>>(), G.Px,
                                                             G.Py, G.Pz, G.Kx, G.Ty, G.Tz, scale);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  G.demag_built = 1;
  return MMX_OK;
}

// ---------------------------------------------------------------------------
// one field evaluation of a group
// ---------------------------------------------------------------------------
struct Combine {
  int ncoef = 0;
  double coef[6] = {0, 0, 0, 0, 0, 0};
  int kidx[6] = {0, 0, 0, 0, 0, 0};  // which k buffer (0..5)
  int normalise = 0;
  int check_finite = 0;  // a normalised result that is a new state: flag non-finite values
  void* mout = nullptr;
};

struct Epilogue {
  int mode = FM_FIELD;
  void* out = nullptr;
  void* k1 = nullptr;
  const void* m0 = nullptr;
  void* mout = nullptr;
  double e[7] = {0, 0, 0, 0, 0, 0, 0};
  int use_k_err = 0;
  int fwd = 0;  // Heun modes: also write the half spectrum of the new state
  // RK stages with fwd: the next stage's combine (coefficients per slope,
  // this stage's slope index, 2 = normalise) written to mnext, from base m0
  double cn[6] = {0, 0, 0, 0, 0, 0};
  int cnext = 0, cstage = 0;
  void* mnext = nullptr;
};

// orthonormal cubic axes from c1 and c2 (c2 orthogonalised against c1)
bool cubic_axes(const mmx_material_ext& e, double c1[3], double c2[3], double c3[3]) {
  double n1 = std::sqrt(e.c1[0] * e.c1[0] + e.c1[1] * e.c1[1] + e.c1[2] * e.c1[2]);
  if (!(n1 > 0)) { c1[0] = 1; c1[1] = 0; c1[2] = 0; n1 = 1; }
  else for (int c = 0; c < 3; ++c) c1[c] = e.c1[c] / n1;
  const double d = e.c2[0] * c1[0] + e.c2[1] * c1[1] + e.c2[2] * c1[2];
  for (int c = 0; c < 3; ++c) c2[c] = e.c2[c] - d * c1[c];
  const double n2 = std::sqrt(c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
  if (!(n2 > 1e-12)) return false;
  for (int c = 0; c < 3; ++c) c2[c] /= n2;
  c3[0] = c1[1] * c2[2] - c1[2] * c2[1];
  c3[1] = c1[2] * c2[0] - c1[0] * c2[2];
  c3[2] = c1[0] * c2[1] - c1[1] * c2[0];
  return true;
}

template <typename T>
FArgs<T> field_args(const mmx_ctx* ctx, const Group& G, uint32_t terms) {
  FArgs<T> a{};
  a.nx = G.nx; a.ny = G.ny; a.nz = G.nz; a.N = G.N; a.Sy = G.Sy; a.Kx = G.Kx; a.hx = G.hx;
  a.L = G.L; a.xone = G.xone;
  const double mu0Ms = kMu0 * G.mat.Ms;
  for (int ax = 0; ax < 3; ++ax) {
    a.pbc[ax] = G.g.pbc[ax];
    a.nax[ax] = G.g.n[ax];
    const double d = G.g.cell[ax];
    a.idd2[ax] = (T)(1.0 / (d * d));
    a.ih2[ax] = (T)(1.0 / (2.0 * d));
    a.hd[ax] = (T)d;
  }
  a.cex = (T)(2.0 * G.mat.A / mu0Ms);
  a.cdmi = (T)(2.0 * G.mat.D / mu0Ms);
  a.kbc = (T)(G.mat.A != 0 ? G.mat.D / (2.0 * G.mat.A) : 0.0);
  a.can = (T)(2.0 * G.mat.Ku / mu0Ms);
  double un = std::sqrt(G.mat.u[0] * G.mat.u[0] + G.mat.u[1] * G.mat.u[1] + G.mat.u[2] * G.mat.u[2]);
  if (un == 0) un = 1;
  for (int c = 0; c < 3; ++c) {
    a.u[c] = (T)(G.mat.u[c] / un);
    a.hz[c] = (T)(G.B[c] / kMu0);
  }
  a.gpm = (T)(kGamma0 / (1.0 + G.mat.alpha * G.mat.alpha) * kMu0);
  a.alpha = (T)G.mat.alpha;
  unsigned t = terms;
  if (G.mat.Ku == 0 && G.cKu.empty()) t &= ~T_ANIS;
  if (G.mat.D == 0 && G.cD.empty()) t &= ~T_DMI;
  if (G.ext.Db == 0) t &= ~T_DMI_BULK;
  if (G.ext.Kc1 == 0 && G.ext.Kc2 == 0) t &= ~T_CUBIC;
  if (G.ext.rkky == 0 || G.nz < 2) t &= ~T_RKKY;
  a.terms = t;
  a.cbulk = (T)(-2.0 * G.ext.Db / mu0Ms);
  a.kbb = (T)(G.mat.A != 0 ? G.ext.Db / (2.0 * G.mat.A) : 0.0);
  a.kc1h = (T)(2.0 * G.ext.Kc1 / mu0Ms);
  a.kc2h = (T)(2.0 * G.ext.Kc2 / mu0Ms);
  a.kc1 = (T)G.ext.Kc1;
  a.kc2 = (T)G.ext.Kc2;
  a.ecub = -2.0 / mu0Ms;
  {
    double c1[3], c2[3], c3[3];
    cubic_axes(G.ext, c1, c2, c3);
    for (int c = 0; c < 3; ++c) {
      a.cax[0][c] = (T)c1[c];
      a.cax[1][c] = (T)c2[c];
      a.cax[2][c] = (T)c3[c];
    }
  }
  a.crkky = (T)(G.ext.rkky / (mu0Ms * G.g.cell[2]));
  a.rkz0 = G.ext.rkky_z[0];
  a.rkz1 = G.ext.rkky_z[1];
  a.Acell = G.acell_on ? G.Acell.as<T>() : nullptr;
  // per-cell Ms, alpha, Ku, D
  a.c2ms = (T)(2.0 / mu0Ms);
  a.Agrp = (T)G.mat.A;
  a.sigunit = 2.0 * kKB / (kMu0 * kMu0 * G.mat.Ms * (G.g.cell[0] * G.g.cell[1] * G.g.cell[2]) * kGamma0);
  if (G.cells_on) {
    const bool ms = !G.cMs.empty(), al = !G.calpha.empty() || ms;
    a.msr = ms ? G.cell[0].as<T>() : nullptr;
    a.mgi = ms ? G.cell[1].as<T>() : nullptr;
    a.gpc = !G.calpha.empty() ? G.cell[2].as<T>() : nullptr;
    a.alc = !G.calpha.empty() ? G.cell[3].as<T>() : nullptr;
    a.sgc = al ? G.cell[4].as<T>() : nullptr;
    a.kuc = !G.cKu.empty() ? G.cell[5].as<T>() : nullptr;
    a.dmc = !G.cD.empty() ? G.cell[6].as<T>() : nullptr;
  }
  a.exs = (T)(2.0 / mu0Ms);
  a.dhalf = (T)(0.5 * G.mat.D);
  a.dbhalf = (T)(0.5 * G.ext.Db);
  const double V = G.g.cell[0] * G.g.cell[1] * G.g.cell[2];
  a.Trep = G.Trep.as<double>();
  a.seeds = G.seeds.as<uint64_t>();
  a.sig2pref = 2.0 * G.mat.alpha * kKB / (kMu0 * kMu0 * G.mat.Ms * V * kGamma0);
  a.S = G.S.as<cpx<T>>();
  a.plan = G.plan_xi;  // inverse transform: full input
  a.tw = G.tw_x.as<cpx<T>>();
  a.wpost = G.wpost.as<cpx<T>>();
  if ((t & T_STT) && G.jrep_on && G.stt_P != 0) {
    const double d = G.g.cell[2] * G.nz;  // free-layer thickness
    a.Jrep = G.Jrep.as<double>();
    a.stt_c = kHbar / (kMu0 * kQe * G.mat.Ms * d);
    for (int c = 0; c < 3; ++c) a.sttp[c] = (T)G.stt_p[c];
    a.stt_P = (T)G.stt_P;
    a.stt_L2 = (T)(G.stt_lambda * G.stt_lambda);
    a.stt_e2 = (T)G.stt_eps2;
  } else {
    a.terms &= ~(unsigned)T_STT;
  }
  a.noprec = ctx->noprec;
  a.nblk_out = G.nblk_dev.as<int>();
  a.nonfinite = ctx->nfflag.as<int>();
  a.rot = ctx->rot;
  if (ctx->refill) {
    a.tgen = G.tgen.as<int>();
    a.tstart = G.tstart.as<unsigned long long>();
  }
  return a;
}

// Heun stages of FP32 grids whose x half-length is 16, 32, 64, 96, 128 or 256
// (4 x 4, 4 x 8, 8 x 8, 8 x 12, 8 x 16, 16 x 16): the register row kernel (mode
// FM_HEUN1 / FM_HEUN2) or its forward-only part (mode -1, the half spectrum
// of the state a.m); false if not applicable.
template <typename T>
bool launch_rows_reg(mmx_ctx* ctx, Group& G, FArgs<T>& a, int mode) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    if (!(mode == FM_HEUN1 || mode == FM_HEUN2 || mode == -1) || !(a.terms & T_DEMAG)) return false;
    if (mode != -1 && !a.fwd) return false;
    if (G.xone || a.hext || a.hd_out || G.cells_on) return false;
    // the register row kernels take neither the further field terms nor the
    // bulk-DMI edge ghosts
    if ((a.terms & (T_DMI_BULK | T_CUBIC | T_RKKY)) || a.kbb != 0 || a.Acell) return false;
    // cell offsets within a replica are formed in 32 bits
    if ((unsigned long long)3 * G.N * sizeof(float) >= (1ull << 32)) return false;
    hipStream_t s = ctx->stream;
    // variants: [stage][rotation][spin-transfer]
    using RowKernel = void (*)(FArgs<float>);
    auto go = [&](const RowKernel (&k)[2][2][2], auto kf, int rpw) {
      const int gx = (G.ny + rpw - 1) / rpw;
      const dim3 grid(gx, G.nz, G.R);
      if (mode == -1) {
        kf<<<grid, 64, 0, s>>>(a);
        return true;
      }
      G.nblk_last = gx * G.nz;
      const RowKernel kern = k[mode == FM_HEUN1 ? 0 : 1][a.rot ? 1 : 0][(a.terms & T_STT) ? 1 : 0];
      const size_t lds = (size_t)rpw * rows_lds_stride(G.nx) * sizeof(cpx<float>);
      kern<<<grid, 64, lds, s>>>(a);
      return true;
    };
#define MMX_ROWS_V(N1, N2, M) \
  {{k_rows_reg<float, N1, N2, M, false, false>, k_rows_reg<float, N1, N2, M, false, true>}, \
   {k_rows_reg<float, N1, N2, M, true, false>, k_rows_reg<float, N1, N2, M, true, true>}}
#define MMX_ROWS(N1, N2, RPW)                                                                 \
  [&]() {                                                                                   \
    static const RowKernel k[2][2][2] = {MMX_ROWS_V(N1, N2, FM_HEUN1),                      \
                                         MMX_ROWS_V(N1, N2, FM_HEUN2)};                     \
    return go(k, k_rows_fwd<float, N1, N2>, RPW);                                           \
  }()
    switch (G.hx) {
      case 16: return MMX_ROWS(4, 4, 16);
      case 32: return MMX_ROWS(4, 8, 16);
      case 64: return MMX_ROWS(8, 8, 8);
      case 96: return MMX_ROWS(8, 12, 8);
      case 128: return MMX_ROWS(8, 16, 8);
      case 256: return MMX_ROWS(16, 16, 4);
      default: return false;
    }
#undef MMX_ROWS
#undef MMX_ROWS_V
  }
}

template <typename T>
mmx_status launch_fields(mmx_ctx* ctx, Group& G, FArgs<T>& a, int mode) {
  static const char* kname_reg[] = {"", "", "k_fields_heun1", "k_fields_heun2"};
  if (mode == FM_HEUN1 || mode == FM_HEUN2) {
    ProfScope ps(ctx->prof, kname_reg[mode], ctx->stream);
    if (launch_rows_reg<T>(ctx, G, a, mode)) {
      HIP_TRY(hipGetLastError());
      return MMX_OK;
    }
    ps.cancel();
  }
  G.nblk_last = G.nblk;
  dim3 grid((G.ny + G.L - 1) / G.L, G.nz, G.R);
  const size_t lds = (a.terms & T_DEMAG) ? (2 * (size_t)3 * G.L * G.hx + G.hx) * cpxb<T>() : 0;
  hipStream_t s = ctx->stream;
  static const char* kname[] = {"k_fields_field", "k_fields_torque", "k_fields_heun1",
                                 "k_fields_heun2", "k_fields_rkk", "k_fields_rk7",
                                 "k_fields_energy"};
  ProfScope ps(ctx->prof, kname[mode], s);
  switch (mode) {
    case FM_FIELD: k_fields<T, FM_FIELD><<<grid, kBlock, lds, s>>>(a); break;
    case FM_TORQUE: k_fields<T, FM_TORQUE><<<grid, kBlock, lds, s>>>(a); break;
    case FM_HEUN1: k_fields<T, FM_HEUN1><<<grid, kBlock, lds, s>>>(a); break;
    case FM_HEUN2: k_fields<T, FM_HEUN2><<<grid, kBlock, lds, s>>>(a); break;
    case FM_RKK: k_fields<T, FM_RKK><<<grid, kBlock, lds, s>>>(a); break;
    case FM_RK7: k_fields<T, FM_RK7><<<grid, kBlock, lds, s>>>(a); break;
    default: k_fields<T, FM_ENERGY><<<grid, kBlock, lds, s>>>(a); break;
  }
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

// Register-resident column convolution for FP32 films whose padded y length
// is 64, 128 or 256 (split 8 x 8, 8 x 16, 16 x 16); false: not applicable.
template <typename T>
bool launch_yconv_reg(const Group& G, const YArgs<T>& y, hipStream_t s) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    const bool prune = G.plan_yf.prune != 0;
    auto go = [&](auto kern, int NC) {
      dim3 grid((G.Kx + NC - 1) / NC, 1, G.R);
      kern<<<grid, 64, 0, s>>>(y);
      return true;
    };
    switch (G.Py) {
      case 64: return prune ? go(k_yconv_reg<float, 8, 8, true>, 8)
                            : go(k_yconv_reg<float, 8, 8, false>, 8);
      case 128: return prune ? go(k_yconv_reg<float, 8, 16, true>, 8)
                             : go(k_yconv_reg<float, 8, 16, false>, 8);
      case 256: return prune ? go(k_yconv_reg<float, 16, 16, true>, 4)
                             : go(k_yconv_reg<float, 16, 16, false>, 4);
      default: return false;
    }
  }
}

// stage combine m + dt sum_j c_j k_j (optionally normalised) fused with the x
// forward transform of the demag convolution when `demag` is set
template <typename T>
mmx_status launch_xfwd(mmx_ctx* ctx, Group& G, const T* mbase, const Combine& cb, bool demag,
                       const double* dtdev, double dth, const int* done) {
  hipStream_t s = ctx->stream;
  XArgs<T> x{};
  x.m = mbase;
  x.ncoef = cb.ncoef;
  for (int j = 0; j < cb.ncoef; ++j) {
    x.kk[j] = G.k[cb.kidx[j]].as<T>();
    x.coef[j] = (T)cb.coef[j];
  }
  x.dtdev = dtdev;
  x.dth = dth;
  x.mout = reinterpret_cast<T*>(cb.mout);
  x.normalise = cb.normalise;
  x.nonfinite = (cb.normalise && cb.check_finite) ? ctx->nfflag.as<int>() : nullptr;
  x.msr = (G.cells_on && !G.cMs.empty()) ? G.cell[0].as<T>() : nullptr;
  x.do_fft = demag ? 1 : 0;
  x.S = G.S.as<cpx<T>>();
  x.tw = G.tw_x.as<cpx<T>>();
  x.wpost = G.wpost.as<cpx<T>>();
  x.plan = G.plan_x;
  x.nx = G.nx; x.ny = G.ny; x.nz = G.nz; x.N = G.N; x.Sy = G.Sy; x.Kx = G.Kx; x.hx = G.hx;
  x.L = G.L; x.xone = G.xone;
  x.done = done;
  dim3 grid((G.ny + G.L - 1) / G.L, G.nz, G.R);
  const size_t lds = demag ? (2 * (size_t)3 * G.L * G.hx + 2 * G.hx + 1) * cpxb<T>() : 0;
  ProfScope ps(ctx->prof, demag ? "k_xfwd" : "k_combine", s);
  k_xfwd<T><<<grid, kBlock, lds, s>>>(x);
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

// Switching check of the previous Heun step, done by the register column
// kernel of the next step's first field evaluation.
struct SwitchFold {
  const double* part = nullptr;
  double* tsw = nullptr;
  const int* nblk = nullptr;  // device: written by the corrector
  int N = 1;
  double dt = 0;
  unsigned long long step = 0;
  const unsigned long long* stepdev = nullptr;
};

// whether launch_yconv_reg takes the 2-D column pass of group G
template <typename T>
bool yconv_reg_applies(const Group& G) {
  return std::is_same<T, float>::value && !G.is3d && (G.Py == 64 || G.Py == 128 || G.Py == 256);
}

// whether the separate z pass of the 3-D group G runs in registers (few
// layers whose fused y-z workgroup does not fit the LDS)
template <typename T>
bool zconv_reg_applies(const Group& G) { return G.is3d && G.nz <= 8 && !yz_applies<T>(G); }

// Register y pass of a 3-D FP32 group (Py = 64, 128, 192, 256 or 512, split
// 8 x 8, 8 x 16, 8 x 24, 16 x 16, 16 x 32); false: not applicable.
template <typename T>
bool launch_ypass_reg(const Group& G, const YArgs<T>& y, bool inv, hipStream_t s) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    if (!G.is3d || (size_t)G.Py * G.Kx >= (1u << 27)) return false;
    const bool prune = G.plan_yf.prune != 0;
    auto go = [&](auto kf, auto kfp, auto ki, auto kip, int NC) {
      const dim3 grid((G.Kx + NC - 1) / NC, 3 * G.nz, G.R);
      if (!inv) {
        if (prune) kfp<<<grid, 64, 0, s>>>(y); else kf<<<grid, 64, 0, s>>>(y);
      } else {
        if (prune) kip<<<grid, 64, 0, s>>>(y); else ki<<<grid, 64, 0, s>>>(y);
      }
      return true;
    };
#define MMX_YP(N1, N2)                                                                          \
  go(k_ypass_reg<float, N1, N2, false, false>, k_ypass_reg<float, N1, N2, false, true>,         \
     k_ypass_reg<float, N1, N2, true, false>, k_ypass_reg<float, N1, N2, true, true>, 64 / N1)
    switch (G.Py) {
      case 64: return MMX_YP(8, 8);
      case 128: return MMX_YP(8, 16);
      case 192: return MMX_YP(8, 24);
      case 256: return MMX_YP(16, 16);
      case 512: return MMX_YP(16, 32);
      default: return false;
    }
#undef MMX_YP
  }
}

// Register z pass with the tensor product of a 3-D FP32 group (Pz = 32, 64
// or 128, split 4 x 8, 8 x 8, 8 x 16); false: not applicable.
template <typename T>
bool launch_zline_reg(const Group& G, const YArgs<T>& z, hipStream_t s) {
  if constexpr (!std::is_same<T, float>::value) {
    return false;
  } else {
    // 32-bit offsets within a replica's spectrum
    if (!G.is3d || (size_t)3 * G.nz * G.Sy * G.Kx * sizeof(cpx<float>) >= (1ull << 31))
      return false;
    const bool prune = G.plan_zf.prune != 0;
    auto go = [&](auto k, auto kp, int NC) {
      const dim3 grid((G.Kx + NC - 1) / NC, G.Py, G.R);
      if (prune) kp<<<grid, 64, 0, s>>>(z); else k<<<grid, 64, 0, s>>>(z);
      return true;
    };
    switch (G.Pz) {
      case 32: return go(k_zline_reg<float, 4, 8, false>, k_zline_reg<float, 4, 8, true>, 16);
      case 64: return go(k_zline_reg<float, 8, 8, false>, k_zline_reg<float, 8, 8, true>, 8);
      case 128: return go(k_zline_reg<float, 8, 16, false>, k_zline_reg<float, 8, 16, true>, 8);
      default: return false;
    }
  }
}

// whether the separate register y passes exist for this group
template <typename T>
bool ypass_reg_applies(const Group& G) {
  return std::is_same<T, float>::value && G.is3d &&
         (G.Py == 64 || G.Py == 128 || G.Py == 192 || G.Py == 256 || G.Py == 512) &&
         (size_t)G.Py * G.Kx < (1u << 27);
}

// m: group-local base pointer of the state used for fields.
template <typename T>
mmx_status eval_group(mmx_ctx* ctx, Group& G, const T* mbase, const Combine& cb, const Epilogue& ep,
                      uint64_t step, double dt_th, const double* dtdev, double dth,
                      const int* done, uint32_t terms_override = 0xFFFFFFFFu,
                      bool spec_ready = false, const SwitchFold* sw = nullptr) {
  uint32_t terms = (terms_override == 0xFFFFFFFFu) ? ctx->terms : terms_override;
  const bool demag = (terms & MMX_DEMAG) != 0;
  if (demag && !G.demag_built) return fail(MMX_ESTATE, "mmx_build_demag has not been called");
  if (spec_ready && cb.mout) return fail(MMX_ESTATE, "spectrum of a combined state");
  hipStream_t s = ctx->stream;
  const T* mfield = mbase;
  // stage 1: combine (+ x forward transform, unless the previous epilogue
  // already wrote the half spectrum of mbase)
  const bool need_fft = demag && !spec_ready;
  if (need_fft || cb.mout) {
    MMX_TRY(launch_xfwd<T>(ctx, G, mbase, cb, need_fft, dtdev, dth, done));
    if (cb.mout) mfield = reinterpret_cast<const T*>(cb.mout);
  }
  // stage 2: y (and z) passes with the tensor product
  if (demag) {
    YArgs<T> y{};
    y.S = G.S.as<cpx<T>>();
    y.Nt = G.Nt.as<T>();
    y.ny = G.ny; y.Py = G.Py; y.Kx = G.Kx; y.Ty = G.Ty; y.Sy = G.Sy; y.nz = G.nz; y.Pz = G.Pz;
    y.Tz = G.Tz;
    y.done = done;
    if (!G.is3d) {
      y.W = G.Wy;
      y.tw = G.tw_y.as<cpx<T>>();
      y.pf = G.plan_yf;
      y.pi = G.plan_yi;
      if (sw) {
        y.sw_part = sw->part;
        y.sw_tsw = sw->tsw;
        y.sw_nblk = sw->nblk;
        y.sw_N = sw->N;
        y.sw_dt = sw->dt;
        y.sw_step = sw->step;
        y.sw_stepdev = sw->stepdev;
      }
      ProfScope ps(ctx->prof, "k_yconv", s);
      if (!launch_yconv_reg<T>(G, y, s)) {
        if (sw) return fail(MMX_ESTATE, "switching check folded into a column kernel without it");
        dim3 grid((G.Kx + G.Wy - 1) / G.Wy, 1, G.R);
        k_yconv<T><<<grid, kBlock, (2 * (size_t)3 * G.Wy * G.Py + G.Py) * cpxb<T>(), s>>>(y);
      }
      HIP_TRY(hipGetLastError());
    } else if (yz_applies<T>(G) && !(G.yz_split && ypass_reg_applies<T>(G))) {
      y.W = G.Wz;
      y.tw = G.tw_y.as<cpx<T>>();
      y.twz = G.tw_z.as<cpx<T>>();
      y.pf = G.plan_yf;
      y.pi = G.plan_yi;
      dim3 g((G.Kx + G.Wz - 1) / G.Wz, 1, G.R);
      const size_t lds = lds_yz<T>(G, G.Wz);
      ProfScope ps(ctx->prof, "k_yzconv", s);
      if (G.nz <= 2)
        k_yzconv<T, 2><<<g, kBlock, lds, s>>>(y);
      else if (G.nz <= 4)
        k_yzconv<T, 4><<<g, kBlock, lds, s>>>(y);
      else
        k_yzconv<T, 8><<<g, kBlock, lds, s>>>(y);
      HIP_TRY(hipGetLastError());
    } else {
      y.W = G.Wy;
      y.tw = G.tw_y.as<cpx<T>>();
      y.pf = G.plan_yf;
      y.pi = G.plan_yi;
      dim3 gy((G.Kx + G.Wy - 1) / G.Wy, 3 * G.nz, G.R);
      const size_t ldy = lds_ycols<T>(true, G.Wy, G.Py);
      {
        ProfScope ps(ctx->prof, "k_ypass_fwd", s);
        if (!launch_ypass_reg<T>(G, y, false, s)) k_ypass<T, false><<<gy, kBlock, ldy, s>>>(y);
      }
      HIP_TRY(hipGetLastError());
      YArgs<T> zz = y;
      zz.W = G.Wz;
      zz.tw = G.tw_z.as<cpx<T>>();
      zz.twz = G.tw_z.as<cpx<T>>();
      zz.pf = G.plan_zf;
      zz.pi = G.plan_zi;
      {
        ProfScope psz(ctx->prof, "k_zconv", s);
        if (G.nz <= 8 && G.is3d) {
          dim3 gz((G.Py * G.Kx + kBlock - 1) / kBlock, G.R);
          if (G.nz <= 2)
            k_zconv_reg<T, 2><<<gz, kBlock, 0, s>>>(zz);
          else if (G.nz <= 4)
            k_zconv_reg<T, 4><<<gz, kBlock, 0, s>>>(zz);
          else
            k_zconv_reg<T, 8><<<gz, kBlock, 0, s>>>(zz);
        } else if (!launch_zline_reg<T>(G, zz, s)) {
          dim3 gz((G.Kx + G.Wz - 1) / G.Wz, G.Py, G.R);
          k_zconv<T><<<gz, kBlock, (2 * (size_t)3 * G.Wz * G.Pz + G.Pz) * cpxb<T>(), s>>>(zz);
        }
      }
      HIP_TRY(hipGetLastError());
      {
        ProfScope ps(ctx->prof, "k_ypass_inv", s);
        if (!launch_ypass_reg<T>(G, y, true, s)) k_ypass<T, true><<<gy, kBlock, ldy, s>>>(y);
      }
      HIP_TRY(hipGetLastError());
    }
  }
  // stage 3: inverse x transform + local fields + epilogue
  FArgs<T> a = field_args<T>(ctx, G, terms);
  a.stepdev = ctx->cur_stepdev;
  a.m = mfield;
  a.step = step;
  a.dt_th = dt_th;
  a.dtdev = dtdev;
  a.dth = dth;
  a.done = done;
  a.out = reinterpret_cast<T*>(ep.out);
  a.k1 = reinterpret_cast<T*>(ep.k1);
  a.m0 = reinterpret_cast<const T*>(ep.m0);
  a.mout = reinterpret_cast<T*>(ep.mout);
  for (int j = 0; j < 7; ++j) a.e[j] = ep.e[j];
  for (int j = 0; j < 6; ++j) a.kk[j] = G.k[j].as<T>();
  a.fwd = ep.fwd;
  for (int j = 0; j < 6; ++j) a.cn[j] = (T)ep.cn[j];
  a.cnext = ep.cnext;
  a.cstage = ep.cstage;
  a.mnext = reinterpret_cast<T*>(ep.mnext);
  a.plan_f = G.plan_x;
  a.st = ctx->st.as<RkState>();
  a.partial = G.partial.as<double>();
  if (!demag && ctx->hext) {
    a.hext = ctx->hext;
    a.hext_scale = (T)ctx->hext_scale;
    a.hext_mz = (T)ctx->hext_mz;
  }
  if (demag) a.hd_out = reinterpret_cast<T*>(ctx->hd_out);
  return launch_fields<T>(ctx, G, a, ep.mode);
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4) coefficients (Dormand & Prince 1980)
// ---------------------------------------------------------------------------
const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
const double DP_B4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                         187.0 / 2100, 1.0 / 40};

// learned-demag hook of an RK45 attempt: stages 2-6 take the demag field from
// `field` (written to h, applied as scale * h + (0, 0, mz m_z)); stage 7 uses
// the exact convolution and also stores it in hd
struct StageHook {
  virtual mmx_status field(mmx_ctx* ctx, Group& G, const float* m) const = 0;
  float* h = nullptr;
  double scale = 0, mz = 0;
  void* hd = nullptr;
};

// validates the arguments, allocates the stage buffers and uploads the initial
// controller state (dt clamped to dt_max, final step landing on t_end)
template <typename T>
mmx_status rk_begin(mmx_ctx* ctx, double t0, double t_end, double tol, double dt0,
                    const double* replay, int64_t n_replay, RkState& h) {
  if (ctx->terms & MMX_THERMAL) return fail(MMX_EUNSUP, "thermal field with RK45");
  if (!(t_end > t0)) return fail(MMX_EINVAL, "t_end must exceed t0");
  if (!(tol > 0) && !replay) return fail(MMX_EINVAL, "tol must be > 0");
  if (replay && n_replay < 1) return fail(MMX_EINVAL, "empty dt replay");
  if (replay && n_replay > kDtsCap)
    return fail(MMX_EINVAL, "dt replay longer than " + std::to_string(kDtsCap) + " steps");
  for (auto& g : ctx->groups) MMX_TRY(ensure_rk_buffers<T>(*g));
  hipStream_t s = ctx->stream;
  // controller state
  h = RkState{};
  h.t = t0;
  h.t_end = t_end;
  h.tol = tol;
  h.dt_max = 1e-11;
  h.dt_min = 1e-20;
  if (replay) {
    h.dt = replay[0];
    h.n_replay = n_replay;
  } else {
    h.dt = std::min(dt0, h.dt_max);
    h.dt_prop = h.dt;
    h.final_flag = (t0 + h.dt >= t_end) ? 1 : 0;
    if (h.final_flag) h.dt = t_end - t0;
  }
  HIP_TRY(hipMemcpyAsync(ctx->st.p, &h, sizeof(RkState), hipMemcpyHostToDevice, s));
  if (replay)
    HIP_TRY(hipMemcpyAsync(ctx->replay.p, replay, n_replay * sizeof(double),
                           hipMemcpyHostToDevice, s));
  return MMX_OK;
}

// stages 2..7 of one Dormand-Prince attempt for group G from its state mg; the
// stage-7 evaluation also yields the embedded error estimate (e = b5 - b4)
template <typename T>
mmx_status rk_stages(mmx_ctx* ctx, Group& G, T* mg, const double e[7], const StageHook* hook) {
  RkState* st = ctx->st.as<RkState>();
  const int* done = &st->done;
  const double* dtdev = &st->dt;
  // Without learned stages every stage's epilogue also forms the next
  // stage's state and its x transform (the states alternate between two
  // buffers, since a stage still reads its own state's neighbours), so only
  // the second stage needs the separate combine pass.
  const bool chain = hook == nullptr && (ctx->terms & MMX_DEMAG);
  void* state[7] = {nullptr, G.ms.p, G.ms2.p, G.ms.p, G.ms2.p, G.ms.p, G.m7.p};
  for (int sidx = 1; sidx < 7; ++sidx) {
    Combine cb;
    for (int j = 0; j < sidx; ++j) {
      const double c = DP_A[sidx][j];
      if (c == 0.0) continue;
      cb.coef[cb.ncoef] = c;
      cb.kidx[cb.ncoef] = j;
      cb.ncoef++;
    }
    Epilogue ep;
    if (sidx < 6) {
      cb.mout = chain ? state[sidx] : G.ms.p;
      ep.mode = FM_RKK;
      ep.out = G.k[sidx].p;
      if (chain) {
        ep.fwd = 1;
        ep.m0 = mg;
        for (int j = 0; j <= sidx; ++j) ep.cn[j] = DP_A[sidx + 1][j];
        ep.cstage = sidx;
        ep.cnext = (sidx + 1 == 6) ? 2 : 1;
        ep.mnext = state[sidx + 1];
      }
    } else {
      cb.mout = G.m7.p;
      cb.normalise = 1;
      ep.mode = FM_RK7;
      ep.out = G.k[6].p;
      for (int j = 0; j < 7; ++j) ep.e[j] = e[j];
    }
    if (hook && sidx < 6) {
      // learned demag: combine, network field at the stage state, local terms
      MMX_TRY(launch_xfwd<T>(ctx, G, mg, cb, false, dtdev, 0.0, done));
      MMX_TRY(hook->field(ctx, G, reinterpret_cast<const float*>(cb.mout)));  // FP32 only
      ctx->hext = hook->h;
      ctx->hext_scale = hook->scale;
      ctx->hext_mz = hook->mz;
      const mmx_status r = eval_group<T>(ctx, G, reinterpret_cast<const T*>(cb.mout), Combine{}, ep,
                                         0, 1.0, dtdev, 0.0, done, ctx->terms & ~MMX_DEMAG);
      ctx->hext = nullptr;
      MMX_TRY(r);
    } else if (chain && sidx > 1) {
      // state and half spectrum written by the previous stage's epilogue
      ctx->hd_out = nullptr;
      MMX_TRY(eval_group<T>(ctx, G, reinterpret_cast<const T*>(state[sidx]), Combine{}, ep, 0, 1.0,
                            dtdev, 0.0, done, 0xFFFFFFFFu, true));
    } else {
      ctx->hd_out = (hook && sidx == 6) ? hook->hd : nullptr;
      const mmx_status r = eval_group<T>(ctx, G, mg, cb, ep, 0, 1.0, dtdev, 0.0, done);
      ctx->hd_out = nullptr;
      MMX_TRY(r);
    }
  }
  return MMX_OK;
}

// controller decision, then m <- m7 and k1 <- k7 if the attempt was accepted
template <typename T>
mmx_status rk_finish(mmx_ctx* ctx, T* mb, const double* replay) {
  RkState* st = ctx->st.as<RkState>();
  {
    ProfScope psc(ctx->prof, "k_rk_controller", ctx->stream);
    k_rk_controller<<<1, 1, 0, ctx->stream>>>(st, replay, ctx->dts.as<double>(), ctx->dts_cap);
    HIP_TRY(hipGetLastError());
  }
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    const size_t n = (size_t)G.R * 3 * G.N;
    const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    ProfScope ps(ctx->prof, "k_rk_commit", ctx->stream);
    k_rk_commit<T><<<nb, 256, 0, ctx->stream>>>(st, mb + G.off, G.m7.as<T>(), G.k[0].as<T>(),
                                               G.k[6].as<T>(), n);
    HIP_TRY(hipGetLastError());
  }
  return MMX_OK;
}

// k1 = f(m) for every group (first stage; later steps reuse k7 of the last accepted one)
template <typename T>
mmx_status rk_first_stage(mmx_ctx* ctx, T* mb) {
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    Epilogue ep;
    ep.mode = FM_RKK;
    ep.out = G.k[0].p;
    MMX_TRY(eval_group<T>(ctx, G, mb + G.off, Combine{}, ep, 0, 1.0, nullptr, 0.0, nullptr));
  }
  return MMX_OK;
}

template <typename T>
mmx_status rk45_impl(mmx_ctx* ctx, void* m, double t0, double t_end, double tol, double dt0,
                     const double* replay, int64_t n_replay, void* trace, int64_t cap,
                     mmx_rk_stats* stats, double* dt_prop = nullptr, bool resume = false) {
  RkState h;
  MMX_TRY(rk_begin<T>(ctx, t0, t_end, tol, dt0, replay, n_replay, h));
  ctx->rk_valid = 0;
  hipStream_t s = ctx->stream;
  RkState* st = ctx->st.as<RkState>();
  T* mb = reinterpret_cast<T*>(m);
  // trace helpers
  int R_total = 0;
  for (auto& g : ctx->groups) R_total += g->R;
  auto energy_into_trace = [&](int force0) -> mmx_status {
    int roff = 0;
    for (auto& gp : ctx->groups) {
      Group& G = *gp;
      Epilogue ep;
      ep.mode = FM_ENERGY;
      MMX_TRY(eval_group<T>(ctx, G, mb + G.off, Combine{}, ep, 0, 1.0, nullptr, 0.0, nullptr));
      const double V = G.g.cell[0] * G.g.cell[1] * G.g.cell[2];
      const double cq = -0.5 * kMu0 * G.mat.Ms * V, cz = -kMu0 * G.mat.Ms * V;
      k_energy_reduce<<<(G.R + 63) / 64, 64, 0, ctx->stream>>>(G.partial.as<double>(), G.nblk, G.R, cq, cz,
                                                      ctx->Etmp.as<double>() + (size_t)roff * 6);
      HIP_TRY(hipGetLastError());
      roff += G.R;
    }
    k_trace_store<<<1, 1, 0, ctx->stream>>>(st, ctx->Etmp.as<double>(), R_total, (double*)trace, cap, force0);
    HIP_TRY(hipGetLastError());
    return MMX_OK;
  };
  // a continuation starts from the saved first-same-as-last slope in k[0]
  if (!resume) MMX_TRY(rk_first_stage<T>(ctx, mb));
  if (trace) MMX_TRY(energy_into_trace(1));
  double e[7];
  for (int j = 0; j < 7; ++j) e[j] = (j < 6 ? DP_A[6][j] : 0.0) - DP_B4[j];
  auto one_step = [&]() -> mmx_status {
    for (auto& gp : ctx->groups) MMX_TRY(rk_stages<T>(ctx, *gp, mb + gp->off, e, nullptr));
    MMX_TRY(rk_finish<T>(ctx, mb, replay ? ctx->replay.as<double>() : nullptr));
    if (trace) MMX_TRY(energy_into_trace(0));
    return MMX_OK;
  };
  const int chunk = 16;  // attempts per host poll of the controller state
  if (ctx->prof.on) {
    for (;;) {
      for (int i = 0; i < chunk; ++i) MMX_TRY(one_step());
      HIP_TRY(hipMemcpyAsync(&h, ctx->st.p, sizeof(RkState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (h.done) break;
    }
  } else {
    // the attempt sequence is static (dt, t and acceptance live on the
    // device), so `chunk` attempts are captured once (and kept for later
    // calls with the same arrays and configuration) and replayed until done
    MMX_TRY(ensure_graph_stream(ctx));
    hipStream_t cs = ctx->cap_stream;
    GraphKey key;
    key.epoch = ctx->epoch;
    key.p[0] = m;
    key.p[1] = trace;
    key.p[2] = replay ? ctx->replay.p : nullptr;
    key.p[3] = ctx->dts.p;
    key.p[4] = ctx->st.p;
    key.p[5] = ctx->Etmp.p;
    key.i[0] = cap;
    key.i[1] = ctx->dts_cap;
    GraphSet& gs = ctx->rk_graphs;
    if (!gs.valid || !(gs.key == key)) {
      HIP_TRY(hipStreamSynchronize(cs));
      gs.clear();
      gs.exec.assign(1, nullptr);
      gs.key = key;
      gs.valid = true;
      MMX_TRY(capture_graph(ctx, [&]() -> mmx_status {
        for (int i = 0; i < chunk; ++i) MMX_TRY(one_step());
        return MMX_OK;
      }, &gs.exec[0]));
    }
    HIP_TRY(hipEventRecord(ctx->ev_user, s));
    HIP_TRY(hipStreamWaitEvent(cs, ctx->ev_user, 0));
    for (;;) {
      HIP_TRY(hipGraphLaunch(gs.exec[0], cs));
      HIP_TRY(hipMemcpyAsync(&h, ctx->st.p, sizeof(RkState), hipMemcpyDeviceToHost, cs));
      HIP_TRY(hipStreamSynchronize(cs));
      if (h.done) break;
    }
  }
  ctx->last_accepted = h.accepted;
  if (dt_prop) *dt_prop = h.dt_prop;
  if (!replay && !h.dtmin_hit) {
    ctx->rk_last = h;
    ctx->rk_valid = 1;
    ctx->rk_epoch = ctx->epoch;
  }
  if (stats) {
    stats->t = h.t;
    stats->dt = h.dt;
    stats->err = h.last_err;
    stats->accepted = h.accepted;
    stats->rejected = h.rejected;
  }
  if (h.dtmin_hit) {
    // every attempt down to dt_min failed on a non-finite error estimate: the
    // state (or its derivative) is not finite, not merely too stiff
    if (!(h.last_err == h.last_err))
      return fail(MMX_ENONFINITE, "non-finite state or derivative in RK45 (step size fell to dt_min)");
    return fail(MMX_EDTMIN, "step size fell below dt_min");
  }
  return MMX_OK;
}

mmx_status ensure_graph_stream(mmx_ctx* ctx) {
  if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  if (!ctx->ev_user) HIP_TRY(hipEventCreateWithFlags(&ctx->ev_user, hipEventDisableTiming));
  if (!ctx->ev_cap) HIP_TRY(hipEventCreateWithFlags(&ctx->ev_cap, hipEventDisableTiming));
  return MMX_OK;
}

// ---------------------------------------------------------------------------
// replica-resident Heun path (2-D films whose half spectrum fits in LDS)
// ---------------------------------------------------------------------------
struct FusedTiles {
  int C = 0, W = 0, nch = 0;
  size_t lds = 0;
  bool ok = false;
};

template <typename T>
FusedTiles fused_tiles(const mmx_ctx* ctx, const Group& G) {
  FusedTiles ft;
  if (G.nz != 1 || G.xone || G.nx > kFusedBlock) return ft;
  int C = 1;
  while (2 * C <= G.ny && 2 * C * G.nx <= kFusedBlock) C *= 2;
  const int nch = (G.ny + C - 1) / C;
  if (nch > kFusedMaxChunks) return ft;
  int W = std::max(1, std::min(G.Kx, C * G.hx / G.Py));
  const size_t scratch = std::max<size_t>((size_t)3 * C * G.hx, (size_t)3 * W * G.Py);
  const size_t elems = (size_t)3 * G.ny * G.Kx + 2 * scratch + G.hx + (G.hx + 1) + G.Py;
  ft.lds = elems * sizeof(cpx<T>);
  if (ft.lds + kFusedBlock / 64 * sizeof(double) > ctx->max_lds) return ft;
  ft.C = C;
  ft.W = W;
  ft.nch = nch;
  ft.ok = true;
  return ft;
}

template <typename T>
mmx_status heun_fused(mmx_ctx* ctx, Group& G, const FusedTiles& ft, T* mg, double dt,
                      int64_t n_steps, uint64_t step0, double* tsw) {
  if ((ctx->terms & MMX_DEMAG) && !G.demag_built)
    return fail(MMX_ESTATE, "mmx_build_demag has not been called");
  HeunFusedArgs<T> a{};
  a.f = field_args<T>(ctx, G, ctx->terms);
  a.pxf = G.plan_x;
  a.pxi = G.plan_xi;
  a.pyf = G.plan_yf;
  a.pyi = G.plan_yi;
  a.tw_x = G.tw_x.as<cpx<T>>();
  a.wpost = G.wpost.as<cpx<T>>();
  a.tw_y = G.tw_y.as<cpx<T>>();
  a.Nt = G.Nt.as<T>();
  a.Ty = G.Ty;
  a.Py = G.Py;
  a.m = mg;
  a.ms = G.ms.as<T>();
  a.tsw = tsw;
  a.dt = dt;
  a.C = ft.C;
  a.W = ft.W;
  a.nch = ft.nch;
  HIP_TRY(hipFuncSetAttribute((const void*)&k_heun_fused<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ft.lds));
  const int64_t per_launch = 64;  // steps per launch
  for (int64_t s0 = 0; s0 < n_steps; s0 += per_launch) {
    a.step0 = step0 + (uint64_t)s0;
    a.nsteps = (int)std::min<int64_t>(per_launch, n_steps - s0);
    ProfScope ps(ctx->prof, "k_heun_fused", ctx->stream);
    k_heun_fused<T><<<G.R, kFusedBlock, ft.lds, ctx->stream>>>(a);
    HIP_TRY(hipGetLastError());
  }
  return MMX_OK;
}

// Retire/refill trials of the rotation scheme: every replica restarts from
// its row of m_init (device, D1) after the step at which its mean m_z turns
// negative; times (device double[R_total][cap]) and counts (device
// int[R_total]) receive the trial durations and the number of finished trials.
struct RefillArgs {
  const void* m_init = nullptr;
  double* times = nullptr;
  int* counts = nullptr;
  int cap = 0;
};

// Sets ctx->rot / ctx->refill for the duration of one integrator call.
struct SchemeScope {
  mmx_ctx* c;
  SchemeScope(mmx_ctx* ctx, int rot, int refill) : c(ctx) {
    c->rot = rot;
    c->refill = refill;
  }
  ~SchemeScope() {
    c->rot = 0;
    c->refill = 0;
  }
};

// Single-cell groups without demag: every replica advances all steps in the
// registers of one thread (k_macrospin), in launches of at most 8192 steps.
template <typename T>
mmx_status heun_macrospin(mmx_ctx* ctx, Group& G, T* mg, double dt, int64_t n_steps,
                          uint64_t step0, double* tsw, int rot, const MacroRefill<T>& mr) {
  FArgs<T> a = field_args<T>(ctx, G, ctx->terms);
  a.dth = dt;
  a.dt_th = dt;
  const dim3 grid((unsigned)((G.R + 255) / 256));
  for (int64_t done = 0; done < n_steps;) {
    const int n = (int)std::min<int64_t>(n_steps - done, 8192);
    ProfScope ps(ctx->prof, "k_macrospin", ctx->stream);
    if (rot)
      k_macrospin<T, true><<<grid, 256, 0, ctx->stream>>>(a, mg, dt, n, step0 + (uint64_t)done,
                                                          tsw, G.R, mr);
    else
      k_macrospin<T, false><<<grid, 256, 0, ctx->stream>>>(a, mg, dt, n, step0 + (uint64_t)done,
                                                           tsw, G.R, mr);
    HIP_TRY(hipGetLastError());
    done += n;
  }
  return MMX_OK;
}

// Trial bookkeeping of a retire/refill call: every replica of the group starts
// trial 0 at step step0; counts zeroed, times set to -1.
template <typename T>
mmx_status refill_begin(mmx_ctx* ctx, Group& G, const RefillArgs& rf, int roff, uint64_t step0) {
  hipStream_t s = ctx->stream;
  const unsigned nb = (unsigned)((G.R + 255) / 256);
  k_fill_i32<<<nb, 256, 0, s>>>(G.tgen.as<int>(), G.R, 0);
  k_fill_i32<<<nb, 256, 0, s>>>(G.tflag.as<int>(), G.R, 0);
  k_fill_i32<<<nb, 256, 0, s>>>(rf.counts + roff, G.R, 0);
  k_fill_u64<<<nb, 256, 0, s>>>(G.tstart.as<unsigned long long>(), G.R,
                                (unsigned long long)step0);
  const size_t nt = (size_t)G.R * rf.cap;
  if (nt)
    k_fill_f64<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(rf.times + (size_t)roff * rf.cap, nt,
                                                            -1.0);
  HIP_TRY(hipGetLastError());
  return MMX_OK;
}

template <typename T>
mmx_status heun_impl(mmx_ctx* ctx, void* m, double dt, int64_t n_steps, uint64_t step0,
                     void* tsw, int rot = 0, const RefillArgs* rf = nullptr) {
  if (!(dt > 0)) return fail(MMX_EINVAL, "dt must be > 0");
  if (n_steps < 0) return fail(MMX_EINVAL, "n_steps must be >= 0");
  ctx->rk_valid = 0;  // the stage buffers are reused
  hipStream_t s = ctx->stream;
  T* mb = reinterpret_cast<T*>(m);
  double* tsw_d = reinterpret_cast<double*>(tsw);
  const bool refill = rf != nullptr;
  if (ctx->noprec)
    return fail(MMX_EUNSUP, "damping-only dynamics are for RK45, RK4 and the relaxer");
  if ((rot || refill) && ctx->path == MMX_PATH_FUSED)
    return fail(MMX_EUNSUP, "the rotation scheme runs on the staged path only");
  SchemeScope scheme(ctx, rot, refill ? 1 : 0);
  // groups on the replica-resident path advance all steps at once
  std::vector<int> staged;
  {
    int roff = 0;
    for (size_t gi = 0; gi < ctx->groups.size(); ++gi) {
      Group& G = *ctx->groups[gi];
      if (G.N == 1 && !(ctx->terms & MMX_DEMAG) && ctx->path != MMX_PATH_STAGED && !G.cells_on) {
        MacroRefill<T> mr{};
        if (refill) {
          MMX_TRY(refill_begin<T>(ctx, G, *rf, roff, step0));
          mr.m_init = reinterpret_cast<const T*>(rf->m_init) + G.off;
          mr.tgen = G.tgen.as<int>();
          mr.tstart = G.tstart.as<unsigned long long>();
          mr.counts = rf->counts + roff;
          mr.times = rf->times + (size_t)roff * rf->cap;
          mr.cap = rf->cap;
        }
        MMX_TRY(heun_macrospin<T>(ctx, G, mb + G.off, dt, n_steps, step0,
                                  tsw_d ? tsw_d + roff : nullptr, rot, mr));
        roff += G.R;
        continue;
      }
      const FusedTiles ft = fused_tiles<T>(ctx, G);
      if (ctx->path == MMX_PATH_FUSED && !ft.ok)
        return fail(MMX_EUNSUP, "group does not fit the replica-resident path");
      const bool stt = ((ctx->terms & MMX_STT) && G.jrep_on && G.stt_P != 0) ||
                       G.ext.Db != 0 || ((ctx->terms & MMX_ANIS_CUBIC) && (G.ext.Kc1 != 0 || G.ext.Kc2 != 0)) ||
                       ((ctx->terms & MMX_RKKY) && G.ext.rkky != 0) || G.acell_on || G.cells_on;
      if (stt && ctx->path == MMX_PATH_FUSED)
        return fail(MMX_EUNSUP, "the spin-transfer torque and further field terms run on the "
                                "staged path only");
      const bool use_fused = !rot && !refill && !stt && ft.ok &&
                             (ctx->path == MMX_PATH_FUSED ||
                              (ctx->path == MMX_PATH_AUTO && G.fused_faster));
      if (use_fused) {
        MMX_TRY(heun_fused<T>(ctx, G, ft, mb + G.off, dt, n_steps, step0,
                              tsw_d ? tsw_d + roff : nullptr));
      } else {
        staged.push_back((int)gi);
      }
      roff += G.R;
    }
  }
  if (staged.empty()) return MMX_OK;
  std::vector<int> roffs;
  {
    int roff = 0;
    for (auto& gp : ctx->groups) {
      roffs.push_back(roff);
      roff += gp->R;
    }
  }
  // groups whose switching check is folded into the next step's column
  // kernel: their partial sums start neutral (positive) so that the first
  // step's check changes nothing; one reduction follows the last step
  std::vector<char> folds(ctx->groups.size(), 0);
  if (tsw_d && !refill && (ctx->terms & MMX_DEMAG) && n_steps > 0) {
    for (int gi : staged) {
      Group& G = *ctx->groups[gi];
      if (!yconv_reg_applies<T>(G)) continue;
      folds[gi] = 1;
      const size_t np = G.partial.bytes / sizeof(double);
      k_fill_f64<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(G.partial.as<double>(), np, 1.0);
      k_fill_i32<<<1, 64, 0, s>>>(G.nblk_dev.as<int>(), 1, 1);
      HIP_TRY(hipGetLastError());
    }
  }
  // one Heun step of every staged group on ctx->stream; with ctx->cur_stepdev
  // set the kernels take the step index *cur_stepdev + step (step: the offset
  // within a captured run, after which the counter is advanced once)
  auto one_step = [&](uint64_t step) -> mmx_status {
    hipStream_t st = ctx->stream;
    for (int gi : staged) {
      Group& G = *ctx->groups[gi];
      const int roff = roffs[gi];
      T* mg = mb + G.off;
      // each epilogue x-transforms the state it writes, so both field
      // evaluations start from a ready half spectrum (the first one of the
      // call is prepared below)
      Epilogue e1;
      e1.mode = FM_HEUN1;
      e1.k1 = G.k[0].p;
      e1.mout = G.ms.p;
      e1.fwd = 1;
      // the previous step's switching check rides on this step's first
      // column kernel (the partial sums are those of the last corrector)
      SwitchFold sf;
      const bool fold = tsw_d && !refill && folds[gi];
      if (fold) {
        sf.part = G.partial.as<double>();
        sf.tsw = tsw_d + roff;
        sf.nblk = G.nblk_dev.as<int>();
        sf.N = G.N;
        sf.dt = dt;
        sf.step = (unsigned long long)step;
        sf.stepdev = ctx->cur_stepdev;
      }
      MMX_TRY(eval_group<T>(ctx, G, mg, Combine{}, e1, step, dt, nullptr, dt, nullptr,
                            0xFFFFFFFFu, true, fold ? &sf : nullptr));
      Epilogue e2;
      e2.mode = FM_HEUN2;
      e2.k1 = G.k[0].p;
      e2.m0 = mg;
      e2.mout = mg;
      e2.fwd = 1;
      MMX_TRY(eval_group<T>(ctx, G, G.ms.as<T>(), Combine{}, e2, step, dt, nullptr, dt, nullptr,
                            0xFFFFFFFFu, true));
      if (refill) {
        ProfScope ps(ctx->prof, "k_refill", st);
        k_refill_check<<<(G.R + 63) / 64, 64, 0, st>>>(
            G.partial.as<double>(), G.nblk_last, G.R, G.N, G.tgen.as<int>(),
            G.tstart.as<unsigned long long>(), G.tflag.as<int>(), rf->counts + roff,
            rf->times + (size_t)roff * rf->cap, rf->cap, (unsigned long long)step,
            ctx->cur_stepdev, dt);
        HIP_TRY(hipGetLastError());
        const size_t n = (size_t)3 * G.N;
        const size_t ns = (ctx->terms & MMX_DEMAG) ? (size_t)3 * G.nz * G.Sy * G.Kx : 0;
        // one workgroup per replica: resets are rare, so the launch is kept
        // small rather than wide
        const dim3 grid(1, (unsigned)G.R);
        k_refill_copy<T><<<grid, 256, 0, st>>>(
            G.tflag.as<int>(), mg, reinterpret_cast<const T*>(rf->m_init) + G.off, n,
            ns ? G.S.as<cpx<T>>() : nullptr, ns ? G.S_init.as<cpx<T>>() : nullptr, ns);
        HIP_TRY(hipGetLastError());
      }
      if (tsw_d && !folds[gi]) {
        ProfScope ps(ctx->prof, "k_switch_reduce", st);
        k_switch_reduce<<<(G.R + 63) / 64, 64, 0, st>>>(G.partial.as<double>(), G.nblk_last, G.R,
                                                         G.N, tsw_d + roff,
                                                         (unsigned long long)(step + 1),
                                                         ctx->cur_stepdev, dt);
        HIP_TRY(hipGetLastError());
      }
    }
    return MMX_OK;
  };
  // half spectrum of a state, with the arithmetic of the row kernel where
  // that kernel will run, so that a run split over several calls equals one
  // call bit for bit
  auto spectrum_of = [&](Group& G, const T* src) -> mmx_status {
    FArgs<T> fa = field_args<T>(ctx, G, ctx->terms);
    fa.m = src;
    bool done_fwd = false;
    {
      ProfScope ps(ctx->prof, "k_xfwd", s);
      done_fwd = launch_rows_reg<T>(ctx, G, fa, -1);
      if (done_fwd) HIP_TRY(hipGetLastError());
    }
    if (!done_fwd) MMX_TRY(launch_xfwd<T>(ctx, G, src, Combine{}, true, nullptr, dt, nullptr));
    return MMX_OK;
  };
  if (refill) {
    // every replica starts trial 0 at step step0; the initial states' half
    // spectra are kept for the resets
    for (int gi : staged) {
      Group& G = *ctx->groups[gi];
      const int roff = roffs[gi];
      MMX_TRY(refill_begin<T>(ctx, G, *rf, roff, step0));
      if (n_steps > 0 && (ctx->terms & MMX_DEMAG)) {
        MMX_TRY(spectrum_of(G, reinterpret_cast<const T*>(rf->m_init) + G.off));
        HIP_TRY(hipMemcpyAsync(G.S_init.p, G.S.p, G.S.bytes, hipMemcpyDeviceToDevice, s));
      }
    }
  }
  if (n_steps > 0 && (ctx->terms & MMX_DEMAG)) {
    for (int gi : staged) {  // half spectrum of the initial state
      Group& G = *ctx->groups[gi];
      MMX_TRY(spectrum_of(G, mb + G.off));
    }
  }
  if (!ctx->prof.on && n_steps > 0) {
    // n_steps = a sum of runs of 2^i steps (i < kHeunGraphs, largest first);
    // each run length is captured once into a graph (the run's first step
    // index lives in device memory, each captured step adds its offset within
    // the run, and the graph's last node advances it by the run length) and
    // kept for later calls
    // with the same arrays and configuration, so every call of any length
    // replays captured steps
    MMX_TRY(ensure_graph_stream(ctx));
    hipStream_t user = ctx->stream, cs = ctx->cap_stream;
    GraphKey key;
    key.epoch = ctx->epoch;
    key.p[0] = m;
    key.p[1] = tsw;
    key.p[2] = refill ? rf->m_init : nullptr;
    key.p[3] = refill ? rf->times : nullptr;
    key.p[4] = refill ? rf->counts : nullptr;
    key.d = dt;
    key.i[0] = rot;
    key.i[1] = refill ? 1 : 0;
    key.i[2] = refill ? rf->cap : 0;
    GraphSet& gs = ctx->heun_graphs;
    if (!gs.valid || !(gs.key == key)) {
      HIP_TRY(hipStreamSynchronize(cs));
      gs.clear();
      gs.exec.assign(kHeunGraphs, nullptr);
      gs.nblk.assign(ctx->groups.size(), 1);
      gs.key = key;
      gs.valid = true;
    }
    std::vector<int> runs;
    for (int64_t left = n_steps; left > 0;) {
      int i = kHeunGraphs - 1;
      while ((int64_t(1) << i) > left) --i;
      runs.push_back(i);
      left -= int64_t(1) << i;
    }
    unsigned long long* sd = ctx->stepdev.as<unsigned long long>();
    for (int i : runs) {
      if (gs.exec[i]) continue;
      ctx->cur_stepdev = sd;
      const mmx_status st = capture_graph(ctx, [&]() -> mmx_status {
        for (int j = 0; j < (1 << i); ++j) MMX_TRY(one_step((uint64_t)j));
        k_inc_u64<<<1, 1, 0, ctx->stream>>>(sd, 1ull << i);
        HIP_TRY(hipGetLastError());
        return MMX_OK;
      }, &gs.exec[i]);
      ctx->cur_stepdev = nullptr;
      MMX_TRY(st);
      for (int gi : staged) gs.nblk[gi] = ctx->groups[gi]->nblk_last;
    }
    HIP_TRY(hipEventRecord(ctx->ev_user, user));
    HIP_TRY(hipStreamWaitEvent(cs, ctx->ev_user, 0));
    k_set_u64<<<1, 1, 0, cs>>>(sd, (unsigned long long)step0);
    HIP_TRY(hipGetLastError());
    for (int i : runs) HIP_TRY(hipGraphLaunch(gs.exec[i], cs));
    HIP_TRY(hipEventRecord(ctx->ev_cap, cs));
    HIP_TRY(hipStreamWaitEvent(user, ctx->ev_cap, 0));
    for (int gi : staged) ctx->groups[gi]->nblk_last = gs.nblk[gi];
  } else {
    for (int64_t i = 0; i < n_steps; ++i) MMX_TRY(one_step(step0 + (uint64_t)i));
  }
  for (int gi : staged) {  // the last step's switching check
    if (!folds[gi]) continue;
    Group& G = *ctx->groups[gi];
    ProfScope ps(ctx->prof, "k_switch_reduce", s);
    k_switch_reduce<<<(G.R + 63) / 64, 64, 0, s>>>(G.partial.as<double>(), G.nblk_last, G.R, G.N,
                                                   tsw_d + roffs[gi],
                                                   (unsigned long long)(step0 + (uint64_t)n_steps),
                                                   nullptr, dt);
    HIP_TRY(hipGetLastError());
  }
  return MMX_OK;
}

// Classical fourth-order Runge-Kutta (fixed dt): stage states m + dt/2 k1,
// m + dt/2 k2, m + dt k3 (not normalised); the new state m + dt (k1/6 + k2/3
// + k3/3 + k4/6) is normalised.
template <typename T>
mmx_status rk4_impl(mmx_ctx* ctx, void* m, double dt, int64_t n_steps) {
  if (!(dt > 0)) return fail(MMX_EINVAL, "dt must be > 0");
  if (n_steps < 0) return fail(MMX_EINVAL, "n_steps must be >= 0");
  if (ctx->terms & MMX_THERMAL) return fail(MMX_EUNSUP, "thermal field with RK4");
  ctx->rk_valid = 0;
  for (auto& gp : ctx->groups) MMX_TRY(ensure_rk_buffers<T>(*gp));
  T* mb = reinterpret_cast<T*>(m);
  for (int64_t i = 0; i < n_steps; ++i) {
    for (auto& gp : ctx->groups) {
      Group& G = *gp;
      T* mg = mb + G.off;
      Epilogue e;
      e.mode = FM_RKK;
      e.out = G.k[0].p;
      MMX_TRY(eval_group<T>(ctx, G, mg, Combine{}, e, 0, dt, nullptr, dt, nullptr));
      for (int st = 1; st < 4; ++st) {
        Combine cb;
        cb.ncoef = 1;
        cb.coef[0] = st == 3 ? 1.0 : 0.5;
        cb.kidx[0] = st - 1;
        cb.mout = G.ms.p;
        e.out = G.k[st].p;
        MMX_TRY(eval_group<T>(ctx, G, mg, cb, e, 0, dt, nullptr, dt, nullptr));
      }
      Combine fc;
      fc.ncoef = 4;
      const double w[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
      for (int j = 0; j < 4; ++j) {
        fc.coef[j] = w[j];
        fc.kidx[j] = j;
      }
      fc.normalise = 1;
      fc.check_finite = 1;
      fc.mout = mg;
      MMX_TRY(launch_xfwd<T>(ctx, G, mg, fc, false, nullptr, dt, nullptr));
    }
  }
  return MMX_OK;
}

// max over all replicas and cells of |dm/dt| (synchronous)
template <typename T>
mmx_status max_torque(mmx_ctx* ctx, const T* mb, double* out) {
  constexpr int nb = 256;
  for (auto& gp : ctx->groups) MMX_TRY(ensure_rk_buffers<T>(*gp));
  double mx = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    Epilogue e;
    e.mode = FM_TORQUE;
    e.out = G.k[6].p;
    MMX_TRY(eval_group<T>(ctx, G, mb + G.off, Combine{}, e, 0, 1.0, nullptr, 1.0, nullptr));
    k_norm_max<T><<<nb, 256, 0, ctx->stream>>>(G.k[6].as<T>(), (size_t)G.N, G.R,
                                                 ctx->maxbuf.as<double>());
    k_max_fold<<<1, 256, 0, ctx->stream>>>(ctx->maxbuf.as<double>(), nb);
    HIP_TRY(hipGetLastError());
    double g = 0;
    HIP_TRY(hipMemcpyAsync(&g, ctx->maxbuf.as<double>() + nb, sizeof(double),
                           hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    mx = std::max(mx, g);
  }
  *out = mx;
  return MMX_OK;
}

// Damping-only relaxation: RK45 on the damping-only dynamics in chunks of
// 10 ps of simulated time (each chunk starting from the controller's last
// unclipped proposal) until max |dm/dt| <= torque_tol or t reaches t_max.
template <typename T>
mmx_status relax_impl(mmx_ctx* ctx, void* m, double torque_tol, double t_max, double tol,
                      mmx_rk_stats* stats, double* tq_out) {
  constexpr double kChunk = 1e-11;
  struct NoPrec {
    mmx_ctx* c;
    int prev;
    ~NoPrec() { c->noprec = prev; }
  } guard{ctx, ctx->noprec};
  ctx->noprec = 1;
  const T* mb = reinterpret_cast<const T*>(m);
  double t = 0, dt = 1e-14, tq = 0;
  int64_t acc = 0, rej = 0;
  MMX_TRY(max_torque<T>(ctx, mb, &tq));
  mmx_rk_stats st{};
  while (tq > torque_tol && t < t_max) {
    const double t1 = std::min(t + kChunk, t_max);
    double prop = dt;
    MMX_TRY(rk45_impl<T>(ctx, m, t, t1, tol, dt, nullptr, 0, nullptr, 0, &st, &prop));
    t = st.t;
    dt = prop;
    acc += st.accepted;
    rej += st.rejected;
    MMX_TRY(max_torque<T>(ctx, mb, &tq));
  }
  if (stats) {
    stats->t = t;
    stats->dt = dt;
    stats->err = st.err;
    stats->accepted = acc;
    stats->rejected = rej;
  }
  if (tq_out) *tq_out = tq;
  ctx->rk_valid = 0;  // the saved slope belongs to the damping-only dynamics
  return MMX_OK;
}

template <typename T>
mmx_status field_impl(mmx_ctx* ctx, const void* m, void* out, uint64_t step, double dt, int mode) {
  if ((ctx->terms & MMX_THERMAL) && !(dt > 0)) return fail(MMX_EINVAL, "thermal term needs dt > 0");
  const T* mb = reinterpret_cast<const T*>(m);
  T* ob = reinterpret_cast<T*>(out);
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    Epilogue ep;
    ep.mode = mode;
    ep.out = ob + G.off;
    MMX_TRY(eval_group<T>(ctx, G, mb + G.off, Combine{}, ep, step, dt > 0 ? dt : 1.0, nullptr,
                          dt, nullptr));
  }
  return MMX_OK;
}

template <typename T>
mmx_status energy_impl(mmx_ctx* ctx, const void* m, void* E) {
  const T* mb = reinterpret_cast<const T*>(m);
  double* Eb = reinterpret_cast<double*>(E);
  int roff = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    Epilogue ep;
    ep.mode = FM_ENERGY;
    MMX_TRY(eval_group<T>(ctx, G, mb + G.off, Combine{}, ep, 0, 1.0, nullptr, 0.0, nullptr,
                          ctx->terms & ~MMX_THERMAL));
    const double V = G.g.cell[0] * G.g.cell[1] * G.g.cell[2];
    k_energy_reduce<<<(G.R + 63) / 64, 64, 0, ctx->stream>>>(
        G.partial.as<double>(), G.nblk, G.R, -0.5 * kMu0 * G.mat.Ms * V, -kMu0 * G.mat.Ms * V,
        Eb + (size_t)roff * 6);
    HIP_TRY(hipGetLastError());
    roff += G.R;
  }
  return MMX_OK;
}

// workgroups per replica of the topological-charge kernel
int topo_blocks(const Group& G) {
  const int plane = G.nx * G.ny;
  return std::max(1, std::min(256, (plane + kBlock - 1) / kBlock));
}

// Q of every replica with the per-workgroup partial sums in `part` (reused
// from its start by every group, in stream order); no allocation, no
// synchronisation
template <typename T>
mmx_status topo_into(mmx_ctx* ctx, const void* m, void* Q, double* part) {
  const T* mb = reinterpret_cast<const T*>(m);
  double* Qb = reinterpret_cast<double*>(Q);
  int roff = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    const int nblk = topo_blocks(G);
    dim3 grid(nblk, G.R);
    k_topo<T><<<grid, kBlock, 0, ctx->stream>>>(mb + G.off, G.nx, G.ny, G.N, G.g.pbc[0],
                                                G.g.pbc[1], 1.0 / (2 * G.g.cell[0]),
                                                1.0 / (2 * G.g.cell[1]), part, nblk);
    HIP_TRY(hipGetLastError());
    k_topo_reduce<<<(G.R + 63) / 64, 64, 0, ctx->stream>>>(
        part, nblk, G.R, G.g.cell[0] * G.g.cell[1] / (4 * kPi), Qb + roff);
    HIP_TRY(hipGetLastError());
    roff += G.R;
  }
  return MMX_OK;
}

template <typename T>
mmx_status topo_impl(mmx_ctx* ctx, const void* m, void* Q) {
  const T* mb = reinterpret_cast<const T*>(m);
  double* Qb = reinterpret_cast<double*>(Q);
  int roff = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    const int nblk = topo_blocks(G);
    double* part = G.topo_part.as<double>();
    dim3 grid(nblk, G.R);
    k_topo<T><<<grid, kBlock, 0, ctx->stream>>>(mb + G.off, G.nx, G.ny, G.N, G.g.pbc[0],
                                                G.g.pbc[1], 1.0 / (2 * G.g.cell[0]),
                                                1.0 / (2 * G.g.cell[1]), part, nblk);
    HIP_TRY(hipGetLastError());
    k_topo_reduce<<<(G.R + 63) / 64, 64, 0, ctx->stream>>>(
        part, nblk, G.R, G.g.cell[0] * G.g.cell[1] / (4 * kPi), Qb + roff);
    HIP_TRY(hipGetLastError());
    roff += G.R;
  }
  return MMX_OK;
}

mmx_status check_ctx(const mmx_ctx* c) {
  if (!c) return fail(MMX_EINVAL, "null context");
  return MMX_OK;
}

// Device address of the static scratch array on each device (taken once per
// device, with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

mmx_status scratch_init(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MMX_EUNSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MMX_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return MMX_OK;
}

// Synchronises the bound stream and reports (and clears) the device flag that
// correctors and normalised combines set when they produce a non-finite state.
mmx_status take_nonfinite(mmx_ctx* ctx) {
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, ctx->nfflag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (!f) return MMX_OK;
  k_fill_i32<<<1, 64, 0, ctx->stream>>>(ctx->nfflag.as<int>(), 1, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return fail(MMX_ENONFINITE, "a non-finite magnetisation was produced since the last check");
}

// ---------------------------------------------------------------------------
// tiles: rows per x workgroup (L), spectrum columns per y / z workgroup
// (Wy, Wz).  Every column and row is transformed by the same arithmetic
// whatever the grouping, so results do not depend on the tiles.
// ---------------------------------------------------------------------------
constexpr size_t kMaxDynLds = 64 * 1024;

template <typename T>
size_t lds_x(const Group& G, int L) {
  return (2 * 3 * (size_t)L * G.hx + 2 * G.hx + 1) * cpxb<T>();
}
template <typename T>
size_t lds_col(int W, int P) {
  return (2 * 3 * (size_t)W * P + P) * cpxb<T>();
}

template <typename T>
mmx_status apply_tiles(Group& G, int L, int Wy, int Wz) {
  if (L < 1 || L > G.ny || Wy < 1 || Wy > G.Kx || Wz < 1 || Wz > G.Kx)
    return fail(MMX_EINVAL, "tile sizes out of range");
  if (lds_x<T>(G, L) > kMaxDynLds || lds_ycols<T>(G.is3d, Wy, G.Py) > kMaxDynLds ||
      !wz_fits<T>(G, Wz))
    return fail(MMX_EINVAL, "tile sizes exceed the LDS budget");
  G.L = L;
  G.Wy = Wy;
  G.Wz = Wz;
  const int nblk = ((G.ny + G.L - 1) / G.L) * G.nz;
  if ((size_t)G.R * nblk * 5 * sizeof(double) > G.partial.bytes)
    return fail(MMX_EINVAL, "tile sizes need more partial sums than reserved");
  G.nblk = nblk;
  return MMX_OK;
}

template <typename T>
mmx_status time_eval(mmx_ctx* ctx, Group& G, float& ms) {
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  Epilogue ep;
  ep.mode = FM_FIELD;
  ep.out = G.k[0].p;
  mmx_status st = MMX_OK;
  float best = 1e30f;
  // five repetitions, the fastest of the last four (the first warms caches):
  // single evaluations of small grids take tens of microseconds
  for (int rep = 0; rep < 5 && st == MMX_OK; ++rep) {
    (void)hipEventRecord(a, ctx->stream);
    st = eval_group<T>(ctx, G, G.ms.as<T>(), Combine{}, ep, 0, 1.0, nullptr, 0.0, nullptr,
                       ctx->terms & ~MMX_THERMAL);
    (void)hipEventRecord(b, ctx->stream);
    (void)hipEventSynchronize(b);
    float t = 0;
    (void)hipEventElapsedTime(&t, a, b);
    if (rep > 0) best = std::min(best, t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ms = best;
  return st;
}

template <typename T>
mmx_status autotune_impl(mmx_ctx* ctx) {
  ctx->rk_valid = 0;
  for (auto& gp : ctx->groups) {
    Group& G = *gp;
    if (!G.demag_built) continue;
    HIP_TRY(hipMemsetAsync(G.ms.p, 0, G.ms.bytes, ctx->stream));
    const int cand[] = {1, 2, 4, 8, 16, 32};
    int bestL = G.L, bestW = G.Wy, bestWz = G.Wz;
    float bt = 1e30f;
    for (int L : cand) {
      if (L > G.ny || lds_x<T>(G, L) > kMaxDynLds || (size_t)L * G.nx > 8 * kBlock) continue;
      MMX_TRY(apply_tiles<T>(G, L, bestW, bestWz));
      float t;
      MMX_TRY(time_eval<T>(ctx, G, t));
      if (t < bt) { bt = t; bestL = L; }
    }
    bt = 1e30f;
    for (int W : cand) {
      if (yz_applies<T>(G)) break;  // the fused y-z pass takes no y tile
      if (W > G.Kx || lds_ycols<T>(G.is3d, W, G.Py) > kMaxDynLds) continue;
      MMX_TRY(apply_tiles<T>(G, bestL, W, bestWz));
      float t;
      MMX_TRY(time_eval<T>(ctx, G, t));
      if (t < bt) { bt = t; bestW = W; }
    }
    // few-layer groups: the fused y-z kernel (its column tile tuned) against
    // the separate register y passes around the z pass
    const bool both_yz = yz_applies<T>(G) && ypass_reg_applies<T>(G);
    if (both_yz) G.yz_split = 0;
    float t_fused = 1e30f;
    if (G.is3d && !zconv_reg_applies<T>(G)) {
      bt = 1e30f;
      for (int W : cand) {
        if (W > G.Kx || !wz_fits<T>(G, W)) continue;
        MMX_TRY(apply_tiles<T>(G, bestL, bestW, W));
        float t;
        MMX_TRY(time_eval<T>(ctx, G, t));
        if (t < bt) { bt = t; bestWz = W; }
      }
      t_fused = bt;
    }
    MMX_TRY(apply_tiles<T>(G, bestL, bestW, bestWz));
    if (both_yz) {
      G.yz_split = 1;
      float t_split = 1e30f;
      MMX_TRY(time_eval<T>(ctx, G, t_split));
      G.yz_split = t_split <= t_fused ? 1 : 0;
    }
    // Heun path: one predictor-corrector step staged (two evaluations) against
    // one replica-resident step, on a zeroed state (scratch buffer m7)
    G.fused_faster = 0;
    const FusedTiles ft = fused_tiles<T>(ctx, G);
    if (ft.ok) {
      MMX_TRY(ensure_rk_buffers<T>(G));
      HIP_TRY(hipMemsetAsync(G.m7.p, 0, G.m7.bytes, ctx->stream));
      float staged_ms = 0, fused_ms = 0;
      MMX_TRY(time_eval<T>(ctx, G, staged_ms));
      staged_ms *= 2.0f;
      hipEvent_t a, b;
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(a, ctx->stream);
        mmx_status st = heun_fused<T>(ctx, G, ft, G.m7.as<T>(), 1e-15, 1, 0, nullptr);
        (void)hipEventRecord(b, ctx->stream);
        (void)hipEventSynchronize(b);
        float t = 0;
        (void)hipEventElapsedTime(&t, a, b);
        if (st != MMX_OK) {
          (void)hipEventDestroy(a);
          (void)hipEventDestroy(b);
          return st;
        }
        if (rep > 0) best = std::min(best, t);
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      fused_ms = best;
      G.fused_faster = fused_ms < staged_ms ? 1 : 0;
    }
  }
  // the timing runs step scratch states (a zero state normalises to NaN):
  // they must not leave the non-finite flag for the caller's next check
  k_fill_i32<<<1, 64, 0, ctx->stream>>>(ctx->nfflag.as<int>(), 1, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return MMX_OK;
}

// Derived per-cell arrays of group G from its per-cell values (FP64 on the
// host, rounded to the context precision once) and the group's material.
template <typename T>
mmx_status upload_cells(mmx_ctx* ctx, Group& G) {
  if (!G.cells_on) return MMX_OK;
  const size_t n = (size_t)G.N;
  std::vector<T> v[7];
  for (auto& x : v) x.assign(n, T(0));
  const double Msg = G.mat.Ms;
  for (size_t i = 0; i < n; ++i) {
    const double Ms = G.cMs.empty() ? Msg : G.cMs[i];
    const double al = G.calpha.empty() ? G.mat.alpha : G.calpha[i];
    const double Ku = G.cKu.empty() ? G.mat.Ku : G.cKu[i];
    const double D = G.cD.empty() ? G.mat.D : G.cD[i];
    v[0][i] = (T)(Ms / Msg);
    v[1][i] = (T)(Msg / Ms);
    v[2][i] = (T)(kGamma0 / (1.0 + al * al) * kMu0);
    v[3][i] = (T)al;
    v[4][i] = (T)std::sqrt(al * Msg / Ms);
    v[5][i] = (T)(2.0 * Ku / (kMu0 * Msg));
    v[6][i] = (T)D;
  }
  for (int j = 0; j < 7; ++j)
    HIP_TRY(hipMemcpyAsync(G.cell[j].p, v[j].data(), n * sizeof(T), hipMemcpyHostToDevice,
                           ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return MMX_OK;
}

mmx_status check_group_idx(const mmx_ctx* c, int32_t g) {
  MMX_TRY(check_ctx(c));
  if (g < 0 || g >= (int)c->groups.size()) return fail(MMX_EINVAL, "group index out of range");
  return MMX_OK;
}

mmx_status check_materials(const mmx_ctx* c) {
  for (auto& g : c->groups)
    if (!g->mat_set) return fail(MMX_ESTATE, "material not set for every group");
  return MMX_OK;
}

}  // namespace

extern "C" {

const char* mmx_last_error(void) { return g_err.c_str(); }

mmx_status mmx_profile_enable(mmx_ctx* ctx, int32_t on) {
  MMX_TRY(check_ctx(ctx));
  ctx->prof.flush();
  if (on) {
    for (auto& v : ctx->prof.ms) v = 0.0;
    for (auto& c : ctx->prof.cnt) c = 0;
  }
  ctx->prof.on = on != 0;
  return MMX_OK;
}

mmx_status mmx_profile_get(mmx_ctx* ctx, int32_t idx, char* name, int32_t name_cap,
                           double* total_ms, int64_t* count, int32_t* n_kernels) {
  MMX_TRY(check_ctx(ctx));
  ctx->prof.flush();
  if (n_kernels) *n_kernels = (int32_t)ctx->prof.names.size();
  if (idx < 0) return MMX_OK;
  if (idx >= (int)ctx->prof.names.size()) return fail(MMX_EINVAL, "kernel index out of range");
  if (name && name_cap > 0) {
    std::strncpy(name, ctx->prof.names[idx].c_str(), name_cap - 1);
    name[name_cap - 1] = 0;
  }
  if (total_ms) *total_ms = ctx->prof.ms[idx];
  if (count) *count = ctx->prof.cnt[idx];
  return MMX_OK;
}

mmx_status mmx_create(const mmx_group* groups, int32_t n_groups, mmx_prec prec, mmx_ctx** out) {
  if (!out) return fail(MMX_EINVAL, "out is null");
  *out = nullptr;
  if (!groups || n_groups < 1) return fail(MMX_EINVAL, "need at least one group");
  if (prec != MMX_F32 && prec != MMX_F64) return fail(MMX_EINVAL, "precision must be F32 or F64");
  for (int i = 0; i < n_groups; ++i) MMX_TRY(check_group(groups[i]));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MMX_EUNSUP, std::string("libmmx is built for gfx950, device is ") + prop.gcnArchName);
  auto ctx = std::make_unique<mmx_ctx>();
  ctx->prec = prec;
  ctx->max_lds = prop.sharedMemPerBlock;
  ctx->device = dev;
  MMX_TRY(scratch_init(dev, &ctx->scratch));
  size_t off = 0;
  for (int i = 0; i < n_groups; ++i) {
    auto G = std::make_unique<Group>();
    G->g = groups[i];
    G->off = off;
    mmx_status s = (prec == MMX_F64) ? setup_group<double>(ctx.get(), *G)
                                     : setup_group<float>(ctx.get(), *G);
    if (s != MMX_OK) return s;
    off += (size_t)G->R * 3 * G->N;
    ctx->groups.push_back(std::move(G));
  }
  ctx->total_elems = off;
  MMX_TRY(arena_init(ctx.get()));
  *out = ctx.release();
  return MMX_OK;
}

void mmx_destroy(mmx_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

mmx_status mmx_set_stream(mmx_ctx* ctx, void* stream) {
  MMX_TRY(check_ctx(ctx));
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return MMX_OK;
}

mmx_status mmx_set_material(mmx_ctx* ctx, int32_t group, const mmx_material* mat) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!mat) return fail(MMX_EINVAL, "material is null");
  if (!(mat->Ms > 0)) return fail(MMX_EINVAL, "Ms must be > 0");
  if (mat->A < 0 || mat->alpha < 0) return fail(MMX_EINVAL, "A and alpha must be >= 0");
  if (mat->D != 0 && mat->A == 0) return fail(MMX_EINVAL, "DMI needs A > 0 (edge condition)");
  Group& G = *ctx->groups[group];
  G.mat = *mat;
  G.mat_set = 1;
  G.demag_built = 0;
  // the derived per-cell arrays are relative to the group's material
  return ctx->prec == MMX_F64 ? upload_cells<double>(ctx, G) : upload_cells<float>(ctx, G);
}

mmx_status mmx_set_material_ext(mmx_ctx* ctx, int32_t group, const mmx_material_ext* ext) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!ext) return fail(MMX_EINVAL, "ext is null");
  Group& G = *ctx->groups[group];
  if (ext->Db != 0 && G.mat.A == 0) return fail(MMX_EINVAL, "bulk DMI needs A > 0 (edge condition)");
  if (ext->Kc1 != 0 || ext->Kc2 != 0) {
    double c1[3], c2[3], c3[3];
    const double n1 = std::sqrt(ext->c1[0] * ext->c1[0] + ext->c1[1] * ext->c1[1] +
                                ext->c1[2] * ext->c1[2]);
    if (!(n1 > 0) || !cubic_axes(*ext, c1, c2, c3))
      return fail(MMX_EINVAL, "cubic axes must be nonzero and not parallel");
  }
  if (ext->rkky != 0) {
    const int z0 = ext->rkky_z[0], z1 = ext->rkky_z[1];
    if (z0 == z1 || z0 < 0 || z1 < 0 || z0 >= G.nz || z1 >= G.nz)
      return fail(MMX_EINVAL, "RKKY layers must be distinct and inside the grid");
  }
  if (!std::isfinite(ext->Kc1) || !std::isfinite(ext->Kc2) || !std::isfinite(ext->Db) ||
      !std::isfinite(ext->rkky))
    return fail(MMX_EINVAL, "non-finite parameter");
  G.ext = *ext;
  return MMX_OK;
}

mmx_status mmx_set_exchange_cells(mmx_ctx* ctx, int32_t group, const double* A) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  Group& G = *ctx->groups[group];
  if (!A) {
    G.acell_on = 0;
    return MMX_OK;
  }
  for (int i = 0; i < G.N; ++i)
    if (!(A[i] >= 0) || !std::isfinite(A[i]))
      return fail(MMX_EINVAL, "per-cell stiffness must be finite and >= 0");
  const size_t es = esize(ctx);
  std::vector<unsigned char> buf((size_t)G.N * es);
  for (int i = 0; i < G.N; ++i) {
    if (es == 8) reinterpret_cast<double*>(buf.data())[i] = A[i];
    else reinterpret_cast<float*>(buf.data())[i] = (float)A[i];
  }
  HIP_TRY(hipMemcpyAsync(G.Acell.p, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  G.acell_on = 1;
  return MMX_OK;
}

mmx_status mmx_set_material_cells(mmx_ctx* ctx, int32_t group, const void* Ms, const void* A,
                                  const void* alpha, const void* Ku, const void* D) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  Group& G = *ctx->groups[group];
  if (!G.mat_set) return fail(MMX_ESTATE, "set the group's material first");
  const size_t n = (size_t)G.N, es = esize(ctx);
  // read each given device array (context element type) to the host
  auto fetch = [&](const void* src, std::vector<double>& out) -> mmx_status {
    out.clear();
    if (!src) return MMX_OK;
    std::vector<unsigned char> raw(n * es);
    HIP_TRY(hipMemcpyAsync(raw.data(), src, raw.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    out.resize(n);
    for (size_t i = 0; i < n; ++i)
      out[i] = es == 8 ? reinterpret_cast<const double*>(raw.data())[i]
                       : (double)reinterpret_cast<const float*>(raw.data())[i];
    return MMX_OK;
  };
  std::vector<double> vMs, vA, val, vKu, vD;
  MMX_TRY(fetch(Ms, vMs));
  MMX_TRY(fetch(A, vA));
  MMX_TRY(fetch(alpha, val));
  MMX_TRY(fetch(Ku, vKu));
  MMX_TRY(fetch(D, vD));
  for (size_t i = 0; i < n; ++i) {
    if (!vMs.empty() && !(vMs[i] > 0 && std::isfinite(vMs[i])))
      return fail(MMX_EINVAL, "per-cell Ms must be finite and > 0");
    if (!vA.empty() && !(vA[i] >= 0 && std::isfinite(vA[i])))
      return fail(MMX_EINVAL, "per-cell A must be finite and >= 0");
    if (!val.empty() && !(val[i] >= 0 && std::isfinite(val[i])))
      return fail(MMX_EINVAL, "per-cell alpha must be finite and >= 0");
    if ((!vKu.empty() && !std::isfinite(vKu[i])) || (!vD.empty() && !std::isfinite(vD[i])))
      return fail(MMX_EINVAL, "per-cell Ku and D must be finite");
  }
  // per-cell A: the exchange stiffness of mmx_set_exchange_cells
  if (!vA.empty()) {
    std::vector<unsigned char> buf(n * es);
    for (size_t i = 0; i < n; ++i) {
      if (es == 8) reinterpret_cast<double*>(buf.data())[i] = vA[i];
      else reinterpret_cast<float*>(buf.data())[i] = (float)vA[i];
    }
    HIP_TRY(hipMemcpyAsync(G.Acell.p, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  G.acell_on = vA.empty() ? 0 : 1;
  G.cMs = std::move(vMs);
  G.calpha = std::move(val);
  G.cKu = std::move(vKu);
  G.cD = std::move(vD);
  G.cells_on = (!G.cMs.empty() || !G.calpha.empty() || !G.cKu.empty() || !G.cD.empty()) ? 1 : 0;
  return ctx->prec == MMX_F64 ? upload_cells<double>(ctx, G) : upload_cells<float>(ctx, G);
}

mmx_status mmx_set_terms(mmx_ctx* ctx, uint32_t mask) {
  MMX_TRY(check_ctx(ctx));
  ctx->epoch++;
  if (mask & ~(uint32_t)MMX_ALL_TERMS) return fail(MMX_EINVAL, "unknown term bits");
  ctx->terms = mask;
  return MMX_OK;
}

mmx_status mmx_set_field(mmx_ctx* ctx, int32_t group, const double B[3]) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!B) return fail(MMX_EINVAL, "B is null");
  for (int c = 0; c < 3; ++c) ctx->groups[group]->B[c] = B[c];
  return MMX_OK;
}

mmx_status mmx_set_thermal(mmx_ctx* ctx, int32_t group, const double* T, const uint64_t* seeds) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!T || !seeds) return fail(MMX_EINVAL, "T and seeds must not be null");
  Group& G = *ctx->groups[group];
  for (int r = 0; r < G.R; ++r)
    if (!(T[r] >= 0)) return fail(MMX_EINVAL, "temperatures must be >= 0");
  HIP_TRY(hipMemcpyAsync(G.Trep.p, T, G.R * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(G.seeds.p, seeds, G.R * sizeof(uint64_t), hipMemcpyHostToDevice,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return MMX_OK;
}

mmx_status mmx_set_stt(mmx_ctx* ctx, int32_t group, const double* J, const double p[3],
                       double P, double Lambda, double eps_prime) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!J || !p) return fail(MMX_EINVAL, "J and p must not be null");
  const double pn = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  if (!(pn > 0) || !std::isfinite(pn)) return fail(MMX_EINVAL, "p must be a nonzero vector");
  if (!(Lambda > 0) || !std::isfinite(P) || !std::isfinite(eps_prime))
    return fail(MMX_EINVAL, "Lambda must be > 0, P and eps' finite");
  Group& G = *ctx->groups[group];
  for (int r = 0; r < G.R; ++r)
    if (!std::isfinite(J[r])) return fail(MMX_EINVAL, "current densities must be finite");
  HIP_TRY(hipMemcpyAsync(G.Jrep.p, J, G.R * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  G.jrep_on = 1;
  for (int c = 0; c < 3; ++c) G.stt_p[c] = p[c] / pn;
  G.stt_P = P;
  G.stt_lambda = Lambda;
  G.stt_eps2 = eps_prime;
  return MMX_OK;
}

mmx_status mmx_build_demag(mmx_ctx* ctx) {
  MMX_TRY(check_ctx(ctx));
  ctx->epoch++;
  MMX_TRY(check_materials(ctx));
  for (auto& g : ctx->groups) {
    mmx_status s = (ctx->prec == MMX_F64) ? build_demag_group<double>(ctx, *g)
                                          : build_demag_group<float>(ctx, *g);
    if (s != MMX_OK) return s;
  }
  return MMX_OK;
}

mmx_status mmx_field(mmx_ctx* ctx, const void* m, void* H, uint64_t step, double dt) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m || !H) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? field_impl<double>(ctx, m, H, step, dt, FM_FIELD)
                              : field_impl<float>(ctx, m, H, step, dt, FM_FIELD);
}

mmx_status mmx_torque(mmx_ctx* ctx, const void* m, void* dmdt, uint64_t step, double dt) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m || !dmdt) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? field_impl<double>(ctx, m, dmdt, step, dt, FM_TORQUE)
                              : field_impl<float>(ctx, m, dmdt, step, dt, FM_TORQUE);
}

mmx_status mmx_heun(mmx_ctx* ctx, void* m, double dt, int64_t n_steps, uint64_t step0,
                    void* t_switch) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? heun_impl<double>(ctx, m, dt, n_steps, step0, t_switch)
                              : heun_impl<float>(ctx, m, dt, n_steps, step0, t_switch);
}

mmx_status mmx_rk4(mmx_ctx* ctx, void* m, double dt, int64_t n_steps) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? rk4_impl<double>(ctx, m, dt, n_steps)
                              : rk4_impl<float>(ctx, m, dt, n_steps);
}

mmx_status mmx_set_precession(mmx_ctx* ctx, int32_t on) {
  MMX_TRY(check_ctx(ctx));
  ctx->epoch++;
  ctx->noprec = on ? 0 : 1;
  return MMX_OK;
}

mmx_status mmx_relax(mmx_ctx* ctx, void* m, double torque_tol, double t_max, double tol,
                     mmx_rk_stats* stats, double* max_torque_out) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  if (!(torque_tol >= 0) || !(t_max > 0) || !(tol > 0))
    return fail(MMX_EINVAL, "torque_tol >= 0, t_max > 0 and tol > 0 required");
  if (ctx->terms & MMX_THERMAL) return fail(MMX_EUNSUP, "thermal field in the relaxer");
  MMX_TRY(ctx->prec == MMX_F64
              ? relax_impl<double>(ctx, m, torque_tol, t_max, tol, stats, max_torque_out)
              : relax_impl<float>(ctx, m, torque_tol, t_max, tol, stats, max_torque_out));
  return take_nonfinite(ctx);
}

mmx_status mmx_depondt(mmx_ctx* ctx, void* m, double dt, int64_t n_steps, uint64_t step0,
                       void* t_switch) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? heun_impl<double>(ctx, m, dt, n_steps, step0, t_switch, 1)
                              : heun_impl<float>(ctx, m, dt, n_steps, step0, t_switch, 1);
}

mmx_status mmx_depondt_refill(mmx_ctx* ctx, void* m, const void* m_init, double dt,
                              int64_t n_steps, uint64_t step0, void* times, int32_t cap,
                              void* counts) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m || !m_init || !counts) return fail(MMX_EINVAL, "null array");
  if (cap < 0) return fail(MMX_EINVAL, "cap must be >= 0");
  if (cap > 0 && !times) return fail(MMX_EINVAL, "null times array");
  RefillArgs rf;
  rf.m_init = m_init;
  rf.times = reinterpret_cast<double*>(times);
  rf.counts = reinterpret_cast<int*>(counts);
  rf.cap = cap;
  return ctx->prec == MMX_F64 ? heun_impl<double>(ctx, m, dt, n_steps, step0, nullptr, 1, &rf)
                              : heun_impl<float>(ctx, m, dt, n_steps, step0, nullptr, 1, &rf);
}

mmx_status mmx_rk45(mmx_ctx* ctx, void* m, double t0, double t_end, double tol, double dt0,
                    const double* dt_replay, int64_t n_replay, void* energy_trace,
                    int64_t trace_cap, mmx_rk_stats* stats) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  if (!dt_replay && !(dt0 > 0)) return fail(MMX_EINVAL, "dt0 must be > 0");
  MMX_TRY(ctx->prec == MMX_F64
              ? rk45_impl<double>(ctx, m, t0, t_end, tol, dt0, dt_replay, n_replay, energy_trace,
                                  trace_cap, stats)
              : rk45_impl<float>(ctx, m, t0, t_end, tol, dt0, dt_replay, n_replay, energy_trace,
                                 trace_cap, stats));
  return take_nonfinite(ctx);
}

mmx_status mmx_workspace_bytes(const mmx_ctx* ctx, size_t* bytes) {
  MMX_TRY(check_ctx(ctx));
  if (!bytes) return fail(MMX_EINVAL, "bytes is null");
  *bytes = ctx->arena_bytes;
  return MMX_OK;
}

mmx_status mmx_bind(mmx_ctx* ctx, void* ws, size_t bytes, void* stream) {
  MMX_TRY(check_ctx(ctx));
  if (ws && bytes < ctx->arena_bytes)
    return fail(MMX_EINVAL, "workspace smaller than mmx_workspace_bytes (" +
                                std::to_string(ctx->arena_bytes) + " bytes)");
  if (ws && (reinterpret_cast<uintptr_t>(ws) % kArenaAlign) != 0)
    return fail(MMX_EINVAL, "workspace must be 256-byte aligned");
  if (ws == ctx->arena) {
    ctx->stream = reinterpret_cast<hipStream_t>(stream);
    return MMX_OK;
  }
  // finish everything that uses the current arena, then move its contents
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->cap_stream) HIP_TRY(hipStreamSynchronize(ctx->cap_stream));
  ctx->heun_graphs.clear();
  ctx->rk_graphs.clear();
  ctx->epoch++;
  void* dst = ws;
  bool owned = false;
  if (!dst) {  // back to a library-owned arena
    HIP_TRY(hipMalloc(&dst, ctx->arena_bytes));
    owned = true;
  }
  const hipError_t e = hipMemcpy(dst, ctx->arena, ctx->arena_bytes, hipMemcpyDeviceToDevice);
  if (e != hipSuccess) {
    if (owned) (void)hipFree(dst);
    return fail(MMX_EHIP, std::string("workspace copy: ") + hipGetErrorString(e));
  }
  if (ctx->arena_owned) HIP_TRY(hipFree(ctx->arena));
  ctx->arena = dst;
  ctx->arena_owned = owned;
  arena_assign(ctx, dst);
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return MMX_OK;
}

// Checkpoint blob: header, then the saved first-same-as-last slope of every
// group (element type of the context, layout D1).
struct CkptHeader {
  char magic[8];
  int32_t prec, n_groups;
  uint64_t total_elems, shape_hash;
  double t, dt_prop, last_err;
  int64_t accepted, rejected;
};

uint64_t shape_hash(const mmx_ctx* ctx) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the group descriptions
  for (auto& gp : ctx->groups) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&gp->g);
    for (size_t i = 0; i < sizeof(mmx_group); ++i) h = (h ^ b[i]) * 1099511628211ull;
  }
  return h;
}

mmx_status mmx_checkpoint(const mmx_ctx* ctx, void* blob, size_t* bytes) {
  MMX_TRY(check_ctx(ctx));
  if (!bytes) return fail(MMX_EINVAL, "bytes is null");
  const size_t need = sizeof(CkptHeader) + ctx->total_elems * esize(ctx);
  if (!blob) {
    *bytes = need;
    return MMX_OK;
  }
  if (*bytes < need) return fail(MMX_EINVAL, "checkpoint buffer too small");
  if (!ctx->rk_valid || ctx->rk_epoch != ctx->epoch)
    return fail(MMX_ESTATE, "no adaptive run to checkpoint (or the configuration changed)");
  CkptHeader hd{};
  std::memcpy(hd.magic, "MMXCKPT1", 8);
  hd.prec = ctx->prec;
  hd.n_groups = (int32_t)ctx->groups.size();
  hd.total_elems = ctx->total_elems;
  hd.shape_hash = shape_hash(ctx);
  hd.t = ctx->rk_last.t;
  hd.dt_prop = ctx->rk_last.dt_prop;
  hd.last_err = ctx->rk_last.last_err;
  hd.accepted = ctx->rk_last.accepted;
  hd.rejected = ctx->rk_last.rejected;
  std::memcpy(blob, &hd, sizeof(hd));
  unsigned char* out = static_cast<unsigned char*>(blob) + sizeof(hd);
  for (auto& gp : ctx->groups) {
    const size_t nb = (size_t)gp->R * 3 * gp->N * esize(ctx);
    HIP_TRY(hipMemcpyAsync(out, gp->k[0].p, nb, hipMemcpyDeviceToHost, ctx->stream));
    out += nb;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  *bytes = need;
  return MMX_OK;
}

mmx_status mmx_restore(mmx_ctx* ctx, const void* blob, size_t bytes) {
  MMX_TRY(check_ctx(ctx));
  if (!blob || bytes < sizeof(CkptHeader)) return fail(MMX_EINVAL, "checkpoint too short");
  CkptHeader hd;
  std::memcpy(&hd, blob, sizeof(hd));
  if (std::memcmp(hd.magic, "MMXCKPT1", 8) != 0) return fail(MMX_EINVAL, "not a checkpoint");
  if (hd.prec != ctx->prec || hd.n_groups != (int32_t)ctx->groups.size() ||
      hd.total_elems != ctx->total_elems || hd.shape_hash != shape_hash(ctx))
    return fail(MMX_ESHAPE, "checkpoint of a different precision or group layout");
  if (bytes < sizeof(CkptHeader) + ctx->total_elems * esize(ctx))
    return fail(MMX_EINVAL, "checkpoint too short");
  const unsigned char* in = static_cast<const unsigned char*>(blob) + sizeof(hd);
  for (auto& gp : ctx->groups) {
    const size_t nb = (size_t)gp->R * 3 * gp->N * esize(ctx);
    HIP_TRY(hipMemcpyAsync(gp->k[0].p, in, nb, hipMemcpyHostToDevice, ctx->stream));
    in += nb;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->rk_last = RkState{};
  ctx->rk_last.t = hd.t;
  ctx->rk_last.dt_prop = hd.dt_prop;
  ctx->rk_last.last_err = hd.last_err;
  ctx->rk_last.accepted = hd.accepted;
  ctx->rk_last.rejected = hd.rejected;
  ctx->rk_valid = 1;
  ctx->rk_epoch = ctx->epoch;
  return MMX_OK;
}

mmx_status mmx_rk45_resume(mmx_ctx* ctx, void* m, double t_end, double tol, void* energy_trace,
                           int64_t trace_cap, mmx_rk_stats* stats) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m) return fail(MMX_EINVAL, "null array");
  if (!ctx->rk_valid || ctx->rk_epoch != ctx->epoch)
    return fail(MMX_ESTATE, "nothing to continue: no adaptive run or restored checkpoint "
                            "with the current configuration");
  const double t0 = ctx->rk_last.t, dt0 = ctx->rk_last.dt_prop;
  MMX_TRY(ctx->prec == MMX_F64
              ? rk45_impl<double>(ctx, m, t0, t_end, tol, dt0, nullptr, 0, energy_trace,
                                  trace_cap, stats, nullptr, true)
              : rk45_impl<float>(ctx, m, t0, t_end, tol, dt0, nullptr, 0, energy_trace,
                                 trace_cap, stats, nullptr, true));
  return take_nonfinite(ctx);
}

mmx_status mmx_sync(mmx_ctx* ctx) {
  MMX_TRY(check_ctx(ctx));
  return take_nonfinite(ctx);
}

mmx_status mmx_rk45_dts(mmx_ctx* ctx, double* dts, int64_t cap, int64_t* count) {
  MMX_TRY(check_ctx(ctx));
  if (!count) return fail(MMX_EINVAL, "count is null");
  const long long n = std::min<long long>(ctx->last_accepted, ctx->dts_cap);
  *count = n;
  if (dts && cap > 0 && n > 0) {
    HIP_TRY(hipMemcpy(dts, ctx->dts.p, std::min<long long>(n, cap) * sizeof(double),
                      hipMemcpyDeviceToHost));
  }
  return MMX_OK;
}

mmx_status mmx_energy(mmx_ctx* ctx, const void* m, void* E) {
  MMX_TRY(check_ctx(ctx));
  MMX_TRY(check_materials(ctx));
  if (!m || !E) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? energy_impl<double>(ctx, m, E) : energy_impl<float>(ctx, m, E);
}

mmx_status mmx_topological_charge(mmx_ctx* ctx, const void* m, void* Q) {
  MMX_TRY(check_ctx(ctx));
  if (!m || !Q) return fail(MMX_EINVAL, "null array");
  return ctx->prec == MMX_F64 ? topo_impl<double>(ctx, m, Q) : topo_impl<float>(ctx, m, Q);
}

mmx_status mmx_topological_charge_noalloc(mmx_ctx* ctx, const void* m, void* Q) {
  MMX_TRY(check_ctx(ctx));
  if (!m || !Q) return fail(MMX_EINVAL, "null array");
  if (!ctx->scratch) return fail(MMX_ESTATE, "static scratch not set up");
  for (auto& gp : ctx->groups) {
    const size_t need = (size_t)gp->R * topo_blocks(*gp);
    if (need > kScratchDoubles)
      return fail(MMX_EINVAL, "mmx_topological_charge_noalloc: a group needs " +
                                  std::to_string(need) + " partial sums (replicas x " +
                                  std::to_string(topo_blocks(*gp)) +
                                  " workgroups), above the static scratch of " +
                                  std::to_string(kScratchDoubles));
  }
  return ctx->prec == MMX_F64 ? topo_into<double>(ctx, m, Q, ctx->scratch)
                              : topo_into<float>(ctx, m, Q, ctx->scratch);
}

mmx_status mmx_set_tiles(mmx_ctx* ctx, int32_t group, const int32_t tiles[3]) {
  MMX_TRY(check_group_idx(ctx, group));
  ctx->epoch++;
  if (!tiles) return fail(MMX_EINVAL, "tiles is null");
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  Group& G = *ctx->groups[group];
  return ctx->prec == MMX_F64 ? apply_tiles<double>(G, tiles[0], tiles[1], tiles[2])
                              : apply_tiles<float>(G, tiles[0], tiles[1], tiles[2]);
}

mmx_status mmx_get_tiles(mmx_ctx* ctx, int32_t group, int32_t tiles[3]) {
  MMX_TRY(check_group_idx(ctx, group));
  if (!tiles) return fail(MMX_EINVAL, "tiles is null");
  const Group& G = *ctx->groups[group];
  tiles[0] = G.L;
  tiles[1] = G.Wy;
  tiles[2] = G.Wz;
  return MMX_OK;
}

mmx_status mmx_set_path(mmx_ctx* ctx, int32_t path) {
  MMX_TRY(check_ctx(ctx));
  ctx->epoch++;
  if (path != MMX_PATH_AUTO && path != MMX_PATH_STAGED && path != MMX_PATH_FUSED)
    return fail(MMX_EINVAL, "unknown path");
  ctx->path = path;
  return MMX_OK;
}

mmx_status mmx_autotune(mmx_ctx* ctx) {
  MMX_TRY(check_ctx(ctx));
  ctx->epoch++;
  MMX_TRY(check_materials(ctx));
  return ctx->prec == MMX_F64 ? autotune_impl<double>(ctx) : autotune_impl<float>(ctx);
}

}  // extern "C"

#include "fno_api.h"
#include "surrogate.h"
