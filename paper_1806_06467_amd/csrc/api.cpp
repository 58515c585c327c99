// Host runtime behind the C ABI of include/fresnel.h: argument checks, the per-context cache
// of float64-built tables, and the launches.
//
// Tables (Sec. 2.3: sin/cos arrays; Sec. 1.1: transfer function and lens chirp): every phase
// is formed from an exact integer (k^2, c^2 or an index product) times a float64 constant,
// reduced to a fraction of a turn in float64, evaluated in float64 and only then rounded to
// float. Separability keeps them O(n) per plane instead of O(n^2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fresnel.h"
#include "fr_internal.h"
#include "fr_runtime.h"

using fr::PlaneArgs;

namespace {

thread_local std::string g_status_text;
thread_local hipError_t g_last_hip = hipSuccess;

}  // namespace

namespace fr {

double frac_turn(double t) { return t - std::nearbyint(t); }

float2 turn_to_c64(double turns, double scale) {
  const double f = frac_turn(turns);
  return make_float2(float(std::cos(2.0 * M_PI * f) * scale), float(std::sin(2.0 * M_PI * f) * scale));
}

int signed_index(int k, int n) { return (2 * k < n) ? k : k - n; }

int record_hip(hipError_t e) {
  if (e == hipSuccess) return FR_OK;
  g_last_hip = e;
  return FR_EHIP;
}

Ctx::~Ctx() {
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  drop_graphs();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  for (auto &kv : tables) (void)hipFree(kv.second);
  tables.clear();
  for (auto &t : timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : event_pool) (void)hipEventDestroy(e);
}

hipEvent_t Ctx::take_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void timing_hook(void *user, hipStream_t s, const char *name, int tag, int phase) {
  Ctx *c = static_cast<Ctx *>(user);
  hipEvent_t e = c->take_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  if (phase == 0) {
    c->pending_start = e;
  } else if (c->pending_start) {
    c->timed.push_back({std::string(name) + "/" + std::to_string(tag), c->pending_start, e});
    c->pending_start = nullptr;
  } else {
    c->event_pool.push_back(e);
  }
}

int Ctx::sweep_variant(int n) const {
  // the autotuner's choice, else variant 0
  int k = 0;
  if (auto it = tuned_variant.find(n); it != tuned_variant.end()) k = it->second;
  if (k < 0 || k >= fr::fresnel_variants(n)) k = 0;
  return k;
}

Ctx::GemmChoice Ctx::gemm_choice(const CGemmArgs &g) const {
  auto it = tuned_gemm.find({g.M, g.N, g.K, g.transA, g.transB});
  return it == tuned_gemm.end() ? default_gemm : it->second;
}

LaunchHook Ctx::hook() {
  LaunchHook h;
  if (profiling) {
    h.fn = timing_hook;
    h.user = this;
  }
  return h;
}

hipGraphExec_t Ctx::find_graph(const std::string &key) {
  for (auto &g : graphs)
    if (g.key == key) return g.exec;
  return nullptr;
}

void Ctx::keep_graph(const std::string &key, hipGraphExec_t exec) {
  if (graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(graphs.front().exec);
    graphs.erase(graphs.begin());
  }
  graphs.push_back({key, exec});
}

void Ctx::drop_graphs() {
  for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

int Ctx::graph_call(const std::string &key, hipStream_t s, const char *name, int tag,
                    const std::function<int(hipStream_t)> &body) {
  if (hipGraphExec_t g = find_graph(key)) {
    const LaunchHook h = hook();
    h(s, name, tag, 0);
    hipError_t e = hipGraphLaunch(g, s);
    h(s, name, tag, 1);
    return record_hip(e);
  }
  int st = body(s);
  if (st < 0) return st;
  if (!capture_stream) {
    hipError_t e = hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return record_hip(e);
  }
  hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return record_hip(e);
  const bool prof = profiling;
  profiling = false;
  capturing = true;
  const int cap = body(capture_stream);
  capturing = false;
  profiling = prof;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(capture_stream, &graph);
  if (cap < 0 || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return cap < 0 ? cap : record_hip(e);
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return record_hip(e);
  keep_graph(key, exec);
  return FR_OK;
}

int Ctx::upload(const TableKey &key, const void *host, size_t bytes, hipStream_t s, void **out) {
  auto it = tables.find(key);
  if (it != tables.end()) {
    *out = it->second;
    return FR_OK;
  }
  if (capturing || no_alloc) return FR_ESTATE;
  void *d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return FR_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return record_hip(e);
  }
  tables.emplace(key, d);
  *out = d;
  return FR_OK;
}

// The cache is bounded at call boundaries only: a call that starts with max_tables or more
// cached waits for the device and drops every table (and the graphs that reference them)
// before it fetches anything, so every table pointer a call holds stays valid to its end
// (upload never frees). The cache thus holds at most max_tables plus what one call adds.
int Ctx::begin_call() {
  if (tables.size() < max_tables) return FR_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return record_hip(e);
  drop_graphs();
  for (auto &kv : tables) (void)hipFree(kv.second);
  tables.clear();
  return FR_OK;
}

static uint64_t bits(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof b);
  return b;
}

// per-pass twiddle table of the FFT plan for edge n (built in float64)
int Ctx::twiddles(int n, hipStream_t s, const float2 **out) {
  TableKey key{kRoots, n, 0, 0, 0, 0};
  if (auto it = tables.find(key); it != tables.end()) {
    *out = static_cast<const float2 *>(it->second);
    return FR_OK;
  }
  std::vector<float2> h(std::max(fresnel_twiddle_count(n), 1));
  fresnel_twiddle_build(n, h.data());
  void *d;
  int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
  *out = static_cast<const float2 *>(d);
  return st;
}

int Ctx::mr(int n, hipStream_t s, MrPlane *out, unsigned plan) {
  int np = 0, rad[kMrMaxPass];
  if (!mr_plan(n, &np, rad)) return FR_EUNSUPPORTED;
  if (plan == 0)
    if (auto it = tuned_plan.find(n); it != tuned_plan.end()) plan = it->second;
  if (plan == 0) plan = mr_default_plan(n);
  if (plan != 0) {
    // another factorisation into supported radices (validated by the caller that chose it)
    np = 0;
    while (np < kMrMaxPass && ((plan >> (5 * np)) & 31u)) {
      rad[np] = int((plan >> (5 * np)) & 31u);
      ++np;
    }
  }
  TableKey key{kMrTw, n, uint64_t(mr_pack(np, rad)), 0, 0, 0};
  void *d = nullptr;
  if (auto it = tables.find(key); it != tables.end()) {
    d = it->second;
  } else {
    std::vector<float2> h(std::max(mr_twiddle_count(np, rad), 1));
    mr_twiddle_build(np, rad, h.data());
    int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
    if (st != FR_OK) return st;
  }
  out->n = n;
  out->npass = np;
  out->plan = mr_pack(np, rad);
  out->tw = static_cast<const float2 *>(d);
  out->first = 0;
  return FR_OK;
}

// h[k] = exp(-i pi lambda z k~^2 / (n dx)^2) / n  (signed index k~; 1/n folds the IFFT scale)
int Ctx::transfer(int n, double dx, double lam, double z, hipStream_t s, const float2 **out) {
  TableKey key{kTransfer, n, bits(dx), bits(lam), bits(z), 0};
  if (auto it = tables.find(key); it != tables.end()) {
    *out = static_cast<const float2 *>(it->second);
    return FR_OK;
  }
  std::vector<float2> h(n);
  const double coef = -lam * z / (2.0 * (double(n) * dx) * (double(n) * dx));
  for (int k = 0; k < n; ++k) {
    const long long kt = signed_index(k, n);
    h[k] = turn_to_c64(double(kt * kt) * coef, 1.0 / double(n));
  }
  void *d;
  int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
  *out = static_cast<const float2 *>(d);
  return st;
}

// l[i] = exp(-i pi c(i)^2 dx^2 / (lambda f)), c(i) = i - n/2
int Ctx::lens(int n, double dx, double lam, double f, hipStream_t s, const float2 **out) {
  TableKey key{kLens, n, bits(dx), bits(lam), bits(f), 0};
  if (auto it = tables.find(key); it != tables.end()) {
    *out = static_cast<const float2 *>(it->second);
    return FR_OK;
  }
  std::vector<float2> h(n);
  const double coef = -dx * dx / (2.0 * lam * f);
  for (int i = 0; i < n; ++i) {
    const long long c = i - n / 2;
    h[i] = turn_to_c64(double(c * c) * coef, 1.0);
  }
  void *d;
  int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
  *out = static_cast<const float2 *>(d);
  return st;
}

// Direct Fresnel step (Sec. 1.1; Sec. 2.3, Eq. 2, the quadratic phase read as
// exp(+i pi r^2 / (lambda z))):
//   pre[i]  = (-1)^i exp(i pi c(i)^2 dx^2 (1/z - 1/f) / lambda)  (a thin lens of focal f folded
//             in; 1/f = 0 without one)
//   post[k] = (-1)^k exp(i pi c(k)^2 dx2^2 / (lambda z)) (dx / sqrt(lambda |z|)) e^{-i pi sign(z)/4},
//             dx2 = lambda |z| / (n dx)   (z of either sign; over z < 0 the transforms' kernel
//             sign flips, kTowardSource)
// so that post[ky] post[kx] DFT2(pre[y] pre[x] U)[ky][kx] is the step: the signs centre the
// transform on pixel n/2 (exp(-2 pi i c(k) c(i) / n) = W^{ki} (-1)^{k + i} (-1)^{n/2}, the last
// factor squaring to 1 over the two axes) and the two roots make the constant dx^2/(i lambda z).
// With `inverse` the output phases of the two axes carry dx2 / dx each: the factor (dx2 / dx)^2
// that turns the adjoint into the inverse step.
int Ctx::direct_phases(int n, double dx, double lam, double z, double f, hipStream_t s, const float2 **pre,
                       const float2 **post, bool inverse) {
  const TableKey kpre{kDirectPre, n, bits(dx), bits(lam), bits(z), bits(f)};
  const TableKey kpost{kDirectPost, n, bits(dx), bits(lam), bits(z), inverse ? 1u : 0u};
  auto build = [&](const TableKey &key, bool input, const float2 **out) -> int {
    if (auto it = tables.find(key); it != tables.end()) {
      *out = static_cast<const float2 *>(it->second);
      return FR_OK;
    }
    std::vector<float2> h(n);
    const double dx2 = lam * std::fabs(z) / (double(n) * dx);
    const double coef = input ? dx * dx * (1.0 / z - (f != 0.0 ? 1.0 / f : 0.0)) / (2.0 * lam)
                              : dx2 * dx2 / (2.0 * lam * z);
    // (the inverse's (dx2 / dx)^2 is split over the two axes' tables)
    const double scale = input ? 1.0 : dx / std::sqrt(lam * std::fabs(z)) * (inverse ? dx2 / dx : 1.0);
    // the root of dx^2 / (i lambda z) is (dx / sqrt(lambda |z|)) exp(-i pi sign(z) / 4)
    const double root_turn = input ? 0.0 : (z > 0 ? -0.125 : 0.125);
    for (int i = 0; i < n; ++i) {
      const long long c = i - n / 2;
      const double turns = double(c * c) * coef + 0.5 * double(i & 1) + root_turn;
      h[i] = turn_to_c64(turns, scale);
    }
    void *d;
    const int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
    *out = static_cast<const float2 *>(d);
    return st;
  };
  const int st = build(kpre, true, pre);
  return st != FR_OK ? st : build(kpost, false, post);
}

// W[k][m] = exp(-2 pi i (k - M/2)(m - N/2) du / n_d), M x N row-major (or its transpose, N x M)
int Ctx::mft_matrix(int m_out, int n_in, double n_d, double du, hipStream_t s, const float2 **out,
                    bool transposed) {
  TableKey key{kMft, m_out, uint64_t(n_in), bits(n_d), bits(du), transposed ? 1u : 0u};
  if (auto it = tables.find(key); it != tables.end()) {
    *out = static_cast<const float2 *>(it->second);
    return FR_OK;
  }
  std::vector<float2> h(size_t(m_out) * n_in);
  const double coef = -du / n_d;
  for (int k = 0; k < m_out; ++k) {
    const long long a = k - m_out / 2;
    for (int m = 0; m < n_in; ++m) {
      const long long b = m - n_in / 2;
      h[transposed ? size_t(m) * m_out + k : size_t(k) * n_in + m] = turn_to_c64(double(a * b) * coef, 1.0);
    }
  }
  void *d;
  int st = upload(key, h.data(), h.size() * sizeof(float2), s, &d);
  *out = static_cast<const float2 *>(d);
  return st;
}

// G[i][a] = exp(-(c(i) - xi_a)^2 / (2 p^2)), xi_a = (a - (n_act-1)/2) p, p = n_d / n_act
// G[i][a] = exp(-(c(i) - xi_a)^2 / (2 p^2)) in float64, rounded once: actuators centred on the
// pupil at pitch p = n_d / n_act, sigma one pitch
static void dm_influence_fill(int n, int n_d, int n_act, float *h) {
  const double p = double(n_d) / double(n_act);
  for (int i = 0; i < n; ++i) {
    const double c = double(i - n / 2);
    for (int a = 0; a < n_act; ++a) {
      const double xi = (double(a) - (n_act - 1) / 2.0) * p;
      const double d = c - xi;
      h[size_t(i) * n_act + a] = float(std::exp(-d * d / (2.0 * p * p)));
    }
  }
}

int Ctx::dm_influence(int n, int n_d, int n_act, hipStream_t s, const float **out) {
  TableKey key{kDm, n, uint64_t(n_d), uint64_t(n_act), 0, 0};
  if (auto it = tables.find(key); it != tables.end()) {
    *out = static_cast<const float *>(it->second);
    return FR_OK;
  }
  std::vector<float> h(size_t(n) * n_act);
  dm_influence_fill(n, n_d, n_act, h.data());
  void *d;
  int st = upload(key, h.data(), h.size() * sizeof(float), s, &d);
  *out = static_cast<const float *>(d);
  return st;
}

void Ctx::dm_band(int n, int n_d, int n_act, int *lo, int *hi) {
  const auto key = std::make_tuple(n, n_d, n_act);
  auto it = dm_bands.find(key);
  if (it == dm_bands.end()) {
    std::vector<float> h(size_t(n) * n_act);
    dm_influence_fill(n, n_d, n_act, h.data());
    int l = n, u = 0;
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < n_act; ++a)
        if (h[size_t(i) * n_act + a] != 0.0f) {
          l = std::min(l, i);
          u = std::max(u, i + 1);
        }
    if (u <= l) l = u = 0;
    it = dm_bands.emplace(key, std::make_pair(l, u)).first;
  }
  *lo = it->second.first;
  *hi = it->second.second;
}


// workspace of one MFT: the n x m c64 intermediate, then (256-byte aligned) the float64
// split-K partials
size_t mft_t_bytes(int n, int m) { return (size_t(n) * size_t(m) * sizeof(float2) + 255) & ~size_t(255); }
size_t mft_ws_bytes(int n, int m) {
  return mft_t_bytes(n, m) + size_t(kMaxSplit) * size_t(n) * size_t(m) * 2 * sizeof(double);
}

static CGemmArgs gemm_args() {
  CGemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.alpha_re = 1.0;
  return g;
}

hipError_t run_gemm(Ctx *ctx, CGemmArgs &g, void *partial, size_t partial_elems, hipStream_t s, int cfg,
                    int split) {
  if (cfg < 0) {
    const Ctx::GemmChoice c = ctx->gemm_choice(g);
    cfg = c.tile;
    split = c.split;
  }
  if (split <= 0) split = cgemm_split_for(g.M, g.N, g.K, cfg);
  split = std::min(split, kMaxSplit);
  while (split > 1 && size_t(split) * size_t(g.M) * size_t(g.N) > partial_elems) split /= 2;
  return launch_cgemm_split(g, split, cfg, partial, s, ctx->hook());
}

int mft_forward_impl(Ctx *ctx, const float2 *in, int n_in, int ld_in, int m_out, double n_d,
                     double du, const MftOut &o, void *ws, hipStream_t s, size_t partial_cap) {
  const float2 *w;
  int st = ctx->mft_matrix(m_out, n_in, n_d, du, s, &w);
  if (st != FR_OK) return st;
  float2 *t = static_cast<float2 *>(ws);
  void *partial = static_cast<char *>(ws) + mft_t_bytes(n_in, m_out);
  const size_t pcap = std::min(size_t(kMaxSplit) * n_in * m_out, partial_cap);
  // T = E W^T  (n_in x m_out)
  CGemmArgs g1 = gemm_args();
  g1.M = n_in; g1.N = m_out; g1.K = n_in;
  g1.A = in; g1.lda = ld_in;
  g1.B = w; g1.ldb = n_in; g1.transB = 1;
  g1.C = t; g1.ldc = m_out;
  hipError_t e = run_gemm(ctx, g1, partial, pcap, s);
  if (e != hipSuccess) return record_hip(e);
  // out = (du / n_d) W T (* mask), optionally + weight |out|^2 into the intensity
  CGemmArgs g2 = gemm_args();
  g2.M = m_out; g2.N = m_out; g2.K = n_in;
  g2.A = w; g2.lda = n_in;
  g2.B = t; g2.ldb = m_out;
  g2.C = o.out; g2.ldc = o.ld_out; g2.skip_c = o.skip_out ? 1 : 0;
  g2.alpha_re = du / n_d;
  g2.mask = o.mask; g2.ldm = m_out;
  g2.intensity = o.intensity; g2.ldi = m_out; g2.weight = o.weight;
  e = run_gemm(ctx, g2, partial, pcap, s);
  return e == hipSuccess ? FR_OK : record_hip(e);
}

int mft_adjoint_impl(Ctx *ctx, const float2 *in, int m_in, int ld_in, float2 *out, int n_out,
                     int ld_out, double n_d, double du, float alpha, float beta,
                     const float2 *cin, int ld_cin, const float *mask, void *ws, hipStream_t s) {
  // with Wt = W^T (n_out x m_in): conj(W) = conj(Wt)^T and W^H = conj(Wt), so both GEMMs read
  // the matrix with k contiguous
  const float2 *wt;
  int st = ctx->mft_matrix(m_in, n_out, n_d, du, s, &wt, true);
  if (st != FR_OK) return st;
  float2 *t = static_cast<float2 *>(ws);
  void *partial = static_cast<char *>(ws) + mft_t_bytes(n_out, m_in);
  const size_t pcap = size_t(kMaxSplit) * n_out * m_in;
  // T = E_B conj(W) = E_B conj(Wt)^T  (m_in x n_out)
  CGemmArgs g1 = gemm_args();
  g1.M = m_in; g1.N = n_out; g1.K = m_in;
  g1.A = in; g1.lda = ld_in;
  g1.B = wt; g1.ldb = m_in; g1.transB = 1; g1.conjB = 1;
  g1.C = t; g1.ldc = n_out;
  hipError_t e = run_gemm(ctx, g1, partial, pcap, s);
  if (e != hipSuccess) return record_hip(e);
  // out = alpha (du / n_d) conj(Wt) T + beta cin (* mask)
  CGemmArgs g2 = gemm_args();
  g2.M = n_out; g2.N = n_out; g2.K = m_in;
  g2.A = wt; g2.lda = m_in; g2.conjA = 1;
  g2.B = t; g2.ldb = n_out;
  g2.C = out; g2.ldc = ld_out;
  g2.alpha_re = double(alpha) * (du / n_d);
  g2.beta = beta; g2.Cin = cin; g2.ldcin = ld_cin;
  g2.mask = mask; g2.ldm = n_out;
  e = run_gemm(ctx, g2, partial, pcap, s);
  return e == hipSuccess ? FR_OK : record_hip(e);
}

bool plane_size_supported(int n) {
  int np, rad[kMrMaxPass];
  return fresnel_size_supported(n) || mr_plan(n, &np, rad);
}

// end of the group that starts at plane i: at most `cap` planes, and either `planes` planes
// (a tuned group size) or, with planes = 0, as many as fit the last-level cache together
static int group_end(const PlaneArgs *args, int count, int i, int cap, int planes = 0) {
  if (planes > 0) return std::min(count, i + std::min(planes, cap));
  size_t bytes = 0;
  int j = i;
  while (j < count && j - i < cap) {
    const size_t b = size_t(args[j].n) * size_t(args[j].n) * sizeof(float2);
    if (j > i && bytes + b > kCacheGroupBytes) break;
    bytes += b;
    ++j;
  }
  return j;
}

// Planes whose edge has a register-resident power-of-two plan go through the two-sweep kernels,
// those of one edge together; the others (mixed-radix edges) through the persistent mixed-radix
// kernels, one launch per sweep for each group of planes, the planes ordered by edge so that a
// group of one edge can take that edge's compile-time plan. The planes of a batch are
// independent, so their order across the paths does not matter.
int run_planes(Ctx *ctx, PlaneArgs *args, int count, hipStream_t s) {
  std::vector<PlaneArgs> rest;
  std::map<int, std::vector<PlaneArgs>> pow2;
  for (int i = 0; i < count; ++i) {
    if (fresnel_size_supported(args[i].n))
      pow2[args[i].n].push_back(args[i]);
    else
      rest.push_back(args[i]);
  }
  std::stable_sort(rest.begin(), rest.end(), [](const PlaneArgs &a, const PlaneArgs &b) { return a.n < b.n; });
  for (auto &[n, v] : pow2) {
    const float2 *root;
    int st = ctx->twiddles(n, s, &root);
    if (st != FR_OK) return st;
    int planes = 0;
    if (auto it = ctx->tuned_group.find(n); it != ctx->tuned_group.end()) planes = it->second;
    const int nv = int(v.size());
    for (int i = 0; i < nv;) {
      const int j = group_end(v.data(), nv, i, kMaxBatch, planes);
      hipError_t e = launch_fresnel_batch(v.data() + i, j - i, n, root, s, ctx->hook(), ctx->sweep_variant(n));
      if (e != hipSuccess) return record_hip(e);
      i = j;
    }
  }
  const int nr = int(rest.size());
  for (int i = 0; i < nr;) {
    const int j = group_end(rest.data(), nr, i, kMrMaxBatch);
    MrBatch b;
    b.count = j - i;
    b.total = 0;
    for (int k = 0; k < b.count; ++k) {
      int st = ctx->mr(rest[i + k].n, s, &b.p[k]);
      if (st != FR_OK) return st;
      b.p[k].pa = rest[i + k];
    }
    hipError_t e = launch_mr_batch(b, ctx->mr_rows_per_cu, ctx->mr_cols_per_cu, ctx->cus, s, ctx->hook());
    if (e != hipSuccess) return record_hip(e);
    i = j;
  }
  return FR_OK;
}

}  // namespace fr

// ============================================================================================
// C ABI
// ============================================================================================
using fr::Ctx;

extern "C" {

int fr_create(fr_ctx **ctx, int device, const char *autotune_path) {
  if (!ctx) return FR_EINVAL;
  *ctx = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return fr::record_hip(e);
  if (device < 0 || device >= ndev) return FR_EINVAL;
  e = hipSetDevice(device);
  if (e != hipSuccess) return fr::record_hip(e);
  // the allocation-free entry point's scratch array: its address on this device (once per device;
  // a failure is kept and reported by that entry point, the other entry points do not need it)
  (void)fr::noalloc_setup(device);
  Ctx *c = new Ctx();
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->cus = cus;
  fr::mr_resident(c->mr_rows_per_cu, c->mr_cols_per_cu);
  if (autotune_path) {
    const int st = fr_autotune_load(reinterpret_cast<fr_ctx *>(c), autotune_path);
    if (st != FR_OK) {
      delete c;
      return st;
    }
  }
  *ctx = reinterpret_cast<fr_ctx *>(c);
  return FR_OK;
}

int fr_destroy(fr_ctx *ctx) {
  delete reinterpret_cast<Ctx *>(ctx);
  return FR_OK;
}

int fr_set_cache_limit(fr_ctx *ctx_, int32_t max_tables) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx || max_tables < 1) return FR_EINVAL;
  ctx->max_tables = size_t(max_tables);
  return FR_OK;
}

const char *fr_status_string(int status) {
  switch (status) {
    case FR_OK: return "ok";
    case FR_EINVAL: return "invalid argument";
    case FR_EUNSUPPORTED: return "unsupported size or combination";
    case FR_EWORKSPACE: return "workspace missing or too small";
    case FR_ENOMEM: return "device allocation for a cached table failed";
    case FR_ESTATE: return "a table was not cached (a graph recording or an allocation-free call cannot build it)";
    case FR_EHIP:
      g_status_text = std::string("HIP error: ") + hipGetErrorString(g_last_hip);
      return g_status_text.c_str();
    default:
      if (status > 0) return "ok with sampling warning";
      return "unknown status";
  }
}

int fr_fft_size_supported(int32_t n) { return fr::plane_size_supported(n) ? 1 : 0; }

static int check_plane(const fr_plane &p) {
  if (!p.field || p.n <= 0) return FR_EINVAL;
  if (!(p.dx_m > 0) || !(p.wavelength_m > 0) || !std::isfinite(p.z_m)) return FR_EINVAL;
  if (!std::isfinite(p.lens_focal_m)) return FR_EINVAL;
  if (p.flags & ~FR_ADJOINT) return FR_EINVAL;
  if (!fr::plane_size_supported(p.n)) return FR_EUNSUPPORTED;
  return FR_OK;
}

static int plane_warnings(const fr_plane &p) {
  return (std::fabs(p.z_m) > double(p.n) * p.dx_m * p.dx_m / p.wavelength_m) ? FR_W_AS_UNDERSAMPLED
                                                                             : 0;
}

// arguments of one batched call, checked before the context is touched: FR_EINVAL /
// FR_EUNSUPPORTED, else the OR of the per-plane warnings
static int check_batch(const fr_plane *planes, int32_t count) {
  if (!planes || count <= 0) return FR_EINVAL;
  int warn = 0;
  for (int i = 0; i < count; ++i) {
    int st = check_plane(planes[i]);
    if (st != FR_OK) return st;
    warn |= plane_warnings(planes[i]);
  }
  return warn;
}

// the tables and launches of one batched call on stream s
static int batch_body(Ctx *ctx, const fr_plane *planes, int32_t count, hipStream_t s) {
  std::vector<PlaneArgs> args(count);
  for (int i = 0; i < count; ++i) {
    const fr_plane &p = planes[i];
    PlaneArgs &a = args[i];
    std::memset(&a, 0, sizeof a);
    a.field = reinterpret_cast<float2 *>(p.field);
    a.amp = p.amp;
    a.opd = p.opd_m;
    a.n = p.n;
    a.win = p.n;
    a.inv_lambda = float(1.0 / p.wavelength_m);
    a.flags = p.flags;
    int st = ctx->transfer(p.n, p.dx_m, p.wavelength_m, p.z_m, s, &a.h);
    if (st != FR_OK) return st;
    if (p.lens_focal_m != 0.0) {
      st = ctx->lens(p.n, p.dx_m, p.wavelength_m, p.lens_focal_m, s, &a.lens);
      if (st != FR_OK) return st;
    }
  }
  return fr::run_planes(ctx, args.data(), count, s);
}

int fresnel_step_batched(fr_ctx *ctx_, const fr_plane *planes, int32_t count, void *stream) {
  const int warn = check_batch(planes, count);
  if (warn < 0) return warn;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  int st = batch_body(ctx, planes, count, s);
  return st != FR_OK ? st : warn;
}

int fresnel_step_batched_graph(fr_ctx *ctx_, const fr_plane *planes, int32_t count, void *stream) {
  const int warn = check_batch(planes, count);
  if (warn < 0) return warn;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  // every value the launches bake in: the plane entries field by field, and the stream
  std::string key("fresnel_batch");
  auto put = [&](const void *p, size_t b) { key.append(static_cast<const char *>(p), b); };
  for (int i = 0; i < count; ++i) {
    const fr_plane &p = planes[i];
    const void *ptrs[3] = {p.field, p.amp, p.opd_m};
    const double vals[4] = {p.dx_m, p.wavelength_m, p.z_m, p.lens_focal_m};
    const int32_t ints[2] = {p.n, p.flags};
    put(ptrs, sizeof ptrs);
    put(vals, sizeof vals);
    put(ints, sizeof ints);
  }
  put(&s, sizeof s);
  int st = ctx->graph_call(key, s, "fresnel_graph", count,
                           [&](hipStream_t cs) { return batch_body(ctx, planes, count, cs); });
  return st != FR_OK ? st : warn;
}

int fresnel_step(fr_ctx *ctx, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                 double z_m, const float *amp, const float *opd_m, double lens_focal_m,
                 int32_t flags, void *stream) {
  fr_plane p;
  p.field = field;
  p.amp = amp;
  p.opd_m = opd_m;
  p.dx_m = dx_m;
  p.wavelength_m = wavelength_m;
  p.z_m = z_m;
  p.lens_focal_m = lens_focal_m;
  p.n = n;
  p.flags = flags;
  return fresnel_step_batched(ctx, &p, 1, stream);
}

int fr_plan_route(double w0_m, double z_waist_m, double wavelength_m, int32_t n, double dx_m, double z_from_m,
                  double z_to_m, fr_route_step *steps, int32_t capacity) {
  if (!steps || capacity < 2 || n <= 0 || !(w0_m > 0) || !(wavelength_m > 0) || !(dx_m > 0)) return FR_EINVAL;
  for (double v : {w0_m, z_waist_m, wavelength_m, dx_m, z_from_m, z_to_m})
    if (!std::isfinite(v)) return FR_EINVAL;
  const double z_r = M_PI * w0_m * w0_m / wavelength_m;
  const double d_from = z_from_m - z_waist_m, d_to = z_to_m - z_waist_m;
  const bool near_from = std::fabs(d_from) <= z_r, near_to = std::fabs(d_to) <= z_r;
  // pitch of the waist plane (near planes share it; a far plane's pitch is lambda |d| / (n dx_w))
  const double dx_w = near_from ? dx_m : wavelength_m * std::fabs(d_from) / (double(n) * dx_m);
  auto far_pitch = [&](double d) { return wavelength_m * std::fabs(d) / (double(n) * dx_w); };
  int k = 0;
  auto add = [&](int kind, double z, double dx_in, double dx_out) {
    steps[k].kind = kind;
    steps[k].z_m = z;
    steps[k].dx_in_m = dx_in;
    steps[k].dx_out_m = dx_out;
    ++k;
  };
  if (z_to_m == z_from_m) return 0;
  if (near_from && near_to) {
    add(FR_ROUTE_AS, z_to_m - z_from_m, dx_w, dx_w);
    return k;
  }
  // through the waist plane
  if (!near_from) add(FR_ROUTE_DIRECT_INVERSE, d_from, dx_m, dx_w);
  if (near_from && d_from != 0.0) add(FR_ROUTE_AS, -d_from, dx_w, dx_w);
  if (near_to && d_to != 0.0) add(FR_ROUTE_AS, d_to, dx_w, dx_w);
  if (!near_to) add(FR_ROUTE_DIRECT, d_to, dx_w, far_pitch(d_to));
  return k;
}

int fresnel_direct(fr_ctx *ctx_, fr_c64 *field, int32_t n, double dx_m, double wavelength_m, double z_m,
                   const float *amp, const float *opd_m, double lens_focal_m, int32_t flags, double *dx_out_m,
                   void *stream) {
  if (!field || !dx_out_m || n <= 0 || (flags & ~(FR_ADJOINT | FR_INVERSE)) || flags == (FR_ADJOINT | FR_INVERSE))
    return FR_EINVAL;
  const bool inverse = flags & FR_INVERSE;
  if (inverse && (amp || opd_m || lens_focal_m != 0.0)) return FR_EINVAL;
  if (!(dx_m > 0) || !(wavelength_m > 0) || z_m == 0.0 || !std::isfinite(dx_m) || !std::isfinite(wavelength_m) ||
      !std::isfinite(z_m) || !std::isfinite(lens_focal_m))
    return FR_EINVAL;
  if (!fr::fresnel_size_supported(n)) return FR_EUNSUPPORTED;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  PlaneArgs a;
  std::memset(&a, 0, sizeof a);
  a.field = reinterpret_cast<float2 *>(field);
  a.amp = amp;
  a.opd = opd_m;
  a.n = n;
  a.win = n;
  a.inv_lambda = float(1.0 / wavelength_m);
  a.flags = (inverse ? FR_ADJOINT : flags) | (z_m < 0 ? fr::kTowardSource : 0);
  int st = ctx->direct_phases(n, dx_m, wavelength_m, z_m, lens_focal_m, s, &a.lens, &a.h, inverse);
  if (st != FR_OK) return st;
  const float2 *root;
  st = ctx->twiddles(n, s, &root);
  if (st != FR_OK) return st;
  e = fr::launch_direct_batch(&a, 1, n, root, s, ctx->hook());
  if (e != hipSuccess) return fr::record_hip(e);
  *dx_out_m = wavelength_m * std::fabs(z_m) / (double(n) * dx_m);
  return std::fabs(z_m) < double(n) * dx_m * dx_m / wavelength_m ? FR_W_DIRECT_UNDERSAMPLED : FR_OK;
}

}  // extern "C"

// ============================================================================================
// MFT entry points
// ============================================================================================
namespace {

int mft_common_checks(const void *in, const void *out, int n, int ld_n, int m, int ld_m,
                      double n_d, double du) {
  if (!in || !out) return FR_EINVAL;
  if (n <= 0 || m <= 0 || ld_n < n || ld_m < m) return FR_EINVAL;
  if (!(n_d > 0) || !std::isfinite(n_d) || !(du > 0) || !std::isfinite(du)) return FR_EINVAL;
  return FR_OK;
}

size_t mft_ws(int32_t n, int32_t m) { return fr::mft_ws_bytes(n, m); }

}  // namespace

extern "C" {

size_t mft_workspace_bytes(int32_t n_pupil, int32_t m_focal) {
  if (n_pupil <= 0 || m_focal <= 0) return 0;
  return mft_ws(n_pupil, m_focal);
}

int mft_forward(fr_ctx *ctx_, const fr_c64 *in, int32_t n_in, int32_t ld_in, fr_c64 *out,
                int32_t m_out, int32_t ld_out, double n_d, double du, const float *out_mask,
                void *ws, size_t ws_bytes, void *stream) {
  int st = mft_common_checks(in, out, n_in, ld_in, m_out, ld_out, n_d, du);
  if (st != FR_OK) return st;
  if (!ws || ws_bytes < mft_ws(n_in, m_out)) return FR_EWORKSPACE;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int c = ctx->begin_call(); c != FR_OK) return c;
  fr::MftOut o;
  o.out = reinterpret_cast<float2 *>(out);
  o.ld_out = ld_out;
  o.mask = out_mask;
  st = fr::mft_forward_impl(ctx, reinterpret_cast<const float2 *>(in), n_in, ld_in, m_out, n_d, du,
                            o, ws, static_cast<hipStream_t>(stream));
  if (st != FR_OK) return st;
  return (du > n_d / double(n_in)) ? FR_W_MFT_ALIASED : FR_OK;
}

int mft_adjoint(fr_ctx *ctx_, const fr_c64 *in, int32_t m_in, int32_t ld_in, fr_c64 *out,
                int32_t n_out, int32_t ld_out, double n_d, double du, float alpha, float beta,
                const float *out_mask, void *ws, size_t ws_bytes, void *stream) {
  int st = mft_common_checks(in, out, n_out, ld_out, m_in, ld_in, n_d, du);
  if (st != FR_OK) return st;
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return FR_EINVAL;
  if (!ws || ws_bytes < mft_ws(n_out, m_in)) return FR_EWORKSPACE;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int c = ctx->begin_call(); c != FR_OK) return c;
  st = fr::mft_adjoint_impl(ctx, reinterpret_cast<const float2 *>(in), m_in, ld_in,
                            reinterpret_cast<float2 *>(out), n_out, ld_out, n_d, du, alpha, beta,
                            nullptr, 0, out_mask, ws, static_cast<hipStream_t>(stream));
  if (st != FR_OK) return st;
  return (du > n_d / double(n_out)) ? FR_W_MFT_ALIASED : FR_OK;
}

}  // extern "C"

// ============================================================================================
// Kernel timing
// ============================================================================================
extern "C" {

int fr_profile_enable(fr_ctx *ctx_, int enable) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  ctx->profiling = enable != 0;
  return FR_OK;
}

int fr_profile_read(fr_ctx *ctx_, int32_t max_entries, char *names, int32_t name_len,
                    double *total_ms, int64_t *launches, int32_t *n_entries) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx || max_entries < 0 || (max_entries > 0 && (!names || name_len <= 1 || !total_ms || !launches)) ||
      !n_entries)
    return FR_EINVAL;
  std::map<std::string, std::pair<double, int64_t>> acc;
  int status = FR_OK;
  for (auto &t : ctx->timed) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) status = fr::record_hip(e);
    auto &a = acc[t.name];
    a.first += ms;
    a.second += 1;
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
  }
  ctx->timed.clear();
  int i = 0;
  for (auto &kv : acc) {
    if (i >= max_entries) break;
    std::snprintf(names + size_t(i) * name_len, size_t(name_len), "%s", kv.first.c_str());
    total_ms[i] = kv.second.first;
    launches[i] = kv.second.second;
    ++i;
  }
  *n_entries = i;
  return status;
}

}  // extern "C"
