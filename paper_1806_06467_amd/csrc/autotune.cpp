// Autotuner: times the candidate kernel configurations of one workload shape and keeps the
// fastest in the context (Sec. 2.1 of the paper: profiling decides what to optimise; here the
// choice among equivalent kernel configurations is made by measurement on the device at hand).
//
// Candidates (all compute the same result up to float32 rounding order):
//   Fresnel plane of edge n: the tile variants of the power-of-two sweeps (row lines per block,
//     column tile width) and the distinct pass orders of the mixed-radix plan;
//   MFT n <-> m: the GEMM tile configurations (64 x 64, 64 x 128, 128 x 128) of the two GEMMs
//     of the forward and of the adjoint transform.
// Each candidate runs once untimed, then kReps times between events; the minimum counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/fresnel.h"
#include "fr_internal.h"
#include "fr_runtime.h"

namespace fr {

namespace {

constexpr int kReps = 3;
constexpr int kMaxOrders = 6;

struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  void *get(size_t bytes, hipStream_t s) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs.push_back(p);
    if (hipMemsetAsync(p, 0, bytes, s) != hipSuccess) return nullptr;
    return p;
  }
};

// milliseconds of the fastest of kReps timed runs of fn(s) (after one untimed run), or -1
template <class F>
float time_min(hipStream_t s, F fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.f;
  float best = -1.f;
  if (fn() == hipSuccess && hipStreamSynchronize(s) == hipSuccess) {
    for (int r = 0; r < kReps; ++r) {
      (void)hipEventRecord(a, s);
      if (fn() != hipSuccess) {
        best = -1.f;
        break;
      }
      (void)hipEventRecord(b, s);
      float ms = 0.f;
      if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        best = -1.f;
        break;
      }
      if (best < 0.f || ms < best) best = ms;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

int tune_fresnel(Ctx *ctx, int n, hipStream_t s) {
  if (!plane_size_supported(n)) return FR_EUNSUPPORTED;
  Scratch mem;
  float2 *field = static_cast<float2 *>(mem.get(size_t(n) * n * sizeof(float2), s));
  if (!field) return FR_ENOMEM;
  PlaneArgs pa;
  std::memset(&pa, 0, sizeof pa);
  pa.field = field;
  pa.n = n;
  pa.win = n;
  pa.inv_lambda = float(1.0 / 550e-9);
  int st = ctx->transfer(n, 25e-6, 550e-9, 1.0, s, &pa.h);
  if (st != FR_OK) return st;
  const LaunchHook none;
  // power-of-two sweeps: tile variants
  if (fresnel_size_supported(n)) {
    const float2 *tw;
    st = ctx->twiddles(n, s, &tw);
    if (st != FR_OK) return st;
    int best = 0;
    float best_ms = -1.f;
    for (int v = 0; v < fresnel_variants(n); ++v) {
      const float ms = time_min(s, [&] { return launch_fresnel_batch(&pa, 1, n, tw, s, none, v); });
      if (ms < 0.f) return record_hip(hipGetLastError());
      if (best_ms < 0.f || ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    ctx->tuned_variant[n] = best;
  }
  // mixed-radix sweeps (used for this edge in batches of mixed edges): pass orders
  unsigned plans[kMaxOrders + 1];
  int np = 0;
  int count = mr_plan_orders(n, kMaxOrders, plans, &np);
  // the edge's default order (a register-resident plan) is always among the candidates
  if (const unsigned d = mr_default_plan(n); d != 0u && std::find(plans, plans + count, d) == plans + count)
    plans[count++] = d;
  unsigned best_plan = 0;
  float best_ms = -1.f;
  for (int c = 0; c < count; ++c) {
    MrBatch b;
    b.count = 1;
    b.total = 0;
    st = ctx->mr(n, s, &b.p[0], plans[c]);
    if (st != FR_OK) return st;
    b.p[0].pa = pa;
    const float ms = time_min(s, [&] { return launch_mr_batch(b, ctx->mr_rows_per_cu, ctx->mr_cols_per_cu, ctx->cus, s, none); });
    if (ms < 0.f) return record_hip(hipGetLastError());
    if (best_ms < 0.f || ms < best_ms) {
      best_ms = ms;
      best_plan = plans[c];
    }
  }
  if (count > 0) ctx->tuned_plan[n] = best_plan;
  return record_hip(hipStreamSynchronize(s));
}

int tune_mft(Ctx *ctx, int n, int m, hipStream_t s) {
  if (n <= 0 || m <= 0) return FR_EINVAL;
  Scratch mem;
  const size_t big = size_t(std::max(n, m)) * std::max(n, m);
  float2 *a = static_cast<float2 *>(mem.get(big * sizeof(float2), s));
  float2 *w = static_cast<float2 *>(mem.get(size_t(n) * m * sizeof(float2), s));
  float2 *t = static_cast<float2 *>(mem.get(size_t(n) * m * sizeof(float2), s));
  float2 *c = static_cast<float2 *>(mem.get(big * sizeof(float2), s));
  const size_t pcap = size_t(kMaxSplit) * n * m;
  void *partial = mem.get(pcap * 2 * sizeof(double), s);
  if (!a || !w || !t || !c || !partial) return FR_ENOMEM;
  // the four GEMM shapes of mft_forward(n -> m) and mft_adjoint(m -> n)
  std::vector<CGemmArgs> shapes;
  auto add = [&](int M, int N, int K, const float2 *A, int lda, int ta, const float2 *B, int ldb, int tb,
                 float2 *C, int ldc) {
    CGemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.M = M, g.N = N, g.K = K;
    g.A = A, g.lda = lda, g.transA = ta;
    g.B = B, g.ldb = ldb, g.transB = tb;
    g.C = C, g.ldc = ldc;
    g.alpha_re = 1.0;
    shapes.push_back(g);
  };
  add(n, m, n, a, n, 0, w, n, 1, t, m);  // forward: T = E W^T
  add(m, m, n, w, n, 0, t, m, 0, c, m);  // forward: W T
  add(m, n, m, a, m, 0, w, m, 1, t, n);  // adjoint: E_B conj(Wt)^T (Wt = W^T, n x m)
  add(n, n, m, w, m, 0, t, n, 0, c, n);  // adjoint: conj(Wt) T
  for (CGemmArgs &g : shapes) {
    Ctx::GemmChoice best{0, 0};
    float best_ms = -1.f;
    for (int cfg = 0; cfg < kGemmTiles; ++cfg) {
      // the tile's default split, and every power of two up to kMaxSplit that leaves slices of
      // at least 64 (the default is tried first, so it wins ties)
      std::vector<int> splits{0};
      for (int sp = 1; sp <= kMaxSplit && g.K / sp >= 64; sp *= 2)
        if (size_t(sp) * size_t(g.M) * size_t(g.N) <= pcap) splits.push_back(sp);
      for (int sp : splits) {
        const float ms = time_min(s, [&] { return run_gemm(ctx, g, partial, pcap, s, cfg, sp); });
        if (ms < 0.f) return record_hip(hipGetLastError());
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          best = {cfg, sp};
        }
      }
    }
    ctx->tuned_gemm[{g.M, g.N, g.K, g.transA, g.transB}] = best;
  }
  return record_hip(hipStreamSynchronize(s));
}

// a pass order read back from a file: radices the sweeps support (2-10, 12, 14, 15, 16), at
// most kMrMaxPass of them, whose product is the edge
bool valid_plan(int n, unsigned plan) {
  int np = 0, greedy[kMrMaxPass];
  if (!mr_plan(n, &np, greedy)) return false;
  long long prod = 1;
  int s = 0;
  for (; s < kMrMaxPass && ((plan >> (5 * s)) & 31u); ++s) {
    const int r = int((plan >> (5 * s)) & 31u);
    if (r < 2 || r == 11 || r == 13 || r > 16) return false;
    prod *= r;
  }
  // nothing after the last radix (shifts of 32 or more bits are avoided)
  const bool tail_clear = 5 * s >= 32 || (plan >> (5 * s)) == 0u;
  return s > 0 && tail_clear && prod == n;
}

}  // namespace

}  // namespace fr

using fr::Ctx;

extern "C" {

int fr_autotune(fr_ctx *ctx_, int32_t kind, int32_t a, int32_t b, void *stream) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  if (kind != FR_TUNE_FRESNEL && kind != FR_TUNE_MFT) return FR_EINVAL;
  if (a <= 0 || (kind == FR_TUNE_MFT && b <= 0)) return FR_EINVAL;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fr::record_hip(e);
  if (int st = ctx->begin_call(); st != FR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  const int st = kind == FR_TUNE_FRESNEL ? fr::tune_fresnel(ctx, a, s) : fr::tune_mft(ctx, a, b, s);
  ctx->profiling = prof;
  // recorded graphs bake in the kernel choices of their time
  (void)hipDeviceSynchronize();
  ctx->drop_graphs();
  return st;
}

int fr_autotune_save(fr_ctx *ctx_, const char *path) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx || !path) return FR_EINVAL;
  FILE *f = std::fopen(path, "w");
  if (!f) return FR_EINVAL;
  std::fprintf(f, "# fresnel autotune v1\n");
  for (auto &kv : ctx->tuned_variant) {
    auto g = ctx->tuned_group.find(kv.first);
    std::fprintf(f, "sweep %d %d %d\n", kv.first, kv.second, g == ctx->tuned_group.end() ? 0 : g->second);
  }
  for (auto &kv : ctx->tuned_plan) std::fprintf(f, "plan %d %u\n", kv.first, kv.second);
  if (ctx->default_gemm.tile >= 0)
    std::fprintf(f, "gemm_default %d %d\n", ctx->default_gemm.tile, ctx->default_gemm.split);
  for (auto &kv : ctx->tuned_gemm) {
    const auto &k = kv.first;
    std::fprintf(f, "gemm %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), kv.second.tile, kv.second.split);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? FR_OK : FR_EINVAL;
}

int fr_autotune_load(fr_ctx *ctx_, const char *path) {
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx || !path) return FR_EINVAL;
  FILE *f = std::fopen(path, "r");
  if (!f) return FR_EINVAL;
  // recorded graphs bake in the kernel choices of their time
  if (hipSetDevice(ctx->device) == hipSuccess) (void)hipDeviceSynchronize();
  ctx->drop_graphs();
  char line[256];
  int st = FR_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int n = 0, v = 0, M = 0, N = 0, K = 0, ta = 0, tb = 0, sp = 0;
    unsigned plan = 0;
    int fields = 0;
    if (std::sscanf(line, "gemm_default %d %d", &v, &sp) == 2) {
      if (v < -1 || v >= fr::kGemmTiles || sp < 0 || sp > fr::kMaxSplit) st = FR_EINVAL;
      else ctx->default_gemm = {v, sp};
    } else if ((fields = std::sscanf(line, "sweep %d %d %d", &n, &v, &sp)) >= 2) {
      if (fields == 2) sp = 0;
      if (!fr::fresnel_size_supported(n) || v < 0 || v >= fr::fresnel_variants(n) || sp < 0 || sp > fr::kMaxBatch)
        st = FR_EINVAL;
      else
        ctx->tuned_variant[n] = v, ctx->tuned_group[n] = sp;
    } else if (std::sscanf(line, "plan %d %u", &n, &plan) == 2) {
      if (!fr::valid_plan(n, plan)) st = FR_EINVAL;
      else ctx->tuned_plan[n] = plan;
    } else if ((fields = std::sscanf(line, "gemm %d %d %d %d %d %d %d", &M, &N, &K, &ta, &tb, &v, &sp)) >= 6) {
      if (fields == 6) sp = 0;
      if (M <= 0 || N <= 0 || K <= 0 || v < 0 || v >= fr::kGemmTiles || (ta & ~1) || (tb & ~1) || sp < 0 ||
          sp > fr::kMaxSplit)
        st = FR_EINVAL;
      else
        ctx->tuned_gemm[{M, N, K, ta, tb}] = {v, sp};
    } else {
      st = FR_EINVAL;
    }
  }
  std::fclose(f);
  return st;
}

}  // extern "C"
