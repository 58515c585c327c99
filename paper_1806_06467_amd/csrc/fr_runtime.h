// Per-context state of the host runtime: the cache of float64-built device tables.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "fr_internal.h"

namespace fr {

// Planes are swept in groups whose fields fit the last-level cache together (at least one plane
// per group), every sweep of a group before the next group: the later sweeps of a plane then
// read what the previous one has just written from that cache instead of from HBM.
constexpr size_t kCacheGroupBytes = size_t(160) << 20;

// the default pass order of a mixed-radix edge n (sweeps_mr.hip): the order of its
// register-resident sweeps when it has them (the per-wavelength grids of a broadband model),
// else 0 (the greedy plan)
unsigned mr_default_plan(int n);

enum TableKind : int {
  kRoots = 1, kTransfer, kLens, kMft, kDm, kMrTw, kDirectPre, kDirectPost, kExactPrm, kMft64,
  kRoots64, kTransfer64, kLens64
};
// (kind, size, then up to four parameter words: sizes or the bits of float64 parameters)
using TableKey = std::tuple<int, int, uint64_t, uint64_t, uint64_t, uint64_t>;

struct Ctx {
  int device = 0;
  int cus = 256;  // compute units of the device
  // resident blocks per compute unit of the mixed-radix sweep instances (mr_resident)
  int mr_rows_per_cu[kMrPolicies] = {2, 2, 2, 2, 2, 2, 2, 2}, mr_cols_per_cu[kMrPolicies] = {1, 1, 1, 1, 1, 1, 1, 1};
  std::map<TableKey, void *> tables;
  size_t max_tables = 4096;  // fr_set_cache_limit
  // start of an entry point that may fetch tables (before the first fetch): trims the cache
  int begin_call();

  // kernel timing: while enabled, every launch is bracketed by HIP events on its stream
  struct Timed {
    std::string name;
    hipEvent_t start, stop;
  };
  bool profiling = false;
  hipEvent_t pending_start = nullptr;
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t take_event();
  LaunchHook hook();
  int sweep_variant(int n) const;

  // instantiated graphs of whole calls, keyed by every argument byte they bake in; dropped
  // together with the tables they reference
  struct GraphEntry {
    std::string key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  static constexpr size_t kMaxGraphs = 8;
  hipStream_t capture_stream = nullptr;
  bool capturing = false;  // table uploads are refused while a capture is open
  bool no_alloc = false;   // ... and during an allocation-free call
  hipGraphExec_t find_graph(const std::string &key);
  void keep_graph(const std::string &key, hipGraphExec_t exec);
  void drop_graphs();
  // Record-or-replay of a whole call: if a graph was recorded under `key`, launch it on `s`;
  // otherwise run `body(s)` eagerly (which builds every table it reads), then record the same
  // launch sequence on the context's own stream (no table may be missing then: FR_ESTATE) and
  // keep the instantiated graph under `key`. `name` / `tag` label the replay for the timing hook.
  int graph_call(const std::string &key, hipStream_t s, const char *name, int tag,
                 const std::function<int(hipStream_t)> &body);

  ~Ctx();
  // copy `bytes` of host data to a new cached device buffer (waits on `s` for the copy)
  int upload(const TableKey &key, const void *host, size_t bytes, hipStream_t s, void **out);
  int twiddles(int n, hipStream_t s, const float2 **out);
  // mixed-radix plan of edge n (radices and device twiddle table); FR_EUNSUPPORTED if none.
  // plan != 0 asks for that packed pass order instead of the tuned or default one.
  int mr(int n, hipStream_t s, MrPlane *out, unsigned plan = 0);

  // choices made by the autotuner (fr_autotune), consulted by every later call
  std::map<int, int> tuned_variant;                 // power-of-two sweep tile variant per edge
  std::map<int, int> tuned_group;                   // planes per launch group per edge (0: cache-sized)
  std::map<int, unsigned> tuned_plan;
  std::map<std::tuple<int, int, int>, std::pair<int, int>> dm_bands;  // dm_band results               // mixed-radix pass order per edge
  struct GemmChoice {
    int tile;   // tile configuration
    int split;  // K slices (0: the default for the tile)
  };
  std::map<std::tuple<int, int, int, int, int>, GemmChoice> tuned_gemm;  // (M, N, K, transA, transB)
  GemmChoice default_gemm{-1, 0};  // for shapes without an entry (tile -1: chosen by shape)
  GemmChoice gemm_choice(const CGemmArgs &g) const;
  int transfer(int n, double dx, double lam, double z, hipStream_t s, const float2 **out);
  int lens(int n, double dx, double lam, double f, hipStream_t s, const float2 **out);
  int direct_phases(int n, double dx, double lam, double z, double f, hipStream_t s, const float2 **pre,
                    const float2 **post, bool inverse = false);
  int mft_matrix(int m_out, int n_in, double n_d, double du, hipStream_t s, const float2 **out,
                 bool transposed = false);
  int dm_influence(int n, int n_d, int n_act, hipStream_t s, const float **out);
  // the rows [lo, hi) of that table with a nonzero entry (the Gaussians underflow float32 to
  // exactly 0 beyond about 14.4 actuator pitches from the outermost actuators); host arithmetic
  void dm_band(int n, int n_d, int n_act, int *lo, int *hi);
};

int record_hip(hipError_t e);

// Internal entry points shared by the C ABI and the train orchestration (arguments already
// validated; tables are fetched from / added to the context cache).
int run_planes(Ctx *ctx, PlaneArgs *args, int count, hipStream_t s);
struct MftOut {
  float2 *out = nullptr;
  int ld_out = 0;
  const float *mask = nullptr;
  double *intensity = nullptr;  // + weight |out|^2 in float64 (det grid, row stride = width)
  double weight = 0.0;
  bool skip_out = false;
};
// one complex GEMM with the tuned (or, cfg >= 0, the given) tile configuration and a split-K
// that fits `partial_elems` float64 complex partial sums
// split > 0 forces that many K slices (at most kMaxSplit, reduced to fit partial_elems)
hipError_t run_gemm(Ctx *ctx, CGemmArgs &g, void *partial, size_t partial_elems, hipStream_t s, int cfg = -1,
                    int split = 0);
// partial_cap: float64 complex split-K partial sums that fit ws after the n_in x m_out product
// (the split factor is reduced to fit; 0 runs every GEMM unsplit)
int mft_forward_impl(Ctx *ctx, const float2 *in, int n_in, int ld_in, int m_out, double n_d,
                     double du, const MftOut &o, void *ws, hipStream_t s, size_t partial_cap = SIZE_MAX);
size_t mft_t_bytes(int n, int m);  // the product T of an MFT pair, 256-byte aligned
// address of the allocation-free entry point's scratch array on `device` (hipGetSymbolAddress once
// per device, then cached); FR_EHIP if the runtime refuses
int noalloc_setup(int device);
// out = alpha (du/n_d) W^H in conj(W) + beta cin, * mask  (cin may alias out)
int mft_adjoint_impl(Ctx *ctx, const float2 *in, int m_in, int ld_in, float2 *out, int n_out,
                     int ld_out, double n_d, double du, float alpha, float beta,
                     const float2 *cin, int ld_cin, const float *mask, void *ws, hipStream_t s);
size_t mft_ws_bytes(int n_pupil, int m_focal);

}  // namespace fr
