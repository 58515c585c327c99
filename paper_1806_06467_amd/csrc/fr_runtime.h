// Per-context state of the host runtime: the cache of float64-built device tables.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "fr_internal.h"

namespace fr {

enum TableKind : int { kRoots = 1, kTransfer, kLens, kMft, kDm };
// (kind, size, then up to four parameter words: sizes or the bits of float64 parameters)
using TableKey = std::tuple<int, int, uint64_t, uint64_t, uint64_t, uint64_t>;

struct Ctx {
  int device = 0;
  std::map<TableKey, void *> tables;
  static constexpr size_t kMaxTables = 4096;

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

  ~Ctx();
  // copy `bytes` of host data to a new cached device buffer (waits on `s` for the copy)
  int upload(const TableKey &key, const void *host, size_t bytes, hipStream_t s, void **out);
  int roots(int n, hipStream_t s, const float2 **out);
  int transfer(int n, double dx, double lam, double z, hipStream_t s, const float2 **out);
  int lens(int n, double dx, double lam, double f, hipStream_t s, const float2 **out);
  int mft_matrix(int m_out, int n_in, double n_d, double du, hipStream_t s, const float2 **out);
  int dm_influence(int n, int n_d, int n_act, hipStream_t s, const float **out);
};

int record_hip(hipError_t e);

}  // namespace fr
