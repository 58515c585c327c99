// The allocation-free entry point: mft_forward with its working memory (the n_in x m_out
// product T of the first GEMM and the split-K partial sums) in a file-scope device array instead
// of a caller workspace, for callers that cannot allocate device memory. Its kernels are those of
// mft_forward (Sec. 1.1: the matrix Fourier transform after Soummer et al.).
//
// The array is a fixed kNoallocScratchBytes per device, held until the process ends. Host code
// never passes the array's name to a kernel or a copy: its device address on each device is
// fetched once, with that device current, by hipGetSymbolAddress (noalloc_setup, called from
// fr_create) and kept per device; only that address is used. Every call on one device shares the
// array: calls that overlap on one device (two streams, two threads) race, so they must be
// ordered by the caller. Nothing in it needs clearing between calls: the first GEMM writes all of
// T and every split slice writes all of its partial sums before they are read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/fresnel.h"
#include "fr_internal.h"
#include "fr_runtime.h"

namespace fr {
namespace {

constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};
int g_status[kMaxDevices] = {};  // 0: not set up yet, FR_OK + 1: ready, < 0: the setup failed

}  // namespace

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return FR_EINVAL;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_status[device] == FR_OK + 1) return FR_OK;
  int current = -1;
  hipError_t e = hipGetDevice(&current);
  if (e == hipSuccess && current != device) e = hipSetDevice(device);
  void *ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (current >= 0 && current != device) (void)hipSetDevice(current);
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    g_status[device] = record_hip(e != hipSuccess ? e : hipErrorInvalidSymbol);
    return g_status[device];
  }
  g_ptr[device] = ptr;
  g_status[device] = FR_OK + 1;
  return FR_OK;
}

}  // namespace fr

using fr::Ctx;

extern "C" {

int mft_forward_noalloc(fr_ctx *ctx_, const fr_c64 *in, int32_t n_in, int32_t ld_in, fr_c64 *out,
                        int32_t m_out, int32_t ld_out, double n_d, double du, const float *out_mask,
                        void *stream) {
  if (!in || !out || n_in <= 0 || m_out <= 0 || ld_in < n_in || ld_out < m_out) return FR_EINVAL;
  if (!(n_d > 0) || !(du > 0) || !std::isfinite(n_d) || !std::isfinite(du)) return FR_EINVAL;
  // the product T must fit the array (the split-K partial sums take what is left, or none)
  const size_t tb = fr::mft_t_bytes(n_in, m_out);
  if (tb > fr::kNoallocScratchBytes) return FR_EWORKSPACE;
  Ctx *ctx = reinterpret_cast<Ctx *>(ctx_);
  if (!ctx) return FR_EINVAL;
  const int dev = ctx->device;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(fr::g_mutex);
    if (dev < 0 || dev >= fr::kMaxDevices) return FR_EINVAL;
    if (fr::g_status[dev] < 0) return fr::g_status[dev];
    if (fr::g_status[dev] != FR_OK + 1) return FR_ESTATE;
    base = fr::g_ptr[dev];
  }
  hipError_t e = hipSetDevice(dev);
  if (e != hipSuccess) return fr::record_hip(e);
  // no cache trim (it would free), no table builds (they would allocate): a missing MFT matrix is
  // FR_ESTATE with nothing launched
  fr::MftOut o;
  o.out = reinterpret_cast<float2 *>(out);
  o.ld_out = ld_out;
  o.mask = out_mask;
  const size_t pcap = (fr::kNoallocScratchBytes - tb) / (2 * sizeof(double));
  ctx->no_alloc = true;
  const int st = fr::mft_forward_impl(ctx, reinterpret_cast<const float2 *>(in), n_in, ld_in, m_out, n_d, du, o,
                                      base, static_cast<hipStream_t>(stream), pcap);
  ctx->no_alloc = false;
  if (st != FR_OK) return st;
  return (du > n_d / double(n_in)) ? FR_W_MFT_ALIASED : FR_OK;
}

}  // extern "C"
