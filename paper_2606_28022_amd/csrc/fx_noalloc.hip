// Embedding field for callers that cannot allocate device memory.
//
// The chunked field pass (k_field_partial, k_field_reduce) needs partial sums
// of nchunk x n_shells doubles.  Here they live in a file-scope device array
// of FX_NOALLOC_SCRATCH_DOUBLES doubles, held by every GPU the library runs
// on until the process ends.  Host code never passes the array's own name to
// a kernel (on the host it is only a stand-in symbol): init_device looks up
// its device address once per device with that device current, and every
// launch takes that address.  Calls on one GPU share the array, so calls
// that overlap on one GPU (other threads or streams) race; the partial sums
// are fully overwritten by every call, nothing has to start at zero.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fx_host.hpp"
#include "fx_kernels.hpp"

namespace fx {

static __device__ __align__(256) double scratch[FX_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void noalloc_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) throw FxError(FX_E_INVALID, "device index out of range");
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw FxError(FX_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(p);
}

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || !g_scratch_ptr[device])
    throw FxError(FX_E_STATE, "scratch of this device not set up");
  return g_scratch_ptr[device];
}

void Ctx::field_noalloc(const double* d_q, double* d_phi) {
  if (Nsh > FX_NOALLOC_SCRATCH_DOUBLES)
    throw FxError(FX_E_INVALID, "system has " + std::to_string(Nsh) + " shells; the allocation-free field pass "
                                "handles at most " + std::to_string((long long)FX_NOALLOC_SCRATCH_DOUBLES));
  double* part = noalloc_scratch(device);
  // as many source chunks as the scratch holds, at most those of the
  // allocating pass
  const int by_grid = std::max(1, std::min(64, (Ne + 255) / 256 > 0 ? 2048 / ((Ne + 255) / 256) : 1));
  const int nchunk = std::max(1, std::min(by_grid, (int)(FX_NOALLOC_SCRATCH_DOUBLES / std::max(1, Nsh))));
  dim3 grid((Ne + 255) / 256, nchunk);
  hipLaunchKernelGGL(k_field_partial, grid, dim3(256), 0, stream, dev_system(), d_q, nchunk, part);
  hipLaunchKernelGGL(k_field_reduce, dim3((Nsh + 255) / 256), dim3(256), 0, stream, Nsh, nchunk,
                     (const double*)part, d_phi);
  check(hipGetLastError(), "field (no allocation)");
}

}  // namespace fx

extern "C" int fx_embedding_field_noalloc(fx_ctx* ctx, const double* d_dq, double* d_phi) {
  if (!ctx || !d_dq || !d_phi) return FX_E_INVALID;
  try {
    fx::Ctx& c = ctx->c;
    if (!c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    c.field_noalloc(d_dq, d_phi);
    c.last_error.clear();
    return FX_OK;
  } catch (const fx::FxError& e) {
    ctx->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return FX_E_INVALID;
  }
}
