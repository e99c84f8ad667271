// qt_contract_batch_noalloc: the contraction of qt_contract_batch for one
// plan with its whole device workspace (intermediates, exponent and max
// slots, step tables, per-slice results) in a static device array, for
// callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy until the process ends.  In host code its name is
// only a stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; every use from
// the host goes through that address.  All calls on one GPU share the array
// and it keeps the last call's contents: the tables are uploaded again
// whenever the array holds another plan's layout, buffers that must start
// at zero are cleared by the kernels of each call, and calls that overlap on
// one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qt_internal.h"

namespace qt {
namespace {

constexpr int64_t kScratchBytes = QT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};         // device address of `scratch` per device
uint64_t g_owner[kMaxDevices] = {};    // workspace layout the device's array holds

// Device address of this device's array (set up on first use).
qt_status scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QT_EUNSUPPORTED, "qt_contract_batch_noalloc: device id too large");
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QT_EHIP, std::string("qt_contract_batch_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_ptr[dev];
  return QT_OK;
}

}  // namespace
}  // namespace qt

using namespace qt;

extern "C" qt_status qt_contract_batch_noalloc(qt_plan* plan, int32_t n_points, const double* gammas,
                                               const double* betas, int64_t slice_begin, int64_t slice_end,
                                               qt_amp* out, double* per_slice_out, void* hip_stream) {
  try {
    if (!plan || n_points <= 0 || !out) return fail(QT_EINVAL, "qt_contract_batch_noalloc: bad arguments");
    const int p = plan->net.p;
    if (p > 0 && (!gammas || !betas)) return fail(QT_EINVAL, "qt_contract_batch_noalloc: null parameters");
    const int64_t ns = 1ll << plan->slice_vars.size();
    if (slice_begin < 0 || slice_end > ns || slice_begin >= slice_end)
      return fail(QT_EINVAL, "qt_contract_batch_noalloc: slice range outside [0, n_slices)");
    if (((slice_end - slice_begin) * n_points << plan->open_vars.size()) > (1ll << 28))
      return fail(QT_EINVAL, "qt_contract_batch_noalloc: slice range too long for one call");
    int dev = 0;
    QT_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    char* region = nullptr;
    QT_TRY(scratch_of(dev, &region));
    return contract_in_region(*plan, region, kScratchBytes, &g_owner[dev], n_points, gammas, betas, slice_begin,
                              slice_end, out, per_slice_out, (hipStream_t)hip_stream);
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_contract_batch_noalloc: ") + ex.what());
  }
}
