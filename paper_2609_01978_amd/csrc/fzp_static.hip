// fzp_propagate_roi_static: fzp_propagate_roi with its workspace in a
// file-scope device array instead of a caller buffer, for callers that cannot
// allocate device memory.  Nothing here allocates: the array belongs to the
// code object (each GPU the library runs on holds its own copy until the
// process ends), and its device address is looked up once per device.

#include <mutex>

#include "fzp_internal.h"

namespace {

// The workspace of every fzp_propagate_roi_static call on a GPU.  In host
// code the name is only a stand-in for the symbol: kernels and copies take
// the address returned by hipGetSymbolAddress for the current device.
static __device__ __align__(256) char scratch[FZP_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
  void *ptr = nullptr;     // device address of `scratch` on this device
  uint64_t owner = 0;      // serial of the plan whose tables it holds (0: none)
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

}  // namespace

extern "C" fzp_status_t fzp_propagate_roi_static(fzp_plan_t p, double *roi_dev, void *stream) {
  if (!p || !roi_dev) {
    fzp::set_last_error("fzp_propagate_roi_static: NULL argument");
    return FZP_E_INVAL;
  }
  const size_t need = fzp::plan_workspace_bytes(p);
  if (need > (size_t)FZP_STATIC_SCRATCH_BYTES) {
    fzp::set_last_error("fzp_propagate_roi_static: the plan's workspace of " + std::to_string(need) +
                        " bytes exceeds FZP_STATIC_SCRATCH_BYTES (" + std::to_string(FZP_STATIC_SCRATCH_BYTES) +
                        "); plan with fewer chunk_rows, fewer instances or smaller ROIs");
    return FZP_E_NOMEM;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fzp::set_last_error(std::string("fzp_propagate_roi_static: current device: ") + hipGetErrorString(e));
    return FZP_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch &ds = g_dev[dev];
  if (!ds.ptr) {
    // once per device, with that device current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fzp::set_last_error(std::string("fzp_propagate_roi_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return FZP_E_DEVICE;
    }
    ds.ptr = ptr;
  }
  const uint64_t serial = fzp::plan_serial(p);
  const bool current = ds.owner == serial;
  ds.owner = 0;  // until the tables are built
  const fzp_status_t s = fzp::propagate_fixed_workspace(p, (char *)ds.ptr, current, roi_dev, (hipStream_t)stream);
  if (s == FZP_OK) ds.owner = serial;
  return s;
}
