// noalloc.hip -- fsmi_eval_poses_noalloc: fsmi_eval_poses for callers that
// cannot allocate device memory.  Its scratch -- the per-beam partial results
// summed into each pose's value, and the queue head the persistent waves take
// their items from -- lives in the file-scope array below instead of the
// context's grow-only work area.  Each device the library runs on holds its
// own copy of the array (kScratchBytes) until the process ends; its device
// address is resolved once per device, with that device current, when a
// context is created, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fsmi_internal.h"

namespace fsmi {
namespace {
constexpr int64_t kScratchItems = (int64_t)1 << 21;   // (pose, beam) items of per-beam partials
constexpr size_t kCounterOffset = (size_t)kScratchItems * 8;
constexpr size_t kScratchBytes = kCounterOffset + 256;  // + the 64-bit queue head
constexpr int kMaxDevices = 64;
}  // namespace
}  // namespace fsmi

static __device__ __align__(256) unsigned char scratch[fsmi::kScratchBytes];

namespace fsmi {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  // with `device` current (fsmi_create has set it): this device's copy
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}
}  // namespace fsmi

extern "C" fsmi_status fsmi_eval_poses_noalloc(fsmi_ctx ctx, const fsmi_params* params,
                                               const fsmi_map* map, int64_t n_poses,
                                               const double* poses, int64_t n_beams,
                                               const double* beam_dir, double sigma,
                                               double max_range, double w, double* mi_pose,
                                               double* mi_beam) {
  using namespace fsmi;
  if (!ctx) return FSMI_E_INVAL;
  if (n_poses < 0 || n_beams < 0) return fail(ctx, FSMI_E_INVAL, "negative count");
  if (!mi_beam && n_beams > 0 && n_poses > kScratchItems / n_beams)
    return fail(ctx, FSMI_E_CAPACITY,
                "fsmi_eval_poses_noalloc: n_poses * n_beams exceeds the static scratch of "
                "2^21 (pose, beam) items (pass mi_beam to lift the limit)");
  void* base = scratch_of(ctx->device);
  if (!base) return fail(ctx, FSMI_E_DEVICE, "fsmi_eval_poses_noalloc: static scratch not resolved");
  PoseScratch ws;
  ws.beams = reinterpret_cast<double*>(base);
  ws.counter = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(base) + kCounterOffset);
  return eval_poses_checked(ctx, params, map, n_poses, poses, n_beams, beam_dir, sigma, max_range,
                            w, mi_pose, mi_beam, &ws);
}
