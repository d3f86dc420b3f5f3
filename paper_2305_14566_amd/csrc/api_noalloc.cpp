// omniseg_stitch_tiles_noalloc: the stand-alone stitch with its tile-index
// grid in a library-owned device array instead of a caller workspace, for
// callers that cannot allocate device memory.
#include <mutex>

#include "plan.h"

using namespace omniseg;

namespace {

// Largest tile grid (ny * nx positions) the array holds: 4 MiB of int32.
constexpr int64_t kNoAllocGridMax = 1 << 20;

// The grid of every call on a device.  Each device holds its own copy for the
// life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device.
static __device__ __align__(256) int32_t scratch[kNoAllocGridMax];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Address of the current device's array, looked up on the first call there.
int32_t scratch_on_current_device(int32_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(OMNISEG_ERR_UNSUPPORTED, "device %d above %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(OMNISEG_ERR_HIP, "hipGetSymbolAddress of the stitch grid failed: %s", hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = static_cast<int32_t*>(g_scratch[dev]);
  return OMNISEG_OK;
}

}  // namespace

extern "C" {

int32_t omniseg_stitch_tiles_noalloc(int32_t tile, int32_t stride, int32_t height, int32_t width,
                                     int32_t vote_threshold, const float* tile_logits, const int32_t* tile_yx,
                                     int32_t n_tiles, uint8_t* mask, int64_t mask_pitch, float* logit,
                                     int64_t logit_pitch, omniseg_stream stream) {
  if (tile < 1 || tile > 4096 || stride < 1 || stride > tile || height < 1 || width < 1)
    return fail(OMNISEG_ERR_ARG, "bad stitch geometry");
  const int64_t ny = grid_count(height, tile, stride), nx = grid_count(width, tile, stride);
  if (ny * nx > kNoAllocGridMax)
    return fail(OMNISEG_ERR_UNSUPPORTED, "stitch grid of %lld tiles above the %lld the library array holds",
                (long long)(ny * nx), (long long)kNoAllocGridMax);
  if (n_tiles < 0) return fail(OMNISEG_ERR_ARG, "n_tiles < 0");
  if (vote_threshold < 0) return fail(OMNISEG_ERR_ARG, "vote_threshold %d < 0", vote_threshold);
  if (n_tiles > 0 && (!tile_logits || !tile_yx)) return fail(OMNISEG_ERR_ARG, "tile arrays are NULL");
  if (!mask || mask_pitch < width) return fail(OMNISEG_ERR_ARG, "bad mask buffer");
  if (logit && logit_pitch < width) return fail(OMNISEG_ERR_ARG, "bad logit pitch");
  if ((int64_t)n_tiles > ny * nx) return fail(OMNISEG_ERR_ARG, "more tiles than grid positions");
  int32_t* grid = nullptr;
  int32_t st = scratch_on_current_device(&grid);
  if (st) return st;
  hipStream_t sm = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  // the fill kernel sets every grid position to -1 before the tiles are
  // entered, so nothing of an earlier call's grid is read
  HIP_TRY(launch_grid_from_list(tile_yx, n_tiles, (int)ny, (int)nx, grid, sm));
  StitchArgs sa{};
  sa.logits = tile_logits;
  sa.tile_stride = (int64_t)tile * tile;
  sa.slot_off = 0;
  sa.index = grid;
  sa.ny = (int)ny;
  sa.nx = (int)nx;
  sa.T = tile;
  sa.s = stride;
  sa.Hk = height;
  sa.Wk = width;
  sa.mask = mask;
  sa.mask_pitch = mask_pitch;
  sa.logit = logit;
  sa.logit_pitch = logit_pitch;
  sa.vote = vote_threshold;
  HIP_TRY(launch_stitch(sa, sm));
  return OMNISEG_OK;
}

}  // extern "C"
