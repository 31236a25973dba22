// Allocation-free variant of the silhouette monitor, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// Its working memory is one file-scope device array, `scratch`, of a fixed
// size: every GPU the library runs on holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel or a copy (in
// host code the name is only a stand-in for the symbol): the device address
// of each GPU's copy is looked up once per device, with that device current,
// by hipGetSymbolAddress, and kept.  Every call on one GPU shares that GPU's
// array, so calls that overlap on one GPU (two host threads, or two streams)
// race; the accumulators are cleared by a kernel at the start of each call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "snaplayout.h"

using namespace snap;

namespace {

// Largest graph the variant takes: 2^18 nodes (a 259k-node graph fits).
constexpr int32_t kMaxNodes = LAYOUT_NOALLOC_MAX_NODES;
// Byte offsets inside the array: two FP64 sums, sorted positions (8 B per
// node), node order, cluster of each sorted node, cluster starts (C + 1 <=
// n + 1 entries).
constexpr size_t kOffAcc = 0;
constexpr size_t kOffYs = 256;
constexpr size_t kOffOrder = kOffYs + 8 * size_t(kMaxNodes);
constexpr size_t kOffCs = kOffOrder + 4 * size_t(kMaxNodes);
constexpr size_t kOffCstart = kOffCs + 4 * size_t(kMaxNodes);
constexpr size_t kScratchBytes = (kOffCstart + 4 * (size_t(kMaxNodes) + 1) + 255) / 256 * 256;

}  // namespace

// 5 MiB + 512 B per GPU.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first call
// on that device, with the device current; the caller's current device is
// restored).
int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LAYOUT_E_UNSUPPORTED, "device %d beyond the %d the variant tracks", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "looking up the scratch array");
    if (!p) return fail(LAYOUT_E_DEVICE, "the scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return LAYOUT_OK;
}

}  // namespace

extern "C" {

int layout_silhouette_noalloc(layout_t* L, const int32_t* labels, double* si_out) {
  g_last_error.clear();
  HandleView v;
  int rc = handle_view(L, &v);
  if (rc != LAYOUT_OK) return rc;
  if (v.dim != 2) return fail(LAYOUT_E_UNSUPPORTED, "the silhouette monitor is 2D");
  if (v.n > kMaxNodes)
    return fail(LAYOUT_E_UNSUPPORTED,
                "layout_silhouette_noalloc takes at most %d nodes (the handle has %d); "
                "use layout_silhouette",
                kMaxNodes, v.n);
  SilhouetteInput in;
  rc = silhouette_input(labels, v.n, si_out, in);
  if (rc != LAYOUT_OK) return rc;
  unsigned char* base = nullptr;
  rc = scratch_address(v.dev, &base);
  if (rc != LAYOUT_OK) return rc;
  SilhouetteBuffers b;
  b.acc = reinterpret_cast<double*>(base + kOffAcc);
  b.Ys = reinterpret_cast<float2*>(base + kOffYs);
  b.order = reinterpret_cast<int32_t*>(base + kOffOrder);
  b.cs = reinterpret_cast<int32_t*>(base + kOffCs);
  b.cstart = reinterpret_cast<int32_t*>(base + kOffCstart);
  return silhouette_run(v.stream, v.Y, v.n, in, b, si_out);
}

}  // extern "C"
