// stk_asm_noalloc: the star-patch solve of stk_asm with its patch-output
// buffer (the scratch between the batched patch solves and the node sums)
// in a fixed device array instead of the hierarchy's own buffer, for callers
// that cannot allocate device memory around the call. The call itself makes
// no allocation of any kind.
#include <mutex>
#include <string>

#include "../../include/stk.h"
#include "stk_internal.h"

using namespace stk;

// Same definition as in stk_api.hip (the opaque handle of the C ABI).
struct stk_hier {
  Hier H;
};

namespace {

// Patch outputs of stk_asm_noalloc: d 3^d values per vertex of the level.
// Each GPU the library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

stk_status fail_na(stk_status st, const std::string& m) {
  set_last_error(m);
  return st;
}

// Device address of `scratch` on the current device, looked up once per
// device (host code never uses the array's own name as an address).
stk_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail_na(STK_EDEVICE, "no current HIP device");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail_na(STK_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return STK_OK;
}

}  // namespace

extern "C" {

stk_status stk_asm_noalloc(stk_hier* h, int level, int dtype, const void* r, void* y, void* stream) {
  if (!h) return fail_na(STK_EINVAL, "hierarchy is NULL");
  Hier& H = h->H;
  if (H.sv.phase == Hier::SV_ARNOLDI || H.sv.phase == Hier::SV_RESIDUAL || H.sv.phase == Hier::SV_FINISH)
    return fail_na(STK_EBUSY, "a resumable solve is in progress on this hierarchy");
  if (level < 1 || level >= H.L) return fail_na(STK_EINVAL, "level out of range");
  if (dtype != STK_F64 && !(dtype == STK_F32 && H.mixed))
    return fail_na(STK_EINVAL, dtype == STK_F32 ? "STK_F32 needs a hierarchy set up with mixed=1" : "unknown dtype");
  if (!r || !y || r == y) return fail_na(STK_EINVAL, "r, y must be distinct non-NULL buffers");
  const Level& L = H.lv[level];
  const size_t per = dtype == STK_F64 ? 8 : 4;
  // patch outputs per vertex: d (2k-1)^d for velocity degree k
  const size_t side = (size_t)(2 * H.deg - 1);
  const size_t need = (size_t)H.dim * (H.dim == 2 ? side * side : side * side * side) * (size_t)L.nvert * per;
  if (need > kScratchBytes)
    return fail_na(STK_EINVAL, "level needs " + std::to_string(need) + " B of patch outputs; the static buffer holds " +
                                   std::to_string(kScratchBytes) + " B");
  void* z = nullptr;
  const stk_status st = scratch_ptr(&z);
  if (st != STK_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  H.stream = s;
  // every entry of the patch outputs that the node sums read is written by
  // the patch solves of the same call, so the previous contents never matter
  if (dtype == STK_F64) launch_asm<double>(H, L, (const double*)r, (double*)y, s, static_cast<double*>(z));
  else launch_asm<float>(H, L, (const float*)r, (float*)y, s, static_cast<float*>(z));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_na(STK_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return STK_OK;
}

}  // extern "C"
