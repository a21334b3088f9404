// noalloc.hip -- lensed_loglike_noalloc: the plain log-likelihood of one point
// (Sec. 3.2 Eq. 17) with every intermediate in a static device array, so that
// no call allocates (for callers that cannot: graph capture, serving loops).
//
// `scratch` below is a device array. In host code its name is a host-side
// stand-in, not a device address: the address of each device's copy comes from
// hipGetSymbolAddress, once per device with that device current, and only that
// pointer is handed to the kernels.
#include <cstring>
#include <mutex>

#include "internal.h"
#include "kernels.h"
#include "plan.h"

namespace lensed {
namespace {

__device__ __align__(256) unsigned char scratch[LENSED_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::once_flag scratch_once[MAX_DEVICES];
void* scratch_ptr[MAX_DEVICES];
hipError_t scratch_err[MAX_DEVICES];

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace
}  // namespace lensed

extern "C" int lensed_loglike_noalloc(const lensed_system* sys, const float* theta, double* logl, void* stream) {
  using namespace lensed;
  const int rc = validate_system(nullptr, sys, true, -1);
  if (rc) return rc;
  if (!theta || !logl) return LENSED_INVALID_ARGUMENT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LENSED_HIP_ERROR;
  if (dev < 0 || dev >= MAX_DEVICES) return LENSED_NOT_SUPPORTED;
  std::call_once(scratch_once[dev], [dev] { scratch_err[dev] = hipGetSymbolAddress(&scratch_ptr[dev], HIP_SYMBOL(scratch)); });
  if (scratch_err[dev] != hipSuccess || !scratch_ptr[dev]) return LENSED_HIP_ERROR;

  // the layout of lensed_loglike's workspace, inside the static array
  const TileShape ts = TileCache::latency_best(*sys);   // the tile lensed_loglike uses
  SysDesc sd = make_desc(*sys, ts);
  const size_t npix = (size_t)sd.H * sd.W;
  const size_t off_pc = 0;
  const size_t off_p64 = up256(off_pc + sizeof(PointConst));
  const size_t off_psf = up256(off_p64 + sizeof(PointConst64));
  const size_t off_cc = up256(off_psf + 3 * sizeof(float) * sd.ph * sd.pw);
  const size_t off_ce = up256(off_cc + sizeof(int));
  const size_t off_L = up256(off_ce + sizeof(CuspEntry) * (size_t)sd.n_rtiles * (RENDER_BLOCK / 64));
  const size_t off_part = up256(off_L + sizeof(float) * npix);
  const size_t total = up256(off_part + sizeof(float2) * sd.n_ptiles);
  if (total > (size_t)LENSED_NOALLOC_SCRATCH_BYTES) return LENSED_TOO_LARGE;

  char* base = (char*)scratch_ptr[dev];
  PointConst* pc = (PointConst*)(base + off_pc);
  PointConst64* p64 = (PointConst64*)(base + off_p64);
  CuspList cl{(CuspEntry*)(base + off_ce), (int*)(base + off_cc)};   // count cleared by the prologue kernel
  sd.psfn = (float*)(base + off_psf);
  float* L = (float*)(base + off_L);
  float2* part = (float2*)(base + off_part);   // every tile writes its own sum
  hipStream_t st = (hipStream_t)stream;
  WorkArgs w;
  std::memset(&w, 0, sizeof(w));
  w.single = sd;
  if (launch_prologue(theta, 1, pc, p64, nullptr, sd, nullptr, 1, cl.count, st) != hipSuccess ||
      launch_render(w, pc, p64, L, sd.n_rtiles, cl, st) != hipSuccess ||
      launch_psf(w, L, nullptr, part, 1, sd.n_ptiles, square_psf_code(sd.ph, sd.pw), sd.TW, sd.TH, sd.ph, sd.pw,
                 st) != hipSuccess ||
      launch_finalize(part, nullptr, nullptr, 1, sd.n_ptiles, logl, st) != hipSuccess)
    return LENSED_HIP_ERROR;
  return LENSED_OK;
}
