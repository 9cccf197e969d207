// Two-site product for callers that cannot allocate device memory (work
// captured into a graph, serving loops, harnesses that forbid hipMalloc): the
// workspace of bsdmrg_heff_apply comes from a library-owned array in device
// memory, one copy per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "bsdmrg_internal.h"

namespace bsd {
int64_t heff_apply_bytes_prec(const bsdmrg_plan_s* P, int prec);
void heff_apply_compact(const bsdmrg_plan_s* P, int prec, const double* L, const double* W1, const double* W2,
                        const double* R, const double* psi, double* out, void* ws, hipStream_t s);
}  // namespace bsd

using namespace bsd;

// The scratch array.  In host code its name is only a stand-in for the
// device symbol: every host use goes through the address returned by
// hipGetSymbolAddress for the current device (scratch_base below).
static __device__ __align__(256) unsigned char scratch[BSDMRG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_base[kMaxDevices] = {};

// Device address of the current device's copy of the scratch array, looked
// up once per device (with that device current) and kept.
void* scratch_base() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) throw Error{BSDMRG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e)};
  if (dev < 0 || dev >= kMaxDevices) throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: device index out of range"};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error{BSDMRG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_base[dev] = p;
  }
  return g_base[dev];
}
}  // namespace

extern "C" bsdmrg_status bsdmrg_heff_apply_noalloc(bsdmrg_plan_t P, int32_t precision, const double* L,
                                                   const double* W1, const double* W2, const double* R,
                                                   const double* psi, double* out, hipStream_t stream) {
  try {
    if (!P) throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: plan is NULL"};
    if (!P->on_device) throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: plan was built host-only"};
    if (precision != BSDMRG_F64 && precision != BSDMRG_F32)
      throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: precision must be F64 or F32"};
    if (!L || !W1 || !W2 || !R || !psi || !out) throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: NULL operand"};
    if (psi == out) throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: out must not alias psi"};
    const int64_t need = heff_apply_bytes_prec(P, precision);
    if (need > (int64_t)BSDMRG_NOALLOC_SCRATCH_BYTES)
      throw Error{BSDMRG_EINVAL, "heff_apply_noalloc: the plan needs " + std::to_string(need) +
                                     " bytes of scratch in this precision; the maximum is " +
                                     std::to_string((int64_t)BSDMRG_NOALLOC_SCRATCH_BYTES)};
    heff_apply_compact(P, precision, L, W1, W2, R, psi, out, scratch_base(), stream);
    return BSDMRG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return BSDMRG_EINVAL;
  } catch (...) {
    set_error("unknown error");
    return BSDMRG_EINVAL;
  }
}
