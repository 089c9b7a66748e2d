// hss_matvec_noalloc: the HSS matrix-vector product of hss_matvec with its
// temporaries in a fixed device array instead of allocations, for callers
// that cannot allocate device memory during the call.
#include <mutex>

#include "driver.h"

using namespace hss;

namespace {

constexpr size_t kScratchBytes = (size_t)HSS_NOALLOC_SCRATCH_BYTES;

// One copy per device, held until the process ends.  In host code the
// name stands for the host-side shadow only; kernels get the address that
// hipGetSymbolAddress returned for the device.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
double* scratch_ptr() {
  int dev = 0;
  HSS_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(HSS_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    HSS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(HSS_ERR_DEVICE, "no device address for the matvec scratch array");
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}

int64_t a256(int64_t elems) { return (elems + 31) & ~int64_t(31); }   // 256-byte steps of doubles

}  // namespace

extern "C" hss_status hss_matvec_noalloc(const hss_matrix* h, int32_t nrhs, const double* X, int64_t ldx,
                                         double* Y, int64_t ldy, void* stream) {
  try {
    if (!h || !X || !Y || nrhs < 1) throw Error(HSS_ERR_INVALID_ARG, "bad arguments");
    const Job& J = *h->job;
    const Problem& P = J.probs[h->k];
    if (ldx < P.n || ldy < P.n) throw Error(HSS_ERR_INVALID_ARG, "leading dimension < n");
    // layout in the array: xp, yp (n x nrhs each), xh, yh (mvtot x nrhs), ws (mvwstot x nrhs)
    const int64_t e_n = a256(P.n * nrhs), e_h = a256(J.mvtot * nrhs), e_w = a256(J.mvwstot * nrhs);
    const int64_t need = 2 * e_n + 2 * e_h + e_w;
    if ((size_t)need * sizeof(double) > kScratchBytes)
      throw Error(HSS_ERR_INVALID_ARG, "hss_matvec_noalloc needs " + std::to_string(need * 8) +
                                           " bytes of scratch for this matrix and nrhs; the fixed array holds " +
                                           std::to_string(kScratchBytes) + " (use fewer right-hand sides)");
    double* base = scratch_ptr();
    double* xp = base;
    double* yp = xp + e_n;
    double* xh = yp + e_n;
    double* yh = xh + e_h;
    double* ws = yh + e_h;
    hipStream_t s = (hipStream_t)stream;
    const int64_t* perm = P.dev.gen.perm;
    launch_gather_rows(X, ldx, perm, P.n, nrhs, xp, P.n, 0, s);
    matvec_permuted(h, nrhs, xp, yp, xh, yh, ws, s);
    launch_gather_rows(yp, P.n, perm, P.n, nrhs, Y, ldy, 1, s);
    HSS_HIP_CHECK(hipGetLastError());
    return HSS_OK;
  } catch (const Error& e) {
    return record_error(e.code, e.msg);
  } catch (...) {
    return record_error(HSS_ERR_INTERNAL, "unknown error");
  }
}
