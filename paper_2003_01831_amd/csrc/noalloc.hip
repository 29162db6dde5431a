// Allocation-free systematic resampling (afq_walkers_comb_noalloc).
//
// The same kernels as afq_walkers_comb (comb_index_kernel, comb_apply_kernel),
// with their scratch -- the running weight sums, the source index of every new
// walker and the {total, new weight} pair -- taken from one file-scope device
// array instead of buffers the walker set allocates on its first comb. The
// array is statically sized for AFQ_COMB_NOALLOC_MAX_WALKERS walkers; every GPU
// the library runs on holds its own copy until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is handed to kernels.
#include <cmath>
#include <mutex>

#include "common.h"
#include "step_kernels.h"

namespace {

constexpr size_t kOutBytes = 256;   // {total, total / n}, padded to keep the next region aligned
constexpr size_t kCumBytes = (size_t)AFQ_COMB_NOALLOC_MAX_WALKERS * sizeof(double);
constexpr size_t kSrcBytes = (size_t)AFQ_COMB_NOALLOC_MAX_WALKERS * sizeof(int);
constexpr size_t kScratchBytes = kOutBytes + kCumBytes + kSrcBytes;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
int scratch_on_device(int dev, unsigned char** out) {
  AFQ_CHECK(dev >= 0 && dev < kMaxDevices, AFQ_E_UNSUPPORTED, "afq_walkers_comb_noalloc: device index too large");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    AFQ_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    AFQ_CHECK(p != nullptr, AFQ_E_HIP, "afq_walkers_comb_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return AFQ_OK;
}

int comb_noalloc(afq_walkers w, double xi, int* src_out, double* total_out) {
  afq_system s = w->sys;
  const int nw = w->nw;
  AFQ_CHECK(nw <= AFQ_COMB_NOALLOC_MAX_WALKERS, AFQ_E_INVALID,
            "afq_walkers_comb_noalloc: " + std::to_string(nw) + " walkers exceed the scratch limit of " +
                std::to_string(AFQ_COMB_NOALLOC_MAX_WALKERS));
  AFQ_CHECK(w->bp_n < 0, AFQ_E_UNSUPPORTED,
            "afq_walkers_comb_noalloc: a back-propagation window is open (its history gather needs a buffer); "
            "use afq_walkers_comb");
  int dev = -1;
  AFQ_TRY_HIP(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  AFQ_RET(scratch_on_device(dev, &base));
  double* out2 = reinterpret_cast<double*>(base);
  double* cum = reinterpret_cast<double*>(base + kOutBytes);
  int* src = reinterpret_cast<int*>(base + kOutBytes + kCumBytes);
  // nothing needs clearing: comb_index_kernel writes out2 and cum[0..nw) before
  // any read, and src[0..nw) whenever the total weight is positive (otherwise
  // the call stops below before src is read)
  hipStream_t st = s->stream;
  AFQ_RET(launch_comb_index(w->weights.as<double>(), nw, xi, cum, src, out2, st));
  double tot[2];
  AFQ_TRY_HIP(hipMemcpyAsync(tot, out2, sizeof(tot), hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  if (total_out) *total_out = tot[0];
  AFQ_CHECK(tot[0] > 0.0 && std::isfinite(tot[0]), AFQ_E_STATE,
            "afq_walkers_comb_noalloc: the walkers carry no positive weight");
  const long per = (long)s->M * s->ntot;
  AFQ_RET(launch_comb_apply(w->W.as<double2>(), w->Wn.as<double2>(), per, nw, src, out2, w->weights.as<double>(),
                            w->alive.as<int>(), st));
  AFQ_TRY_HIP(hipMemcpyAsync(w->W.p, w->Wn.p, (size_t)nw * per * 16, hipMemcpyDeviceToDevice, st));
  w->s_carried = false;
  if (src_out) {
    AFQ_TRY_HIP(hipMemcpyAsync(src_out, src, (size_t)nw * sizeof(int), hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
  }
  return AFQ_OK;
}

}  // namespace

extern "C" int afq_walkers_comb_noalloc(afq_walkers w, double xi, int32_t* src_out, double* total_out) {
  AFQ_CHECK(w, AFQ_E_INVALID, "afq_walkers_comb_noalloc: walkers is NULL");
  AFQ_CHECK(xi >= 0.0 && xi < 1.0, AFQ_E_INVALID, "afq_walkers_comb_noalloc: xi must be in [0, 1)");
  try {
    int dev = -1;
    AFQ_TRY_HIP(hipGetDevice(&dev));
    AFQ_CHECK(dev == w->sys->device, AFQ_E_STATE, "the current HIP device differs from the system's device");
    return comb_noalloc(w, xi, src_out, total_out);
  } catch (const std::exception& e) {
    afq_set_error(std::string("internal error: ") + e.what());
    return AFQ_E_HIP;
  } catch (...) {
    afq_set_error("internal error");
    return AFQ_E_HIP;
  }
}
