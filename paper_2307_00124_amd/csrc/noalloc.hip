// mg_fmg_f64_noalloc: the FP64-in, FP64-out FMG solve for callers that
// cannot allocate device memory. The solver hierarchy (every level's blocks,
// the recorded coarse-level programs, the reduction slots) lives in a
// file-scope device array; each GPU holds its own copy of it, found once per
// device with hipGetSymbolAddress. The host keeps, per device, the hierarchy
// object built on that array for the last parameter set.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/bfpmg.h"
#include "api_internal.hpp"

using namespace bfpk;

// the solver hierarchy of mg_fmg_f64_noalloc (host code must use the
// per-device address from hipGetSymbolAddress, never this name)
static __device__ __align__(256) char scratch[MG_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceState {
  bool ready = false;        // ptr holds this device's address of `scratch`
  void* ptr = nullptr;
  mg_hierarchy* h = nullptr; // built on ptr for prm
  mg_params prm{};
  int exec_points = -1;
  bool diag = false;
};

DeviceState g_state[kMaxDevices];
std::mutex g_mutex;

}  // namespace

extern "C" int mg_fmg_f64_noalloc(const mg_params* prm, const double* const* rhs_dev,
                                  double* x_out_dev, void* stream) {
  if (!prm || !rhs_dev || !x_out_dev) return fail(BFP_EINVAL, "NULL argument");
  int rc = params_ok(prm);
  if (rc) return rc;
  for (int j = 1; j <= prm->L; ++j)
    if (!rhs_dev[j - 1]) return fail(BFP_EINVAL, "right-hand side of level %d is NULL", j);
  size_t need = 0;
  if ((rc = hierarchy_bytes_ex(prm, exec_max_points(), &need))) return rc;
  if (need > MG_NOALLOC_BYTES)
    return fail(BFP_ENOMEM,
                "mg_fmg_f64_noalloc: this problem needs %zu bytes of solver state, more than the "
                "static %zu-byte array (use mg_hierarchy_create with an arena)",
                need, (size_t)MG_NOALLOC_BYTES);
  int dev = 0;
  if ((rc = hip_check(hipGetDevice(&dev), "hipGetDevice"))) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(BFP_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mutex);
  DeviceState& st = g_state[dev];
  if (!st.ready) {
    void* p = nullptr;
    if ((rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")))
      return rc;
    st.ptr = p;
    st.ready = true;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool same = st.h && !std::memcmp(&st.prm, prm, sizeof(mg_params)) &&
                    st.exec_points == exec_max_points() && st.diag == diagnostics_on();
  if (!same) {
    if (st.h) {
      mg_hierarchy_destroy(st.h);
      st.h = nullptr;
    }
    // lays the hierarchy out in the array and zeroes it on `stream`
    if ((rc = hierarchy_create_ex(prm, st.ptr, MG_NOALLOC_BYTES, stream, exec_max_points(), &st.h)))
      return rc;
    st.prm = *prm;
    st.exec_points = exec_max_points();
    st.diag = diagnostics_on();
  }
  if ((rc = fmg_f64_one_stream(st.h, rhs_dev, s))) return rc;
  bfp_vec x;
  if ((rc = mg_get_vec(st.h, prm->L, 0, &x))) return rc;
  return bfp_vec_to_f64(&x, x_out_dev, stream);
}
