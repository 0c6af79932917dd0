// top_solve_static: a whole solve (create, k sweeps, outputs) that allocates no device memory.  The
// problem's state, shape tables and lane map live in `scratch`, a fixed array compiled into the
// library (one copy per device, held until the process ends).  See include/top.h for the contract.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "api_internal.h"
#include "top.h"

constexpr size_t kStaticScratchBytes = size_t(TOP_STATIC_SCRATCH_BYTES);

// Host code names this array only to look up its device address (once per device); kernels and
// copies get that address.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

struct StaticScratch {
  std::mutex mu;        // serialises this process's calls on the device
  char* ptr = nullptr;  // device address of `scratch` on the device
};
std::mutex g_static_mu;
// Never destroyed (records of devices may be used until the process ends).
std::map<int, StaticScratch*>& g_static = *new std::map<int, StaticScratch*>();

// The current device's record; the first call on a device looks the array's address up there.
top_status static_scratch(StaticScratch** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return top::internal_error(TOP_E_HIP, (std::string("hipGetDevice failed: ") + hipGetErrorString(e)).c_str());
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticScratch*& r = g_static[dev];
  if (r == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return top::internal_error(TOP_E_HIP, (std::string("static scratch address: ") + hipGetErrorString(e)).c_str());
    r = new StaticScratch();
    r->ptr = static_cast<char*>(p);
  }
  *out = r;
  return TOP_OK;
}

}  // namespace

extern "C" top_status top_solve_static(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                                       const double* durations, const double* bc, const double* box_lo,
                                       const double* box_hi, const double* vmax, const double* rho,
                                       const top_options* opt_in, int32_t k, double* coeffs, double* cost,
                                       double* r_primal, double* r_dual, hipStream_t stream) {
  if (k < 0) return top::internal_error(TOP_E_INVALID, "k must be >= 0");
  if (k == 0 && (r_primal != nullptr || r_dual != nullptr))
    return top::internal_error(TOP_E_STATE, "residuals need at least one sweep (k = 0)");
  top_options opt;
  if (opt_in != nullptr) opt = *opt_in; else top_default_options(&opt);
  if (opt.checkpoint_every != 0) return top::internal_error(TOP_E_UNSUPPORTED, "top_solve_static records no tape");
  opt.use_graph = 0;  // direct launches: a graph would be instantiated (allocated) per call
  opt.chain = 1;      // ordinary launches only (the runtime may set up state for a cooperative one)
  StaticScratch* sc = nullptr;
  top_status st = static_scratch(&sc);
  if (st != TOP_OK) return st;
  std::lock_guard<std::mutex> lk(sc->mu);
  top_problem* h = nullptr;
  st = top::internal_create(n_traj, seg_offsets, waypoints, durations, bc, box_lo, box_hi, vmax, rho, &opt, sc->ptr,
                            kStaticScratchBytes, stream, &h, top::Mem::kStatic);
  if (st == TOP_E_WORKSPACE)
    return top::internal_error(TOP_E_WORKSPACE, (std::string("problem too large for the static scratch (") +
                                                 std::to_string(kStaticScratchBytes) + " bytes): " + top_last_error())
                                                    .c_str());
  if (st != TOP_OK) return st;
  st = top_iterate(h, k);
  if (st == TOP_OK && (r_primal != nullptr || r_dual != nullptr)) st = top_residuals(h, r_primal, r_dual);
  if (st == TOP_OK && cost != nullptr) st = top_cost(h, cost);
  if (st == TOP_OK && coeffs != nullptr) st = top_coeffs(h, coeffs);
  // The next call reuses the scratch: wait for this call's work (top_sync_status synchronises the
  // stream and reports a non-finite iterate).
  if (st == TOP_OK) {
    st = top_sync_status(h);
  } else {
    const std::string msg = top_last_error();
    (void)hipStreamSynchronize(stream);
    (void)top::internal_error(st, msg.c_str());
  }
  top_destroy(h);
  return st;
}
