// fa_apply_noalloc: fa_apply for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).  Its workspace -- the Krylov basis, the chain vectors and the
// reduction scratch of fa_apply -- is one file-scope device array of
// FA_NOALLOC_MAX_BYTES; the caller passes only b and x.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "fa_internal.hpp"
#include "solver.hpp"

// Every device the library runs on holds its own copy, from the first use of
// the code object on it until the process ends.  In host code this name is
// only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress (device_scratch below), once per device.
static __device__ __align__(256) unsigned char scratch[FA_NOALLOC_MAX_BYTES];

namespace {

struct DeviceScratch {
  std::mutex mu;              // serializes the calls on one device
  void* ptr = nullptr;        // device address of `scratch` on that device
};

std::mutex g_table_mu;
std::vector<DeviceScratch*> g_table;  // per device, never freed

// the current device's entry; its scratch address is taken on the first call
// on that device, with the device current
int device_scratch(DeviceScratch** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return FA_ERR_HIP;
  std::lock_guard<std::mutex> g(g_table_mu);
  if ((int)g_table.size() <= dev) g_table.resize(dev + 1, nullptr);
  if (!g_table[dev]) g_table[dev] = new DeviceScratch;
  DeviceScratch* d = g_table[dev];
  if (!d->ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return FA_ERR_HIP;
    d->ptr = p;
  }
  *out = d;
  return FA_OK;
}

}  // namespace

extern "C" int fa_apply_noalloc(fa_op op, int kind, const void* d_b, void* d_x, int m_max,
                                double tol, int check_every, uint32_t flags, void* hip_stream,
                                fa_stats* stats) {
  if (!op || !d_b || !d_x || d_b == d_x || m_max < 1 || check_every < 0 ||
      (kind != FA_INVSQRT && kind != FA_SQRT) || !std::isfinite(tol) ||
      (flags & ~uint32_t(FA_FORCE_ARNOLDI | FA_NO_FUSION | FA_FUSE2 | FA_FUSE3 | FA_MIXED |
                         FA_TWO_PASS | FA_RIGHT_PREC | FA_CGS2)))
    return FA_ERR_ARG;  // FA_PROFILE is refused: its timing events are created on demand
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  if ((int64_t)m_max > op->op.n) return FA_ERR_ARG;
  const size_t need = fa::make_layout(op->op, m_max, flags).bytes;
  if (need > FA_NOALLOC_MAX_BYTES) return FA_ERR_WORKSPACE;
  DeviceScratch* d = nullptr;
  int st = device_scratch(&d);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(d->mu);
  try {
    st = fa::apply(op->op, kind, d_b, d_x, m_max, tol, check_every, d->ptr, FA_NOALLOC_MAX_BYTES,
                   flags | fa::kApplyNoAlloc, s, stats);
  } catch (...) {
    st = FA_ERR_ARG;
  }
  // the next call may reuse the array only once this call's work is done
  // (an error return can leave launches in flight)
  if (hipStreamSynchronize(s) != hipSuccess && st >= 0) st = FA_ERR_HIP;
  return st;
}
