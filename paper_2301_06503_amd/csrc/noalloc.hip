// Static device scratch of the allocation-free linear solve
// (lgdm_solve_linear_noalloc).
//
// The solve's per-workgroup reduction partials and its device scalars live in
// one file-scope device array instead of buffers the library allocates.  Host code never passes the array's name to a
// kernel or a copy: on the host the name is only a stand-in for the symbol.
// noalloc_init resolves the array's address on each device once (with that
// device current) and every later use goes through that address.
#include <algorithm>
#include <mutex>

#include "lgdm_internal.h"

namespace lgdm {
namespace {

static __device__ __align__(256) double scratch[LGDM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each GPU

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(scratch_mutex);
  if (scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(scratch_mutex);
  return scratch_ptr[device];
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  fill_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace lgdm
