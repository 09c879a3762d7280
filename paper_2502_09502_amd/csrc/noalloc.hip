// cgl_prox_batch_noalloc: the batched prox of cgl_prox_node_batch for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops). Inputs and outputs
// are the caller's device buffers; the per-vector prox states and the shared row of class codes
// live in a file-scope device array (`scratch`) of fixed size, one copy per GPU, whose device
// address is taken once per device when a context is created on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/certglm.h"
#include "engine.h"
#include "kernels.h"
#include "prox.h"

namespace cgl {

constexpr int32_t kNoAllocMaxVectors = 4096;
constexpr int64_t kNoAllocMaxP = 32768;
constexpr size_t kNoAllocStateBytes = (size_t)kNoAllocMaxVectors * sizeof(NodeDev);
constexpr size_t kNoAllocScratchBytes = kNoAllocStateBytes + (size_t)kNoAllocMaxP;  // 992 KiB

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this GPU's copy of the array (the array's name in host code is only a
// host-side stand-in). Called with the device current.
void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) invalid("device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  CGL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
  g_scratch_ptr[device] = ptr;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// The state of every vector as cgl_prox_node_batch sets it for a node without fixed sets
// (k' = k, |F| = p, no iteration or monitor limits), and the class row (all free). Every field
// is written, so nothing left by an earlier call survives.
__global__ void k_noalloc_init(NodeDev* __restrict__ st, int count, int k, int64_t p,
                               uint8_t* __restrict__ cls) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) {
    NodeDev s;
    __builtin_memset(&s, 0, sizeof(s));
    s.phi = 1.0;
    s.c = 0.25;
    s.L_prev = HUGE_VAL;
    s.P_best = HUGE_VAL;
    s.D_best = -HUGE_VAL;
    s.iter = 1;
    s.status = kRunning;
    s.kp = k;
    s.nfree = (int)p;
    s.max_iter = 1 << 30;
    s.check_every = 1 << 30;
    s.tol = 1e-6;
    s.incumbent = HUGE_VAL;
    st[t] = s;
  }
  for (int64_t j = t; j < p; j += (int64_t)gridDim.x * blockDim.x) cls[j] = CLS_FREE;
}

__global__ void k_noalloc_gval(const NodeDev* __restrict__ st, int count,
                               double* __restrict__ gval) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) gval[t] = st[t].g_new;
}

}  // namespace cgl

using namespace cgl;

extern "C" int cgl_prox_batch_noalloc(cgl_ctx* ctx, double rho, double M, int32_t k,
                                      const double* W, int32_t count, int64_t p, double* beta_out,
                                      double* gval_out) {
  CGL_API_BEGIN
  if (!ctx || !W || !beta_out) invalid("NULL argument");
  if (count < 0 || p < 1) invalid("count < 0 or p < 1");
  if (count > kNoAllocMaxVectors)
    invalid("count > " + std::to_string(kNoAllocMaxVectors) +
            ": beyond the fixed scratch of the allocation-free prox");
  if (p > kNoAllocMaxP)
    invalid("p > " + std::to_string(kNoAllocMaxP) +
            ": beyond the fixed scratch of the allocation-free prox");
  if (!(rho > 0.0) || !(M > 0.0) || k < 0 || !std::isfinite(rho) || !std::isfinite(M))
    invalid("need rho > 0, M > 0, k >= 0");
  if (k > kMaxHead && k < p) invalid("k > 256 with more coordinates than that is not supported");
  if (count == 0) return CGL_OK;
  CGL_HIP(hipSetDevice(ctx->device));
  unsigned char* base = static_cast<unsigned char*>(scratch_of(ctx->device));
  if (!base) invalid("no scratch address for this device (create a context on it first)");
  NodeDev* st = reinterpret_cast<NodeDev*>(base);
  uint8_t* cls = base + kNoAllocStateBytes;
  hipStream_t s = ctx->stream;
  const int threads = 256;
  const int blocks = (int)((std::max<int64_t>(count, p) + threads - 1) / threads);
  hipLaunchKernelGGL(k_noalloc_init, dim3(blocks), dim3(threads), 0, s, st, count, k, p, cls);
  CGL_HIP(hipGetLastError());
  // cls_ld = 0: every vector reads the one class row
  launch_prox(count, W, p, nullptr, 0, cls, 0, p, rho, M, 1.0, st, beta_out, 0, p, s);
  CGL_HIP(hipGetLastError());
  if (gval_out) {
    hipLaunchKernelGGL(k_noalloc_gval, dim3((count + threads - 1) / threads), dim3(threads), 0, s,
                       st, count, gval_out);
    CGL_HIP(hipGetLastError());
  }
  return CGL_OK;
  CGL_API_END
}
