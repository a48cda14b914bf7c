// pfmm_plan_direct_noalloc: the direct periodic convolution of Eq. 4 with a
// plan's G, for callers that cannot allocate device memory (code under graph
// capture, serving loops, harnesses that forbid hipMalloc).  pfmm_plan_direct
// allocates its lattice table on the first call; this variant tabulates it on
// every call into a file-scope device array instead, and allocates nothing.
//
// The array holds, one after another (256-byte aligned): the FP64 lattice
// table G(h j), j in [-C, C]^3; its FP32 copy; the n^3 packed block offsets;
// and the partial Fourier sums of G_K / G_E.  Each device holds its own copy
// of the array, at its own address, looked up once per device with
// hipGetSymbolAddress; host code uses only that address.  Every call on a
// device overwrites the whole table before it is read (stream order), so
// nothing carries over from the previous call; calls that overlap on one
// device (different streams, or threads) race on the array.
#include "../../include/pfmm.h"
#include "internal.h"

#include <mutex>

namespace {

constexpr int kMaxN = 64;                      // largest mesh the array serves
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's array (looked up on the first call).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// The source blocks of the whole box, d in [-n/2, n/2)^3, packed as the
// block-Toeplitz kernel reads them (pack_offset's byte layout), x slowest.
__global__ void k_direct_offsets(int n, int* __restrict__ offs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n * n) return;
  const int dx = i / (n * n) - n / 2, dy = (i / n) % n - n / 2, dz = i % n - n / 2;
  offs[i] = ((dx + 128) & 255) << 16 | ((dy + 128) & 255) << 8 | ((dz + 128) & 255);
}

}  // namespace

extern "C" pfmm_status pfmm_plan_direct_noalloc(pfmm_plan_t plan, const float* density,
                                                float* potential) {
  using namespace pfmm;
  clear_error();
  DirectSpec sp{};
  const int st0 = plan_direct_spec(plan, &sp);
  if (st0 != PFMM_OK) return (pfmm_status)st0;
  if (sp.isolated) return (pfmm_status)set_error(PFMM_ERR_UNSUPPORTED, "direct solve of an isolated plan");
  if (!density || !potential || (const void*)density == (const void*)potential)
    return (pfmm_status)set_error(PFMM_ERR_INVALID_ARG,
                                  "density and potential must be distinct device arrays");
  if (sp.N > kMaxN)
    return (pfmm_status)set_error(PFMM_ERR_UNSUPPORTED,
                                  "pfmm_plan_direct_noalloc serves N <= 64 (its 8 MiB device array)");
  const int N = sp.N;
  const int q = N >= 16 ? 8 : N / 2, n = N / q;
  const int C = N / 2 + q - 1;
  const int64_t E3 = (int64_t)(2 * C + 1) * (2 * C + 1) * (2 * C + 1);
  const size_t b64 = up256((size_t)E3 * sizeof(double));
  const size_t b32 = up256((size_t)E3 * sizeof(float));
  const size_t boffs = up256((size_t)n * n * n * sizeof(int));
  const size_t bws = tabulate_workspace_doubles(sp.green.kind, N, C) * sizeof(double);
  if (b64 + b32 + boffs + bws > kScratchBytes)
    return (pfmm_status)set_error(PFMM_ERR_UNSUPPORTED, "table larger than the device array");
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess)
    return (pfmm_status)set_error(PFMM_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  unsigned char* b = static_cast<unsigned char*>(base);
  double* tab64 = reinterpret_cast<double*>(b);
  float* tab32 = reinterpret_cast<float*>(b + b64);
  int* offs = reinterpret_cast<int*>(b + b64 + b32);
  double* ws = bws ? reinterpret_cast<double*>(b + b64 + b32 + boffs) : nullptr;
  hipStream_t st = sp.stream;
  e = tabulate_green_ws(sp.green, N, C, N, 1.0 / N, tab64, ws, st);
  if (e == hipSuccess) e = cast_f64_f32(tab64, tab32, E3, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_direct_offsets, dim3((n * n * n + 255) / 256), dim3(256), 0, st, n, offs);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    ToepArgs a{};
    a.n = n;
    a.m = 1;
    a.q = q;
    a.noff = n * n * n;
    a.offs = offs;
    a.tab = tab32;
    a.C = C;
    a.X = density;
    a.Y = potential;
    a.grid_in = 1;
    a.grid_out = 1;
    a.xscale = 1.0 / ((double)N * N * N);
    a.accumulate = 0;
    a.groups = 1;
    e = launch_toeplitz(a, st);
  }
  if (e != hipSuccess)
    return (pfmm_status)set_error(PFMM_ERR_HIP, std::string("direct solve: ") + hipGetErrorString(e));
  return PFMM_OK;
}
