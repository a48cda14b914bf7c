// G_* as one grid-valued function everywhere (Sec. 3, Eq. 8; Sec. 4).
//
// The paper defines the optimal Green's function G_* as the one with which
// the FMM and PM, both using G_*, give the same potential (Eq. 8 follows
// from requiring it for every gridlet mass), and proposes to represent G_*
// by a grid of free values.  Here G_*(x) = G(x) (1 + delta[orbit(x)]) on the
// periodic mesh, one free value per orbit of mesh separations under the
// cube's 48 symmetries, and the same G_* enters every place the method
// samples G: the near-zone table G(h m), every level's interaction-zone
// table G(eta_l j) (mesh points when p divides the leaf width), and the PM
// solution the FMM is compared with (the exact periodic convolution).
//
// With r = 2 (phi_FMM - phi_PM - mean) / B the loss gradient of the FMM side
// and q = r + 2 (loss / B) (phi_PM - mean phi_PM) that of the PM side
// (B = sum (phi_PM - mean)^2, which also moves with G_*),
//   d loss / d G_*(x) = [FMM adjoint at x] - h^3 sum_t q_t rho(t - x).
// The FMM adjoint of the level tables is the learned tables' (adjoint sweep
// and table gradient); this file adds the near-zone table's, a direct sum
// over the pairs of neighbouring leaves, and the PM side, a periodic
// cross-correlation by FP64 FFT.
#include "internal.h"

#include <hipfft/hipfft.h>

#include <utility>

namespace pfmm {
namespace {

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t ferr(hipfftResult r) { return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown; }

// floor(a / s) for a > -4s
__device__ __forceinline__ int fdiv(int a, int s) { return (a + 4 * s) / s - 4; }

// Near-zone table gradient: g[m] = h^3 sum over target cells t whose source
// cell t - m lies in one of the 27 leaves around t's leaf of r[t] rho[t - m],
// for every separation m of the table (|m_i| <= C = 2s - 1), one block each.
__global__ __launch_bounds__(256) void k_near_grad(const float* __restrict__ r,
                                                   const float* __restrict__ rho, int N, int s,
                                                   int C, double h3, double* __restrict__ g) {
  const int E = 2 * C + 1;
  const int id = blockIdx.x;
  const int mx = id / (E * E) - C, my = (id / E) % E - C, mz = id % E - C;
  const int64_t n3 = (int64_t)N * N * N;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < n3; t += blockDim.x) {
    const int tx = (int)(t / ((int64_t)N * N)), ty = (int)((t / N) % N), tz = (int)(t % N);
    const int ux = tx - mx, uy = ty - my, uz = tz - mz;
    const int ex = tx / s - fdiv(ux, s), ey = ty / s - fdiv(uy, s), ez = tz / s - fdiv(uz, s);
    if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ez < -1 || ez > 1) continue;
    const int sx = (ux + N) % N, sy = (uy + N) % N, sz = (uz + N) % N;
    acc += (double)r[t] * (double)rho[((int64_t)sx * N + sy) * N + sz];
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[id] = h3 * red[0];
}

// q = r + 2 (loss / B) (t - mean t) and the density, both in FP64;
// stats = {mean(phi - t), loss, B, mean t}
__global__ void k_qfield(const float* __restrict__ r, const float* __restrict__ t,
                         const float* __restrict__ rho, const double* __restrict__ stats,
                         int64_t n, double* __restrict__ q, double* __restrict__ rho64) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  q[i] = (double)r[i] + 2.0 * stats[1] / stats[2] * ((double)t[i] - stats[3]);
  rho64[i] = (double)rho[i];
}

// qhat <- qhat conj(rhohat) (the transform of sum_t q_t rho(t - x))
__global__ void k_corr_mul(hipfftDoubleComplex* __restrict__ qh,
                           const hipfftDoubleComplex* __restrict__ rh, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const hipfftDoubleComplex a = qh[i], b = rh[i];
  qh[i].x = a.x * b.x + a.y * b.y;
  qh[i].y = a.y * b.x - a.x * b.y;
}

// scale G(x) at every mesh point x in [0, N)^3 from a centred table of
// extent C (C >= N / 2), x folded to the representative in [-N/2, N/2)
__global__ void k_mesh_values(const double* __restrict__ tab, int C, int N, double scale,
                              double* __restrict__ out) {
  const int64_t n3 = (int64_t)N * N * N;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  int x = (int)(i / ((int64_t)N * N)), y = (int)((i / N) % N), z = (int)(i % N);
  if (2 * x >= N) x -= N;
  if (2 * y >= N) y -= N;
  if (2 * z >= N) z -= N;
  const int E = 2 * C + 1;
  out[i] = scale * tab[((int64_t)(x + C) * E + (y + C)) * E + (z + C)];
}

}  // namespace

// Orbit index of an integer mesh separation on the periodic N^3 mesh: each
// component folded to min(|x| mod N, N - |x| mod N), sorted c <= b <= a,
// index a (a + 1) (a + 2) / 6 + b (b + 1) / 2 + c.
int gstar_orbit(int x, int y, int z, int N) {
  int v[3] = {x, y, z};
  for (int& a : v) {
    a = ((a % N) + N) % N;
    if (N - a < a) a = N - a;
  }
  if (v[0] > v[1]) std::swap(v[0], v[1]);
  if (v[1] > v[2]) std::swap(v[1], v[2]);
  if (v[0] > v[1]) std::swap(v[0], v[1]);
  const int a = v[2], b = v[1], c = v[0];
  return a * (a + 1) * (a + 2) / 6 + b * (b + 1) / 2 + c;
}

int gstar_orbits(int N) {
  const int K = N / 2 + 1;
  return K * (K + 1) * (K + 2) / 6;
}

struct GStarFft {
  int N = 0;
  hipfftHandle fwd = 0, inv = 0;
  double* q = nullptr;
  double* rho = nullptr;
  hipfftDoubleComplex* qh = nullptr;
  hipfftDoubleComplex* rh = nullptr;
};

void gstar_fft_destroy(GStarFft* f) {
  if (!f) return;
  if (f->fwd) (void)hipfftDestroy(f->fwd);
  if (f->inv) (void)hipfftDestroy(f->inv);
  (void)hipFree(f->q);
  (void)hipFree(f->rho);
  (void)hipFree(f->qh);
  (void)hipFree(f->rh);
  delete f;
}

hipError_t gstar_fft_create(int N, GStarFft** out) {
  *out = nullptr;
  GStarFft* f = new GStarFft;
  f->N = N;
  const size_t n3 = (size_t)N * N * N, nh = (size_t)N * N * (N / 2 + 1);
  hipError_t e = hipMalloc(&f->q, n3 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&f->rho, n3 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&f->qh, nh * sizeof(hipfftDoubleComplex));
  if (e == hipSuccess) e = hipMalloc(&f->rh, nh * sizeof(hipfftDoubleComplex));
  if (e == hipSuccess) e = ferr(hipfftPlan3d(&f->fwd, N, N, N, HIPFFT_D2Z));
  if (e == hipSuccess) e = ferr(hipfftPlan3d(&f->inv, N, N, N, HIPFFT_Z2D));
  if (e != hipSuccess) {
    gstar_fft_destroy(f);
    return e;
  }
  *out = f;
  return hipSuccess;
}

hipError_t gstar_near_grad(const float* r, const float* rho, int N, int s, double h3, double* g,
                           hipStream_t st) {
  const int C = 2 * s - 1, E = 2 * C + 1;
  hipLaunchKernelGGL(k_near_grad, dim3(E * E * E), dim3(256), 0, st, r, rho, N, s, C, h3, g);
  return hipGetLastError();
}

hipError_t gstar_pm_corr(GStarFft* f, const float* r, const float* t, const float* rho,
                         const double* stats, double* corr, hipStream_t st) {
  const int N = f->N;
  const int64_t n3 = (int64_t)N * N * N, nh = (int64_t)N * N * (N / 2 + 1);
  hipLaunchKernelGGL(k_qfield, dim3(nb(n3, 256)), dim3(256), 0, st, r, t, rho, stats, n3, f->q,
                     f->rho);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = ferr(hipfftSetStream(f->fwd, st));
  if (e == hipSuccess) e = ferr(hipfftSetStream(f->inv, st));
  if (e == hipSuccess) e = ferr(hipfftExecD2Z(f->fwd, f->q, f->qh));
  if (e == hipSuccess) e = ferr(hipfftExecD2Z(f->fwd, f->rho, f->rh));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_corr_mul, dim3(nb(nh, 256)), dim3(256), 0, st, f->qh, f->rh, nh);
  e = hipGetLastError();
  if (e == hipSuccess) e = ferr(hipfftExecZ2D(f->inv, f->qh, corr));
  return e;
}

hipError_t gstar_mesh_values(const double* tab, int C, int N, double scale, double* out,
                             hipStream_t st) {
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_mesh_values, dim3(nb(n3, 256)), dim3(256), 0, st, tab, C, N, scale, out);
  return hipGetLastError();
}

}  // namespace pfmm
