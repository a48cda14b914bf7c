// FP64 tabulation of the periodic Green's functions on the device (plan time).
//
// Real-space kinds (one thread per entry):
//   G_X  (Eq. 2):  -1 / (4 pi |x wrapped|),  wrap(x) = x - nint(x)
//   G_S  (Sec. 3 ansatz, n <= 2): G_X of x_hat_i = xi(x_i),
//        xi(t) = sin(pi t)/pi + a1 (sin(3 pi t)/(3 pi) - sin(pi t)/pi)
//                             + a2 (sin(5 pi t)/(5 pi) - sin(pi t)/pi)
//   G_S1 (Eq. 9):  x_hat = 9/(8 pi) sin(pi x) - 1/(24 pi) sin(3 pi x)
//   G_0  (the non-periodic twin of Eq. 3): -1 / (4 pi |x|), no wrap
//   G_E  (Ewald, Sec. 1), real-space part: G_X(x) erfc(r / r_S) + 1/(2 pi^(3/2) r_S)
//        on the nearest image (r_S << L), added to its Fourier part below
// The zero separation takes the potential at the centre of a uniform cube
// cell of side h: -c0/(4 pi h), c0 = 3 ln((sqrt3+1)/(sqrt3-1)) - pi/2.
//
// G_K (Eq. 1) is the trigonometric sum of -1/k^2 over the mesh frequencies
// with k = 0 removed.  The sum is even in every frequency component, so it is
// folded onto n_i in [0, N/2] with per-axis weights 1 (n = 0), 2 (0 < n < N/2)
// and 1 (n = N/2: the Nyquist term split equally between +N/2 and -N/2), and
// evaluated as three successive 1D cosine contractions on the product grid of
// table coordinates.  Cosines take exactly reduced rational arguments.  The
// Fourier part of G_E is the same sum with -1/k^2 damped by exp(-k^2 r_S^2 / 4).
// At zero separation G_E keeps the cube self value for its Newtonian part;
// the rest of its real-space part tends to 1/(2 pi^(3/2) r_S) there.
//
// For accelerations taken from the expansion, the near zone sums the
// acceleration of each source cell with the 4th-order central difference of
// the lattice G along each axis (what differencing the potential gives for
// that cell), tabulated from G over a table two cells wider.
#include "internal.h"

#include <cmath>

namespace pfmm {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline double self_potential(double h) {
  const double r3 = sqrt(3.0);
  const double c0 = 3.0 * log((r3 + 1.0) / (r3 - 1.0)) - 0.5 * kPi;
  return -c0 / (4.0 * kPi * h);
}

__device__ inline double xi_s1(double t) {
  return (9.0 / (8.0 * kPi)) * sinpi(t) - (1.0 / (24.0 * kPi)) * sinpi(3.0 * t);
}

__device__ inline double xi_s(double t, double a1, double a2) {
  const double s1 = sinpi(t) / kPi;
  const double s3 = sinpi(3.0 * t) / (3.0 * kPi);
  const double s5 = sinpi(5.0 * t) / (5.0 * kPi);
  return s1 + a1 * (s3 - s1) + a2 * (s5 - s1);
}

__global__ void tab_real_space(int kind, double a1, double a2, double rs, int C, int64_t den,
                               double self_h, double* __restrict__ dst) {
  const int E = 2 * C + 1;
  const int64_t total = (int64_t)E * E * E;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int jz = (int)(i % E) - C;
  const int jy = (int)((i / E) % E) - C;
  const int jx = (int)(i / ((int64_t)E * E)) - C;
  const double ewald_c = kind == GK_E ? 1.0 / (2.0 * kPi * sqrt(kPi) * rs) : 0.0;
  if (jx == 0 && jy == 0 && jz == 0) {
    const double v = self_h > 0.0 ? self_potential(self_h) + 2.0 * ewald_c : 0.0;
    dst[i] = kind == GK_E ? dst[i] + v : v;
    return;
  }
  const double inv = 1.0 / (double)den;
  double x = jx * inv, y = jy * inv, z = jz * inv;
  if (kind == GK_S1) {
    x = xi_s1(x); y = xi_s1(y); z = xi_s1(z);
  } else if (kind == GK_S) {
    x = xi_s(x, a1, a2); y = xi_s(y, a1, a2); z = xi_s(z, a1, a2);
  }
  if (kind != GK_N) {
    x -= rint(x); y -= rint(y); z -= rint(z);
  }
  const double r = sqrt(x * x + y * y + z * z);
  if (kind == GK_E)
    dst[i] += -erfc(r / rs) / (4.0 * kPi * r) + ewald_c;
  else
    dst[i] = -1.0 / (4.0 * kPi * r);
}

// CS[n][j] = w(n) cos(2 pi n j / den), n in [0, H], j in [0, C]
__global__ void gk_cos(int H, int C, int64_t den, double* __restrict__ cs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (H + 1) * (C + 1)) return;
  const int n = i / (C + 1), j = i % (C + 1);
  const int64_t r = (2 * (int64_t)n * j) % (2 * den);  // cos(pi r / den), exact reduction
  const double w = (n == 0 || n == H) ? 1.0 : 2.0;
  cs[i] = w * cospi((double)r / (double)den);
}

// U[nx][ny][jz] = sum_nz CS[nz][jz] Gt(nx, ny, nz),
// Gt = -exp(-damp |n|^2) / (4 pi^2 |n|^2), Gt(0) = 0  (damp = pi^2 r_S^2 for G_E, else 0)
__global__ void gk_step1(int H, int C, double damp, const double* __restrict__ cs,
                         double* __restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)(H + 1) * (H + 1) * (C + 1);
  if (i >= total) return;
  const int jz = (int)(i % (C + 1));
  const int ny = (int)((i / (C + 1)) % (H + 1));
  const int nx = (int)(i / ((int64_t)(C + 1) * (H + 1)));
  const double n2xy = (double)nx * nx + (double)ny * ny;
  double acc = 0.0;
  for (int nz = 0; nz <= H; ++nz) {
    const double n2 = n2xy + (double)nz * nz;
    if (n2 == 0.0) continue;
    const double w = damp > 0.0 ? exp(-damp * n2) : 1.0;
    acc += cs[nz * (C + 1) + jz] * (-w / (4.0 * kPi * kPi * n2));
  }
  U[i] = acc;
}

// V[nx][jy][jz] = sum_ny CS[ny][jy] U[nx][ny][jz]
__global__ void gk_step2(int H, int C, const double* __restrict__ cs, const double* __restrict__ U,
                         double* __restrict__ V) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)(H + 1) * (C + 1) * (C + 1);
  if (i >= total) return;
  const int jz = (int)(i % (C + 1));
  const int jy = (int)((i / (C + 1)) % (C + 1));
  const int nx = (int)(i / ((int64_t)(C + 1) * (C + 1)));
  double acc = 0.0;
  for (int ny = 0; ny <= H; ++ny)
    acc += cs[ny * (C + 1) + jy] * U[((int64_t)nx * (H + 1) + ny) * (C + 1) + jz];
  V[i] = acc;
}

// dst[jx][jy][jz] (j in [-C, C]) = sum_nx CS[nx][|jx|] V[nx][|jy|][|jz|]
__global__ void gk_step3(int H, int C, const double* __restrict__ cs, const double* __restrict__ V,
                         double* __restrict__ dst) {
  const int E = 2 * C + 1;
  const int64_t total = (int64_t)E * E * E;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int jz = abs((int)(i % E) - C);
  const int jy = abs((int)((i / E) % E) - C);
  const int jx = abs((int)(i / ((int64_t)E * E)) - C);
  double acc = 0.0;
  for (int nx = 0; nx <= H; ++nx)
    acc += cs[nx * (C + 1) + jx] * V[((int64_t)nx * (C + 1) + jy) * (C + 1) + jz];
  dst[i] = acc;
}

__global__ void k_cast(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// D_i(j) = -(8 (G(j + e_i) - G(j - e_i)) - (G(j + 2 e_i) - G(j - 2 e_i))) N / 12 for
// j in [-C, C]^3, from G on [-C-2, C+2]^3
__global__ void k_accel_tab(const double* __restrict__ g, int C, double n12,
                            double* __restrict__ dx, double* __restrict__ dy,
                            double* __restrict__ dz) {
  const int E = 2 * C + 1, Eg = 2 * C + 5;
  const int64_t total = (int64_t)E * E * E;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int jz = (int)(i % E) + 2;
  const int jy = (int)((i / E) % E) + 2;
  const int jx = (int)(i / ((int64_t)E * E)) + 2;
  auto at = [&](int x, int y, int z) { return g[((int64_t)x * Eg + y) * Eg + z]; };
  dx[i] = -(8.0 * (at(jx + 1, jy, jz) - at(jx - 1, jy, jz)) -
            (at(jx + 2, jy, jz) - at(jx - 2, jy, jz))) * n12;
  dy[i] = -(8.0 * (at(jx, jy + 1, jz) - at(jx, jy - 1, jz)) -
            (at(jx, jy + 2, jz) - at(jx, jy - 2, jz))) * n12;
  dz[i] = -(8.0 * (at(jx, jy, jz + 1) - at(jx, jy, jz - 1)) -
            (at(jx, jy, jz + 2) - at(jx, jy, jz - 2))) * n12;
}

}  // namespace

namespace {
// The three partial sums of the Fourier kinds (doubles each).
void fourier_sizes(int N, int C, int64_t& ncs, int64_t& nU, int64_t& nV) {
  const int H = N / 2;
  ncs = (int64_t)(H + 1) * (C + 1);
  nU = (int64_t)(H + 1) * (H + 1) * (C + 1);
  nV = (int64_t)(H + 1) * (C + 1) * (C + 1);
}

// Tabulation with the Fourier kinds' partial sums in `ws` (cs, U, V one
// after another); enqueued on `st` only.
hipError_t tabulate_into(const GreenSpec& g, int N, int C, int64_t den, double self_h, double* dst,
                         double* ws, hipStream_t st) {
  const int E = 2 * C + 1;
  const int64_t total = (int64_t)E * E * E;
  if (g.kind == GK_K || g.kind == GK_E) {  // Fourier sum (the whole G_K; G_E's long-range part)
    const int H = N / 2;
    const double damp = g.kind == GK_E ? kPi * kPi * g.rs * g.rs : 0.0;
    int64_t ncs, nU, nV;
    fourier_sizes(N, C, ncs, nU, nV);
    double* cs = ws;
    double* U = cs + ncs;
    double* V = U + nU;
    hipLaunchKernelGGL(gk_cos, dim3(nblocks(ncs, 256)), dim3(256), 0, st, H, C, den, cs);
    hipLaunchKernelGGL(gk_step1, dim3(nblocks(nU, 256)), dim3(256), 0, st, H, C, damp, cs, U);
    hipLaunchKernelGGL(gk_step2, dim3(nblocks(nV, 256)), dim3(256), 0, st, H, C, cs, U, V);
    hipLaunchKernelGGL(gk_step3, dim3(nblocks(total, 256)), dim3(256), 0, st, H, C, cs, V, dst);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || g.kind == GK_K) return e;
  }
  hipLaunchKernelGGL(tab_real_space, dim3(nblocks(total, 256)), dim3(256), 0, st, g.kind, g.a1,
                     g.a2, g.rs, C, den, self_h, dst);
  return hipGetLastError();
}
}  // namespace

size_t tabulate_workspace_doubles(int kind, int N, int C) {
  if (kind != GK_K && kind != GK_E) return 0;
  int64_t ncs, nU, nV;
  fourier_sizes(N, C, ncs, nU, nV);
  return (size_t)(ncs + nU + nV);
}

hipError_t tabulate_green_ws(const GreenSpec& g, int N, int C, int64_t den, double self_h,
                             double* dst, double* ws, hipStream_t st) {
  return tabulate_into(g, N, C, den, self_h, dst, ws, st);
}

hipError_t tabulate_green(const GreenSpec& g, int N, int C, int64_t den, double self_h,
                          double* dst, hipStream_t st) {
  const size_t nws = tabulate_workspace_doubles(g.kind, N, C);
  double* ws = nullptr;
  hipError_t e = nws ? hipMalloc(&ws, nws * sizeof(double)) : hipSuccess;
  if (e == hipSuccess) e = tabulate_into(g, N, C, den, self_h, dst, ws, st);
  if (ws) {
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(ws);
  }
  return e;
}

hipError_t tabulate_accel(const GreenSpec& gs, int N, int C, double* d[3], hipStream_t st) {
  const int64_t ng = (int64_t)(2 * C + 5) * (2 * C + 5) * (2 * C + 5);
  const int64_t total = (int64_t)(2 * C + 1) * (2 * C + 1) * (2 * C + 1);
  double* g = nullptr;
  hipError_t e = hipMalloc(&g, ng * sizeof(double));
  if (e != hipSuccess) return e;
  e = tabulate_green(gs, N, C + 2, N, 1.0 / N, g, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_accel_tab, dim3(nblocks(total, 256)), dim3(256), 0, st, g, C,
                       (double)N / 12.0, d[0], d[1], d[2]);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(g);
  return e;
}

hipError_t cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast, dim3(nblocks(n, 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace pfmm
