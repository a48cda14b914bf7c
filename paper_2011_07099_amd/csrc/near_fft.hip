// The leaf near zone by FFT convolution on a doubled grid: the paper's own
// route (Sec. 2 adds a leaf's near zone by a PM solver with non-periodic
// boundary conditions; Sec. 3 names grid doubling as the way it does so).
//
// Target leaf b, source leaf b + e (e in {-1, 0, 1}^3, 27 neighbours), cells
// c and c' inside their leaves: the near zone is
//   phi[b s + c] = h^3 sum_e sum_c' G(h (c - c' - s e)) rho[(b + e) s + c'].
// For one e this is a linear convolution of an s^3 block with the kernel
// K_e[m] = G(h (m - s e)), m = c - c' in [-(s-1), s-1]^3.  On a cyclic grid of
// 2s points per axis every needed m has its own residue (2s - 1 of the 2s
// slots), so the cyclic convolution of the zero-padded block equals the
// linear one at the s^3 target cells.  In Fourier space the 27 neighbours
// then add pointwise:
//   phi_hat_b(k) = sum_e K_hat_e(k) rho_hat_{b+e}(k),
// one forward transform per leaf, a 27-point stencil over the leaf grid at
// every frequency, one inverse transform per leaf.  Against the direct sum's
// 2 (s^3)^2 flops per leaf pair this costs O(s^3 log s) per leaf.
//
// The kernels are transformed once per table (plan time) by a separable
// FP64 DFT; the per-solve transforms are rocFFT R2C / C2R in FP32.  The same
// machinery serves the acceleration kernels D_i (they replace G).
#include "internal.h"

#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>

namespace pfmm {

struct NearFft {
  int N = 0, s = 0, nb = 0;  // cells per axis, leaf edge, leaves per axis
  int64_t nleaf = 0;
  int64_t R = 0;             // (2s)^3 real points per leaf
  int64_t F = 0;             // 2s * 2s * (s + 1) frequencies per leaf (half spectrum)
  hipfftHandle fwd = 0, inv = 0;
  float* pad = nullptr;      // [nleaf][R]: padded blocks, then inverse transforms
  float2* rhat = nullptr;    // [nleaf][F]
  float2* yhat = nullptr;    // [nleaf][F]
  float2* khat[4] = {nullptr, nullptr, nullptr, nullptr};  // [27][F] per kernel
  double2* dft[2] = {nullptr, nullptr};                    // [F] FP64 DFT passes
};

namespace {

constexpr int kThreads = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

hipError_t fft_err(hipfftResult r) { return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown; }

// Signed cyclic index of slot u on 2s points: u for u < s, u - 2s for u > s;
// slot s carries no separation (returned as `bad`).
__device__ inline int signed_slot(int u, int s, bool& bad) {
  bad = bad || u == s;
  return u < s ? u : u - 2 * s;
}

// First DFT pass, along z (real input, half spectrum kz in [0, s]):
//   A[x][y][kz] = sum_z K_e[x][y][z] exp(-2 pi i kz z / 2s),
// K_e[x][y][z] = tab[w(x) - s ex][w(y) - s ey][w(z) - s ez] (tab centred, edge
// 2C + 1, C = 2s - 1), zero on the unused slot.
__global__ void k_kdft_z(const double* __restrict__ tab, int s, int ex, int ey, int ez,
                         double2* __restrict__ A) {
  const int M = 2 * s, H = s + 1;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)M * M * H) return;
  const int kz = (int)(i % H), y = (int)((i / H) % M), x = (int)(i / ((int64_t)H * M));
  const int C = 2 * s - 1, E = 2 * C + 1;
  bool bad = false;
  const int jx = signed_slot(x, s, bad) - s * ex;
  const int jy = signed_slot(y, s, bad) - s * ey;
  double re = 0.0, im = 0.0;
  if (!bad) {
    const double* row = tab + ((int64_t)(jx + C) * E + (jy + C)) * E;
    for (int z = 0; z < M; ++z) {
      if (z == s) continue;
      const int jz = (z < s ? z : z - M) - s * ez;
      const double v = row[jz + C];
      double sn, cs;
      sincospi(-(double)((kz * z) % M) / s, &sn, &cs);
      re += v * cs;
      im += v * sn;
    }
  }
  A[i] = make_double2(re, im);
}

// Complex DFT pass along y (axis 1) or x (axis 0) of a [2s][2s][s + 1] array.
__global__ void k_kdft_axis(const double2* __restrict__ in, int s, int axis, double2* __restrict__ out) {
  const int M = 2 * s, H = s + 1;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)M * M * H) return;
  const int kz = (int)(i % H), b = (int)((i / H) % M), a = (int)(i / ((int64_t)H * M));
  const int k = axis ? b : a;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < M; ++j) {
    const int64_t src = axis ? ((int64_t)a * M + j) * H + kz : ((int64_t)j * M + b) * H + kz;
    const double2 v = in[src];
    double sn, cs;
    sincospi(-(double)((k * j) % M) / s, &sn, &cs);
    re += v.x * cs - v.y * sn;
    im += v.x * sn + v.y * cs;
  }
  out[i] = make_double2(re, im);
}

__global__ void k_kdft_store(const double2* __restrict__ in, int64_t F, double scale,
                             float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F) return;
  out[i] = make_float2((float)(in[i].x * scale), (float)(in[i].y * scale));
}

// pad[leaf][x][y][z] = rho of the leaf's cell (x, y, z) for x, y, z < s, else 0
__global__ void k_pack(const float* __restrict__ rho, int N, int s, int nb, int64_t total,
                       float* __restrict__ pad) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total) return;
  const int M = 2 * s;
  const int64_t R = (int64_t)M * M * M;
  const int64_t leaf = i / R;
  const int u = (int)(i % R);
  const int z = u % M, y = (u / M) % M, x = u / (M * M);
  float v = 0.0f;
  if (x < s && y < s && z < s) {
    const int bz = (int)(leaf % nb), by = (int)((leaf / nb) % nb), bx = (int)(leaf / ((int64_t)nb * nb));
    v = rho[((int64_t)(bx * s + x) * N + (by * s + y)) * N + (bz * s + z)];
  }
  pad[i] = v;
}

// out[cell] (+)= the target block of the inverse transform of the cell's leaf
__global__ void k_unpack(const float* __restrict__ pad, int N, int s, int nb, int accumulate,
                         float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t N3 = (int64_t)N * N * N;
  if (i >= N3) return;
  const int Z = (int)(i % N), Y = (int)((i / N) % N), X = (int)(i / ((int64_t)N * N));
  const int M = 2 * s;
  const int64_t leaf = ((int64_t)(X / s) * nb + (Y / s)) * nb + (Z / s);
  const float v = pad[leaf * ((int64_t)M * M * M) + ((int64_t)(X % s) * M + (Y % s)) * M + (Z % s)];
  out[i] = accumulate ? out[i] + v : v;
}

// yhat_b(k) = sum_e khat_e(k) rhat_{b+e}(k).  Block = 256 consecutive
// frequencies of one pencil of leaves (bx, by), swept along z with the
// 3 z-neighbours of each of the 9 (ex, ey) columns held in registers.  The
// pencils of one frequency chunk go to one XCD (blocks are dealt to the 8
// XCDs round robin), so its L2 serves the 9 column re-reads.
__global__ void __launch_bounds__(kThreads) k_near_mac(const float2* __restrict__ rhat,
                                                        const float2* __restrict__ khat, int nb,
                                                        int64_t F, int nchunk, int isolated,
                                                        float2* __restrict__ yhat) {
  const int g = blockIdx.x;
  const int np = nb * nb;
  const int j = g >> 3;
  const int chunk = (j / np) * 8 + (g & 7);
  if (chunk >= nchunk) return;
  const int64_t k = (int64_t)chunk * kThreads + threadIdx.x;
  if (k >= F) return;
  const int pencil = j % np;
  const int bx = pencil / nb, by = pencil % nb;
  float2 kk[27];
#pragma unroll
  for (int e = 0; e < 27; ++e) kk[e] = khat[(int64_t)e * F + k];
  int64_t col[9];
  bool ok[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    int sx = bx + c / 3 - 1, sy = by + c % 3 - 1;
    ok[c] = !isolated || (sx >= 0 && sx < nb && sy >= 0 && sy < nb);
    sx = (sx + nb) % nb;
    sy = (sy + nb) % nb;
    col[c] = ((int64_t)sx * nb + sy) * nb;
  }
  auto load = [&](int c, int z) -> float2 {
    if (isolated && (z < 0 || z >= nb || !ok[c])) return make_float2(0.0f, 0.0f);
    const int zw = (z + nb) % nb;
    return rhat[(col[c] + zw) * F + k];
  };
  float2 r0[9], r1[9], r2[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    r0[c] = load(c, -1);
    r1[c] = load(c, 0);
  }
  for (int bz = 0; bz < nb; ++bz) {
#pragma unroll
    for (int c = 0; c < 9; ++c) r2[c] = load(c, bz + 1);
    float re = 0.0f, im = 0.0f;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const float2 a = kk[3 * c], b = kk[3 * c + 1], d = kk[3 * c + 2];
      re += a.x * r0[c].x - a.y * r0[c].y + b.x * r1[c].x - b.y * r1[c].y + d.x * r2[c].x - d.y * r2[c].y;
      im += a.x * r0[c].y + a.y * r0[c].x + b.x * r1[c].y + b.y * r1[c].x + d.x * r2[c].y + d.y * r2[c].x;
    }
    yhat[(((int64_t)bx * nb + by) * nb + bz) * F + k] = make_float2(re, im);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      r0[c] = r1[c];
      r1[c] = r2[c];
    }
  }
}

}  // namespace

void near_fft_destroy(NearFft* f) {
  if (!f) return;
  if (f->fwd) (void)hipfftDestroy(f->fwd);
  if (f->inv) (void)hipfftDestroy(f->inv);
  (void)hipFree(f->pad);
  (void)hipFree(f->rhat);
  (void)hipFree(f->yhat);
  for (float2* k : f->khat) (void)hipFree(k);
  for (double2* d : f->dft) (void)hipFree(d);
  delete f;
}

hipError_t near_fft_create(int N, int s, NearFft** out) {
  *out = nullptr;
  if (s < 1 || N % s) return hipErrorInvalidValue;
  NearFft* f = new NearFft;
  f->N = N;
  f->s = s;
  f->nb = N / s;
  f->nleaf = (int64_t)f->nb * f->nb * f->nb;
  const int M = 2 * s;
  f->R = (int64_t)M * M * M;
  f->F = (int64_t)M * M * (s + 1);
  hipError_t e = hipMalloc(&f->pad, (size_t)(f->nleaf * f->R) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&f->rhat, (size_t)(f->nleaf * f->F) * sizeof(float2));
  if (e == hipSuccess) e = hipMalloc(&f->yhat, (size_t)(f->nleaf * f->F) * sizeof(float2));
  if (e == hipSuccess) {
    int nn[3] = {M, M, M};
    e = fft_err(hipfftPlanMany(&f->fwd, 3, nn, nullptr, 1, (int)f->R, nullptr, 1, (int)f->F,
                               HIPFFT_R2C, (int)f->nleaf));
    if (e == hipSuccess)
      e = fft_err(hipfftPlanMany(&f->inv, 3, nn, nullptr, 1, (int)f->F, nullptr, 1, (int)f->R,
                                 HIPFFT_C2R, (int)f->nleaf));
  }
  if (e != hipSuccess) {
    near_fft_destroy(f);
    return e;
  }
  *out = f;
  return hipSuccess;
}

hipError_t near_fft_tables(NearFft* f, const double* const* tabs, int ntabs, double scale,
                           hipStream_t st) {
  if (ntabs < 1 || ntabs > 4) return hipErrorInvalidValue;
  const int s = f->s;
  hipError_t e = hipSuccess;
  for (int d = 0; d < 2 && e == hipSuccess; ++d)
    if (!f->dft[d]) e = hipMalloc(&f->dft[d], (size_t)f->F * sizeof(double2));
  for (int t = 0; t < ntabs && e == hipSuccess; ++t)
    if (!f->khat[t]) e = hipMalloc(&f->khat[t], (size_t)(27 * f->F) * sizeof(float2));
  // the inverse transform is unnormalised: fold 1 / (2s)^3 into the kernels
  const double sc = scale / (double)f->R;
  for (int t = 0; t < ntabs && e == hipSuccess; ++t)
    for (int ei = 0; ei < 27 && e == hipSuccess; ++ei) {
      const int ex = ei / 9 - 1, ey = (ei / 3) % 3 - 1, ez = ei % 3 - 1;
      k_kdft_z<<<nblk(f->F), kThreads, 0, st>>>(tabs[t], s, ex, ey, ez, f->dft[0]);
      k_kdft_axis<<<nblk(f->F), kThreads, 0, st>>>(f->dft[0], s, 1, f->dft[1]);
      k_kdft_axis<<<nblk(f->F), kThreads, 0, st>>>(f->dft[1], s, 0, f->dft[0]);
      k_kdft_store<<<nblk(f->F), kThreads, 0, st>>>(f->dft[0], f->F, sc, f->khat[t] + (int64_t)ei * f->F);
      e = hipGetLastError();
    }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

int near_fft_kernels(const NearFft* f) {
  int n = 0;
  while (n < 4 && f->khat[n]) ++n;
  return n;
}

hipError_t near_fft_run(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                        hipStream_t st) {
  if (nout < 1 || nout > near_fft_kernels(f)) return hipErrorInvalidValue;
  const int64_t total = f->nleaf * f->R;
  k_pack<<<nblk(total), kThreads, 0, st>>>(rho, f->N, f->s, f->nb, total, f->pad);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->fwd, st));
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->inv, st));
  if (e == hipSuccess) e = fft_err(hipfftExecR2C(f->fwd, f->pad, (hipfftComplex*)f->rhat));
  const int nchunk = (int)((f->F + kThreads - 1) / kThreads);
  const int64_t blocks = (int64_t)((nchunk + 7) / 8) * 8 * f->nb * f->nb;
  const int64_t N3 = (int64_t)f->N * f->N * f->N;
  for (int t = 0; t < nout && e == hipSuccess; ++t) {
    k_near_mac<<<(unsigned)blocks, kThreads, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F, nchunk,
                                                     isolated, f->yhat);
    e = hipGetLastError();
    if (e == hipSuccess) e = fft_err(hipfftExecC2R(f->inv, (hipfftComplex*)f->yhat, f->pad));
    if (e == hipSuccess) {
      k_unpack<<<nblk(N3), kThreads, 0, st>>>(f->pad, f->N, f->s, f->nb, 0, out[t]);
      e = hipGetLastError();
    }
  }
  return e;
}

}  // namespace pfmm
