// Interaction-zone sums by FFT convolution: the M2L of the Hierarchical
// Particle-Mesh flavour of the FMM that the paper runs (Sec. 2).  The
// effective masses of a target node's whole interaction zone are placed on
// one uniform grid and the potential at the target's gridlet points is one
// FFT convolution of that grid with G, as in PM.  This is the comparator of
// the block-Toeplitz GEMM M2L: same sums and tables, each level in the
// precision the plan keeps it in (FP64 transforms for the FP64 coarse levels).
//
// Levels >= 3: the zone of target t lies in the 6^3 children of the parent's
// 27 neighbours; that region's gridlet points, with t's own 27 neighbours
// zeroed, form a (6p)^3 grid, zero-padded to M = 8p per axis so that the
// cyclic convolution equals the linear one at the target's points (every
// target-source separation is below 4p = M/2 gridlet spacings).  Level 2:
// the whole periodic 4^3 level is one (4p)^3 grid and the cyclic convolution
// with the periodic G is the periodic zone sum itself.
//
// Per batch of B targets: scatter (masked masses -> real grids), batched R2C
// FFT, multiply by the transformed kernel (K[m] = G(eta w(m)), w the signed
// cyclic index), batched C2R FFT, gather (add to the target's potentials).
#include "internal.h"

#include <hipfft/hipfft.h>

#include <algorithm>

namespace pfmm {
namespace {

constexpr int kThreads = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

template <class T> struct Cplx;
template <> struct Cplx<float> { using type = hipfftComplex; };
template <> struct Cplx<double> { using type = hipfftDoubleComplex; };

// K[m] = tab[w(m)] for |w_i| <= C, else 0; tab is the level table, (2C+1)^3
template <class T>
__global__ void k_fft_kernel(const double* __restrict__ tab, int C, int M, T* __restrict__ K) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t M3 = (int64_t)M * M * M;
  if (i >= M3) return;
  const int mz = (int)(i % M), my = (int)((i / M) % M), mx = (int)(i / ((int64_t)M * M));
  const int wx = mx < M / 2 ? mx : mx - M;
  const int wy = my < M / 2 ? my : my - M;
  const int wz = mz < M / 2 ? mz : mz - M;
  const int E = 2 * C + 1;
  T v = 0;
  if (abs(wx) <= C && abs(wy) <= C && abs(wz) <= C)
    v = (T)tab[((int64_t)(wx + C) * E + (wy + C)) * E + (wz + C)];
  K[i] = v;
}

// x[b][u]: the masked interaction-zone masses of target t0 + b (zero for
// b beyond the level's targets)
template <class T>
__global__ void k_fft_scatter(const T* __restrict__ Ml, int n, int p, int M, int level2,
                              int64_t t0, int64_t ntarg, int B, T* __restrict__ x) {
  const int64_t M3 = (int64_t)M * M * M;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)B * M3) return;
  const int64_t b = i / M3;
  const int64_t u = i % M3;
  const int64_t t = t0 + b;
  T v = 0;
  if (t < ntarg) {
    const int tx = (int)(t / ((int64_t)n * n)), ty = (int)((t / n) % n), tz = (int)(t % n);
    const int ux = (int)(u / ((int64_t)M * M)), uy = (int)((u / M) % M), uz = (int)(u % M);
    int kx, ky, kz;   // source node (before the periodic wrap)
    int dx, dy, dz;   // its offset from the target node
    bool inside;
    if (level2) {
      kx = ux / p; ky = uy / p; kz = uz / p;
      inside = true;
      dx = ((kx - tx + 2) & 3) - 2;  // nearest image on the periodic 4^3 level
      dy = ((ky - ty + 2) & 3) - 2;
      dz = ((kz - tz + 2) & 3) - 2;
    } else {
      inside = ux < 6 * p && uy < 6 * p && uz < 6 * p;
      kx = 2 * (tx >> 1) - 2 + ux / p;
      ky = 2 * (ty >> 1) - 2 + uy / p;
      kz = 2 * (tz >> 1) - 2 + uz / p;
      dx = kx - tx; dy = ky - ty; dz = kz - tz;
    }
    const bool zone = abs(dx) > 1 || abs(dy) > 1 || abs(dz) > 1;
    if (inside && zone) {
      const int sx = (kx + n) & (n - 1), sy = (ky + n) & (n - 1), sz = (kz + n) & (n - 1);
      const int ax = ux % p, ay = uy % p, az = uz % p;
      v = Ml[(((int64_t)sx * n + sy) * n + sz) * p * p * p + (ax * p + ay) * p + az];
    }
  }
  x[i] = v;
}

// X[b][f] *= Kf[f] * scale (the inverse transform is unnormalised)
template <class C, class T>
__global__ void k_fft_mul(C* __restrict__ X, const C* __restrict__ Kf, int64_t nf, int B, T scale) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)B * nf) return;
  const C k = Kf[i % nf];
  const C a = X[i];
  C r;
  r.x = (a.x * k.x - a.y * k.y) * scale;
  r.y = (a.x * k.y + a.y * k.x) * scale;
  X[i] = r;
}

// Phi[t][a] (+)= y[b][target point a]
template <class T>
__global__ void k_fft_gather(const T* __restrict__ y, int n, int p, int M, int level2,
                             int64_t t0, int64_t ntarg, int B, int accumulate,
                             T* __restrict__ Pl) {
  const int p3 = p * p * p;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)B * p3) return;
  const int64_t b = i / p3;
  const int a = (int)(i % p3);
  const int64_t t = t0 + b;
  if (t >= ntarg) return;
  const int tx = (int)(t / ((int64_t)n * n)), ty = (int)((t / n) % n), tz = (int)(t % n);
  const int ax = a / (p * p), ay = (a / p) % p, az = a % p;
  int ux, uy, uz;
  if (level2) {
    ux = tx * p + ax; uy = ty * p + ay; uz = tz * p + az;
  } else {  // the target node sits at child position 2 + (t & 1) of its region
    ux = (2 + (tx & 1)) * p + ax; uy = (2 + (ty & 1)) * p + ay; uz = (2 + (tz & 1)) * p + az;
  }
  const T v = y[b * (int64_t)M * M * M + ((int64_t)ux * M + uy) * M + uz];
  T* o = Pl + t * p3 + a;
  *o = accumulate ? *o + v : v;
}

hipError_t fft_err(hipfftResult r) { return r == HIPFFT_SUCCESS ? hipSuccess : hipErrorUnknown; }
int64_t nfreq(int M) { return (int64_t)M * M * (M / 2 + 1); }

}  // namespace

struct M2LFft {
  int p = 0, L = 0;
  // per grid size (index 0: level 2, M = 4p; index 1: levels >= 3, M = 8p),
  // per precision (index 0: FP32, 1: FP64)
  int M[2] = {0, 0};
  int B[2] = {0, 0};
  hipfftHandle fwd[2][2] = {{0, 0}, {0, 0}}, inv[2][2] = {{0, 0}, {0, 0}};
  void* x = nullptr;              // real grids, max over sizes of B M^3 doubles
  void* X = nullptr;              // their transforms
  std::vector<void*> Kf[2];       // per precision, per level: transformed kernel
  std::vector<void*> owned;
};

void m2l_fft_destroy(M2LFft* f) {
  if (!f) return;
  for (int k = 0; k < 2; ++k)
    for (int d = 0; d < 2; ++d) {
      if (f->fwd[k][d]) (void)hipfftDestroy(f->fwd[k][d]);
      if (f->inv[k][d]) (void)hipfftDestroy(f->inv[k][d]);
    }
  for (void* q : f->owned) (void)hipFree(q);
  delete f;
}

hipError_t m2l_fft_create(int L, int p, size_t budget_bytes, M2LFft** out) {
  *out = nullptr;
  M2LFft* f = new M2LFft;
  f->p = p;
  f->L = L;
  f->M[0] = 4 * p;
  f->M[1] = 8 * p;
  size_t xb = 0, Xb = 0;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    if (k == 1 && L < 3) break;
    const int M = f->M[k];
    const int64_t M3 = (int64_t)M * M * M;
    // sized for FP64 grids; FP32 batches use the same count
    const size_t per = (size_t)M3 * sizeof(double) + (size_t)nfreq(M) * sizeof(hipfftDoubleComplex);
    const int64_t maxt = k == 0 ? 64 : (int64_t)1 << (3 * L);
    int64_t B = 1;
    while (B * 2 <= maxt && (size_t)(B * 2) * per <= budget_bytes) B *= 2;
    f->B[k] = (int)B;
    int nn[3] = {M, M, M};
    const hipfftType tf[2] = {HIPFFT_R2C, HIPFFT_D2Z}, ti[2] = {HIPFFT_C2R, HIPFFT_Z2D};
    for (int d = 0; d < 2 && e == hipSuccess; ++d) {
      e = fft_err(hipfftPlanMany(&f->fwd[k][d], 3, nn, nullptr, 1, (int)M3, nullptr, 1,
                                 (int)nfreq(M), tf[d], (int)B));
      if (e == hipSuccess)
        e = fft_err(hipfftPlanMany(&f->inv[k][d], 3, nn, nullptr, 1, (int)nfreq(M), nullptr, 1,
                                   (int)M3, ti[d], (int)B));
    }
    xb = std::max(xb, (size_t)(B * M3) * sizeof(double));
    Xb = std::max(Xb, (size_t)(B * nfreq(M)) * sizeof(hipfftDoubleComplex));
  }
  void* q = nullptr;
  if (e == hipSuccess) e = hipMalloc(&q, xb);
  if (e == hipSuccess) {
    f->owned.push_back(q);
    f->x = q;
    e = hipMalloc(&q, Xb);
  }
  if (e == hipSuccess) {
    f->owned.push_back(q);
    f->X = q;
  }
  for (int d = 0; d < 2; ++d) f->Kf[d].assign(L + 1, nullptr);
  for (int l = 2; l <= L && e == hipSuccess; ++l)
    for (int d = 0; d < 2 && e == hipSuccess; ++d) {
      const size_t c = d ? sizeof(hipfftDoubleComplex) : sizeof(hipfftComplex);
      e = hipMalloc(&q, (size_t)nfreq(f->M[l == 2 ? 0 : 1]) * c);
      if (e == hipSuccess) {
        f->owned.push_back(q);
        f->Kf[d][l] = q;
      }
    }
  if (e != hipSuccess) {
    m2l_fft_destroy(f);
    return e;
  }
  *out = f;
  return hipSuccess;
}

namespace {
template <class T>
hipError_t exec_fwd(hipfftHandle h, void* in, void* out);
template <>
hipError_t exec_fwd<float>(hipfftHandle h, void* in, void* out) {
  return fft_err(hipfftExecR2C(h, (hipfftReal*)in, (hipfftComplex*)out));
}
template <>
hipError_t exec_fwd<double>(hipfftHandle h, void* in, void* out) {
  return fft_err(hipfftExecD2Z(h, (hipfftDoubleReal*)in, (hipfftDoubleComplex*)out));
}
template <class T>
hipError_t exec_inv(hipfftHandle h, void* in, void* out);
template <>
hipError_t exec_inv<float>(hipfftHandle h, void* in, void* out) {
  return fft_err(hipfftExecC2R(h, (hipfftComplex*)in, (hipfftReal*)out));
}
template <>
hipError_t exec_inv<double>(hipfftHandle h, void* in, void* out) {
  return fft_err(hipfftExecZ2D(h, (hipfftDoubleComplex*)in, (hipfftDoubleReal*)out));
}

template <class T>
hipError_t kernel_transform(M2LFft* f, int l, const double* tab64, hipStream_t st) {
  const int d = sizeof(T) == 8 ? 1 : 0;
  const int k = l == 2 ? 0 : 1;
  const int M = f->M[k];
  const int64_t M3 = (int64_t)M * M * M;
  T* x = (T*)f->x;
  // the batch plan transforms every slot: zero them, the kernel in slot 0
  hipLaunchKernelGGL(k_fft_scatter<T>, dim3(nblk((int64_t)f->B[k] * M3)), dim3(kThreads), 0, st,
                     (const T*)nullptr, 1, f->p, M, 1, (int64_t)0, (int64_t)0, f->B[k], x);
  hipLaunchKernelGGL(k_fft_kernel<T>, dim3(nblk(M3)), dim3(kThreads), 0, st, tab64, 4 * f->p - 1,
                     M, x);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->fwd[k][d], st));
  if (e == hipSuccess) e = exec_fwd<T>(f->fwd[k][d], f->x, f->X);
  const size_t c = sizeof(typename Cplx<T>::type);
  if (e == hipSuccess)
    e = hipMemcpyAsync(f->Kf[d][l], f->X, (size_t)nfreq(M) * c, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

template <class T>
hipError_t level_sums(M2LFft* f, int l, const T* Ml, T* Pl, int accumulate, hipStream_t st) {
  using C = typename Cplx<T>::type;
  const int d = sizeof(T) == 8 ? 1 : 0;
  const int k = l == 2 ? 0 : 1;
  const int M = f->M[k], B = f->B[k], p = f->p, n = 1 << l;
  const int64_t M3 = (int64_t)M * M * M, nf = nfreq(M);
  const int64_t ntarg = (int64_t)1 << (3 * l);
  T* x = (T*)f->x;
  hipError_t e = fft_err(hipfftSetStream(f->fwd[k][d], st));
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->inv[k][d], st));
  for (int64_t t0 = 0; t0 < ntarg && e == hipSuccess; t0 += B) {
    hipLaunchKernelGGL(k_fft_scatter<T>, dim3(nblk((int64_t)B * M3)), dim3(kThreads), 0, st, Ml,
                       n, p, M, l == 2 ? 1 : 0, t0, ntarg, B, x);
    e = hipGetLastError();
    if (e == hipSuccess) e = exec_fwd<T>(f->fwd[k][d], f->x, f->X);
    if (e == hipSuccess) {
      hipLaunchKernelGGL((k_fft_mul<C, T>), dim3(nblk((int64_t)B * nf)), dim3(kThreads), 0, st,
                         (C*)f->X, (const C*)f->Kf[d][l], nf, B, (T)1 / (T)M3);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = exec_inv<T>(f->inv[k][d], f->X, f->x);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_fft_gather<T>, dim3(nblk((int64_t)B * p * p * p)), dim3(kThreads), 0,
                         st, (const T*)x, n, p, M, l == 2 ? 1 : 0, t0, ntarg, B, accumulate, Pl);
      e = hipGetLastError();
    }
  }
  return e;
}
}  // namespace

hipError_t m2l_fft_tables(M2LFft* f, const std::vector<double*>& tab64, hipStream_t st) {
  for (int l = 2; l <= f->L; ++l) {
    hipError_t e = kernel_transform<float>(f, l, tab64[l], st);
    if (e == hipSuccess) e = kernel_transform<double>(f, l, tab64[l], st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t m2l_fft_level(M2LFft* f, int l, const void* Ml, void* Pl, int fp64, int accumulate,
                         hipStream_t st) {
  if (fp64) return level_sums<double>(f, l, (const double*)Ml, (double*)Pl, accumulate, st);
  return level_sums<float>(f, l, (const float*)Ml, (float*)Pl, accumulate, st);
}

}  // namespace pfmm
