// Learned correction of the interaction-zone Green's-function tables.
//
// The paper defines an "optimal" Green's function G_* as the one with which
// the FMM reproduces the PM solution (Sec. 3, Eq. 8), approximates it by the
// closed form G_S1 (Eq. 9), and suggests parameterising G_* by many values
// and minimising the FMM-vs-PM error (Sec. 4).  Here a small MLP
// f_theta(|j| sorted / (4p), (|j| sorted mod p) / p, level / 8, p / 10) of the
// table offset j = a - a' - p d (its cube invariants and in-gridlet residues),
// the level and p gives every table entry
// T_l[j] = G(eta_l j) (1 + delta), delta = kappa f_theta with the fixed output
// scale kappa = 1e-4 (the corrections that matter are of the size of the
// FMM-vs-PM residual), of the interaction-zone convolution (Eq. 6); the near
// zone keeps G.  The network is invariant under the 48
// symmetries of the cube, so the corrected operator keeps the FMM symmetric.
// An untrained network (zero output layer) is exactly the uncorrected G.
//
// Training minimises the mean-removed relative residual
//     loss = sum_i r_i^2 / sum_i (phi_t,i - mean)^2,   r = phi - phi_t - mean(phi - phi_t)
// The FMM potential is linear in every table, so
//     d loss / d T_l[j] = sum_t sum_{d in IZ(t)} sum_{a - a' - p d = j} lambda_l[t][a] M_l[t+d][a']
// with the adjoint lambda_l = (M2M)^(L-l) P2M(2 r / norm): the transposes of
// L2L (Eq. 7) and L2P.  The kernels below compute the residual, the table
// gradient, its pull-back to the network output, the network's gradient, and
// Adam; the forward solve and the adjoint sweep reuse the solve's kernels.
#include "internal.h"

#include <cstdint>

namespace pfmm {
namespace {

constexpr int kH = 64;           // hidden width
constexpr float kKappa = 1e-4f;  // output scale: delta = kappa * network output

__device__ inline float silu(float z) { return z / (1.f + expf(-z)); }
__device__ inline float dsilu(float z) {
  const float s = 1.f / (1.f + expf(-z));
  return s * (1.f + z * (1.f - s));
}
__device__ inline float rb(float x, int bf16) { return bf16 ? (float)(__bf16)x : x; }

// theta layout: W1[64][kMlpIn] b1[64] W2[64][64] b2[64] W3[64] b3
constexpr int oW1 = 0, oB1 = kH * kMlpIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;
static_assert(oB3 + 1 == kMlpParams, "network layout");

// Network output for every entry; with bf16 = 1 the weights, inputs and
// activations are rounded to bf16 before each product (FP32 accumulation).
__global__ void k_mlp_forward(const float* __restrict__ theta, const float* __restrict__ feats,
                              int n, int bf16, float* __restrict__ delta) {
  __shared__ float w[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = rb(theta[i], bf16);
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float x[kMlpIn];
  for (int k = 0; k < kMlpIn; ++k) x[k] = rb(feats[e * kMlpIn + k], bf16);
  float h1[kH];
  for (int i = 0; i < kH; ++i) {
    float z = w[oB1 + i];
    for (int k = 0; k < kMlpIn; ++k) z += w[oW1 + i * kMlpIn + k] * x[k];
    h1[i] = rb(silu(z), bf16);
  }
  float out = w[oB3];
  for (int i = 0; i < kH; ++i) {
    float z = w[oB2 + i];
    for (int k = 0; k < kH; ++k) z += w[oW2 + i * kH + k] * h1[k];
    out += w[oW3 + i] * rb(silu(z), bf16);
  }
  delta[e] = kKappa * out;
}

// T[j] = G0[j] (1 + delta[uidx[j]]) in FP64 and FP32
__global__ void k_apply_correction(const double* __restrict__ g0, const float* __restrict__ delta,
                                   const int* __restrict__ uidx, int64_t n,
                                   double* __restrict__ t64, float* __restrict__ t32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = g0[i] * (1.0 + (double)delta[uidx[i]]);
  t64[i] = v;
  t32[i] = (float)v;
}

// Partial sums over the mesh of d = phi - t, d^2, t, t^2 (FP64), one block each.
__global__ void k_resid_partial(const float* __restrict__ phi, const float* __restrict__ t,
                                int64_t n, double* __restrict__ part) {
  __shared__ double sd[256], sdd[256], st[256], stt[256];
  double a = 0, b = 0, c = 0, e = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)phi[i] - (double)t[i], tv = t[i];
    a += d;
    b += d * d;
    c += tv;
    e += tv * tv;
  }
  sd[threadIdx.x] = a;
  sdd[threadIdx.x] = b;
  st[threadIdx.x] = c;
  stt[threadIdx.x] = e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sd[threadIdx.x] += sd[threadIdx.x + s];
      sdd[threadIdx.x] += sdd[threadIdx.x + s];
      st[threadIdx.x] += st[threadIdx.x + s];
      stt[threadIdx.x] += stt[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = sd[0];
    part[blockIdx.x * 4 + 1] = sdd[0];
    part[blockIdx.x * 4 + 2] = st[0];
    part[blockIdx.x * 4 + 3] = stt[0];
  }
}

// out[0] = mean d, out[1] = loss, out[2] = norm, out[3] = mean t (sum over the block
// partials in order)
__global__ void k_resid_final(const double* __restrict__ part, int nblk, int64_t n,
                              double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0, b = 0, c = 0, e = 0;
  for (int i = 0; i < nblk; ++i) {
    a += part[i * 4 + 0];
    b += part[i * 4 + 1];
    c += part[i * 4 + 2];
    e += part[i * 4 + 3];
  }
  const double md = a / (double)n, mt = c / (double)n;
  const double norm = e - (double)n * mt * mt;
  out[0] = md;
  out[1] = (b - (double)n * md * md) / norm;
  out[2] = norm;
  out[3] = mt;
}

// r = 2 (phi - t - mean) / norm  (d loss / d phi)
__global__ void k_resid_scale(const float* __restrict__ phi, const float* __restrict__ t,
                              const double* __restrict__ stats, int64_t n, float* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  r[i] = (float)(2.0 * ((double)phi[i] - (double)t[i] - stats[0]) / stats[2]);
}

// Table gradient, one block per (class, offset): window entries w of the
// (2q-1)^3 slice around -q d get sum over the class's targets t and points a
// of lambda[t][a] M[t+d][a - w'] (w' = w - (q-1) per axis).
template <class T>
__global__ __launch_bounds__(256) void k_table_grad(int n, int m, int q, int noff,
                                                    const int* __restrict__ offs,
                                                    const T* __restrict__ lam,
                                                    const T* __restrict__ M,
                                                    double* __restrict__ part) {
  extern __shared__ __align__(8) unsigned char smraw[];
  T* sl = reinterpret_cast<T*>(smraw);     // lambda of 8 targets
  T* sm = sl + 8 * q * q * q;              // M of their sources
  const int cls = blockIdx.x / noff, k = blockIdx.x % noff;
  const int pk = offs[(size_t)cls * noff + k];
  const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
  const int cx = cls / (m * m), cy = (cls / m) % m, cz = cls % m;
  const int nk = n / m, ntarg = nk * nk * nk, q3 = q * q * q, S = 2 * q - 1;
  const int nw = S * S * S;
  constexpr int kPer = 28;  // window entries per thread: 15^3 / 256 < 14, (2q-1)^3 <= 3375
  double acc[kPer];
  for (int r = 0; r < kPer; ++r) acc[r] = 0.0;
  for (int t0 = 0; t0 < ntarg; t0 += 8) {
    __syncthreads();
    for (int i = threadIdx.x; i < 8 * q3; i += blockDim.x) {
      const int tl = i / q3, e = i % q3, t = t0 + tl;
      T lv = 0, mv = 0;
      if (t < ntarg) {
        const int kx = t / (nk * nk), ky = (t / nk) % nk, kz = t % nk;
        const int tx = cx + m * kx, ty = cy + m * ky, tz = cz + m * kz;
        const int ux = (tx + dx) & (n - 1), uy = (ty + dy) & (n - 1), uz = (tz + dz) & (n - 1);
        lv = lam[(((size_t)tx * n + ty) * n + tz) * q3 + e];
        mv = M[(((size_t)ux * n + uy) * n + uz) * q3 + e];
      }
      sl[i] = lv;
      sm[i] = mv;
    }
    __syncthreads();
    for (int r = 0; r < kPer; ++r) {
      const int w = threadIdx.x + r * blockDim.x;
      if (w >= nw) break;
      const int wx = w / (S * S) - (q - 1), wy = (w / S) % S - (q - 1), wz = w % S - (q - 1);
      double s = 0.0;
      for (int tl = 0; tl < 8; ++tl) {
        const T* L = sl + tl * q3;
        const T* Ms = sm + tl * q3;
        for (int ax = max(0, wx); ax < min(q, q + wx); ++ax)
          for (int ay = max(0, wy); ay < min(q, q + wy); ++ay)
            for (int az = max(0, wz); az < min(q, q + wz); ++az)
              s += (double)L[(ax * q + ay) * q + az] *
                   (double)Ms[((ax - wx) * q + (ay - wy)) * q + (az - wz)];
      }
      acc[r] += s;
    }
  }
  for (int r = 0; r < kPer; ++r) {
    const int w = threadIdx.x + r * blockDim.x;
    if (w >= nw) break;
    part[(size_t)blockIdx.x * nw + w] = acc[r];
  }
}

// g[j] = sum over (class, offset) windows holding j, in order; table extent
// E = 2C+1, window offset: table index of window entry w is w' - q d + C.
__global__ void k_table_grad_gather(const double* __restrict__ part, int m3, int noff,
                                    const int* __restrict__ offs, int q, int C,
                                    double* __restrict__ g) {
  const int E = 2 * C + 1;
  const int64_t total = (int64_t)E * E * E;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int jx = (int)(i / ((int64_t)E * E)) - C, jy = (int)((i / E) % E) - C, jz = (int)(i % E) - C;
  const int S = 2 * q - 1, nw = S * S * S;
  double s = 0.0;
  for (int c = 0; c < m3; ++c)
    for (int k = 0; k < noff; ++k) {
      const int pk = offs[(size_t)c * noff + k];
      const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
      const int wx = jx + q * dx, wy = jy + q * dy, wz = jz + q * dz;  // w' = j + q d
      if (wx < -(q - 1) || wx > q - 1 || wy < -(q - 1) || wy > q - 1 || wz < -(q - 1) || wz > q - 1)
        continue;
      const int w = ((wx + q - 1) * S + (wy + q - 1)) * S + (wz + q - 1);
      s += part[((size_t)c * noff + k) * nw + w];
    }
  g[i] = s;
}

// d loss / d delta[u] += sum_{j in orbit(u)} g[j] G0[j]
__global__ void k_orbit_gather(const double* __restrict__ g, const double* __restrict__ g0,
                               const int* __restrict__ ptr, const int* __restrict__ pos, int nu,
                               float* __restrict__ ddelta) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  double s = 0.0;
  for (int k = ptr[u]; k < ptr[u + 1]; ++k) s += g[pos[k]] * g0[pos[k]];
  ddelta[u] += (float)s;
}

// Network gradient for 64 entries per block (FP32), written as one partial
// gradient per block; every gradient component is summed by one thread in
// entry order.
__global__ __launch_bounds__(64) void k_mlp_backward(const float* __restrict__ theta,
                                                     const float* __restrict__ feats,
                                                     const float* __restrict__ ddelta, int n,
                                                     float* __restrict__ part) {
  __shared__ float w[kMlpParams];
  __shared__ float X[64][kMlpIn], H1[64][kH + 1], H2[64][kH + 1], DZ2[64][kH + 1], DZ1[64][kH + 1];
  __shared__ float DD[64];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = theta[i];
  __syncthreads();
  const int tid = threadIdx.x;
  const int e = blockIdx.x * 64 + tid;
  const bool ok = e < n;
  float x[kMlpIn], z1[kH], z2[kH];
  for (int k = 0; k < kMlpIn; ++k) x[k] = ok ? feats[e * kMlpIn + k] : 0.f;
  const float dd = ok ? kKappa * ddelta[e] : 0.f;  // d loss / d (network output)
  for (int i = 0; i < kH; ++i) {
    float z = w[oB1 + i];
    for (int k = 0; k < kMlpIn; ++k) z += w[oW1 + i * kMlpIn + k] * x[k];
    z1[i] = z;
    H1[tid][i] = silu(z);
  }
  for (int i = 0; i < kH; ++i) {
    float z = w[oB2 + i];
    for (int k = 0; k < kH; ++k) z += w[oW2 + i * kH + k] * H1[tid][k];
    z2[i] = z;
    H2[tid][i] = silu(z);
    DZ2[tid][i] = dd * w[oW3 + i] * dsilu(z);
  }
  for (int k = 0; k < kH; ++k) {
    float s = 0.f;
    for (int i = 0; i < kH; ++i) s += w[oW2 + i * kH + k] * DZ2[tid][i];
    DZ1[tid][k] = s * dsilu(z1[k]);
  }
  for (int k = 0; k < kMlpIn; ++k) X[tid][k] = x[k];
  DD[tid] = dd;
  __syncthreads();
  // thread tid owns hidden unit tid: W2 row, W1 row, biases, W3 entry
  float* out = part + (size_t)blockIdx.x * kMlpParams;
  const int i = tid;
  for (int k = 0; k < kH; ++k) {
    float s = 0.f;
    for (int r = 0; r < 64; ++r) s += DZ2[r][i] * H1[r][k];
    out[oW2 + i * kH + k] = s;
  }
  for (int k = 0; k < kMlpIn; ++k) {
    float s = 0.f;
    for (int r = 0; r < 64; ++r) s += DZ1[r][i] * X[r][k];
    out[oW1 + i * kMlpIn + k] = s;
  }
  float b1 = 0.f, b2 = 0.f, w3 = 0.f;
  for (int r = 0; r < 64; ++r) {
    b1 += DZ1[r][i];
    b2 += DZ2[r][i];
    w3 += DD[r] * H2[r][i];
  }
  out[oB1 + i] = b1;
  out[oB2 + i] = b2;
  out[oW3 + i] = w3;
  if (i == 0) {
    float b3 = 0.f;
    for (int r = 0; r < 64; ++r) b3 += DD[r];
    out[oB3] = b3;
  }
}

__global__ void k_sum_partials(const float* __restrict__ part, int nblk, float* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * kMlpParams + i];
  g[i] += s;
}

// Adam (Kingma & Ba) on the averaged gradient g / count over n parameters;
// clears g.
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m1, float* __restrict__ m2,
                       float* __restrict__ g, int n, float count, float lr, float b1, float b2,
                       float eps, int step) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] / count;
  m1[i] = b1 * m1[i] + (1.f - b1) * gi;
  m2[i] = b2 * m2[i] + (1.f - b2) * gi * gi;
  const float mh = m1[i] / (1.f - powf(b1, (float)step));
  const float vh = m2[i] / (1.f - powf(b2, (float)step));
  th[i] -= lr * mh / (sqrtf(vh) + eps);
  g[i] = 0.f;
}

__global__ void k_add_into(float* __restrict__ dst, const float* __restrict__ src, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += src[i];
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t mlp_forward(const float* theta, const float* feats, int n, int bf16, float* delta,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb(n, 64)), dim3(64), 0, st, theta, feats, n, bf16, delta);
  return hipGetLastError();
}

hipError_t apply_correction(const double* g0, const float* delta, const int* uidx, int64_t n,
                            double* t64, float* t32, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_correction, dim3(nb(n, 256)), dim3(256), 0, st, g0, delta, uidx, n,
                     t64, t32);
  return hipGetLastError();
}

hipError_t residual(const float* phi, const float* t, int64_t n, double* part, double* stats,
                    float* r, hipStream_t st) {
  const int nblk = 1024;
  hipLaunchKernelGGL(k_resid_partial, dim3(nblk), dim3(256), 0, st, phi, t, n, part);
  hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(64), 0, st, part, nblk, n, stats);
  hipLaunchKernelGGL(k_resid_scale, dim3(nb(n, 256)), dim3(256), 0, st, phi, t, stats, n, r);
  return hipGetLastError();
}

size_t table_grad_partial_doubles(int m, int q, int noff) {
  const size_t S = 2 * q - 1;
  return (size_t)m * m * m * noff * S * S * S;
}

hipError_t table_grad(int n, int m, int q, int noff, const int* offs, const void* lam,
                      const void* M, int fp64, int C, double* part, double* g, hipStream_t st) {
  const int m3 = m * m * m;
  const size_t q3 = (size_t)q * q * q;
  if (fp64)
    hipLaunchKernelGGL((k_table_grad<double>), dim3(m3 * noff), dim3(256), 16 * q3 * sizeof(double),
                       st, n, m, q, noff, offs, (const double*)lam, (const double*)M, part);
  else
    hipLaunchKernelGGL((k_table_grad<float>), dim3(m3 * noff), dim3(256), 16 * q3 * sizeof(float),
                       st, n, m, q, noff, offs, (const float*)lam, (const float*)M, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t E = 2 * C + 1;
  hipLaunchKernelGGL(k_table_grad_gather, dim3(nb(E * E * E, 256)), dim3(256), 0, st, part, m3,
                     noff, offs, q, C, g);
  return hipGetLastError();
}

hipError_t orbit_gather(const double* g, const double* g0, const int* ptr, const int* pos, int nu,
                        float* ddelta, hipStream_t st) {
  hipLaunchKernelGGL(k_orbit_gather, dim3(nb(nu, 256)), dim3(256), 0, st, g, g0, ptr, pos, nu,
                     ddelta);
  return hipGetLastError();
}

size_t mlp_backward_partial_floats(int n) { return (size_t)nb(n, 64) * kMlpParams; }

hipError_t mlp_backward(const float* theta, const float* feats, const float* ddelta, int n,
                        float* part, float* grad, hipStream_t st) {
  const int nblk = (int)nb(n, 64);
  hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(64), 0, st, theta, feats, ddelta, n, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(nb(kMlpParams, 256)), dim3(256), 0, st, part, nblk, grad);
  return hipGetLastError();
}

hipError_t adam_step(float* theta, float* m1, float* m2, float* grad, int n, float count,
                     float lr, int step, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, st, theta, m1, m2, grad, n, count,
                     lr, 0.9f, 0.999f, 1e-8f, step);
  return hipGetLastError();
}

hipError_t add_into(float* dst, const float* src, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_into, dim3(nb(n, 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace pfmm
