// Block-Toeplitz operator of the FMM's two contraction-heavy steps.
//
// For every target block t of a level (n^3 blocks of q^3 points) and every
// offset d of its zone,
//     Y[t][a] += sum_{a'} tab[a - a' - q d] * X[(t + d) mod n][a'],
// which is the interaction-zone convolution of Eq. 6 when the blocks are
// gridlets (tab = G sampled at the gridlet spacing of the level) and the
// direct near-zone sum of a leaf when the blocks are mesh cells (tab = G on
// the mesh).  The zone D depends on the target's class t mod m: at levels
// >= 3 the interaction zone of a node depends on its position in its parent
// (Sec. 2, Fig. 2).
//
// This file holds the portable form, used for every block edge q and for
// FP32 or FP64 operands: it stages the (2q-1)^3 slice of the table that one
// offset touches and the sources of a tile of targets in LDS and accumulates
// z-rows of outputs in registers.  Each offset's contribution is summed in the
// operand type and then added to an FP64 running total: a single FP32
// accumulator over all ~10^5 terms of a level would leave rounding noise that
// the extrapolating interpolation of the downward pass (Eq. 7) amplifies.
#include "internal.h"

namespace pfmm {
namespace {

constexpr int kThreads = 256;

__device__ inline void unpack_offset(int pk, int& dx, int& dy, int& dz) {
  dx = ((pk >> 16) & 255) - 128;
  dy = ((pk >> 8) & 255) - 128;
  dz = (pk & 255) - 128;
}

template <int Q, int TPT, int GMAX, class T>
__global__ __launch_bounds__(kThreads) void k_toeplitz(ToepArgs a) {
  constexpr int R = Q * Q;                                   // z-rows of a block
  constexpr int Q3 = Q * Q * Q;
  constexpr int S = 2 * Q - 1;                               // slice extent per axis
  // slice rows per x plane: 24 for q = 8 spreads the 64 lanes (ax, ay) of a
  // wave over 8 ax + ay (mod 16) bank groups (conflict-free slice reads)
  constexpr int SY = Q == 8 ? 24 : S;
  constexpr int G = (kThreads / R) < GMAX ? (kThreads / R) : GMAX;  // thread groups
  constexpr int TT = G * TPT;                                // targets per workgroup
  __shared__ T sl[S * SY * S];
  __shared__ T xs[TT * Q3];

  const T* tab = static_cast<const T*>(a.tab);
  const int tid = threadIdx.x;
  const int m = a.m;
  const int cls = blockIdx.y;
  const int cx = cls / (m * m), cy = (cls / m) % m, cz = cls % m;
  const int nk = a.n / m;
  const int ntarg = nk * nk * nk;
  const int t0 = blockIdx.x * TT;
  const int E = 2 * a.C + 1;
  const int nmask = a.n - 1;
  const int* offs = a.offs + (size_t)cls * a.noff;
  const size_t NN = (size_t)a.n * Q;  // mesh size in grid mode
  const T xscale = (T)a.xscale;
  const int g = blockIdx.z;
  const int ob = (a.noff * g) / a.groups, oe = (a.noff * (g + 1)) / a.groups;

  const int grp = tid / R, row = tid % R;
  const bool active = grp < G;
  const int ax = row / Q, ay = row % Q;

  double tot[TPT][Q];
#pragma unroll
  for (int i = 0; i < TPT; ++i)
#pragma unroll
    for (int j = 0; j < Q; ++j) tot[i][j] = 0.0;

  for (int k = ob; k < oe; ++k) {
    int dx, dy, dz;
    unpack_offset(offs[k], dx, dy, dz);
    __syncthreads();
    for (int i = tid; i < S * S * S; i += kThreads) {
      const int jx = i / (S * S), jy = (i / S) % S, jz = i % S;
      const int li = (jx * SY + jy) * S + jz;  // padded slice position
      const int ix = -Q * dx + jx - (Q - 1) + a.C;
      const int iy = -Q * dy + jy - (Q - 1) + a.C;
      const int iz = -Q * dz + jz - (Q - 1) + a.C;
      sl[li] = tab[((size_t)ix * E + iy) * E + iz];
    }
    for (int i = tid; i < TT * Q3; i += kThreads) {
      const int tl = i / Q3, e = i % Q3;
      const int t = t0 + tl;
      T v = 0;
      const int kx = t / (nk * nk), ky = (t / nk) % nk, kz = t % nk;
      const int ux0 = cx + m * kx + dx, uy0 = cy + m * ky + dy, uz0 = cz + m * kz + dz;
      const bool inside = !a.isolated || ((unsigned)ux0 < (unsigned)a.n &&
                                          (unsigned)uy0 < (unsigned)a.n && (unsigned)uz0 < (unsigned)a.n);
      if (t < ntarg && inside) {
        const int ux = ux0 & nmask, uy = uy0 & nmask, uz = uz0 & nmask;
        size_t src;
        if (a.grid_in) {
          const int ex = e / (Q * Q), ey = (e / Q) % Q, ez = e % Q;
          src = ((size_t)(ux * Q + ex) * NN + (uy * Q + ey)) * NN + (uz * Q + ez);
        } else {
          src = (((size_t)ux * a.n + uy) * a.n + uz) * Q3 + e;
        }
        // a mesh source is FP32 unless the FP64 solve hands in an FP64 mesh
        const T x = !a.grid_in ? static_cast<const T*>(a.X)[src]
                    : a.mesh64 ? (T) static_cast<const double*>(a.X)[src]
                               : (T) static_cast<const float*>(a.X)[src];
        v = x * xscale;
      }
      xs[i] = v;
    }
    __syncthreads();
    if (active) {
      T acc[TPT][Q];
#pragma unroll
      for (int i = 0; i < TPT; ++i)
#pragma unroll
        for (int j = 0; j < Q; ++j) acc[i][j] = 0;
      for (int bx = 0; bx < Q; ++bx) {
        for (int by = 0; by < Q; ++by) {
          T sv[S];
          const T* sp = sl + ((ax - bx + Q - 1) * SY + (ay - by + Q - 1)) * S;
#pragma unroll
          for (int j = 0; j < S; ++j) sv[j] = sp[j];
#pragma unroll
          for (int i = 0; i < TPT; ++i) {
            const T* xp = xs + (grp * TPT + i) * Q3 + (bx * Q + by) * Q;
            T xv[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) xv[j] = xp[j];
#pragma unroll
            for (int az = 0; az < Q; ++az)
#pragma unroll
              for (int bz = 0; bz < Q; ++bz) acc[i][az] += sv[az - bz + Q - 1] * xv[bz];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < TPT; ++i)
#pragma unroll
        for (int j = 0; j < Q; ++j) tot[i][j] += (double)acc[i][j];
    }
  }

  if (!active) return;
  T* Y = static_cast<T*>(a.Y);
  const bool to_part = a.groups > 1;
  if (to_part) Y = static_cast<T*>(a.partial) + (size_t)g * a.n * a.n * a.n * Q3;
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int t = t0 + grp * TPT + i;
    if (t >= ntarg) continue;
    const int kx = t / (nk * nk), ky = (t / nk) % nk, kz = t % nk;
    const int tx = cx + m * kx, ty = cy + m * ky, tz = cz + m * kz;
#pragma unroll
    for (int az = 0; az < Q; ++az) {
      if (a.grid_out) {  // the mesh: FP32, or FP64 for the FP64 solve with FP64 buffers
        const size_t o = ((size_t)(tx * Q + ax) * NN + (ty * Q + ay)) * NN + (tz * Q + az);
        if (a.mesh64) {
          double* Yd = static_cast<double*>(a.Y);
          Yd[o] = a.accumulate ? Yd[o] + tot[i][az] : tot[i][az];
        } else {
          float* Yf = static_cast<float*>(a.Y);
          Yf[o] = a.accumulate ? (float)((double)Yf[o] + tot[i][az]) : (float)tot[i][az];
        }
        continue;
      }
      const size_t o = (((size_t)tx * a.n + ty) * a.n + tz) * Q3 + (ax * Q + ay) * Q + az;
      Y[o] = (a.accumulate && !to_part) ? (T)((double)Y[o] + tot[i][az]) : (T)tot[i][az];
    }
  }
}

// Y (+)= sum_g partial[g], groups in order, in the operand type.
template <class T>
__global__ void k_reduce(const T* __restrict__ part, int groups, int64_t n, T* __restrict__ Y,
                         int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = accumulate ? Y[i] : (T)0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * n + i];
  Y[i] = s;
}

template <int Q, int TPT, int GMAX, class T>
hipError_t launch_q(const ToepArgs& a, hipStream_t st) {
  constexpr int R = Q * Q;
  constexpr int G = (kThreads / R) < GMAX ? (kThreads / R) : GMAX;
  constexpr int TT = G * TPT;
  constexpr int SY = Q == 8 ? 24 : 2 * Q - 1;
  static_assert(((2 * Q - 1) * SY * (2 * Q - 1) + TT * Q * Q * Q) * sizeof(T) <= 65536,
                "LDS budget");
  const int nk = a.n / a.m;
  const int ntarg = nk * nk * nk;
  dim3 grid((ntarg + TT - 1) / TT, a.m * a.m * a.m, a.groups);
  hipLaunchKernelGGL((k_toeplitz<Q, TPT, GMAX, T>), grid, dim3(kThreads), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.groups <= 1) return e;
  const int64_t n = (int64_t)a.n * a.n * a.n * Q * Q * Q;
  hipLaunchKernelGGL((k_reduce<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     static_cast<const T*>(a.partial), a.groups, n, static_cast<T*>(a.Y),
                     a.accumulate);
  return hipGetLastError();
}

template <int Q, int TPT, int GMAX, class T>
int workgroups_q(int n, int m) {
  constexpr int R = Q * Q;
  constexpr int G = (kThreads / R) < GMAX ? (kThreads / R) : GMAX;
  constexpr int TT = G * TPT;
  const int nk = n / m;
  return ((nk * nk * nk + TT - 1) / TT) * m * m * m;
}

template <int Q>
int workgroups_q2(int fp64, int n, int m) {
  if (fp64) return workgroups_q<Q, 1, (Q >= 10 ? 1 : 4), double>(n, m);
  return workgroups_q<Q, 2, 256, float>(n, m);
}

template <int Q>
hipError_t launch_q2(const ToepArgs& a, hipStream_t st) {
  if (a.fp64) return launch_q<Q, 1, (Q >= 10 ? 1 : 4), double>(a, st);
  return launch_q<Q, 2, 256, float>(a, st);
}

}  // namespace

int toeplitz_workgroups(int q, int fp64, int n, int m) {
  switch (q) {
    case 1: return workgroups_q2<1>(fp64, n, m);
    case 2: return workgroups_q2<2>(fp64, n, m);
    case 3: return workgroups_q2<3>(fp64, n, m);
    case 4: return workgroups_q2<4>(fp64, n, m);
    case 5: return workgroups_q2<5>(fp64, n, m);
    case 6: return workgroups_q2<6>(fp64, n, m);
    case 7: return workgroups_q2<7>(fp64, n, m);
    case 8: return workgroups_q2<8>(fp64, n, m);
    case 9: return workgroups_q2<9>(fp64, n, m);
    case 10: return workgroups_q2<10>(fp64, n, m);
    default: return 0;
  }
}

hipError_t launch_toeplitz(const ToepArgs& a, hipStream_t st) {
  if (a.mesh64 && !a.fp64) return hipErrorInvalidValue;  // an FP64 mesh needs FP64 arithmetic
  if (a.groups < 1 || (a.groups > 1 && (a.grid_out || !a.partial))) return hipErrorInvalidValue;
  switch (a.q) {
    case 1: return launch_q2<1>(a, st);
    case 2: return launch_q2<2>(a, st);
    case 3: return launch_q2<3>(a, st);
    case 4: return launch_q2<4>(a, st);
    case 5: return launch_q2<5>(a, st);
    case 6: return launch_q2<6>(a, st);
    case 7: return launch_q2<7>(a, st);
    case 8: return launch_q2<8>(a, st);
    case 9: return launch_q2<9>(a, st);
    case 10: return launch_q2<10>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pfmm
