// Persistent block-Toeplitz kernel for batches of independent fields.
//
// For a batch, every interaction-zone level of every field writes its own
// gridlet-potential buffer and every near zone writes its mesh: these
// contractions depend only on the upward pass and the density, not on each
// other (Sec. 2: the three parts of a target's potential are summed after
// the fact, the parent part by Eq. 7).  They are therefore one pool of
// independent work items (field, level or near zone, class, tile of
// targets), drained by a grid of resident workgroups through an atomic
// counter, largest items first.  No workgroup ever waits on another.
//
// An item applies  Y[t] = sum_{d in D(class)} tab[a - a' - q d] X[(t+d) mod n]
// to a tile of targets; the block edge q (1..8) and the tile width (targets
// per thread, TPT = 1, 2 or 4, chosen by timing per group of items) are fields
// of the item.
// Items of FP32 levels sum each offset's contribution in FP32 and add it to an
// FP64 running total, as in the single-field portable kernel; items of the
// FP64 coarse levels run the same body in FP64 with one target per thread.
#include "internal.h"

namespace pfmm {
namespace {

constexpr int kThreads = 256;

__device__ inline void unpack_offset(int pk, int& dx, int& dy, int& dz) {
  dx = ((pk >> 16) & 255) - 128;
  dy = ((pk >> 8) & 255) - 128;
  dz = (pk & 255) - 128;
}

template <int Q, int TPT, class T>
__device__ __forceinline__ void item_body(const BatchItem& it, T* sl, T* xs) {
  constexpr int R = Q * Q;
  constexpr int Q3 = Q * Q * Q;
  constexpr int S = 2 * Q - 1;
  constexpr int SY = Q == 8 ? 24 : S;  // padded slice rows per x plane (bank spread)
  constexpr int G = kThreads / R;
  constexpr int TT = G * TPT;
  const int tid = threadIdx.x;
  const int m = it.m;
  const int cx = it.cls / (m * m), cy = (it.cls / m) % m, cz = it.cls % m;
  const int nk = it.n / m;
  const int ntarg = nk * nk * nk;
  const int E = 2 * it.C + 1;
  const int nmask = it.n - 1;
  const int* offs = it.offs + (size_t)it.cls * it.noff;
  const size_t NN = (size_t)it.n * Q;
  const int grp = tid / R, row = tid % R;
  const bool active = grp < G;
  const int ax = row / Q, ay = row % Q;

  double tot[TPT][Q];
#pragma unroll
  for (int i = 0; i < TPT; ++i)
#pragma unroll
    for (int j = 0; j < Q; ++j) tot[i][j] = 0.0;

  for (int k = 0; k < it.noff; ++k) {
    int dx, dy, dz;
    unpack_offset(offs[k], dx, dy, dz);
    __syncthreads();
    for (int i = tid; i < S * S * S; i += kThreads) {
      const int jx = i / (S * S), jy = (i / S) % S, jz = i % S;
      const int li = (jx * SY + jy) * S + jz;  // padded slice position
      const int ix = -Q * dx + jx - (Q - 1) + it.C;
      const int iy = -Q * dy + jy - (Q - 1) + it.C;
      const int iz = -Q * dz + jz - (Q - 1) + it.C;
      sl[li] = static_cast<const T*>(it.tab)[((size_t)ix * E + iy) * E + iz];
    }
    for (int i = tid; i < TT * Q3; i += kThreads) {
      const int tl = i / Q3, e = i % Q3;
      const int t = it.t0 + tl;
      T v = 0;
      if (t < ntarg) {
        const int kx = t / (nk * nk), ky = (t / nk) % nk, kz = t % nk;
        const int ux = (cx + m * kx + dx) & nmask;
        const int uy = (cy + m * ky + dy) & nmask;
        const int uz = (cz + m * kz + dz) & nmask;
        size_t src;
        if (it.grid) {
          const int ex = e / (Q * Q), ey = (e / Q) % Q, ez = e % Q;
          src = ((size_t)(ux * Q + ex) * NN + (uy * Q + ey)) * NN + (uz * Q + ez);
        } else {
          src = (((size_t)ux * it.n + uy) * it.n + uz) * Q3 + e;
        }
        v = static_cast<const T*>(it.X)[src] * (T)it.xscale;
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
  if (active) {
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      const int t = it.t0 + grp * TPT + i;
      if (t >= ntarg) continue;
      const int kx = t / (nk * nk), ky = (t / nk) % nk, kz = t % nk;
      const int tx = cx + m * kx, ty = cy + m * ky, tz = cz + m * kz;
#pragma unroll
      for (int az = 0; az < Q; ++az) {
        size_t o;
        if (it.grid)
          o = ((size_t)(tx * Q + ax) * NN + (ty * Q + ay)) * NN + (tz * Q + az);
        else
          o = (((size_t)tx * it.n + ty) * it.n + tz) * Q3 + (ax * Q + ay) * Q + az;
        static_cast<T*>(it.Y)[o] = (T)tot[i][az];
      }
    }
  }
  __syncthreads();  // the LDS staging is reused by the next item
}

// LDS bytes for the largest block edge (8): slice + targets of a tile, for
// FP32 items with tile width TPT and FP64 items with tile width 1
template <int TPT>
struct BatchLds {
  static constexpr int kSlice = 15 * 24 * 15;  // padded slice of q = 8
  static constexpr int kF32 = (kSlice + (kThreads / 64) * TPT * 512) * 4;
  static constexpr int kF64 = (kSlice + (kThreads / 64) * 512) * 8;
  static constexpr int kBytes = kF32 > kF64 ? kF32 : kF64;
};

template <int TPT>
__device__ __forceinline__ void run_f32(const BatchItem& it, float* slf, float* xsf) {
  switch (it.q) {
    case 1: item_body<1, TPT, float>(it, slf, xsf); break;
    case 2: item_body<2, TPT, float>(it, slf, xsf); break;
    case 3: item_body<3, TPT, float>(it, slf, xsf); break;
    case 4: item_body<4, TPT, float>(it, slf, xsf); break;
    case 5: item_body<5, TPT, float>(it, slf, xsf); break;
    case 6: item_body<6, TPT, float>(it, slf, xsf); break;
    case 7: item_body<7, TPT, float>(it, slf, xsf); break;
    case 8: item_body<8, TPT, float>(it, slf, xsf); break;
    default: break;
  }
}

__global__ __launch_bounds__(kThreads, 2) void k_batch_toeplitz(const BatchItem* __restrict__ items,
                                                             int nitems,
                                                             unsigned* __restrict__ counter) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[BatchLds<4>::kBytes];
  __shared__ int cur;
  float* slf = reinterpret_cast<float*>(lds);
  float* xsf = slf + BatchLds<4>::kSlice;
  double* sld = reinterpret_cast<double*>(lds);
  double* xsd = sld + BatchLds<4>::kSlice;
  for (;;) {
    if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int idx = cur;
    __syncthreads();  // every thread has read `cur` before thread 0 overwrites it
    if (idx >= nitems) break;  // uniform: the whole workgroup leaves together
    const BatchItem it = items[idx];
    if (it.fp64) {
      switch (it.q) {
        case 1: item_body<1, 1, double>(it, sld, xsd); break;
        case 2: item_body<2, 1, double>(it, sld, xsd); break;
        case 3: item_body<3, 1, double>(it, sld, xsd); break;
        case 4: item_body<4, 1, double>(it, sld, xsd); break;
        case 5: item_body<5, 1, double>(it, sld, xsd); break;
        case 6: item_body<6, 1, double>(it, sld, xsd); break;
        case 7: item_body<7, 1, double>(it, sld, xsd); break;
        case 8: item_body<8, 1, double>(it, sld, xsd); break;
        default: break;
      }
    } else if (it.tpt == 4) {
      run_f32<4>(it, slf, xsf);
    } else if (it.tpt == 2) {
      run_f32<2>(it, slf, xsf);
    } else {
      run_f32<1>(it, slf, xsf);
    }
  }
}

__global__ void k_reset_counter(unsigned* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

int resident_grid() {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_toeplitz, kThreads, 0) !=
      hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

}  // namespace

int batch_targets_per_item(int q, int tpt, int fp64) {
  return (kThreads / (q * q)) * (fp64 ? 1 : tpt);
}

int batch_resident_grid() { return resident_grid(); }

hipError_t launch_batch_toeplitz(const BatchItem* items, int nitems, unsigned* counter, int grid,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grid > nitems) grid = nitems;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_toeplitz, dim3(grid), dim3(kThreads), 0, st, items, nitems, counter);
  return hipGetLastError();
}

}  // namespace pfmm
