// Upward and downward passes of the FMM on the uniform tree (Sec. 2):
//   P2M  leaf cells -> leaf gridlet (effective masses with the same Cartesian
//        moments 0 <= n_i < p; the 1D weights are the Lagrange basis of the
//        gridlet nodes evaluated at the cell centres),
//   M2M  Eq. 5, child gridlets -> parent gridlet,
//   L2L  Eq. 7, parent local field -> child gridlets (the transposed operator,
//        i.e. Lagrange interpolation),
//   L2P  leaf gridlet -> cells (transpose of P2M); with derivative weights on
//        one axis, the gradient of the leaf's local expansion (accelerations
//        from the expansion, Sec. 3),
//   FD4  a = -grad(phi) by periodic 4th-order central differences (Sec. 3).
// Every operator is a tensor product of 1D operators and is applied as three
// successive 1D contractions on a block staged in LDS.  These stages move a
// few bytes per cell and are bound by memory traffic, not arithmetic.
//
// Gridlet buffers of a level are FP32 or FP64 (coarse levels can be kept in
// FP64: the interpolation of Eq. 7 extrapolates past the parent's outermost
// gridlet nodes, so rounding noise of a parent's field is amplified in its
// children); each kernel computes in the wider of its operand types.
#include "internal.h"

namespace pfmm {
namespace {

constexpr int kThreads = 256;

template <class W> __device__ inline const W* wsel(Weights w);
template <> __device__ inline const float* wsel<float>(Weights w) { return w.f; }
template <> __device__ inline const double* wsel<double>(Weights w) { return w.d; }

// S, P: leaf width and gridlet size fixed at compile time (0: the arguments),
// so that the index arithmetic folds and the contraction loops unroll.
template <class TO, class W, int S = 0, int P = 0, class TR = float>
__global__ __launch_bounds__(kThreads) void k_p2m(const TR* __restrict__ rho,
                                                   TO* __restrict__ M, Weights Aw, int N, int s_,
                                                   int p_, W h3) {
  const int s = S ? S : s_, p = P ? P : p_;
  // LDS rows of the weights and of the cell block padded by one word, so
  // that lanes reading different rows at one column hit different banks
  const int sp = s + 1;
  // compile-time rows of FP32 cells, one per thread: each thread contracts
  // its own row along z from registers, and the cell block never goes
  // through LDS (a third of the LDS, so more leaves per CU)
  constexpr bool kRowRegs = S % 4 == 0 && S > 0 && P > 0 && S * S <= kThreads &&
                            sizeof(TR) == 4;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sm = reinterpret_cast<W*>(smraw);
  W* sA = sm;               // [p][s + 1]
  W* sr = sA + p * sp;      // [s][s][s + 1] (not with rows in registers)
  W* t1 = kRowRegs ? sr : sr + s * s * sp;  // [cx][cy][az]
  W* t2 = t1 + s * s * p;   // [cx][ay][az]
  const W* A = wsel<W>(Aw);
  const int nL = N / s;
  const int b = (int)xcd_leaf(blockIdx.x, (int64_t)nL * nL * nL);
  const int bx = b / (nL * nL), by = (b / nL) % nL, bz = b % nL;
  const int tid = threadIdx.x;
  if constexpr (kRowRegs) {
    float4 rowv[S / 4];
    if (tid < S * S) {
      const int cx = tid / S, cy = tid % S;
      const float4* src = reinterpret_cast<const float4*>(
          rho + ((size_t)(bx * S + cx) * N + (by * S + cy)) * N + (size_t)bz * S);
#pragma unroll
      for (int q = 0; q < S / 4; ++q) rowv[q] = src[q];
    }
    for (int i = tid; i < P * S; i += kThreads) sA[(i / S) * sp + i % S] = A[i];
    __syncthreads();
    if (tid < S * S) {
#pragma unroll
      for (int az = 0; az < P; ++az) {
        const W* w = sA + az * sp;
        W acc = 0;
#pragma unroll
        for (int q = 0; q < S / 4; ++q)
          acc += w[4 * q] * (W)rowv[q].x + w[4 * q + 1] * (W)rowv[q].y +
                 w[4 * q + 2] * (W)rowv[q].z + w[4 * q + 3] * (W)rowv[q].w;
        t1[tid * P + az] = acc;
      }
    }
    __syncthreads();
  } else {
    for (int i = tid; i < p * s; i += kThreads) sA[(i / s) * sp + i % s] = A[i];
    if constexpr (S % 4 == 0 && S > 0) {  // rows of s cells as float4 (16-byte aligned: s | N)
      for (int i = tid; i < s * s * (s / 4); i += kThreads) {
        const int row = i / (s / 4), q = i % (s / 4);
        const int cx = row / s, cy = row % s;
        const TR* src = rho + ((size_t)(bx * s + cx) * N + (by * s + cy)) * N + (size_t)bz * s + 4 * q;
        W* dst = sr + row * sp + 4 * q;
        if constexpr (sizeof(TR) == 4) {
          const float4 v = *reinterpret_cast<const float4*>(src);
          dst[0] = (W)v.x;
          dst[1] = (W)v.y;
          dst[2] = (W)v.z;
          dst[3] = (W)v.w;
        } else {
          for (int c = 0; c < 4; ++c) dst[c] = (W)src[c];
        }
      }
    } else {
      for (int i = tid; i < s * s * s; i += kThreads) {
        const int cx = i / (s * s), cy = (i / s) % s, cz = i % s;
        sr[(cx * s + cy) * sp + cz] = (W)rho[((size_t)(bx * s + cx) * N + (by * s + cy)) * N + (bz * s + cz)];
      }
    }
    __syncthreads();
    for (int i = tid; i < s * s * p; i += kThreads) {
      const int cxy = i / p, az = i % p;
      W acc = 0;
      for (int cz = 0; cz < s; ++cz) acc += sA[az * sp + cz] * sr[cxy * sp + cz];
      t1[i] = acc;
    }
    __syncthreads();
  }
  for (int i = tid; i < s * p * p; i += kThreads) {
    const int cx = i / (p * p), ay = (i / p) % p, az = i % p;
    W acc = 0;
    for (int cy = 0; cy < s; ++cy) acc += sA[ay * sp + cy] * t1[(cx * s + cy) * p + az];
    t2[i] = acc;
  }
  __syncthreads();
  const int p3 = p * p * p;
  for (int i = tid; i < p3; i += kThreads) {
    const int ax = i / (p * p), ayz = i % (p * p);
    W acc = 0;
    for (int cx = 0; cx < s; ++cx) acc += sA[ax * sp + cx] * t2[cx * p * p + ayz];
    M[(size_t)b * p3 + i] = (TO)(h3 * acc);
  }
}

template <class TI, class TO, class W, int PP = 0>
__global__ __launch_bounds__(kThreads) void k_m2m(const TI* __restrict__ Mc,
                                                   TO* __restrict__ Mp, Weights Tw, int np,
                                                   int p_) {
  const int p = PP ? PP : p_;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sm = reinterpret_cast<W*>(smraw);
  const int p3 = p * p * p;
  W* sT = sm;  // [o][a][a']
  W* c = sT + 2 * p * p;
  W* u1 = c + p3;
  W* u2 = u1 + p3;
  const W* T = wsel<W>(Tw);
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * p * p; i += kThreads) sT[i] = T[i];
  const int B = blockIdx.x;
  const int Bx = B / (np * np), By = (B / np) % np, Bz = B % np;
  const int nc = 2 * np;
  W acc[4] = {0, 0, 0, 0};  // p^3 <= 1000 <= 4 * kThreads
  for (int o = 0; o < 8; ++o) {
    const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
    const size_t child = ((size_t)(2 * Bx + ox) * nc + (2 * By + oy)) * nc + (2 * Bz + oz);
    __syncthreads();
    for (int i = tid; i < p3; i += kThreads) c[i] = (W)Mc[child * p3 + i];
    __syncthreads();
    const W* Tz = sT + oz * p * p;
    const W* Ty = sT + oy * p * p;
    const W* Tx = sT + ox * p * p;
    for (int i = tid; i < p3; i += kThreads) {  // u1[a'x][a'y][az]
      const int xy = i / p, az = i % p;
      W v = 0;
      for (int k = 0; k < p; ++k) v += Tz[az * p + k] * c[xy * p + k];
      u1[i] = v;
    }
    __syncthreads();
    for (int i = tid; i < p3; i += kThreads) {  // u2[a'x][ay][az]
      const int x = i / (p * p), ay = (i / p) % p, az = i % p;
      W v = 0;
      for (int k = 0; k < p; ++k) v += Ty[ay * p + k] * u1[(x * p + k) * p + az];
      u2[i] = v;
    }
    __syncthreads();
    for (int i = tid, r = 0; i < p3; i += kThreads, ++r) {  // out[ax][ay][az]
      const int ax = i / (p * p), yz = i % (p * p);
      W v = 0;
      for (int k = 0; k < p; ++k) v += Tx[ax * p + k] * u2[k * p * p + yz];
      acc[r] += v;
    }
  }
  for (int i = tid, r = 0; i < p3; i += kThreads, ++r) Mp[(size_t)B * p3 + i] = (TO)acc[r];
}

template <class TI, class TO, class W, int PP = 0>
__global__ __launch_bounds__(kThreads) void k_l2l(const TI* __restrict__ Pp,
                                                   TO* __restrict__ Pc, Weights Tw, int np,
                                                   int p_, int accumulate) {
  const int p = PP ? PP : p_;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sm = reinterpret_cast<W*>(smraw);
  const int p3 = p * p * p;
  W* sT = sm;
  W* par = sT + 2 * p * p;
  W* v1 = par + p3;
  W* v2 = v1 + p3;
  const W* T = wsel<W>(Tw);
  const int tid = threadIdx.x;
  const int B = blockIdx.x;
  const int Bx = B / (np * np), By = (B / np) % np, Bz = B % np;
  const int nc = 2 * np;
  for (int i = tid; i < 2 * p * p; i += kThreads) sT[i] = T[i];
  for (int i = tid; i < p3; i += kThreads) par[i] = (W)Pp[(size_t)B * p3 + i];
  for (int o = 0; o < 8; ++o) {
    const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
    const W* Tz = sT + oz * p * p;
    const W* Ty = sT + oy * p * p;
    const W* Tx = sT + ox * p * p;
    __syncthreads();
    for (int i = tid; i < p3; i += kThreads) {  // v1[ax][ay][a'z] = sum_az Tz[az][a'z] par
      const int xy = i / p, bz = i % p;
      W v = 0;
      for (int k = 0; k < p; ++k) v += Tz[k * p + bz] * par[xy * p + k];
      v1[i] = v;
    }
    __syncthreads();
    for (int i = tid; i < p3; i += kThreads) {  // v2[ax][a'y][a'z]
      const int x = i / (p * p), by = (i / p) % p, bz = i % p;
      W v = 0;
      for (int k = 0; k < p; ++k) v += Ty[k * p + by] * v1[(x * p + k) * p + bz];
      v2[i] = v;
    }
    __syncthreads();
    const size_t child = ((size_t)(2 * Bx + ox) * nc + (2 * By + oy)) * nc + (2 * Bz + oz);
    for (int i = tid; i < p3; i += kThreads) {  // out[a'x][a'y][a'z]
      const int bx = i / (p * p), yz = i % (p * p);
      W v = 0;
      for (int k = 0; k < p; ++k) v += Tx[k * p + bx] * v2[k * p * p + yz];
      Pc[child * p3 + i] = accumulate ? (TO)((W)Pc[child * p3 + i] + v) : (TO)v;
    }
  }
}

// M2M and L2L with the gridlet size fixed at compile time, the eight
// children in one pass per axis instead of one child after another.  The
// child operators are T_o = T_ox (x) T_oy (x) T_oz with two 1D matrices
// T_0, T_1, so along each axis the two children of a pair share the pass:
// M2M contracts x over (ox, kx) for the four (oy, oz), then y over (oy, ky)
// for the two oz, then z over (oz, kz) (14 p^4 multiply-adds against
// 24 p^4 child by child, three barriers against 32); L2L expands x into the
// two ox, y into four (ox, oy), z into the eight children.
template <class TI, class TO, class W, int P>
__global__ __launch_bounds__(kThreads) void k_m2m_pairs(const TI* __restrict__ Mc,
                                                         TO* __restrict__ Mp, Weights Tw, int np) {
  constexpr int P2 = P * P, P3 = P2 * P;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sT = reinterpret_cast<W*>(smraw);  // [o][a][k]
  W* sTt = sT + 2 * P2;                 // [o][k][a]
  W* c = sTt + 2 * P2;                  // children [ox][oy][oz][kx][ky][kz]
  W* w = c + 8 * P3;                    // [oy][oz][ax][ky][kz]
  W* v = c;                             // [oz][ax][ay][kz], over the children
  const W* T = wsel<W>(Tw);
  const int tid = threadIdx.x;
  for (int i = tid; i < 2 * P2; i += kThreads) {
    const int o = i / P2, a = (i / P) % P, k = i % P;
    sT[i] = T[i];
    sTt[(o * P + k) * P + a] = T[i];
  }
  const int B = blockIdx.x;
  const int Bx = B / (np * np), By = (B / np) % np, Bz = B % np;
  const int nc = 2 * np;
  for (int i = tid; i < 8 * P3; i += kThreads) {
    const int o = i / P3;
    const size_t child = ((size_t)(2 * Bx + (o >> 2)) * nc + (2 * By + ((o >> 1) & 1))) * nc +
                         (2 * Bz + (o & 1));
    c[i] = (W)Mc[child * P3 + i % P3];
  }
  __syncthreads();
  for (int i = tid; i < 4 * P3; i += kThreads) {
    const int q = i / P3, ax = (i / P2) % P, kyz = i % P2;
    W acc = 0;
#pragma unroll
    for (int ox = 0; ox < 2; ++ox)
#pragma unroll
      for (int kx = 0; kx < P; ++kx)
        acc += sT[(ox * P + ax) * P + kx] * c[((ox * 4 + q) * P + kx) * P2 + kyz];
    w[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < 2 * P3; i += kThreads) {
    const int oz = i / P3, ax = (i / P2) % P, ay = (i / P) % P, kz = i % P;
    W acc = 0;
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ky = 0; ky < P; ++ky)
        acc += sT[(oy * P + ay) * P + ky] * w[(oy * 2 + oz) * P3 + (ax * P + ky) * P + kz];
    v[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < P3; i += kThreads) {
    const int axy = i / P, az = i % P;
    W acc = 0;
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
      for (int kz = 0; kz < P; ++kz) acc += sTt[(oz * P + kz) * P + az] * v[oz * P3 + axy * P + kz];
    Mp[(size_t)B * P3 + i] = (TO)acc;
  }
}

template <class TI, class TO, class W, int P>
__global__ __launch_bounds__(kThreads) void k_l2l_pairs(const TI* __restrict__ Pp,
                                                         TO* __restrict__ Pc, Weights Tw, int np,
                                                         int accumulate) {
  constexpr int P2 = P * P, P3 = P2 * P;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sT = reinterpret_cast<W*>(smraw);  // [o][a][b]: child node b from parent node a
  W* par = sT + 2 * P2;                 // [ax][ay][az]
  W* w = par + P3;                      // [ox][bx][ay][az]
  W* v = w + 2 * P3;                    // [ox][oy][bx][by][az]
  const W* T = wsel<W>(Tw);
  const int tid = threadIdx.x;
  const int B = blockIdx.x;
  const int Bx = B / (np * np), By = (B / np) % np, Bz = B % np;
  const int nc = 2 * np;
  for (int i = tid; i < 2 * P2; i += kThreads) sT[i] = T[i];
  for (int i = tid; i < P3; i += kThreads) par[i] = (W)Pp[(size_t)B * P3 + i];
  __syncthreads();
  for (int i = tid; i < 2 * P3; i += kThreads) {
    const int ox = i / P3, bx = (i / P2) % P, ayz = i % P2;
    W acc = 0;
#pragma unroll
    for (int ax = 0; ax < P; ++ax) acc += sT[(ox * P + ax) * P + bx] * par[ax * P2 + ayz];
    w[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < 4 * P3; i += kThreads) {
    const int q = i / P3, bx = (i / P2) % P, by = (i / P) % P, az = i % P;
    const int ox = q >> 1, oy = q & 1;
    W acc = 0;
#pragma unroll
    for (int ay = 0; ay < P; ++ay)
      acc += sT[(oy * P + ay) * P + by] * w[ox * P3 + (bx * P + ay) * P + az];
    v[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < 8 * P3; i += kThreads) {
    const int o = i / P3, bxy = (i / P) % P2, bz = i % P;
    const int oz = o & 1;
    W acc = 0;
#pragma unroll
    for (int az = 0; az < P; ++az) acc += sT[(oz * P + az) * P + bz] * v[(o >> 1) * P3 + bxy * P + az];
    const size_t child = ((size_t)(2 * Bx + (o >> 2)) * nc + (2 * By + ((o >> 1) & 1))) * nc +
                         (2 * Bz + oz);
    TO* dst = Pc + child * P3 + i % P3;
    *dst = accumulate ? (TO)((W)*dst + acc) : (TO)acc;
  }
}

// out[b s + c] (+)= scale sum_a Wx[ax][cx] Wy[ay][cy] Wz[az][cz] P[b][a]: L2P
// with Wx = Wy = Wz = A and scale 1, or one component of the gradient of the
// leaf's local expansion with the derivative weights on that axis
template <class TI, class W, int S = 0, int PP = 0, class TP = float>
__global__ __launch_bounds__(kThreads) void k_l2p(const TI* __restrict__ P,
                                                   TP* __restrict__ phi, Weights Wxw,
                                                   Weights Wyw, Weights Wzw, W scale, int N,
                                                   int s_, int p_, int accumulate) {
  const int s = S ? S : s_, p = PP ? PP : p_;
  extern __shared__ __align__(8) unsigned char smraw[];
  W* sm = reinterpret_cast<W*>(smraw);
  const int p3 = p * p * p;
  W* sAx = sm;             // [p][s] per axis
  W* sAy = sAx + p * s;
  W* sAz = sAy + p * s;
  W* sp = sAz + p * s;     // [ax][ay][az]
  W* w1 = sp + p3;         // [ax][ay][cz]
  W* w2 = w1 + p * p * s;  // [ax][cy][cz]
  const W* Ax = wsel<W>(Wxw);
  const W* Ay = wsel<W>(Wyw);
  const W* Az = wsel<W>(Wzw);
  const int nL = N / s;
  const int b = (int)xcd_leaf(blockIdx.x, (int64_t)nL * nL * nL);
  const int bx = b / (nL * nL), by = (b / nL) % nL, bz = b % nL;
  const int tid = threadIdx.x;
  // with rows of float4 and accumulation, the mesh values this thread will
  // update are read first, so their latency overlaps the two LDS passes
  constexpr int kRows = (S % 4 == 0 && S > 0 && sizeof(TP) == 4)
                            ? (S * S * (S / 4) + kThreads - 1) / kThreads : 1;
  float4 prior[kRows];
  auto row_ptr = [&](int i) {
    const int cx = i / (s * (s / 4)), cy = (i / (s / 4)) % s, cz0 = 4 * (i % (s / 4));
    return reinterpret_cast<float4*>(phi + ((size_t)(bx * s + cx) * N + (by * s + cy)) * N +
                                     (bz * s + cz0));
  };
  if constexpr (S % 4 == 0 && S > 0 && sizeof(TP) == 4) {
    if (accumulate) {
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = tid + k * kThreads;
        if (i < s * s * (s / 4)) prior[k] = *row_ptr(i);
      }
    }
  }
  for (int i = tid; i < p * s; i += kThreads) {
    sAx[i] = Ax[i];
    sAy[i] = Ay[i];
    sAz[i] = Az[i];
  }
  for (int i = tid; i < p3; i += kThreads) sp[i] = (W)P[(size_t)b * p3 + i];
  __syncthreads();
  for (int i = tid; i < p * p * s; i += kThreads) {
    const int xy = i / s, cz = i % s;
    W v = 0;
    for (int k = 0; k < p; ++k) v += sAz[k * s + cz] * sp[xy * p + k];
    w1[i] = v;
  }
  __syncthreads();
  for (int i = tid; i < p * s * s; i += kThreads) {
    const int ax = i / (s * s), cy = (i / s) % s, cz = i % s;
    W v = 0;
    for (int k = 0; k < p; ++k) v += sAy[k * s + cy] * w1[(ax * p + k) * s + cz];
    w2[i] = v;
  }
  __syncthreads();
  if constexpr (S % 4 == 0 && S > 0 && sizeof(TP) == 4) {
    // four consecutive cells of a row per thread, read and written as float4
    // (16-byte aligned: the launcher checks the mesh pointer)
#pragma unroll
    for (int kr = 0; kr < kRows; ++kr) {
      const int i = tid + kr * kThreads;
      if (i >= s * s * (s / 4)) break;
      const int cx = i / (s * (s / 4)), cy = (i / (s / 4)) % s, cz0 = 4 * (i % (s / 4));
      W v[4] = {0, 0, 0, 0};
      for (int k = 0; k < p; ++k) {
        const W a = sAx[k * s + cx];
        const W* w = w2 + k * s * s + cy * s + cz0;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] += a * w[c];
      }
      float4 r = make_float4((float)(v[0] * scale), (float)(v[1] * scale), (float)(v[2] * scale),
                             (float)(v[3] * scale));
      if (accumulate) {
        const float4 q = prior[kr];
        r = make_float4((float)((W)q.x + v[0] * scale), (float)((W)q.y + v[1] * scale),
                        (float)((W)q.z + v[2] * scale), (float)((W)q.w + v[3] * scale));
      }
      *row_ptr(i) = r;
    }
  } else {
    for (int i = tid; i < s * s * s; i += kThreads) {
      const int cx = i / (s * s), cyz = i % (s * s);
      W v = 0;
      for (int k = 0; k < p; ++k) v += sAx[k * s + cx] * w2[k * s * s + cyz];
      v *= scale;
      const int cy = cyz / s, cz = cyz % s;
      TP* o = phi + ((size_t)(bx * s + cx) * N + (by * s + cy)) * N + (bz * s + cz);
      *o = accumulate ? (TP)((W)*o + v) : (TP)v;
    }
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_fd4(const T* __restrict__ phi,
                                                   T* __restrict__ acc, int N) {
  const size_t n3 = (size_t)N * N * N;
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n3) return;
  const int z = (int)(i % N), y = (int)((i / N) % N), x = (int)(i / ((size_t)N * N));
  const int mk = N - 1;
  const T inv12h = (T)N / (T)12;
  auto at = [&](int xx, int yy, int zz) {
    return phi[((size_t)(xx & mk) * N + (yy & mk)) * N + (zz & mk)];
  };
  const T gx = -at(x + 2, y, z) + (T)8 * at(x + 1, y, z) - (T)8 * at(x - 1, y, z) + at(x - 2, y, z);
  const T gy = -at(x, y + 2, z) + (T)8 * at(x, y + 1, z) - (T)8 * at(x, y - 1, z) + at(x, y - 2, z);
  const T gz = -at(x, y, z + 2) + (T)8 * at(x, y, z + 1) - (T)8 * at(x, y, z - 1) + at(x, y, z - 2);
  acc[i] = -gx * inv12h;
  acc[n3 + i] = -gy * inv12h;
  acc[2 * n3 + i] = -gz * inv12h;
}

__global__ void k_d2f(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

}  // namespace

// LDS words of P2M: the padded weights and cell block, and the two partial
// contractions; without the cell block for the instances that keep the
// rows in registers.
inline size_t p2m_words(int s, int p) {
  return (size_t)(p * (s + 1) + s * s * (s + 1) + s * s * p + s * p * p);
}
inline size_t p2m_words_rows(int s, int p) {
  return (size_t)(p * (s + 1) + s * s * p + s * p * p);
}

hipError_t launch_p2m(const float* rho, void* M, int m64, Weights A, int N, int s, int p,
                      double h3, hipStream_t st) {
  const int nL = N / s;
  const size_t words = p2m_words(s, p);
  if (m64)
    hipLaunchKernelGGL((k_p2m<double, double>), dim3(nL * nL * nL), dim3(kThreads),
                       words * sizeof(double), st, rho, (double*)M, A, N, s, p, h3);
  else {
    const dim3 g(nL * nL * nL), b(kThreads);
    size_t sh = words * sizeof(float);
    const float hf = (float)h3;
    // the compile-time instances read rows of cells as float4
    const bool aligned = ((uintptr_t)rho & 15) == 0;
    if (aligned && (s == 16 || s == 8) && (p == 8 || p == 4))
      sh = p2m_words_rows(s, p) * sizeof(float);
    if (!aligned)
      hipLaunchKernelGGL((k_p2m<float, float>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
    else if (s == 16 && p == 8)
      hipLaunchKernelGGL((k_p2m<float, float, 16, 8>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
    else if (s == 8 && p == 8)
      hipLaunchKernelGGL((k_p2m<float, float, 8, 8>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
    else if (s == 16 && p == 4)
      hipLaunchKernelGGL((k_p2m<float, float, 16, 4>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
    else if (s == 8 && p == 4)
      hipLaunchKernelGGL((k_p2m<float, float, 8, 4>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
    else
      hipLaunchKernelGGL((k_p2m<float, float>), g, b, sh, st, rho, (float*)M, A, N, s, p, hf);
  }
  return hipGetLastError();
}

// M2M / L2L instance with the gridlet size fixed at compile time for p = 4
// and 8 (index arithmetic folded, loops unrolled), else the generic one.
#define PFMM_BY_P(KERNEL, TI, TO, W, ...)                        \
  do {                                                            \
    if (p == 8)                                                   \
      hipLaunchKernelGGL((KERNEL<TI, TO, W, 8>), __VA_ARGS__);    \
    else if (p == 4)                                              \
      hipLaunchKernelGGL((KERNEL<TI, TO, W, 4>), __VA_ARGS__);    \
    else                                                          \
      hipLaunchKernelGGL((KERNEL<TI, TO, W>), __VA_ARGS__);       \
  } while (0)

// The pairwise kernels at p = 4, 8 (LDS words: the weights twice, eight
// children and the four x-contracted pairs).
#define PFMM_PAIRS(KERNEL, TI, TO, W, ...)                        \
  do {                                                            \
    if (p == 8)                                                   \
      hipLaunchKernelGGL((KERNEL<TI, TO, W, 8>), __VA_ARGS__);    \
    else                                                          \
      hipLaunchKernelGGL((KERNEL<TI, TO, W, 4>), __VA_ARGS__);    \
  } while (0)

hipError_t launch_m2m(const void* Mc, int c64, void* Mp, int p64, Weights T, int np, int p,
                      hipStream_t st) {
  const dim3 g(np * np * np), b(kThreads);
  if (p == 4 || p == 8) {
    const size_t pw = (size_t)(4 * p * p + 12 * p * p * p);
    if (!c64 && !p64)
      PFMM_PAIRS(k_m2m_pairs, float, float, float, g, b, pw * 4, st, (const float*)Mc, (float*)Mp, T, np);
    else if (!c64 && p64)
      PFMM_PAIRS(k_m2m_pairs, float, double, double, g, b, pw * 8, st, (const float*)Mc, (double*)Mp, T, np);
    else if (c64 && p64)
      PFMM_PAIRS(k_m2m_pairs, double, double, double, g, b, pw * 8, st, (const double*)Mc, (double*)Mp, T,
                 np);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  const size_t words = (size_t)(2 * p * p + 3 * p * p * p);
  if (!c64 && !p64)
    PFMM_BY_P(k_m2m, float, float, float, g, b, words * 4, st, (const float*)Mc, (float*)Mp, T, np, p);
  else if (!c64 && p64)
    PFMM_BY_P(k_m2m, float, double, double, g, b, words * 8, st, (const float*)Mc, (double*)Mp, T, np, p);
  else if (c64 && p64)
    PFMM_BY_P(k_m2m, double, double, double, g, b, words * 8, st, (const double*)Mc, (double*)Mp, T,
              np, p);
  else
    return hipErrorInvalidValue;  // a finer level is never wider than its parent
  return hipGetLastError();
}

hipError_t launch_l2l(const void* Pp, int p64, void* Pc, int c64, Weights T, int np, int p,
                      hipStream_t st, int accumulate) {
  const dim3 g(np * np * np), b(kThreads);
  if (p == 4 || p == 8) {
    const size_t pw = (size_t)(2 * p * p + 7 * p * p * p);
    if (!p64 && !c64)
      PFMM_PAIRS(k_l2l_pairs, float, float, float, g, b, pw * 4, st, (const float*)Pp, (float*)Pc, T, np,
                 accumulate);
    else if (p64 && !c64)
      PFMM_PAIRS(k_l2l_pairs, double, float, double, g, b, pw * 8, st, (const double*)Pp, (float*)Pc, T,
                 np, accumulate);
    else if (p64 && c64)
      PFMM_PAIRS(k_l2l_pairs, double, double, double, g, b, pw * 8, st, (const double*)Pp, (double*)Pc,
                 T, np, accumulate);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  const size_t words = (size_t)(2 * p * p + 3 * p * p * p);
  if (!p64 && !c64)
    PFMM_BY_P(k_l2l, float, float, float, g, b, words * 4, st, (const float*)Pp, (float*)Pc, T, np, p,
              accumulate);
  else if (p64 && !c64)
    PFMM_BY_P(k_l2l, double, float, double, g, b, words * 8, st, (const double*)Pp, (float*)Pc, T, np,
              p, accumulate);
  else if (p64 && c64)
    PFMM_BY_P(k_l2l, double, double, double, g, b, words * 8, st, (const double*)Pp, (double*)Pc, T,
              np, p, accumulate);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
#undef PFMM_BY_P
#undef PFMM_PAIRS

namespace {
hipError_t l2p_axes(const void* P, int p64, float* out, Weights Wx, Weights Wy, Weights Wz,
                    double scale, int N, int s, int p, hipStream_t st, int accumulate) {
  const int nL = N / s;
  const size_t words = (size_t)(3 * p * s + p * p * p + p * p * s + p * s * s);
  if (p64)
    hipLaunchKernelGGL((k_l2p<double, double>), dim3(nL * nL * nL), dim3(kThreads),
                       words * sizeof(double), st, (const double*)P, out, Wx, Wy, Wz, scale, N, s,
                       p, accumulate);
  else {
    const dim3 g(nL * nL * nL), b(kThreads);
    const size_t sh = words * sizeof(float);
    const float sc = (float)scale;
    const float* Pf = (const float*)P;
    if (((uintptr_t)out & 15) != 0)  // the compile-time instances write float4
      hipLaunchKernelGGL((k_l2p<float, float>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
    else if (s == 16 && p == 8)
      hipLaunchKernelGGL((k_l2p<float, float, 16, 8>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
    else if (s == 8 && p == 8)
      hipLaunchKernelGGL((k_l2p<float, float, 8, 8>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
    else if (s == 16 && p == 4)
      hipLaunchKernelGGL((k_l2p<float, float, 16, 4>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
    else if (s == 8 && p == 4)
      hipLaunchKernelGGL((k_l2p<float, float, 8, 4>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
    else
      hipLaunchKernelGGL((k_l2p<float, float>), g, b, sh, st, Pf, out, Wx, Wy, Wz, sc, N, s, p, accumulate);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_l2p(const void* P, int p64, float* phi, Weights A, int N, int s, int p,
                      hipStream_t st, int accumulate) {
  return l2p_axes(P, p64, phi, A, A, A, 1.0, N, s, p, st, accumulate);
}

hipError_t launch_l2p_grad(const void* P, int p64, float* acc, Weights A, Weights Ad,
                           double scale, int N, int s, int p, hipStream_t st) {
  const size_t n3 = (size_t)N * N * N;
  for (int c = 0; c < 3; ++c) {
    const hipError_t e = l2p_axes(P, p64, acc + c * n3, c == 0 ? Ad : A, c == 1 ? Ad : A,
                                  c == 2 ? Ad : A, scale, N, s, p, st, 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fd4(const float* phi, float* acc, int N, hipStream_t st) {
  const size_t n3 = (size_t)N * N * N;
  hipLaunchKernelGGL(k_fd4<float>, dim3((unsigned)((n3 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     st, phi, acc, N);
  return hipGetLastError();
}

hipError_t launch_fd4_f64(const double* phi, double* acc, int N, hipStream_t st) {
  const size_t n3 = (size_t)N * N * N;
  hipLaunchKernelGGL(k_fd4<double>, dim3((unsigned)((n3 + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, st, phi, acc, N);
  return hipGetLastError();
}

hipError_t launch_p2m_f64in(const double* rho, void* M, Weights A, int N, int s, int p, double h3,
                            hipStream_t st) {
  const int nL = N / s;
  const size_t words = p2m_words(s, p);
  hipLaunchKernelGGL((k_p2m<double, double, 0, 0, double>), dim3(nL * nL * nL), dim3(kThreads),
                     words * sizeof(double), st, rho, (double*)M, A, N, s, p, h3);
  return hipGetLastError();
}

namespace {
hipError_t l2p_axes_f64out(const void* P, double* out, Weights Wx, Weights Wy, Weights Wz,
                           double scale, int N, int s, int p, hipStream_t st, int accumulate) {
  const int nL = N / s;
  const size_t words = (size_t)(3 * p * s + p * p * p + p * p * s + p * s * s);
  hipLaunchKernelGGL((k_l2p<double, double, 0, 0, double>), dim3(nL * nL * nL), dim3(kThreads),
                     words * sizeof(double), st, (const double*)P, out, Wx, Wy, Wz, scale, N, s, p,
                     accumulate);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_l2p_f64out(const void* P, double* phi, Weights A, int N, int s, int p,
                             hipStream_t st, int accumulate) {
  return l2p_axes_f64out(P, phi, A, A, A, 1.0, N, s, p, st, accumulate);
}

hipError_t launch_l2p_grad_f64out(const void* P, double* acc, Weights A, Weights Ad, double scale,
                                  int N, int s, int p, hipStream_t st) {
  const size_t n3 = (size_t)N * N * N;
  for (int c = 0; c < 3; ++c) {
    const hipError_t e = l2p_axes_f64out(P, acc + c * n3, c == 0 ? Ad : A, c == 1 ? Ad : A,
                                         c == 2 ? Ad : A, scale, N, s, p, st, 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cast_d2f(const double* src, float* dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_d2f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace pfmm
