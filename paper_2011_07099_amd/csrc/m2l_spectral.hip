// Interaction zones (Eq. 6) as spectral stencils over the nodes of a level.
//
// Target node t, source node t + d (d in the zone of t's parity class, 189
// offsets at levels >= 3; the periodic level-2 zone), gridlet points a, a':
//   Phi_l[t][a] += sum_d sum_a' G(eta_l (a - a' - p d)) M_l[t + d][a'].
// For one d this is a linear convolution of a p^3 block with the kernel
// K_d[m] = G(eta_l (m - p d)), |m_i| <= p - 1, so, as for the leaf near zone,
// it is exact as a cyclic convolution on 2p points per axis, and the zone's
// offsets add per frequency:
//   Phi_hat_t(k) = sum_{d in IZ(t)} K_hat_d(k) M_hat_{t+d}(k).
// One forward transform per node, a stencil of 189 (37 at level 2) terms per
// target and frequency, one inverse per node.  Against the block-Toeplitz
// GEMM's 2 p^6 flops per target and offset this is 8 flops per frequency
// ((2p)^2 (p + 1) of them) plus the transforms.
//
// Everything here is FP64 (transforms, kernel spectra, stencil), on the
// vector ALUs; masses are read and potentials added in the level's own
// precision.  Kernel spectra (all 343 offsets of [-3, 3]^3) are transformed
// once per table by the same separable FP64 DFT as the near zone's.
//
// Layout: spectra of a level as [frequency / 8][node][frequency % 8]: a
// node's transform writes (and its inverse reads) 128-byte runs, and the 8
// frequencies of a chunk, whose stencil workgroups run on one XCD, share
// every line of it.  In the stencil each wave handles
// one parity class, so the offset, and with it the kernel value, is the same
// across the wave.
#include "internal.h"

#include <vector>

namespace pfmm {

struct M2LSpectral {
  int L = 0, p = 0;
  int64_t F = 0;                 // (2p)^2 (p + 1) frequencies per node
  double2* spec = nullptr;       // [F][nodes] of the level being summed
  double2* out = nullptr;        // [F][nodes]
  std::vector<double2*> khat;    // per level: [343][F], offsets of [-3, 3]^3
  std::vector<double2*> khatT;   // per level: [F][kKT], the same values frequency by frequency
  float2* khatT32 = nullptr;     // the leaf level's khatT in FP32 (the FP32 16^3 stencil)
  int f32 = 0;                   // the 16^3 level's stencil in FP32 with FP64 column totals
  double2* dft[2] = {nullptr, nullptr};  // [343][F] DFT passes of the kernels
};

namespace {

constexpr int kThreads = 256;
constexpr int kKT = 344;  // kernel values per frequency in khatT (343 offsets, padded)

inline unsigned nblk(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// cos(2 pi j / 96) for j = 0 .. 24 (96 = lcm of the grid sizes 2p = 8, 12, 16)
__device__ constexpr double kQuarterD[25] = {
    1.0,                    0.997858923238603506738, 0.991444861373810411145,
    0.980785280403230449126, 0.96592582628906828675,  0.946930129495105664256,
    0.923879532511286756128, 0.896872741532688303894, 0.866025403784438646764,
    0.831469612302545237079, 0.79335334029123516458,  0.751839807478977396408,
    0.707106781186547524401, 0.659345815100068868425, 0.608761429008720639416,
    0.555570233019602224743, 0.5,                     0.442288690219001281995,
    0.382683432365089771728, 0.321439465303161580701, 0.258819045102520762349,
    0.195090322016128267848, 0.130526192220051591548, 0.0654031292301430668153,
    0.0};
__device__ __forceinline__ double cosd96(int j) {
  j %= 96;
  if (j < 0) j += 96;
  if (j <= 24) return kQuarterD[j];
  if (j <= 48) return -kQuarterD[48 - j];
  if (j <= 72) return -kQuarterD[j - 48];
  return kQuarterD[96 - j];
}

// (cos, sin) of 2 pi j / M, M | 96
template <int M>
__device__ __forceinline__ double2 twd(int j) {
  constexpr int r = 96 / M;
  return make_double2(cosd96(j * r), cosd96(j * r - 24));
}

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// a exp(-2 pi i j / P) (forward) or a exp(+2 pi i j / P) (INV)
template <int P, bool INV>
__device__ __forceinline__ double2 dtwiddle(double2 a, int j) {
  const double2 w = twd<P>(j);
  return INV ? make_double2(a.x * w.x - a.y * w.y, a.y * w.x + a.x * w.y)
             : make_double2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

template <bool INV>
__device__ __forceinline__ void ddft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 b0 = dadd(a0, a2), b1 = dsub(a0, a2), b2 = dadd(a1, a3), b3 = dsub(a1, a3);
  const double2 ib3 = make_double2(-b3.y, b3.x);
  a0 = dadd(b0, b2);
  a2 = dsub(b0, b2);
  a1 = INV ? dadd(b1, ib3) : dsub(b1, ib3);
  a3 = INV ? dsub(b1, ib3) : dadd(b1, ib3);
}

// In-place DFT of P values: P = 4Q (Q = 1, 2) by the split n = Q n1 + n2,
// m = m1 + 4 m2; P = 6 directly.
template <int P, bool INV>
__device__ __forceinline__ void ddft(double2 (&v)[P]) {
  if constexpr (P == 6) {
    double2 u[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) u[n] = v[n];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double2 acc = u[0];
#pragma unroll
      for (int n = 1; n < 6; ++n) acc = dadd(acc, dtwiddle<6, INV>(u[n], n * m));
      v[m] = acc;
    }
    return;
  }
  constexpr int Q = P / 4;
  double2 T[Q][4];
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    T[n2][0] = v[n2];
    T[n2][1] = v[Q + n2];
    T[n2][2] = v[2 * Q + n2];
    T[n2][3] = v[3 * Q + n2];
    ddft4<INV>(T[n2][0], T[n2][1], T[n2][2], T[n2][3]);
#pragma unroll
    for (int m1 = 1; m1 < 4; ++m1)
      if (n2) T[n2][m1] = dtwiddle<P, INV>(T[n2][m1], n2 * m1);
  }
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) {
    if constexpr (Q == 1) {
      v[m1] = T[0][m1];
    } else {
      v[m1] = dadd(T[0][m1], T[1][m1]);
      v[m1 + 4] = dsub(T[0][m1], T[1][m1]);
    }
  }
}

template <int P>
constexpr int node_threads() { return (P * (P + 1) + 63) / 64 * 64; }

// Node of block g: the 8 XCDs (blocks dealt round robin) take contiguous runs
// of nodes, so that the [frequency][node] writes of neighbouring nodes meet in
// one L2.
__device__ __forceinline__ int64_t xcd_node(int64_t g, int64_t nn) { return (g & 7) * (nn >> 3) + (g >> 3); }

// Spectrum element (frequency f, node) of a level with nn nodes.
__device__ __forceinline__ int64_t sidx(int f, int64_t node, int64_t nn) {
  return ((int64_t)(f >> 3) * nn + node) * 8 + (f & 7);
}

// Stencil block g: the 8 XCDs (blocks dealt round robin) take whole
// 8-frequency chunks, all of a chunk's frequencies and tiles back to back.
// The grid covers the chunks rounded up to a multiple of 8; false for the
// blocks beyond the last chunk.
__device__ __forceinline__ bool zone_block(int g, int tiles, int nchunk, int& k, int& tile) {
  const int j = g >> 3;
  const int chunk = (j / (8 * tiles)) * 8 + (g & 7);
  k = chunk * 8 + (j / tiles) % 8;
  tile = j % tiles;
  return chunk < nchunk;
}

// Forward transform of one node's p^3 gridlet (on the 2p cyclic grid, zero
// beyond p) to its half spectrum; frequency order
// ((kx * 2 + ky % 2) * p + ky / 2) * (p + 1) + kz.
// Spectra are stored as TS: double2, or float2 for the 16^3 leaf level
// summed in FP32 columns (half the bytes; its stencil rounds them to FP32
// anyway).
__device__ __forceinline__ double2 as_d2(double2 v) { return v; }
__device__ __forceinline__ double2 as_d2(float2 v) { return make_double2(v.x, v.y); }
template <class TS> __device__ __forceinline__ TS from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) {
  return make_float2((float)v.x, (float)v.y);
}

template <int P, class TIN, class TS = double2>
__global__ void __launch_bounds__(node_threads<P>()) k_node_fwd(const TIN* __restrict__ Ml, int64_t nn,
                                                                TS* __restrict__ spec) {
  constexpr int M = 2 * P, H = P + 1, NT = node_threads<P>();
  __shared__ double2 A1[P * P * H];
  __shared__ double2 A2[P * P * H];
  const int64_t node = xcd_node(blockIdx.x, nn);
  const TIN* src = Ml + node * (P * P * P);
  for (int r = threadIdx.x; r < P * P; r += NT) {
    double2 e[P], o[P];
#pragma unroll
    for (int z = 0; z < P; ++z) {
      e[z] = make_double2((double)src[r * P + z], 0.0);
      o[z] = dtwiddle<M, false>(e[z], z);
    }
    ddft<P, false>(e);
    ddft<P, false>(o);
    double2* row = A1 + r * H;
#pragma unroll
    for (int m = 0; m < P / 2; ++m) {
      row[2 * m] = e[m];
      row[2 * m + 1] = o[m];
    }
    row[P] = e[P / 2];
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    for (int r = threadIdx.x; r < P * H; r += NT) {
      const int x = r / H, kz = r % H;
      double2 u[P];
#pragma unroll
      for (int y = 0; y < P; ++y) {
        u[y] = A1[(x * P + y) * H + kz];
        if (h) u[y] = dtwiddle<M, false>(u[y], y);
      }
      ddft<P, false>(u);
#pragma unroll
      for (int m = 0; m < P; ++m) A2[(x * P + m) * H + kz] = u[m];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < P * H; r += NT) {
      const int m = r / H, kz = r % H;
      double2 e[P], o[P];
#pragma unroll
      for (int x = 0; x < P; ++x) {
        e[x] = A2[(x * P + m) * H + kz];
        o[x] = dtwiddle<M, false>(e[x], x);
      }
      ddft<P, false>(e);
      ddft<P, false>(o);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        spec[sidx((4 * j + h) * P * H + r, node, nn)] = from_d2<TS>(e[j]);
        spec[sidx((4 * j + 2 + h) * P * H + r, node, nn)] = from_d2<TS>(o[j]);
      }
    }
    __syncthreads();
  }
}

// Inverse of k_node_fwd at the p^3 gridlet points, added to (or written into)
// the node's potentials; unnormalised (the kernel spectra carry 1 / (2p)^3).
template <int P, class TOUT, class TS = double2>
__global__ void __launch_bounds__(node_threads<P>()) k_node_inv(const TS* __restrict__ spec,
                                                                int64_t nn, int accumulate,
                                                                TOUT* __restrict__ Pl) {
  constexpr int M = 2 * P, H = P + 1, NT = node_threads<P>();
  __shared__ double2 B1[P * P * H];
  __shared__ double2 B2[P * P * H];
  const int64_t node = xcd_node(blockIdx.x, nn);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    for (int r = threadIdx.x; r < P * H; r += NT) {
      const int m = r / H, kz = r % H;
      double2 e[P], o[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        e[j] = as_d2(spec[sidx((4 * j + h) * P * H + r, node, nn)]);
        o[j] = as_d2(spec[sidx((4 * j + 2 + h) * P * H + r, node, nn)]);
      }
      ddft<P, true>(e);
      ddft<P, true>(o);
#pragma unroll
      for (int x = 0; x < P; ++x) B1[(x * P + m) * H + kz] = dadd(e[x], dtwiddle<M, true>(o[x], x));
    }
    __syncthreads();
    for (int r = threadIdx.x; r < P * H; r += NT) {
      const int x = r / H, kz = r % H;
      double2 v[P];
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = B1[(x * P + m) * H + kz];
      ddft<P, true>(v);
#pragma unroll
      for (int y = 0; y < P; ++y) {
        double2& d = B2[(x * P + y) * H + kz];
        d = h ? dadd(d, dtwiddle<M, true>(v[y], y)) : v[y];
      }
    }
    __syncthreads();
  }
  TOUT* dst = Pl + node * (P * P * P);
  for (int r = threadIdx.x; r < P * P; r += NT) {
    double2 u[H];
#pragma unroll
    for (int k = 0; k < H; ++k) u[k] = B2[r * H + k];
#pragma unroll
    for (int z = 0; z < P; ++z) {
      double b = 0.0;
#pragma unroll
      for (int k = 1; k < P; ++k) {
        const double2 w = twd<M>(k * z);
        b += u[k].x * w.x - u[k].y * w.y;
      }
      const double v = u[0].x + ((z & 1) ? -u[P].x : u[P].x) + 2.0 * b;
      dst[r * P + z] = accumulate ? (TOUT)((double)dst[r * P + z] + v) : (TOUT)v;
    }
  }
}

// (re, im) += k s, one complex multiply-add as four FMAs
__device__ __forceinline__ void cmac(double& re, double& im, double2 k, double2 s) {
  re = fma(k.x, s.x, re);
  re = fma(-k.y, s.y, re);
  im = fma(k.x, s.y, im);
  im = fma(k.y, s.x, im);
}
__device__ __forceinline__ void cmac(float& re, float& im, float2 k, float2 s) {
  re = fmaf(k.x, s.x, re);
  re = fmaf(-k.y, s.y, re);
  im = fmaf(k.x, s.y, im);
  im = fmaf(k.y, s.x, im);
}

// A wave-uniform FP32 value copied into a vector register, so that the
// multiply-adds that use it take the two-operand form with all operands in
// vector registers, which gfx950 issues at twice the rate of the forms with
// a scalar operand or a negation modifier.
__device__ __forceinline__ float vreg(float x) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// out_t(k) = sum_{d in zone(class of t)} khat_d(k) spec_{t+d}(k) for one
// frequency k and one tile of T^3 targets; T = 8, or T = n = 4 on the 4^3
// level (one class).  Blocks are dealt to the 8 XCDs round robin; block g
// takes frequency 8 (g / 8 / tiles) + g % 8 and tile (g / 8) % tiles, so each
// XCD runs all tiles of a frequency back to back and their overlapping halos
// come from its L2.  The tile's source spectra with a
// 3-node halo are staged in LDS (wrapped, or zero outside an isolated box).
// Wave w handles the targets of class w (levels >= 3), so the offset list,
// and the kernel value at k, is uniform across the wave.
__global__ void __launch_bounds__(512) k_zone_spec(const double2* __restrict__ spec,
                                                   const double2* __restrict__ khat,
                                                   const int* __restrict__ offs, int noff, int n,
                                                   int classes, int isolated, int64_t F,
                                                   double2* __restrict__ out) {
  __shared__ double2 box[14 * 14 * 14];
  __shared__ double2 kk[343];        // this frequency's kernel values, all offsets of [-3, 3]^3
  __shared__ int sof[8 * 316];       // the zone's offsets per class, as box steps and kernel index
  const int T = n < 8 ? n : 8;
  const int B = T + 6;
  const int Bh = B / 2, H3 = Bh * Bh * Bh;  // parity-split box
  const int64_t nn = (int64_t)n * n * n;
  const int tpa = n / T;  // tiles per axis
  const int tiles = tpa * tpa * tpa;
  int k, tile;
  if (!zone_block(blockIdx.x, tiles, (int)(F >> 3), k, tile)) return;
  const int ox = (tile / (tpa * tpa)) * T, oy = ((tile / tpa) % tpa) * T, oz = (tile % tpa) * T;
  const double2* sk = spec + sidx(k, 0, nn);  // node v at sk[8 v]
  for (int i = threadIdx.x; i < 343; i += blockDim.x) kk[i] = khat[(int64_t)i * F + k];
  // per (class, offset): the box position of the source of the class's first
  // target (the others follow it by the lane's lattice step), and the kernel
  for (int i = threadIdx.x; i < classes * noff; i += blockDim.x) {
    const int pk = offs[i];
    const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
    int pos;
    if (classes == 8) {
      const int c = i / noff;
      const int sx = (c >> 2) + dx + 3, sy = ((c >> 1) & 1) + dy + 3, sz = (c & 1) + dz + 3;
      pos = (((sx & 1) * 2 + (sy & 1)) * 2 + (sz & 1)) * H3 + ((sx >> 1) * Bh + (sy >> 1)) * Bh + (sz >> 1);
    } else {
      pos = ((dx + 3) * B + (dy + 3)) * B + (dz + 3);
    }
    sof[i] = pos * 512 + ((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3));
  }
  // With 8 classes the box is stored split by parity, [px][py][pz][hx][hy][hz]
  // (coordinate 2h + p): for one offset, the 64 targets of a class (a 4^3
  // lattice of step 2) then read 64 consecutive entries.  On the 4^3 level it
  // is stored plainly.
  for (int i = threadIdx.x; i < B * B * B; i += blockDim.x) {
    const int bx = i / (B * B), by = (i / B) % B, bz = i % B;
    const int x = ox + bx - 3, y = oy + by - 3, z = oz + bz - 3;
    double2 v = make_double2(0.0, 0.0);
    if (!isolated || ((unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n)) {
      const int xw = x & (n - 1), yw = y & (n - 1), zw = z & (n - 1);
      v = sk[(((int64_t)xw * n + yw) * n + zw) * 8];
    }
    const int dst = classes == 8 ? (((bx & 1) * 2 + (by & 1)) * 2 + (bz & 1)) * H3 +
                                       ((bx >> 1) * Bh + (by >> 1)) * Bh + (bz >> 1)
                                 : i;
    box[dst] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int tx, ty, tz, cls;
  if (classes == 8) {  // 4^3 targets of class `wave` in the 8^3 tile
    cls = wave;
    tx = 2 * (lane >> 4) + (cls >> 2);
    ty = 2 * ((lane >> 2) & 3) + ((cls >> 1) & 1);
    tz = 2 * (lane & 3) + (cls & 1);
  } else {             // one class, the whole 4^3 level
    cls = 0;
    tx = lane >> 4;
    ty = (lane >> 2) & 3;
    tz = lane & 3;
  }
  const int* o = sof + cls * noff;
  const int base = classes == 8 ? ((lane >> 4) * Bh + ((lane >> 2) & 3)) * Bh + (lane & 3)
                                : (tx * B + ty) * B + tz;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int i = 0; i < noff; ++i) {
    const int w = o[i];
    const double2 kd = kk[w & 511];
    const double2 s = box[base + (w >> 9)];
    re += kd.x * s.x - kd.y * s.y;
    im += kd.x * s.y + kd.y * s.x;
  }
  out[sidx(k, ((int64_t)(ox + tx) * n + (oy + ty)) * n + (oz + tz), nn)] = make_double2(re, im);
}

// The same sums on levels with n >= 8 nodes per axis (levels >= 3), tiles
// of 8 x 8 x TZ targets (TZ = 16, or 8 on the 8^3 level): each lane owns two
// targets of its class, 2 apart in z, and walks the zone by (dx, dy)
// columns.  With TZ = 16 a wave is one class; with TZ = 8 a wave holds two
// classes that differ only in z parity, so the column loops stay uniform.  Stored split by
// parity, a full column (six consecutive dz) is two runs of three entries
// per target, and the second target's runs are the first's shifted by one,
// so four loads per parity plane serve both (8 loads for 12 multiply-adds).
// Columns next to the target (|dx|, |dy| <= 1) keep the three dz outside the
// near zone.  The zone of class c is {d : d_i in [-2 - c_i, 3 - c_i],
// max |d_i| > 1} (Sec. 2), enumerated here directly.
template <int TZ>
__global__ void __launch_bounds__(TZ * 32) k_zone_spec2(const double2* __restrict__ spec,
                                                        const double2* __restrict__ khat, int n,
                                                        int isolated, int64_t F,
                                                        double2* __restrict__ out) {
  constexpr int TX = 8, BX = TX + 6, BZ = TZ + 6;
  constexpr int KZ = TZ / 4;       // target pairs along z per class and (x, y)
  constexpr int LPC = 16 * KZ;     // lanes per class
  constexpr int HX = BX / 2, HZ = BZ / 2, H3 = HX * HX * HZ;
  __shared__ double2 box[8 * H3];
  __shared__ double2 kk[343];
  const int64_t nn = (int64_t)n * n * n;
  const int tpx = n / TX, tpz = n / TZ;
  const int tiles = tpx * tpx * tpz;
  int k, tile;
  if (!zone_block(blockIdx.x, tiles, (int)(F >> 3), k, tile)) return;
  const int ox = (tile / (tpx * tpz)) * TX, oy = ((tile / tpz) % tpx) * TX, oz = (tile % tpz) * TZ;
  const double2* sk = spec + sidx(k, 0, nn);  // node v at sk[8 v]
  for (int i = threadIdx.x; i < 343; i += blockDim.x) kk[i] = khat[(int64_t)i * F + k];
  for (int i = threadIdx.x; i < BX * BX * BZ; i += blockDim.x) {
    const int bx = i / (BX * BZ), by = (i / BZ) % BX, bz = i % BZ;
    const int x = ox + bx - 3, y = oy + by - 3, z = oz + bz - 3;
    double2 v = make_double2(0.0, 0.0);
    if (!isolated || ((unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n && (unsigned)z < (unsigned)n))
      v = sk[(((int64_t)(x & (n - 1)) * n + (y & (n - 1))) * n + (z & (n - 1))) * 8];
    box[(((bx & 1) * 2 + (by & 1)) * 2 + (bz & 1)) * H3 + ((bx >> 1) * HX + (by >> 1)) * HZ + (bz >> 1)] = v;
  }
  __syncthreads();
  const int cls = threadIdx.x / LPC, lane = threadIdx.x % LPC;
  const int cx = cls >> 2, cy = (cls >> 1) & 1, cz = cls & 1;
  const int kx = lane / (4 * KZ), ky = (lane / KZ) % 4, kz = 2 * (lane % KZ);
  const int base = (kx * HX + ky) * HZ + kz;
  double r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0;
  const int dz0 = -2 - cz;
  for (int dx = -2 - cx; dx <= 3 - cx; ++dx) {
    const int sx = cx + dx + 3;
    for (int dy = -2 - cy; dy <= 3 - cy; ++dy) {
      const int sy = cy + dy + 3;
      const int pxy = ((sx & 1) * 2 + (sy & 1)) * 2;
      const int col = base + ((sx >> 1) * HX + (sy >> 1)) * HZ;
      const double2* kc = kk + (dx + 3) * 49 + (dy + 3) * 7 + (dz0 + 3);
      if (abs(dx) > 1 || abs(dy) > 1) {
        // dz0 + 2m: source z 1 + 2m (odd plane, h = m); dz0 + 2m + 1: z 2 + 2m (even, h = m + 1)
        const double2* pa = box + (pxy + 1) * H3 + col;
        const double2* pb = box + pxy * H3 + col + 1;
        double2 a[4], b[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          a[m] = pa[m];
          b[m] = pb[m];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double2 ka = kc[2 * m], kb = kc[2 * m + 1];
          cmac(r1, i1, ka, a[m]);
          cmac(r1, i1, kb, b[m]);
          cmac(r2, i2, ka, a[m + 1]);
          cmac(r2, i2, kb, b[m + 1]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const int dz = dz0 + q;
          if (dz >= -1 && dz <= 1) continue;
          const int sz = 1 + q;
          const double2* ps = box + (pxy + (sz & 1)) * H3 + col + (sz >> 1);
          const double2 kd = kc[q], s1 = ps[0], s2 = ps[1];
          cmac(r1, i1, kd, s1);
          cmac(r2, i2, kd, s2);
        }
      }
    }
  }
  const int tx = ox + 2 * kx + cx, ty = oy + 2 * ky + cy, tz = oz + 2 * kz + cz;
  double2* o = out + sidx(k, ((int64_t)tx * n + ty) * n + tz, nn);
  o[0] = make_double2(r1, i1);
  o[16] = make_double2(r2, i2);  // node tz + 2
}

// Whole-level stencil, targets in runs along y (used for the 16^3 level, n =
// 2H = 16): one workgroup per frequency holds the level's whole spectrum at that
// frequency in LDS (n^3 values: periodic wrap, no halo) and sums every
// target's zone.  Stored split by parity, [px][py][pz][hx][hy][hz] (node
// coordinate 2h + p), hz fastest.  With H = 8 and TY = 8 one wave per
// parity class: the class, the zone's offsets and so every kernel value are
// uniform across a wave, and the kernel values come from the frequency's
// contiguous row of khatT by scalar loads, leaving LDS to the sources.  The
// 64 lanes of a wave span (hx, hz), so that one load instruction reads H
// consecutive entries per row; a lane owns TY targets of its class
// consecutive in hy (2 apart in y).  Walking the zone by (dx, dz) columns,
// each parity plane of a column is one run of TY + 2 source rows along hy
// shared by the TY targets (three offsets per target and plane); with
// TY = H the run's rows are the same for the whole wave, so their offsets
// fold into the load instructions.  Columns
// next to the target (|dx|, |dz| <= 1) skip the three dy of the near zone.
// Blocks are dealt to the 8 XCDs so that the 8 frequencies of a chunk, which
// share every 128-byte line of the spectra, run on one XCD back to back.
//
// T = float: the sources and kernel values in FP32 (with TS = float2 the
// level's spectra are stored in FP32 too; the transforms compute in FP64),
// the terms of each (dx, dz) column summed in FP32 and the 36 column sums
// of a target added in FP64.
template <int H, int TY, class T = double, class TS = double2>
__global__ void __launch_bounds__(8 * (H * H * H / TY), sizeof(T) == 4 ? 4 : 8) k_zone_level_y(
    const TS* __restrict__ spec, const typename Vec2<T>::type* __restrict__ khatT, int64_t F,
    int nchunk, TS* __restrict__ out) {
  using T2 = typename Vec2<T>::type;
  constexpr bool kSplit = sizeof(T) == 4;  // FP32 column sums into FP64 totals
  constexpr int n = 2 * H, nn = n * n * n, H3 = H * H * H;
  constexpr int LPC = H3 / TY;   // lanes per class
  constexpr int NT = 8 * LPC;
  static_assert(LPC % 64 == 0, "a class fills whole waves");
  static_assert(H % TY == 0, "whole target runs");
  __shared__ T2 box[nn];
  const int g = blockIdx.x;
  const int chunk = ((g >> 3) >> 3) * 8 + (g & 7);
  if (chunk >= nchunk) return;
  const int k = chunk * 8 + ((g >> 3) & 7);
  const TS* sk = spec + (int64_t)(k >> 3) * nn * 8 + (k & 7);  // node v at sk[8 v]
  // stage: LDS slot i = ((p * H + hx) * H + (hy ^ (hx & 1))) * H + hz,
  // consecutive threads writing consecutive slots.  Flipping the low bit of
  // hy on odd hx puts the two hx of a 16-lane group on different halves of
  // the 64 banks when all lanes read one hy.
  for (int i = threadIdx.x; i < nn; i += NT) {
    const int hz = i % H, hx = (i / (H * H)) % H, hy = ((i / H) % H) ^ (hx & 1), p = i / H3;
    const int x = 2 * hx + (p >> 2), y = 2 * hy + ((p >> 1) & 1), z = 2 * hz + (p & 1);
    const TS v = sk[(int64_t)((x * n + y) * n + z) * 8];
    box[i] = T2{(T)v.x, (T)v.y};
  }
  __syncthreads();
  const int cls = __builtin_amdgcn_readfirstlane(threadIdx.x / LPC);
  const int cx = cls >> 2, cy = (cls >> 1) & 1, cz = cls & 1;
  const int lane = threadIdx.x % LPC;
  const int hz = lane % H, hx = (lane / H) % H, hy0 = (lane / (H * H)) * TY;
  const T2* kf = khatT + (int64_t)k * kKT;
  double re[TY], im[TY];
  T cr[TY], ci[TY];  // the current column's sums (FP32 with kSplit)
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    re[t] = im[t] = 0.0;
    cr[t] = ci[t] = (T)0;
  }
  int fl = 0;  // 1 when the current source column's hx' is odd
  // one parity plane (py) of a column: rows hy0 - 1 + j (j < TY + 2) of the
  // column's (px, pz, hx', hz'); target t reads j = t + m with the kernel of
  // offset dy = 2 m - 2 + py - cy
  auto plane = [&](int col, int kbase, int py, bool m0, bool m1, bool m2) {
    // row hy sits at slot row hy ^ (hx' & 1): one base per parity of hy
    // (32-bit LDS slot offsets, no pointer arithmetic)
    const int pl = col + py * 2 * H3;
    const int pe = pl + fl * H;   // even hy: +H on odd hx'
    const int po = pl - fl * H;   // odd hy: -H on odd hx'
    T2 src[TY + 2];
#pragma unroll
    for (int j = 0; j < TY + 2; ++j) {
      const int hy = (hy0 - 1 + j) & (H - 1);
      src[j] = box[((hy & 1) ? po : pe) + hy * H];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if ((m == 0 && !m0) || (m == 1 && !m1) || (m == 2 && !m2)) continue;
      const T2 kd = kf[kbase + 7 * (2 * m - 2 + py - cy + 3)];
      if constexpr (kSplit) {
        // k s = (kx sx - ky sy, kx sy + ky sx) with -ky kept as its own value
        const float kx = vreg(kd.x), ky = vreg(kd.y), nky = vreg(-kd.y);
#pragma unroll
        for (int t = 0; t < TY; ++t) {
          cr[t] = fmaf(kx, src[t + m].x, cr[t]);
          cr[t] = fmaf(nky, src[t + m].y, cr[t]);
          ci[t] = fmaf(kx, src[t + m].y, ci[t]);
          ci[t] = fmaf(ky, src[t + m].x, ci[t]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < TY; ++t) cmac(re[t], im[t], kd, src[t + m]);
      }
    }
  };
  // with kSplit, a finished column's sums go into the FP64 totals
  auto flush = [&]() {
    if constexpr (kSplit) {
#pragma unroll
      for (int t = 0; t < TY; ++t) {
        re[t] += (double)cr[t];
        im[t] += (double)ci[t];
        cr[t] = ci[t] = (T)0;
      }
    }
  };
  for (int sx = -2; sx <= 3; ++sx) {      // source x = 2 hx + cx + dx, sx = cx + dx
    const int dx = sx - cx;
    const int hxs = (hx + (sx >> 1)) & (H - 1);
    fl = hxs & 1;
    const int cxo = (sx & 1) * 4 * H3 + hxs * H * H;
    for (int sz = -2; sz <= 3; ++sz) {
      const int dz = sz - cz;
      const int col = cxo + (sz & 1) * H3 + ((hz + (sz >> 1)) & (H - 1));
      const int kbase = (dx + 3) * 49 + (dz + 3);
      if (abs(dx) > 1 || abs(dz) > 1) {
        plane(col, kbase, 0, true, true, true);
        plane(col, kbase, 1, true, true, true);
      } else if (cy == 0) {  // keep sy = -2, 2 (even) and 3 (odd)
        plane(col, kbase, 0, true, false, true);
        plane(col, kbase, 1, false, false, true);
      } else {               // keep sy = -2 (even), -1 and 3 (odd)
        plane(col, kbase, 0, true, false, false);
        plane(col, kbase, 1, true, false, true);
      }
      flush();
    }
  }
  TS* o = out + (int64_t)(k >> 3) * nn * 8 + (k & 7);
#pragma unroll
  for (int t = 0; t < TY; ++t) {
    const int y = 2 * (hy0 + t) + cy;
    const int v = ((2 * hx + cx) * n + y) * n + (2 * hz + cz);
    o[(int64_t)v * 8] = from_d2<TS>(make_double2(re[t], im[t]));
  }
}

// Whole-level stencil, targets in runs along z (used for the 8^3 level, n =
// 2H = 8): one workgroup per frequency holds the level's whole spectrum at that
// frequency in LDS (n^3 values: periodic wrap, no halo) and sums every
// target's zone.  Stored split by parity ([px][py][pz][hx][hy][hz], node
// coordinate 2h + p), rows of H values (hz) XOR-swizzled by the row index so
// that the lanes of a wave, which read one hz from H different rows, hit
// distinct banks.  Two (H = 8) or one (H = 4) waves per parity class: the
// class, the zone's offsets and so every kernel value are uniform across a
// wave, and the kernel values come from the frequency's contiguous row of
// khatT by scalar loads, leaving LDS to the sources.  A lane owns TZ targets
// of its class consecutive in hz (2 apart in z); walking the zone by (dx, dy)
// columns, each parity plane of a column is one run of TZ + 2 source values
// shared by the TZ targets (three offsets per target and plane).  Columns
// next to the target (|dx|, |dy| <= 1) skip the three dz of the near zone.
// Blocks are dealt to the 8 XCDs so that the 8 frequencies of a chunk, which
// share every 128-byte line of the spectra, run on one XCD back to back.
template <int H, int TZ>
__global__ void __launch_bounds__(8 * (H * H * H / TZ), 8) k_zone_level_z(
    const double2* __restrict__ spec, const double2* __restrict__ khatT, int64_t F, int nchunk,
    double2* __restrict__ out) {
  constexpr int n = 2 * H, nn = n * n * n;
  constexpr int LPC = H * H * H / TZ;   // lanes per class
  constexpr int NT = 8 * LPC;
  static_assert(LPC % 64 == 0, "a class fills whole waves");
  static_assert(H % TZ == 0, "whole target runs");
  __shared__ double2 box[nn];
  const int g = blockIdx.x;
  const int chunk = ((g >> 3) >> 3) * 8 + (g & 7);
  if (chunk >= nchunk) return;
  const int k = chunk * 8 + ((g >> 3) & 7);
  const double2* sk = spec + (int64_t)(k >> 3) * nn * 8 + (k & 7);  // node v at sk[8 v]
  // stage: node (x, y, z) -> parity block, row (hx, hy), swizzled hz
  for (int v = threadIdx.x; v < nn; v += NT) {
    const int x = v / (n * n), y = (v / n) % n, z = v % n;
    const int row = (((x & 1) * 2 + (y & 1)) * 2 + (z & 1)) * H * H + (x >> 1) * H + (y >> 1);
    box[row * H + ((z >> 1) ^ (row & (H - 1)))] = sk[(int64_t)v * 8];
  }
  __syncthreads();
  const int cls = __builtin_amdgcn_readfirstlane(threadIdx.x / LPC);
  const int cx = cls >> 2, cy = (cls >> 1) & 1, cz = cls & 1;
  const int lane = threadIdx.x % LPC;
  const int hx = lane / (H * (H / TZ)), hy = (lane / (H / TZ)) % H, hz0 = (lane % (H / TZ)) * TZ;
  const double2* kf = khatT + (int64_t)k * kKT;
  double re[TZ], im[TZ];
#pragma unroll
  for (int t = 0; t < TZ; ++t) re[t] = im[t] = 0.0;
  // one parity plane of a column: source half-z hz0 - 1 + j (j < TZ + 2);
  // target t reads j = t + m with the kernel of offset index kidx[m]
  auto plane = [&](int rowbase, int kbase, int pz, bool m0, bool m1, bool m2) {
    double2 src[TZ + 2];
    const int row = rowbase + pz * H * H;
#pragma unroll
    for (int j = 0; j < TZ + 2; ++j)
      src[j] = box[row * H + (((hz0 - 1 + j) & (H - 1)) ^ (row & (H - 1)))];
    // offset dz = sz - cz with sz = 2 m - 2 + pz (m = 0, 1, 2)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if ((m == 0 && !m0) || (m == 1 && !m1) || (m == 2 && !m2)) continue;
      const double2 kd = kf[kbase + (2 * m - 2 + pz - cz + 3)];
#pragma unroll
      for (int t = 0; t < TZ; ++t) cmac(re[t], im[t], kd, src[t + m]);
    }
  };
  for (int sx = -2; sx <= 3; ++sx) {      // source x = 2 hx + cx + dx, sx = cx + dx
    const int dx = sx - cx;
    const int rx = ((hx + (sx >> 1)) & (H - 1)) * H;
    for (int sy = -2; sy <= 3; ++sy) {
      const int dy = sy - cy;
      const int rowbase = ((sx & 1) * 4 + (sy & 1) * 2) * H * H + rx + ((hy + (sy >> 1)) & (H - 1));
      const int kbase = (dx + 3) * 49 + (dy + 3) * 7;
      if (abs(dx) > 1 || abs(dy) > 1) {
        plane(rowbase, kbase, 0, true, true, true);
        plane(rowbase, kbase, 1, true, true, true);
      } else if (cz == 0) {  // keep sz = -2, 2 (even) and 3 (odd)
        plane(rowbase, kbase, 0, true, false, true);
        plane(rowbase, kbase, 1, false, false, true);
      } else {               // keep sz = -2 (even), -1 and 3 (odd)
        plane(rowbase, kbase, 0, true, false, false);
        plane(rowbase, kbase, 1, true, false, true);
      }
    }
  }
  double2* o = out + (int64_t)(k >> 3) * nn * 8 + (k & 7);
#pragma unroll
  for (int t = 0; t < TZ; ++t) {
    const int z = 2 * (hz0 + t) + cz;
    const int v = ((2 * hx + cx) * n + (2 * hy + cy)) * n + z;
    o[(int64_t)v * 8] = make_double2(re[t], im[t]);
  }
}

// The 4^3 level (37 offsets periodic, 316 isolated), one workgroup per
// 8-frequency chunk: each thread loads one node's 8 frequencies (one 128-byte
// line) and then sums one target's zone at one frequency.  Kernel values of
// the zone's offsets for the chunk come from khatT.
__global__ void __launch_bounds__(512) k_zone_l2(const double2* __restrict__ spec,
                                                 const double2* __restrict__ khatT,
                                                 const int* __restrict__ offs, int noff, int isolated,
                                                 int nchunk, double2* __restrict__ out) {
  __shared__ double2 box[8 * 64];        // [frequency in chunk][node]
  __shared__ double2 kk[8 * 316];        // [frequency in chunk][zone offset]
  __shared__ int so[316];                // packed offsets
  const int chunk = blockIdx.x;
  if (chunk >= nchunk) return;
  const double2* sk = spec + (int64_t)chunk * 64 * 8;
  for (int i = threadIdx.x; i < 512; i += 512) box[(i & 7) * 64 + (i >> 3)] = sk[i];
  for (int i = threadIdx.x; i < noff; i += 512) so[i] = offs[i];
  __syncthreads();
  for (int i = threadIdx.x; i < 8 * noff; i += 512) {
    const int f = i / noff, d = i % noff;
    const int pk = so[d];
    const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
    kk[f * 316 + d] = khatT[(int64_t)(chunk * 8 + f) * kKT + (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)];
  }
  __syncthreads();
  const int f = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int tx = t >> 4, ty = (t >> 2) & 3, tz = t & 3;
  double re = 0.0, im = 0.0;
  for (int d = 0; d < noff; ++d) {
    const int pk = so[d];
    const int x = tx + ((pk >> 16) & 255) - 128, y = ty + ((pk >> 8) & 255) - 128,
              z = tz + (pk & 255) - 128;
    if (isolated && ((unsigned)x > 3u || (unsigned)y > 3u || (unsigned)z > 3u)) continue;
    const double2 kd = kk[f * 316 + d];
    const double2 sv = box[f * 64 + (((x & 3) * 4 + (y & 3)) * 4 + (z & 3))];
    re = fma(kd.x, sv.x, re);
    re = fma(-kd.y, sv.y, re);
    im = fma(kd.x, sv.y, im);
    im = fma(kd.y, sv.x, im);
  }
  out[(int64_t)chunk * 64 * 8 + t * 8 + f] = make_double2(re, im);
}

// khatT in FP32.
__global__ void k_khat_f32(const double2* __restrict__ in, int64_t n, float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// khatT[f][d] = khat[d][f] (d < 343; the pad entry is zero).
__global__ void k_khat_transpose(const double2* __restrict__ khat, int64_t F,
                                 double2* __restrict__ khatT) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F * kKT) return;
  const int64_t f = i / kKT;
  const int d = (int)(i % kKT);
  khatT[i] = d < 343 ? khat[(int64_t)d * F + f] : make_double2(0.0, 0.0);
}

// Kernel spectrum of offset d (FP64 separable DFT): first pass along z of
// K_d[x][y][z] = tab[w(x) - p dx][w(y) - p dy][w(z) - p dz] (tab centred at
// C), zero on the unused slot p; then y and x (k_sdft_axis); stored scaled in
// the frequency order of k_node_fwd.
__global__ void k_sdft_z(const double* __restrict__ tab, int p, int C, double2* __restrict__ A) {
  const int M = 2 * p, H = p + 1;
  const int64_t F = (int64_t)M * M * H;
  const int di = blockIdx.y;  // offset (dx, dy, dz) in [-3, 3]^3
  const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
  A += di * F;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F) return;
  const int kz = (int)(i % H), y = (int)((i / H) % M), x = (int)(i / ((int64_t)H * M));
  const int E = 2 * C + 1;
  double re = 0.0, im = 0.0;
  if (x != p && y != p) {
    const int jx = (x < p ? x : x - M) - p * dx, jy = (y < p ? y : y - M) - p * dy;
    const double* row = tab + ((int64_t)(jx + C) * E + (jy + C)) * E;
    for (int z = 0; z < M; ++z) {
      if (z == p) continue;
      const double v = row[(z < p ? z : z - M) - p * dz + C];
      double sn, cs;
      sincospi(-(double)((kz * z) % M) / p, &sn, &cs);
      re += v * cs;
      im += v * sn;
    }
  }
  A[i] = make_double2(re, im);
}

__global__ void k_sdft_axis(const double2* __restrict__ in, int p, int axis, double2* __restrict__ out) {
  const int M = 2 * p, H = p + 1;
  const int64_t F = (int64_t)M * M * H;
  in += blockIdx.y * F;
  out += blockIdx.y * F;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F) return;
  const int kz = (int)(i % H), b = (int)((i / H) % M), a = (int)(i / ((int64_t)H * M));
  const int kk = axis ? b : a;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < M; ++j) {
    const double2 v = in[axis ? ((int64_t)a * M + j) * H + kz : ((int64_t)j * M + b) * H + kz];
    double sn, cs;
    sincospi(-(double)((kk * j) % M) / p, &sn, &cs);
    re += v.x * cs - v.y * sn;
    im += v.x * sn + v.y * cs;
  }
  out[i] = make_double2(re, im);
}

__global__ void k_sdft_store(const double2* __restrict__ in, int p, double scale, double2* __restrict__ out) {
  const int M = 2 * p, H = p + 1;
  const int64_t F = (int64_t)M * M * H;
  in += blockIdx.y * F;
  out += blockIdx.y * F;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F) return;
  const int kz = (int)(i % H), ky = (int)((i / H) % M), kx = (int)(i / ((int64_t)H * M));
  const int64_t d = ((int64_t)(kx * 2 + (ky & 1)) * p + (ky >> 1)) * H + kz;
  out[d] = make_double2(in[i].x * scale, in[i].y * scale);
}

inline hipError_t tbegin(KernelTimer* kt, hipStream_t st) { return kt ? kt->begin(st) : hipSuccess; }
inline hipError_t tend(KernelTimer* kt, hipStream_t st, int part, hipError_t e) {
  if (e != hipSuccess || !kt) return e;
  return kt->end(st, part);
}

template <int P>
hipError_t run_level(M2LSpectral* f, int l, const void* Ml, int m64, void* Pl, int p64,
                     int accumulate, const int* offs, int noff, int isolated, hipStream_t st,
                     KernelTimer* kt) {
  const int n = 1 << l;
  const int64_t nn = (int64_t)n * n * n;
  constexpr int NT = node_threads<P>();
  // the 16^3 leaf level in FP32 columns: its spectra stored as float2
  const bool f32 = n == 16 && !isolated && f->f32 && l == f->L && f->khatT32;
  float2* spec32 = reinterpret_cast<float2*>(f->spec);
  float2* out32 = reinterpret_cast<float2*>(f->out);
  hipError_t e = tbegin(kt, st);
  if (e != hipSuccess) return e;
  if (m64 && f32)
    k_node_fwd<P, double, float2><<<(unsigned)nn, NT, 0, st>>>((const double*)Ml, nn, spec32);
  else if (f32)
    k_node_fwd<P, float, float2><<<(unsigned)nn, NT, 0, st>>>((const float*)Ml, nn, spec32);
  else if (m64)
    k_node_fwd<P, double><<<(unsigned)nn, NT, 0, st>>>((const double*)Ml, nn, f->spec);
  else
    k_node_fwd<P, float><<<(unsigned)nn, NT, 0, st>>>((const float*)Ml, nn, f->spec);
  e = tend(kt, st, 0, hipGetLastError());
  if (e == hipSuccess) e = tbegin(kt, st);
  if (e != hipSuccess) return e;
  const int classes = l == 2 ? 1 : 8;
  // blocks per tile: the 8-frequency chunks rounded up to a multiple of 8, times 8
  const int64_t per_tile = (f->F / 8 + 7) / 8 * 64;
  const int nchunk = (int)(f->F / 8);
  const unsigned cgrid = (unsigned)((nchunk + 7) / 8 * 64);  // chunks rounded up to 8, times 8
  if (f32) {  // FP32 columns
    k_zone_level_y<8, 8, float, float2><<<cgrid, 512, 0, st>>>(spec32, f->khatT32, f->F, nchunk, out32);
  } else if (n == 16 && !isolated) {  // the whole level per frequency, eight targets per lane
    k_zone_level_y<8, 8><<<cgrid, 512, 0, st>>>(f->spec, f->khatT[l], f->F, nchunk, f->out);
  } else if (n == 8 && !isolated) {
    k_zone_level_z<4, 1><<<cgrid, 512, 0, st>>>(f->spec, f->khatT[l], f->F, nchunk, f->out);
  } else if (n == 4) {
    k_zone_l2<<<(unsigned)nchunk, 512, 0, st>>>(f->spec, f->khatT[l], offs, noff, isolated, nchunk,
                                                 f->out);
  } else if (n >= 16) {  // 8 x 8 x 16 tiles, two targets per lane
    const unsigned grid = (unsigned)(per_tile * (n / 8) * (n / 8) * (n / 16));
    k_zone_spec2<16><<<grid, 512, 0, st>>>(f->spec, f->khat[l], n, isolated, f->F, f->out);
  } else if (n == 8) {  // the 8^3 level as one tile, two targets per lane
    k_zone_spec2<8><<<(unsigned)per_tile, 256, 0, st>>>(f->spec, f->khat[l], n, isolated, f->F, f->out);
  } else {
    const int T = n < 8 ? n : 8;
    const unsigned grid = (unsigned)(per_tile * (n / T) * (n / T) * (n / T));
    k_zone_spec<<<grid, classes == 8 ? 512 : 64, 0, st>>>(f->spec, f->khat[l], offs, noff, n, classes,
                                                           isolated, f->F, f->out);
  }
  e = tend(kt, st, 1, hipGetLastError());
  if (e == hipSuccess) e = tbegin(kt, st);
  if (e != hipSuccess) return e;
  if (p64 && f32)
    k_node_inv<P, double, float2><<<(unsigned)nn, NT, 0, st>>>(out32, nn, accumulate, (double*)Pl);
  else if (f32)
    k_node_inv<P, float, float2><<<(unsigned)nn, NT, 0, st>>>(out32, nn, accumulate, (float*)Pl);
  else if (p64)
    k_node_inv<P, double><<<(unsigned)nn, NT, 0, st>>>(f->out, nn, accumulate, (double*)Pl);
  else
    k_node_inv<P, float><<<(unsigned)nn, NT, 0, st>>>(f->out, nn, accumulate, (float*)Pl);
  return tend(kt, st, 2, hipGetLastError());
}

}  // namespace

void m2l_spectral_destroy(M2LSpectral* f) {
  if (!f) return;
  (void)hipFree(f->spec);
  (void)hipFree(f->out);
  for (double2* k : f->khat) (void)hipFree(k);
  for (double2* k : f->khatT) (void)hipFree(k);
  (void)hipFree(f->khatT32);
  for (double2* d : f->dft) (void)hipFree(d);
  delete f;
}

hipError_t m2l_spectral_create(int L, int p, M2LSpectral** out) {
  *out = nullptr;
  if (p != 4 && p != 6 && p != 8) return hipErrorInvalidValue;
  M2LSpectral* f = new M2LSpectral;
  f->L = L;
  f->p = p;
  f->F = (int64_t)(2 * p) * (2 * p) * (p + 1);
  const int64_t nodes = (int64_t)1 << (3 * L);
  f->khat.assign(L + 1, nullptr);
  f->khatT.assign(L + 1, nullptr);
  hipError_t e = hipMalloc(&f->spec, (size_t)(f->F * nodes) * sizeof(double2));
  if (e == hipSuccess) e = hipMalloc(&f->out, (size_t)(f->F * nodes) * sizeof(double2));
  for (int d = 0; d < 2 && e == hipSuccess; ++d) e = hipMalloc(&f->dft[d], (size_t)(343 * f->F) * sizeof(double2));
  for (int l = 2; l <= L && e == hipSuccess; ++l)
    e = hipMalloc(&f->khat[l], (size_t)(343 * f->F) * sizeof(double2));
  for (int l = 2; l <= L && e == hipSuccess; ++l)
    e = hipMalloc(&f->khatT[l], (size_t)(kKT * f->F) * sizeof(double2));
  if (e == hipSuccess && L == 4) e = hipMalloc(&f->khatT32, (size_t)(kKT * f->F) * sizeof(float2));
  if (e != hipSuccess) {
    m2l_spectral_destroy(f);
    return e;
  }
  *out = f;
  return hipSuccess;
}

void m2l_spectral_set_f32(M2LSpectral* f, int on) { f->f32 = on; }

hipError_t m2l_spectral_tables(M2LSpectral* f, const std::vector<double*>& tab64, hipStream_t st) {
  const int p = f->p, C = 4 * p - 1;
  const double scale = 1.0 / (double)((2 * p) * (2 * p) * (2 * p));
  hipError_t e = hipSuccess;
  const dim3 grid(nblk(f->F), 343);  // all offsets of [-3, 3]^3 at once
  for (int l = 2; l <= f->L && e == hipSuccess; ++l) {
    k_sdft_z<<<grid, kThreads, 0, st>>>(tab64[l], p, C, f->dft[0]);
    k_sdft_axis<<<grid, kThreads, 0, st>>>(f->dft[0], p, 1, f->dft[1]);
    k_sdft_axis<<<grid, kThreads, 0, st>>>(f->dft[1], p, 0, f->dft[0]);
    k_sdft_store<<<grid, kThreads, 0, st>>>(f->dft[0], p, scale, f->khat[l]);
    k_khat_transpose<<<nblk(f->F * kKT), kThreads, 0, st>>>(f->khat[l], f->F, f->khatT[l]);
    if (l == f->L && f->khatT32)
      k_khat_f32<<<nblk(f->F * kKT), kThreads, 0, st>>>(f->khatT[l], f->F * kKT, f->khatT32);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

hipError_t m2l_spectral_level(M2LSpectral* f, int l, const void* Ml, int m64, void* Pl, int p64,
                              int accumulate, const int* offs, int noff, int isolated, hipStream_t st,
                              KernelTimer* kt) {
  if (l < 2 || l > f->L) return hipErrorInvalidValue;
  if (f->p == 4) return run_level<4>(f, l, Ml, m64, Pl, p64, accumulate, offs, noff, isolated, st, kt);
  if (f->p == 6) return run_level<6>(f, l, Ml, m64, Pl, p64, accumulate, offs, noff, isolated, st, kt);
  return run_level<8>(f, l, Ml, m64, Pl, p64, accumulate, offs, noff, isolated, st, kt);
}

}  // namespace pfmm
