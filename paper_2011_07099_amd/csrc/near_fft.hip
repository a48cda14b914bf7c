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
// FP64 DFT.  Per solve, for leaf edges s = 4, 8, 16 one workgroup per leaf
// reads the leaf's cells straight from the mesh and transforms them in LDS,
// skipping the zero half of every axis (only s of the 2s inputs of a forward
// pass, and only s of the 2s outputs of an inverse pass, are ever nonzero or
// needed), and the inverse writes the target cells straight into the mesh;
// spectra are stored in chunks of 64 frequencies over all leaves, so that
// the 27-point stencil of one chunk reads 64 x 8 B contiguous per leaf and
// its whole working set (64 x 8 B x leaves: 2 MiB at 16^3 leaves) stays in
// one XCD's L2.  Other leaf edges use rocFFT R2C / C2R on zero-padded blocks.
// The same machinery serves the acceleration kernels D_i (they replace G).
#include "internal.h"

#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <vector>

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
  int fused = 0;             // s in {4, 8, 16}: fused LDS transforms, chunked spectra
  int lgnb = 0;              // log2 of leaves per axis
  int sym[4] = {0, 0, 0, 0};  // per kernel: +1 even, -1 odd, 0 neither (k_near_mac)
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

// Scaled FP32 copy of a transformed kernel.  With `fused` the frequencies
// go to the order of the fused transforms, ky split into parity and half
// and the parity of kx innermost (kx = 2j and 2j + 1 side by side):
// (kx, ky, kz) -> (((kx / 2 * 2 + ky % 2) * s + ky / 2) * (s + 1) + kz) * 2 + kx % 2.
__global__ void k_kdft_store(const double2* __restrict__ in, int s, int fused, double scale,
                             float2* __restrict__ out) {
  const int M = 2 * s, H = s + 1;
  const int64_t F = (int64_t)M * M * H;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= F) return;
  int64_t d = i;
  if (fused) {
    const int kz = (int)(i % H), ky = (int)((i / H) % M), kx = (int)(i / ((int64_t)H * M));
    d = ((((int64_t)(kx >> 1) * 2 + (ky & 1)) * s + (ky >> 1)) * H + kz) * 2 + (kx & 1);
  }
  out[d] = make_float2((float)(in[i].x * scale), (float)(in[i].y * scale));
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

// exp(-2 pi i j / 32) = cos32(j) - i sin32(j).  With the DFT loops below
// fully unrolled, j is a compile-time constant and these fold to literals.
__device__ constexpr float kQuarter[9] = {1.0f, 0.98078528040f, 0.92387953251f, 0.83146961230f,
                                          0.70710678119f, 0.55557023302f, 0.38268343237f,
                                          0.19509032202f, 0.0f};
__device__ __forceinline__ float cos32(int j) {
  j &= 31;
  if (j <= 8) return kQuarter[j];
  if (j <= 16) return -kQuarter[16 - j];
  if (j <= 24) return -kQuarter[j - 16];
  return kQuarter[32 - j];
}
__device__ __forceinline__ float sin32(int j) { return cos32(j - 8); }

// Twiddle exp(-2 pi i j / M) as (cos, sin) of the positive angle, M | 32.
template <int M>
__device__ __forceinline__ float2 tw(int j) {
  constexpr int r = 32 / M;
  return make_float2(cos32(j * r), sin32(j * r));
}

// Fourth word of a raw buffer resource (32-bit data format, no swizzle) and
// the two-dword vector the 64-bit buffer builtins move.
constexpr int kBufferDword3 = 0x00020000;
typedef unsigned v2u32 __attribute__((ext_vector_type(2)));
typedef unsigned v4u32 __attribute__((ext_vector_type(4)));

// Address of frequency f of leaf `leaf` in the chunked spectrum layout:
// [F / 64][leaves][64].
__device__ __forceinline__ int64_t chunk_addr(int f, int64_t leaf, int64_t nleaf) {
  return ((int64_t)(f >> 6) * nleaf + leaf) * 64 + (f & 63);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// a exp(-2 pi i j / P) (forward) or a exp(+2 pi i j / P) (INV)
template <int P, bool INV>
__device__ __forceinline__ float2 twiddle(float2 a, int j) {
  const float2 w = tw<P>(j);
  return INV ? make_float2(a.x * w.x - a.y * w.y, a.y * w.x + a.x * w.y)
             : make_float2(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3), b3 = csub(a1, a3);
  const float2 ib3 = make_float2(-b3.y, b3.x);
  a0 = cadd(b0, b2);
  a2 = csub(b0, b2);
  a1 = INV ? cadd(b1, ib3) : csub(b1, ib3);
  a3 = INV ? csub(b1, ib3) : cadd(b1, ib3);
}

// In-place DFT of P = 4Q values (Q = 1, 2, 4), v[m] <- sum_n v[n] exp(-+2 pi i n m / P),
// by the split n = Q n1 + n2, m = m1 + 4 m2: length-4 DFTs over n1, twiddles
// exp(-+2 pi i n2 m1 / P), length-Q DFTs over n2.
template <int P, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[P]) {
  constexpr int Q = P / 4;
  float2 T[Q][4];
#pragma unroll
  for (int n2 = 0; n2 < Q; ++n2) {
    T[n2][0] = v[n2];
    T[n2][1] = v[Q + n2];
    T[n2][2] = v[2 * Q + n2];
    T[n2][3] = v[3 * Q + n2];
    dft4<INV>(T[n2][0], T[n2][1], T[n2][2], T[n2][3]);
#pragma unroll
    for (int m1 = 1; m1 < 4; ++m1)
      if (n2) T[n2][m1] = twiddle<P, INV>(T[n2][m1], n2 * m1);
  }
#pragma unroll
  for (int m1 = 0; m1 < 4; ++m1) {
    if constexpr (Q == 1) {
      v[m1] = T[0][m1];
    } else if constexpr (Q == 2) {
      v[m1] = cadd(T[0][m1], T[1][m1]);
      v[m1 + 4] = csub(T[0][m1], T[1][m1]);
    } else {
      float2 c0 = T[0][m1], c1 = T[1][m1], c2 = T[2][m1], c3 = T[3][m1];
      dft4<INV>(c0, c1, c2, c3);
      v[m1] = c0;
      v[m1 + 4] = c1;
      v[m1 + 8] = c2;
      v[m1 + 12] = c3;
    }
  }
}

// Threads per leaf: every pass has at most s (s + 1) tasks, one per thread.
template <int S>
constexpr int leaf_threads() { return (S * (S + 1) + 63) / 64 * 64; }

// Forward transform of one leaf: its s^3 cells (read from the mesh) on the
// (2s)^3 cyclic grid, zero beyond s on every axis, to the half spectrum
// X[kx][ky][kz], kz <= s, written in the chunked layout.  z: direct real DFT
// of the s inputs to s + 1 outputs.  y and x: s inputs to 2s outputs, split
// by output parity, X[2m] = DFT_s(u)[m] and X[2m + 1] = DFT_s(u_n w^n)[m]
// with w = exp(-2 pi i / 2s).  The work runs once per parity of ky in one
// LDS buffer of s^2 (s + 1) values: the z pass fills it, the y pass of that
// parity transforms every (x, kz) column in place (one thread per column),
// the x pass reads it out.  The second parity redoes the z pass from the
// row each thread keeps in registers instead of keeping a second buffer, so
// four leaves fit in a CU's LDS at s = 16 and the mesh is read once.
//
// With P > 0 the kernel first does the leaf's P2M from the same rows (the
// gridlet masses h^3 sum_c A[ax][cx] A[ay][cy] A[az][cz] rho[c], A[a][c] the
// Lagrange basis of gridlet node a at cell centre c): z is contracted from
// each thread's row in registers, y and x through the LDS buffer before the
// transform takes it over, so the density is read from HBM once for both.
template <int S, int P = 0>
__global__ void __launch_bounds__(leaf_threads<S>()) k_leaf_fwd(const float* __restrict__ rho, int N, int lgnb,
                                                        int64_t nleaf, float2* __restrict__ rhat,
                                                        LeafTree tree) {
  constexpr int M = 2 * S, H = S + 1, NT = leaf_threads<S>();
  __shared__ float2 A[S * S * H];  // [x][y][kz], then [x][m][kz] with ky = 2m + parity
  const int64_t leaf = xcd_leaf(blockIdx.x, nleaf);
  const int msk = (1 << lgnb) - 1;
  const int bz = (int)(leaf & msk), by = (int)((leaf >> lgnb) & msk), bx = (int)(leaf >> (2 * lgnb));
  static_assert(NT >= S * S, "one row per thread");
  const int tr = threadIdx.x;
  float4 rowv[S / 4];
  if (tr < S * S) {
    const int x = tr / S, y = tr % S;
    const float4* src = reinterpret_cast<const float4*>(
        rho + ((int64_t)(bx * S + x) * N + (by * S + y)) * N + (int64_t)bz * S);
#pragma unroll
    for (int q = 0; q < S / 4; ++q) rowv[q] = src[q];
  }
  if constexpr (P > 0) {
    constexpr int SP = S + 1;  // weight rows padded by one word
    static_assert((P * SP + S * S * P + S * P * P) * sizeof(float) <= sizeof(A), "P2M fits in the buffer");
    float* sw = reinterpret_cast<float*>(A);  // [a][c]
    float* t1 = sw + P * SP;                  // [cx][cy][az]
    float* t2 = t1 + S * S * P;               // [cx][ay][az]
    for (int i = tr; i < P * S; i += NT) sw[(i / S) * SP + i % S] = tree.A[i];
    __syncthreads();
    if (tr < S * S) {
#pragma unroll
      for (int az = 0; az < P; ++az) {
        const float* w = sw + az * SP;
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < S / 4; ++q)
          acc += w[4 * q] * rowv[q].x + w[4 * q + 1] * rowv[q].y + w[4 * q + 2] * rowv[q].z +
                 w[4 * q + 3] * rowv[q].w;
        t1[tr * P + az] = acc;
      }
    }
    __syncthreads();
    for (int i = tr; i < S * P * P; i += NT) {
      const int cx = i / (P * P), ay = (i / P) % P, az = i % P;
      float acc = 0.0f;
#pragma unroll
      for (int cy = 0; cy < S; ++cy) acc += sw[ay * SP + cy] * t1[(cx * S + cy) * P + az];
      t2[i] = acc;
    }
    __syncthreads();
    for (int i = tr; i < P * P * P; i += NT) {
      const int ax = i / (P * P), ayz = i % (P * P);
      float acc = 0.0f;
#pragma unroll
      for (int cx = 0; cx < S; ++cx) acc += sw[ax * SP + cx] * t2[cx * P * P + ayz];
      tree.M[leaf * (P * P * P) + i] = tree.h3 * acc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (tr < S * S) {
      const int x = tr / S, y = tr % S;
      // kz = 2m: DFT_s of the row; kz = 2m + 1: DFT_s of the row times w^z
      float2 e[S], o[S];
#pragma unroll
      for (int q = 0; q < S / 4; ++q) {
        const float4 a = rowv[q];
        e[4 * q] = make_float2(a.x, 0.0f);
        e[4 * q + 1] = make_float2(a.y, 0.0f);
        e[4 * q + 2] = make_float2(a.z, 0.0f);
        e[4 * q + 3] = make_float2(a.w, 0.0f);
      }
#pragma unroll
      for (int z = 0; z < S; ++z) o[z] = twiddle<M, false>(e[z], z);
      dft<S, false>(e);
      dft<S, false>(o);
      float2* row = A + (x * S + y) * H;
#pragma unroll
      for (int m = 0; m < S / 2; ++m) {
        row[2 * m] = e[m];
        row[2 * m + 1] = o[m];
      }
      row[S] = e[S / 2];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < S * H; r += leaf_threads<S>()) {
      const int x = r / H, kz = r % H;
      float2 u[S];
#pragma unroll
      for (int y = 0; y < S; ++y) {
        u[y] = A[(x * S + y) * H + kz];
        if (h) u[y] = twiddle<M, false>(u[y], y);
      }
      dft<S, false>(u);
#pragma unroll
      for (int m = 0; m < S; ++m) A[(x * S + m) * H + kz] = u[m];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < S * H; r += leaf_threads<S>()) {
      const int m = r / H, kz = r % H;
      float2 e[S], o[S];
#pragma unroll
      for (int x = 0; x < S; ++x) {
        e[x] = A[(x * S + m) * H + kz];
        o[x] = twiddle<M, false>(e[x], x);
      }
      dft<S, false>(e);
      dft<S, false>(o);
      // frequency order (((j * 2 + parity) * s + m) * (s + 1) + kz) * 2 + kx % 2
      // (kx = 2j, 2j + 1; ky = 2m + parity): one 16-byte store writes both kx
#pragma unroll
      for (int j = 0; j < S; ++j)
        *reinterpret_cast<float4*>(rhat + chunk_addr(((2 * j + h) * S * H + r) * 2, leaf, nleaf)) =
            make_float4(e[j].x, e[j].y, o[j].x, o[j].y);
    }
    __syncthreads();
  }
}

// Inverse transform of one leaf's half spectrum (chunked layout), kept only
// at the s^3 target cells and written into the mesh: x and y passes keep s
// of the 2s outputs, v[x] = IDFT_s(Y_even)[x] + exp(2 pi i x / 2s) IDFT_s(Y_odd)[x];
// the z pass is the real inverse of the half spectrum,
//   v[z] = Re Y[0] + (-1)^z Re Y[s] + 2 sum_{0 < k < s} Re(Y[k] exp(2 pi i k z / 2s)),
// unnormalised (the kernels carry 1 / (2s)^3), done as one complex inverse
// DFT of length s whose real and imaginary parts are the even and odd z
// (the Hermitian half spectrum packed into s values).  One LDS buffer of s^2 (s + 1)
// values: per parity of ky the x pass fills it, then the thread of each
// (x, kz) column does that column's y pass; the first parity's result waits
// in the thread's registers, and the second parity's sum is written back over
// the column in place for the z pass.  Every pass has at most one task per
// thread (leaf_threads >= s (s + 1)).  The second parity's spectra are
// loaded as soon as the first parity's x pass has consumed its registers,
// so they arrive while the first parity's y pass runs.
//
// With P > 0 the leaf's L2P is added before the write (the far field
// sum_a A[ax][x] A[ay][y] A[az][z] P[a] of the leaf locals P, A as in the
// forward kernel): the locals are read at the start, and once the z pass
// has its spectra in registers the buffer holds the weights, the locals and
// their x contraction; each thread then contracts y and z for its row.
template <int S, int P = 0>
__global__ void __launch_bounds__(leaf_threads<S>()) k_leaf_inv(const float2* __restrict__ yhat, int N, int lgnb,
                                                        int64_t nleaf, float* __restrict__ out,
                                                        LeafTree tree) {
  constexpr int M = 2 * S, H = S + 1, NT = leaf_threads<S>();
  static_assert(NT >= S * H, "one column per thread");
  __shared__ float2 B[S * S * H];  // [x][m][kz], then [x][y][kz]
  const int64_t leaf = xcd_leaf(blockIdx.x, nleaf);
  const int msk = (1 << lgnb) - 1;
  const int bz = (int)(leaf & msk), by = (int)((leaf >> lgnb) & msk), bx = (int)(leaf >> (2 * lgnb));
  const int r = threadIdx.x;
  constexpr int P3 = P * P * P, NPL = P > 0 ? (P3 + NT - 1) / NT : 1;
  float loc[NPL];
  if constexpr (P > 0) {
#pragma unroll
    for (int j = 0; j < NPL; ++j)
      if (r + j * NT < P3) loc[j] = tree.Pl[leaf * P3 + r + j * NT];
  }
  float2 acc[S];
  float2 e[S], o[S];
  if (r < S * H) {
#pragma unroll
    for (int j = 0; j < S; ++j) {  // kx = 2j and 2j + 1 side by side: one 16-byte load
      const float4 q = *reinterpret_cast<const float4*>(yhat + chunk_addr((2 * j * S * H + r) * 2, leaf, nleaf));
      e[j] = make_float2(q.x, q.y);
      o[j] = make_float2(q.z, q.w);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (r < S * H) {
      const int m = r / H, kz = r % H;
      dft<S, true>(e);
      dft<S, true>(o);
#pragma unroll
      for (int x = 0; x < S; ++x) B[(x * S + m) * H + kz] = cadd(e[x], twiddle<M, true>(o[x], x));
      if (h == 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const float4 q =
              *reinterpret_cast<const float4*>(yhat + chunk_addr(((2 * j + 1) * S * H + r) * 2, leaf, nleaf));
          e[j] = make_float2(q.x, q.y);
          o[j] = make_float2(q.z, q.w);
        }
      }
    }
    __syncthreads();
    if (r < S * H) {
      const int x = r / H, kz = r % H;
      float2 v[S];
#pragma unroll
      for (int m = 0; m < S; ++m) v[m] = B[(x * S + m) * H + kz];
      dft<S, true>(v);
      if (h == 0) {
#pragma unroll
        for (int y = 0; y < S; ++y) acc[y] = v[y];
      } else {
#pragma unroll
        for (int y = 0; y < S; ++y) B[(x * S + y) * H + kz] = cadd(acc[y], twiddle<M, true>(v[y], y));
      }
    }
    __syncthreads();
  }
  float v[S];
  if (r < S * S) {
    float2 u[H];
#pragma unroll
    for (int k = 0; k < H; ++k) u[k] = B[r * H + k];
    // with X[k + s] = conj Y[s - k] and w = exp(2 pi i / 2s),
    // Z[k] = (Y[k] + X[k + s]) + i w^k (Y[k] - X[k + s]) has
    // IDFT_s(Z)[n] = v[2n] + i v[2n + 1]; n < s / 2 are the target cells
    float2 zz[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const float2 ys = make_float2(u[S - k].x, -u[S - k].y);
      const float2 e = cadd(u[k], ys);
      const float2 o = twiddle<M, true>(csub(u[k], ys), k);
      zz[k] = make_float2(e.x - o.y, e.y + o.x);
    }
    dft<S, true>(zz);
#pragma unroll
    for (int n = 0; n < S / 2; ++n) {
      v[2 * n] = zz[n].x;
      v[2 * n + 1] = zz[n].y;
    }
  }
  if constexpr (P > 0) {
    static_assert((P * S + P3 + S * P * P) * sizeof(float) <= sizeof(B), "L2P fits in the buffer");
    float* sw = reinterpret_cast<float*>(B);  // [a][c]
    float* sl = sw + P * S;                   // locals [ax][ay][az]
    float* su = sl + P3;                      // [x][ay][az]
    __syncthreads();  // every row of the buffer is in registers
    for (int i = r; i < P * S; i += NT) sw[i] = tree.A[i];
#pragma unroll
    for (int j = 0; j < NPL; ++j)
      if (r + j * NT < P3) sl[r + j * NT] = loc[j];
    __syncthreads();
    for (int i = r; i < S * P * P; i += NT) {
      const int x = i / (P * P), yz = i % (P * P);
      float a = 0.0f;
#pragma unroll
      for (int ax = 0; ax < P; ++ax) a += sw[ax * S + x] * sl[ax * P * P + yz];
      su[i] = a;
    }
    __syncthreads();
    if (r < S * S) {
      const int x = r / S, y = r % S;
      float t[P];
#pragma unroll
      for (int az = 0; az < P; ++az) {
        float a = 0.0f;
#pragma unroll
        for (int ay = 0; ay < P; ++ay) a += sw[ay * S + y] * su[(x * P + ay) * P + az];
        t[az] = a;
      }
#pragma unroll
      for (int z = 0; z < S; ++z) {
        float a = 0.0f;
#pragma unroll
        for (int az = 0; az < P; ++az) a += sw[az * S + z] * t[az];
        v[z] += a;
      }
    }
  }
  if (r < S * S) {
    const int x = r / S, y = r % S;
    float4* dst = reinterpret_cast<float4*>(
        out + ((int64_t)(bx * S + x) * N + (by * S + y)) * N + (int64_t)bz * S);
#pragma unroll
    for (int q = 0; q < S / 4; ++q) dst[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
}

// yhat_b(k) = sum_e khat_e(k) rhat_{b+e}(k).  A thread owns one frequency
// and a 2 x 2 block of pencils of leaves (bx, by), swept along z: the 4 x 4
// source columns around the block are each read once per z and serve all
// four targets (4 reads per output instead of 9), three z-planes of them in
// registers.  Each step first adds the lowest plane's terms, then reloads
// that plane's registers with the plane two above (in flight while the other
// two planes' terms are added), so three register sets rotate.  The
// thread's kernel values sit in its own slots of LDS (no barrier: only the
// writing thread reads them).  The pencil blocks of one frequency chunk go
// to one XCD (blocks are dealt to the 8 XCDs round robin), so its L2 serves
// the column re-reads between neighbouring blocks.
//
// The stencil is bound by its vector memory instructions (the texture
// units' address and data paths, not the bytes), so in the chunked layout
// every load and store moves 16 bytes per lane: lane l takes frequency
// 2 (l mod 32) + l / 32 of its chunk, a half-wave reads or writes one
// leaf's 64 frequencies, and a swap of values between the half-waves
// (v_permlane32_swap) gives each lane its frequency of two columns, or
// gathers two targets' outputs, per instruction.
//
// SYM = +1 (-1): the kernel is even (odd) in the cell separation, so the
// transform of neighbour -e is the conjugate (minus the conjugate) of that of
// e, and only the 14 kernels from the centre up in index order are kept in
// LDS (half the LDS per thread).  SYM = 0: all 27.
template <bool CHUNKED, bool ISO, int SYM = 0>
__global__ void __launch_bounds__(CHUNKED ? 64 : kThreads) k_near_mac(
    const float2* __restrict__ rhat, const float2* __restrict__ khat, int nb, int64_t F,
    int nchunk, float2* __restrict__ yhat) {
  constexpr bool isolated = ISO;  // sources outside the box are absent
  constexpr int W = CHUNKED ? 64 : kThreads;  // frequencies per block
  constexpr int NK = SYM ? 14 : 27;           // kernels kept
  __shared__ float2 kks[NK * W];
  const int g = blockIdx.x;
  const int hb = nb >> 1;
  const int np = hb * hb;  // 2 x 2 pencil blocks
  const int j = g >> 3;
  const int chunk = (j / np) * 8 + (g & 7);
  if (chunk >= nchunk) return;
  // chunked: lane l takes frequency 2 (l mod 32) + l / 32 of the chunk (the
  // even ones in the lower half-wave, the odd ones in the upper), which lets
  // one 16-byte load per lane serve two columns (see load_plane)
  const int phi = CHUNKED ? (int)(((threadIdx.x & 31) << 1) | (threadIdx.x >> 5)) : (int)threadIdx.x;
  const int64_t k = (int64_t)chunk * W + phi;
  if (k >= F) return;
  // this frequency of leaf l is at base[l * stride + lane] (leaves per axis
  // are a power of two, so wrapping is a mask).  In the chunked layout a
  // chunk's spectra of all leaves span nleaf * 512 bytes, so every access
  // goes through a buffer resource on the chunk with 32-bit offsets: no
  // per-lane 64-bit address arithmetic or registers holding the columns'
  // addresses.
  const int64_t nleaf = (int64_t)nb * nb * nb;
  const int64_t off = CHUNKED ? (int64_t)chunk * nleaf * 64 : (int64_t)chunk * W;
  const float2* __restrict__ base = rhat + off;
  float2* __restrict__ obase = yhat + off;
  const unsigned lane = threadIdx.x;
  const int stride = CHUNKED ? 64 : (int)F;
  const unsigned chunk_bytes = (unsigned)(nleaf * 64 * sizeof(float2));
  __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float2*>(base), (short)0, (int)chunk_bytes, kBufferDword3);
  __amdgpu_buffer_rsrc_t rout =
      __builtin_amdgcn_make_buffer_rsrc(obase, (short)0, (int)chunk_bytes, kBufferDword3);
  const int msk = nb - 1;
  const int blk = j % np;
  const int bx0 = 2 * (blk / hb), by0 = 2 * (blk % hb);
  float2* kk = kks + threadIdx.x;  // kernel e at kk[slot(e) * W]
  // e = (ex, ey, ez) in {0, 1, 2}^3 (offset e - 1), index 9 ex + 3 ey + ez;
  // its opposite is 26 - e.  With SYM the kernels e >= 13 sit at slot
  // e - 13 and e < 13 reads slot 13 - e (its opposite's) conjugated.
#pragma unroll
  for (int e = SYM ? 13 : 0; e < 27; ++e) kk[(SYM ? e - 13 : e) * W] = khat[(int64_t)e * F + k];
  // columns (bx0 - 1 + ix, by0 - 1 + iy), ix, iy in [0, 4), c = 4 ix + iy
  auto load = [&](int c, int z) -> float2 {
    const int sx = bx0 - 1 + c / 4, sy = by0 - 1 + c % 4;
    if (isolated && (z < 0 || z >= nb || sx < 0 || sx >= nb || sy < 0 || sy >= nb))
      return make_float2(0.0f, 0.0f);
    const int leaf = (((sx & msk) * nb + (sy & msk)) * nb) + (z & msk);
    if constexpr (CHUNKED) {
      return __builtin_bit_cast(
          float2, __builtin_amdgcn_raw_buffer_load_b64(rin, phi * 8, leaf * 512, 0));
    } else {
      return base[(int64_t)leaf * stride + lane];
    }
  };
  // a z-plane of the 16 columns.  Chunked: the lower half-wave loads column
  // c with 16 bytes per lane (frequencies 2j and 2j + 1 in lane j), the
  // upper half column c + 1; swapping the lower half's odd values with the
  // upper half's even ones leaves every lane its own frequency of both
  // columns, with half the load instructions of one 8-byte load per column.
  const unsigned hi = lane >> 5, lo16 = (lane & 31) * 16;
  auto load_plane = [&](float2 (&dst)[16], int z) {
    if constexpr (CHUNKED) {
#pragma unroll
      for (int c = 0; c < 16; c += 2) {
        const int sxa = bx0 - 1 + c / 4, sya = by0 - 1 + c % 4, syb = sya + 1;
        const int la = (((sxa & msk) * nb + (sya & msk)) * nb) + (z & msk);
        const int lb = (((sxa & msk) * nb + (syb & msk)) * nb) + (z & msk);
        v4u32 q = __builtin_amdgcn_raw_buffer_load_b128(rin, (unsigned)((hi ? lb : la) * 512) + lo16, 0, 0);
        if (isolated) {
          const bool zin = z >= 0 && z < nb && sxa >= 0 && sxa < nb;
          const bool ok = zin && (hi ? (syb >= 0 && syb < nb) : (sya >= 0 && sya < nb));
          if (!ok) q = v4u32{0u, 0u, 0u, 0u};
        }
        const auto sre = __builtin_amdgcn_permlane32_swap(q[0], q[2], false, false);
        const auto sim = __builtin_amdgcn_permlane32_swap(q[1], q[3], false, false);
        dst[c] = make_float2(__uint_as_float(sre[0]), __uint_as_float(sim[0]));
        dst[c + 1] = make_float2(__uint_as_float(sre[1]), __uint_as_float(sim[1]));
      }
    } else {
#pragma unroll
      for (int c = 0; c < 16; ++c) dst[c] = load(c, z);
    }
  };
  float2 r0[16], r1[16], r2[16];
  load_plane(r0, -1);
  load_plane(r1, 0);
  load_plane(r2, 1);
  // one complex multiply-add as four FMAs
  auto cmac = [](float& re, float& im, float2 kv, float2 sv) {
    re = fmaf(kv.x, sv.x, re);
    re = fmaf(-kv.y, sv.y, re);
    im = fmaf(kv.x, sv.y, im);
    im = fmaf(kv.y, sv.x, im);
  };
  // plane `ez` (0: z - 1, 1: z, 2: z + 1) of the four targets' sums
  auto plane = [&](float (&re)[4], float (&im)[4], const float2 (&zz)[16], int ez) {
    // the kernel values are read from LDS here, every time: an empty asm
    // statement with a memory clobber keeps the compiler from hoisting them
    // into registers for the whole sweep (it emits no instruction)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int ex = 0; ex < 3; ++ex)
#pragma unroll
      for (int ey = 0; ey < 3; ++ey) {
        const int e = ex * 9 + ey * 3 + ez;
        const bool kept = !SYM || e >= 13;
        float2 kv = kk[(SYM ? (kept ? e - 13 : 13 - e) : e) * W];
        if (!kept) kv = SYM > 0 ? make_float2(kv.x, -kv.y) : make_float2(-kv.x, kv.y);
#pragma unroll
        for (int tx = 0; tx < 2; ++tx)
#pragma unroll
          for (int ty = 0; ty < 2; ++ty)
            cmac(re[tx * 2 + ty], im[tx * 2 + ty], kv, zz[(tx + ex) * 4 + (ty + ey)]);
      }
  };
  // targets at z = bz: planes zm (bz - 1), z0 (bz), zp (bz + 1); zm is
  // reloaded with bz + 2 once its terms are in
  auto step = [&](int bz, float2 (&zm)[16], float2 (&z0)[16], float2 (&zp)[16]) {
    float re[4] = {0.0f, 0.0f, 0.0f, 0.0f}, im[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    plane(re, im, zm, 0);
    if (bz + 1 < nb) load_plane(zm, bz + 2);
    plane(re, im, z0, 1);
    plane(re, im, zp, 2);
#pragma unroll
    for (int tx = 0; tx < 2; ++tx) {
      if constexpr (CHUNKED) {
        // the two targets (tx, 0), (tx, 1) with one 16-byte store per lane:
        // after the swap the lower half-wave holds frequencies 2j, 2j + 1 of
        // the first, the upper half those of the second
        const int l0 = ((bx0 + tx) * nb + by0) * nb + bz, l1 = l0 + nb;
        const auto sre = __builtin_amdgcn_permlane32_swap(__float_as_uint(re[tx * 2]),
                                                          __float_as_uint(re[tx * 2 + 1]), false, false);
        const auto sim = __builtin_amdgcn_permlane32_swap(__float_as_uint(im[tx * 2]),
                                                          __float_as_uint(im[tx * 2 + 1]), false, false);
        const v4u32 q = {sre[0], sim[0], sre[1], sim[1]};
        __builtin_amdgcn_raw_buffer_store_b128(q, rout, (unsigned)((hi ? l1 : l0) * 512) + lo16, 0, 0);
      } else {
#pragma unroll
        for (int ty = 0; ty < 2; ++ty) {
          const int leaf = ((bx0 + tx) * nb + by0 + ty) * nb + bz;
          obase[(int64_t)leaf * stride + lane] = make_float2(re[tx * 2 + ty], im[tx * 2 + ty]);
        }
      }
    }
  };
  int bz = 0;
  for (; bz + 3 <= nb; bz += 3) {
    step(bz, r0, r1, r2);
    step(bz + 1, r1, r2, r0);
    step(bz + 2, r2, r0, r1);
  }
  if (bz < nb) step(bz, r0, r1, r2);
  if (bz + 1 < nb) step(bz + 1, r1, r2, r0);
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
  f->fused = s == 4 || s == 8 || s == 16;
  while ((1 << f->lgnb) < f->nb) ++f->lgnb;
  if ((1 << f->lgnb) != f->nb) f->fused = 0;
  hipError_t e = hipMalloc(&f->rhat, (size_t)(f->nleaf * f->F) * sizeof(float2));
  if (e == hipSuccess) e = hipMalloc(&f->yhat, (size_t)(f->nleaf * f->F) * sizeof(float2));
  if (e == hipSuccess && !f->fused) e = hipMalloc(&f->pad, (size_t)(f->nleaf * f->R) * sizeof(float));
  if (e == hipSuccess && !f->fused) {
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
      k_kdft_store<<<nblk(f->F), kThreads, 0, st>>>(f->dft[0], s, f->fused, sc,
                                                    f->khat[t] + (int64_t)ei * f->F);
      e = hipGetLastError();
    }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  // parity of each kernel: its neighbour -e is the conjugate (even kernel)
  // or minus the conjugate (odd) of neighbour e at every frequency, to FP32
  // rounding of the largest value
  std::vector<float2> h((size_t)27 * f->F);
  for (int t = 0; t < ntabs && e == hipSuccess; ++t) {
    e = hipMemcpy(h.data(), f->khat[t], h.size() * sizeof(float2), hipMemcpyDeviceToHost);
    if (e != hipSuccess) break;
    double big = 0.0, de = 0.0, dodd = 0.0;
    for (int ei = 0; ei < 27; ++ei)
      for (int64_t k = 0; k < f->F; ++k) {
        const float2 a = h[(size_t)ei * f->F + k], b = h[(size_t)(26 - ei) * f->F + k];
        big = std::max(big, (double)std::hypot(a.x, a.y));
        de = std::max(de, std::hypot((double)a.x - b.x, (double)a.y + b.y));
        dodd = std::max(dodd, std::hypot((double)a.x + b.x, (double)a.y - b.y));
      }
    f->sym[t] = de <= 1e-6 * big ? 1 : dodd <= 1e-6 * big ? -1 : 0;
  }
  return e;
}

int near_fft_fused(const NearFft* f) { return f->fused; }

int near_fft_kernels(const NearFft* f) {
  int n = 0;
  while (n < 4 && f->khat[n]) ++n;
  return n;
}

// Timer hooks that do nothing without a timer.
inline hipError_t tbegin(KernelTimer* kt, hipStream_t st) { return kt ? kt->begin(st) : hipSuccess; }
inline hipError_t tend(KernelTimer* kt, hipStream_t st, int part, hipError_t e) {
  if (e != hipSuccess || !kt) return e;
  return kt->end(st, part);
}

template <int S, int P>
hipError_t leaf_fwd(NearFft* f, const float* rho, const LeafTree& tree, hipStream_t st) {
  k_leaf_fwd<S, P><<<(unsigned)f->nleaf, leaf_threads<S>(), 0, st>>>(rho, f->N, f->lgnb, f->nleaf,
                                                                     f->rhat, tree);
  return hipGetLastError();
}

template <int S, int P>
hipError_t leaf_inv(NearFft* f, float* out, const LeafTree& tree, hipStream_t st) {
  k_leaf_inv<S, P><<<(unsigned)f->nleaf, leaf_threads<S>(), 0, st>>>(f->yhat, f->N, f->lgnb, f->nleaf,
                                                                     out, tree);
  return hipGetLastError();
}

// The fused leaf transforms at the plan's leaf edge, with the P2M or L2P of
// gridlet size p folded in (p = 0: none; p = 4 or 8 at s = 8, 16).
hipError_t fwd_any(NearFft* f, const float* rho, const LeafTree& tree, int p, hipStream_t st) {
  switch (f->s * 16 + p) {
    case 4 * 16: return leaf_fwd<4, 0>(f, rho, tree, st);
    case 8 * 16: return leaf_fwd<8, 0>(f, rho, tree, st);
    case 8 * 16 + 4: return leaf_fwd<8, 4>(f, rho, tree, st);
    case 8 * 16 + 8: return leaf_fwd<8, 8>(f, rho, tree, st);
    case 16 * 16: return leaf_fwd<16, 0>(f, rho, tree, st);
    case 16 * 16 + 4: return leaf_fwd<16, 4>(f, rho, tree, st);
    case 16 * 16 + 8: return leaf_fwd<16, 8>(f, rho, tree, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t inv_any(NearFft* f, float* out, const LeafTree& tree, int p, hipStream_t st) {
  switch (f->s * 16 + p) {
    case 4 * 16: return leaf_inv<4, 0>(f, out, tree, st);
    case 8 * 16: return leaf_inv<8, 0>(f, out, tree, st);
    case 8 * 16 + 4: return leaf_inv<8, 4>(f, out, tree, st);
    case 8 * 16 + 8: return leaf_inv<8, 8>(f, out, tree, st);
    case 16 * 16: return leaf_inv<16, 0>(f, out, tree, st);
    case 16 * 16 + 4: return leaf_inv<16, 4>(f, out, tree, st);
    case 16 * 16 + 8: return leaf_inv<16, 8>(f, out, tree, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool ISO>
hipError_t near_mac_iso(NearFft* f, int t, hipStream_t st) {
  const int nchunk = (int)(f->F / 64);
  const unsigned blocks = (unsigned)((int64_t)((nchunk + 7) / 8) * 8 * (f->nb / 2) * (f->nb / 2));
  if (f->sym[t] > 0)
    k_near_mac<true, ISO, 1><<<blocks, 64, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F, nchunk, f->yhat);
  else if (f->sym[t] < 0)
    k_near_mac<true, ISO, -1><<<blocks, 64, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F, nchunk, f->yhat);
  else
    k_near_mac<true, ISO, 0><<<blocks, 64, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F, nchunk, f->yhat);
  return hipGetLastError();
}

hipError_t near_mac(NearFft* f, int t, int isolated, hipStream_t st) {
  return isolated ? near_mac_iso<true>(f, t, st) : near_mac_iso<false>(f, t, st);
}

hipError_t run_fused(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                     hipStream_t st, KernelTimer* kt) {
  const LeafTree none{};
  hipError_t e = tbegin(kt, st);
  if (e == hipSuccess) e = tend(kt, st, 0, fwd_any(f, rho, none, 0, st));
  for (int t = 0; t < nout && e == hipSuccess; ++t) {
    e = tbegin(kt, st);
    if (e == hipSuccess) e = tend(kt, st, 1 + 2 * t, near_mac(f, t, isolated, st));
    if (e == hipSuccess) e = tbegin(kt, st);
    if (e == hipSuccess) e = tend(kt, st, 2 + 2 * t, inv_any(f, out[t], none, 0, st));
  }
  return e;
}

int near_fft_folds(const NearFft* f, int p) {
  return f->fused && (f->s == 8 || f->s == 16) && (p == 4 || p == 8);
}

hipError_t near_fft_begin(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                          const LeafTree& tree, hipEvent_t after_fwd, hipStream_t st,
                          KernelTimer* kt) {
  if (nout < 1 || nout > near_fft_kernels(f) || !near_fft_folds(f, tree.p) || !tree.A)
    return hipErrorInvalidValue;
  const LeafTree none{};
  hipError_t e = tbegin(kt, st);
  if (e == hipSuccess) e = tend(kt, st, 0, fwd_any(f, rho, tree, tree.M ? tree.p : 0, st));
  if (e == hipSuccess && after_fwd) e = hipEventRecord(after_fwd, st);
  for (int t = 1; t < nout && e == hipSuccess; ++t) {
    e = tbegin(kt, st);
    if (e == hipSuccess) e = tend(kt, st, 1 + 2 * t, near_mac(f, t, isolated, st));
    if (e == hipSuccess) e = tbegin(kt, st);
    if (e == hipSuccess) e = tend(kt, st, 2 + 2 * t, inv_any(f, out[t], none, 0, st));
  }
  if (e == hipSuccess) e = tbegin(kt, st);
  if (e == hipSuccess) e = tend(kt, st, 1, near_mac(f, 0, isolated, st));
  return e;
}

hipError_t near_fft_end(NearFft* f, float* out0, const LeafTree& tree, hipStream_t st,
                        KernelTimer* kt) {
  if (!near_fft_folds(f, tree.p) || !tree.A) return hipErrorInvalidValue;
  hipError_t e = tbegin(kt, st);
  if (e == hipSuccess) e = tend(kt, st, 2, inv_any(f, out0, tree, tree.Pl ? tree.p : 0, st));
  return e;
}

hipError_t near_fft_run(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                        hipStream_t st, KernelTimer* kt) {
  if (nout < 1 || nout > near_fft_kernels(f)) return hipErrorInvalidValue;
  if (f->fused) return run_fused(f, rho, out, nout, isolated, st, kt);
  const int64_t total = f->nleaf * f->R;
  hipError_t e = tbegin(kt, st);
  if (e != hipSuccess) return e;
  k_pack<<<nblk(total), kThreads, 0, st>>>(rho, f->N, f->s, f->nb, total, f->pad);
  e = hipGetLastError();
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->fwd, st));
  if (e == hipSuccess) e = fft_err(hipfftSetStream(f->inv, st));
  if (e == hipSuccess) e = fft_err(hipfftExecR2C(f->fwd, f->pad, (hipfftComplex*)f->rhat));
  e = tend(kt, st, 0, e);
  const int nchunk = (int)((f->F + kThreads - 1) / kThreads);
  const int64_t blocks = (int64_t)((nchunk + 7) / 8) * 8 * (f->nb / 2) * (f->nb / 2);
  const int64_t N3 = (int64_t)f->N * f->N * f->N;
  for (int t = 0; t < nout && e == hipSuccess; ++t) {
    e = tbegin(kt, st);
    if (e != hipSuccess) break;
    if (isolated)
      k_near_mac<false, true><<<(unsigned)blocks, kThreads, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F,
                                                                     nchunk, f->yhat);
    else
      k_near_mac<false, false><<<(unsigned)blocks, kThreads, 0, st>>>(f->rhat, f->khat[t], f->nb, f->F,
                                                                      nchunk, f->yhat);
    e = tend(kt, st, 1 + 2 * t, hipGetLastError());
    if (e == hipSuccess) e = tbegin(kt, st);
    if (e == hipSuccess) e = fft_err(hipfftExecC2R(f->inv, (hipfftComplex*)f->yhat, f->pad));
    if (e == hipSuccess) {
      k_unpack<<<nblk(N3), kThreads, 0, st>>>(f->pad, f->N, f->s, f->nb, 0, out[t]);
      e = tend(kt, st, 2 + 2 * t, hipGetLastError());
    }
  }
  return e;
}

}  // namespace pfmm
