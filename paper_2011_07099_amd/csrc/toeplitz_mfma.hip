// Block-Toeplitz operator for 8^3 blocks on the BF16 matrix cores with split
// precision: each operand is held as NT bf16 terms (x = x0 + x1 [+ x2]) and
// the products of terms whose combined order is below NT are accumulated in
// FP32 -- 3 MFMAs per product for NT = 2 (~2^-17 relative per product), 6 for
// NT = 3 (~2^-24, FP32 class).  It serves the interaction-zone convolution of
// Eq. 6 at p = 8 (blocks = gridlets; NT = 3, because the effective masses of
// a gridlet alternate in sign and cancel by 10^2-10^3 within a sum, and the
// downward interpolation amplifies the residue) and the leaf near zone
// (blocks = 8^3 cells; NT = 2).
//
// For one class of targets (same zone) and one offset d the operation is the
// GEMM  C[a][t] += sum_a' K_d[a][a'] X[t + d][a'],  a, a' in [0, 512),
// K_d[a][a'] = G((a - a' - 8 d) * spacing).  Mapping onto
// v_mfma_f32_32x32x16_bf16:
//   * M = output points a of a block (512 = 16 tiles of 32 rows: a tile is a
//     fixed x index, 4 y indices, all 8 z indices),
//   * N = targets (a workgroup holds 64 targets of one class, a 4x4x4 cube),
//   * K = source points a' (16 per step: a fixed x, 2 y, all 8 z indices).
// The A operand is never stored densely: a lane's 8 consecutive K entries
// are G at 8 consecutive z separations, read from a 15^3 window of the table
// around -8d that is kept in LDS z-reversed as packed (v, v+1) bf16 pairs, so
// every fragment is four aligned 32-bit LDS reads.  Sources are staged in LDS
// in chunks of 128 K entries, double-buffered with the windows.
#include "internal.h"

#include <cstdint>

namespace pfmm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWinPairs = 15 * 15 * 14;   // packed pairs per window term
constexpr int kWinPart = 3152;            // dwords per window term (padded to 16 B)
constexpr int kTN = 64;                   // targets per workgroup

__device__ inline uint16_t bf16_bits(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(uint16_t, b);
}
__device__ inline float bf16_float(uint16_t u) { return (float)__builtin_bit_cast(__bf16, u); }

__device__ inline void unpack_offset(int pk, int& dx, int& dy, int& dz) {
  dx = ((pk >> 16) & 255) - 128;
  dy = ((pk >> 8) & 255) - 128;
  dz = (pk & 255) - 128;
}

// Windows of an FP64 table (centre C, extent E per axis) for the 343 offsets
// d in [-3, 3]^3: slot = ((dx+3)*7 + (dy+3))*7 + (dz+3), nt terms per slot.
// Local indices jx, jy in [0, 15) stand for separations jx - 7 - 8 dx; z is
// reversed: local v stands for the z separation 7 - v - 8 dz.  Dword
// (jx, jy, v) of a term packs the bf16 values at v (low half) and v + 1 (high
// half), v in [0, 14).  Out-of-range windows (small tables) are zero; they
// are never used.
__global__ void k_make_windows(const double* __restrict__ tab, int C, int nt,
                               uint32_t* __restrict__ win) {
  const int slot = blockIdx.x;
  const int dx = slot / 49 - 3, dy = (slot / 7) % 7 - 3, dz = slot % 7 - 3;
  const int E = 2 * C + 1;
  uint32_t* w = win + (size_t)slot * nt * kWinPart;
  for (int i = threadIdx.x; i < nt * kWinPart; i += blockDim.x) {
    uint32_t out = 0;
    const int term = i / kWinPart, r = i % kWinPart;
    if (r < kWinPairs) {
      const int jx = r / (15 * 14), jy = (r / 14) % 15, v = r % 14;
      const int ix = jx - 7 - 8 * dx + C, iy = jy - 7 - 8 * dy + C;
      uint16_t h2[2];
      for (int e = 0; e < 2; ++e) {
        const int iz = 7 - (v + e) - 8 * dz + C;
        double x = 0.0;
        if (ix >= 0 && ix < E && iy >= 0 && iy < E && iz >= 0 && iz < E)
          x = tab[((size_t)ix * E + iy) * E + iz];
        uint16_t t = 0;
        for (int q = 0; q <= term; ++q) {  // residual splitting x = t0 + t1 + t2
          t = bf16_bits((float)x);
          x -= (double)bf16_float(t);
        }
        h2[e] = t;
      }
      out = (uint32_t)h2[0] | ((uint32_t)h2[1] << 16);
    }
    w[i] = out;
  }
}

// FP32 blocks [nodes][512] -> nt bf16 terms, term q at X + q * n.
__global__ void k_split_blocks(const float* __restrict__ X, uint16_t* __restrict__ out, int nt,
                               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x = X[i];
  for (int q = 0; q < nt; ++q) {
    const uint16_t t = bf16_bits(x);
    out[(int64_t)q * n + i] = t;
    x -= bf16_float(t);
  }
}

// Mesh [N]^3 (times scale) -> 8^3-cell sub-blocks [(N/8)^3][512], nt terms.
__global__ void k_split_mesh(const float* __restrict__ rho, float scale, int N, int nt,
                             uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n3 = (int64_t)N * N * N;
  if (i >= n3) return;
  const int z = (int)(i % N), y = (int)((i / N) % N), x = (int)(i / ((int64_t)N * N));
  const int nb = N / 8;
  const int64_t blk = ((int64_t)(x >> 3) * nb + (y >> 3)) * nb + (z >> 3);
  const int64_t o = blk * 512 + ((x & 7) * 64 + (y & 7) * 8 + (z & 7));
  float v = rho[i] * scale;
  for (int q = 0; q < nt; ++q) {
    const uint16_t t = bf16_bits(v);
    out[(int64_t)q * n3 + o] = t;
    v -= bf16_float(t);
  }
}

// Y[node][a] (+)= sum_g partial[g][node][a], groups summed in order.
__global__ void k_reduce_groups(const float* __restrict__ part, int groups, int64_t n,
                                float* __restrict__ Y, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = accumulate ? (double)Y[i] : 0.0;  // the group partials are added in FP64
  for (int g = 0; g < groups; ++g) s += (double)part[(int64_t)g * n + i];
  Y[i] = (float)s;
}

struct Tile {
  int tx, ty, tz;  // target node
};

__device__ inline Tile tile_target(int tile, int nt4, int cls, int m, int local) {
  // tile = 4x4x4 cube of class-lattice points; nt4 tiles per axis
  const int Tx = tile / (nt4 * nt4), Ty = (tile / nt4) % nt4, Tz = tile % nt4;
  const int kx = 4 * Tx + (local >> 4), ky = 4 * Ty + ((local >> 2) & 3), kz = 4 * Tz + (local & 3);
  const int cx = cls / (m * m), cy = (cls / m) % m, cz = cls % m;
  Tile t;
  t.tx = cx + m * kx;
  t.ty = cy + m * ky;
  t.tz = cz + m * kz;
  return t;
}

// Staged source rows hold KCH bf16 values as 16-byte slots, slot j of row r
// holding segment j ^ swz(r): 16 consecutive rows (the lanes of one B
// fragment read) then fall in distinct banks without row padding.
template <int NT>
__device__ inline int swz(int row) {
  return NT == 2 ? (row & 15) : ((row >> 1) & 7);
}

template <int NT>
struct SplitCfg {
  static constexpr int KCH = NT == 2 ? 128 : 64;              // source points per staged chunk
  static constexpr int AW = (NT * kWinPart + 255) / 256 * 256;  // staged window dwords
};

// LDS of one workgroup of the split kernel.  Operands go from global memory
// straight into LDS (global_load_lds), so the copies of the next chunk are in
// flight while this chunk's MFMAs run and hold no registers.  Each buffer is
// its own LDS object: the copies into one never alias the reads from the
// other.
#define PFMM_SPLIT_LDS(NT)                                                             \
  __shared__ __attribute__((aligned(16))) uint32_t Aw0[SplitCfg<NT>::AW];              \
  __shared__ __attribute__((aligned(16))) uint32_t Aw1[SplitCfg<NT>::AW];              \
  __shared__ __attribute__((aligned(16))) uint16_t Bs0[NT][kTN][SplitCfg<NT>::KCH];    \
  __shared__ __attribute__((aligned(16))) uint16_t Bs1[NT][kTN][SplitCfg<NT>::KCH];    \
  __shared__ int Os[kSplitMaxOffs]; /* the class's offsets (read by every copy) */

// One workgroup's share of the operator: 512 outputs x 64 targets (tile
// `lin` = class * tiles + tile) over offset group g.  Ends with a barrier, so
// the caller may reuse the LDS at once.
template <int NT>
__device__ __forceinline__ void split_tile(const ToepMfmaArgs& a, int lin, int g, uint32_t* Aw0,
                                           uint32_t* Aw1, uint16_t (*Bs0)[kTN][SplitCfg<NT>::KCH],
                                           uint16_t (*Bs1)[kTN][SplitCfg<NT>::KCH], int* Os) {
  constexpr int KCH = SplitCfg<NT>::KCH;
  constexpr int NCH = 512 / KCH;                 // chunks per offset (even)
  constexpr int SLOTS = KCH / 8;                 // 16-byte slots per staged row
  constexpr int RPI = 64 / SLOTS;                // rows per wave copy instruction
  constexpr int IPT = 16 / RPI;                  // copy instructions per term and wave
  constexpr int AW = SplitCfg<NT>::AW;
  constexpr int AI = AW / 256;                   // 1 KB window pieces

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, h = l >> 5, l32 = l & 31;
  const int m = a.m;
  const int nk = a.n / m;                    // class lattice points per axis
  const int nt4 = nk / 4;                    // tiles per axis
  const int tiles_per_class = nt4 * nt4 * nt4;
  const int cls = lin / tiles_per_class, tile = lin % tiles_per_class;

  const int ob = (a.noff * g) / a.groups, oe = (a.noff * (g + 1)) / a.groups;
  const int nmask = a.n - 1;
  const size_t nterm = (size_t)a.n * a.n * a.n * 512;  // stride between source terms
  for (int i = tid; i < a.noff; i += kThreads) Os[i] = a.offs[(size_t)cls * a.noff + i];
  __syncthreads();

  // copy map: instruction i of a term and wave covers rows 16w + RPI i ..
  // + RPI - 1; lane l takes row 16w + RPI i + l / SLOTS, slot l % SLOTS
  Tile st[IPT];
  int seg[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int row = 16 * w + RPI * i + l / SLOTS;
    st[i] = tile_target(tile, nt4, cls, m, row);
    seg[i] = (l % SLOTS) ^ swz<NT>(row);
  }

  typedef const void __attribute__((address_space(1)))* gptr;
  typedef void __attribute__((address_space(3)))* lptr;
  auto copy_A = [&](uint32_t* dst, int k) {
    int dx, dy, dz;
    unpack_offset(Os[k], dx, dy, dz);
    const int slot = ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3);
    const uint32_t* src = a.win + (size_t)slot * NT * kWinPart;
    for (int r = w; r < AI; r += 4)
      __builtin_amdgcn_global_load_lds((gptr)(src + 256 * r + 4 * l), (lptr)(dst + 256 * r), 16, 0,
                                       0);
  };
  auto copy_B = [&](uint16_t (*dst)[kTN][KCH], int k, int c) {
    int dx, dy, dz;
    unpack_offset(Os[k], dx, dy, dz);
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int ux0 = st[i].tx + dx, uy0 = st[i].ty + dy, uz0 = st[i].tz + dz;
      const bool inside = !a.isolated || ((unsigned)ux0 < (unsigned)a.n &&
                                          (unsigned)uy0 < (unsigned)a.n && (unsigned)uz0 < (unsigned)a.n);
      const int ux = ux0 & nmask, uy = uy0 & nmask, uz = uz0 & nmask;
      const uint16_t* src = a.X + (((size_t)ux * a.n + uy) * a.n + uz) * 512 + KCH * c + 8 * seg[i];
#pragma unroll
      for (int q = 0; q < NT; ++q)  // a source outside an isolated box is the zero block
        __builtin_amdgcn_global_load_lds((gptr)(inside ? src + q * nterm : a.zero + 8 * seg[i]),
                                         (lptr)&dst[q][16 * w + RPI * i][0], 16, 0, 0);
    }
  };

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // A addresses: for M-tile i and k-step s the window dword is
  //   ((ax - bx + 7) * 15 + (ay - by + 7)) * 14 + 7 - az
  // with ax = 2w + i/2, ay = 4(i%2) + l32/8, az = l32%8, bx = s/4,
  // by = 2(s%4) + h.  The lane part is one base; the rest is a constant.
  const int abase = (210 * (2 * w + 7) + 14 * ((l32 >> 3) + 7 - h) + 7 - (l32 & 7));
  // B rows: target 32j + l32; k offset 16 sl + 8h is segment 2 sl + h
  const int bswz = h ^ swz<NT>(l32);

  struct Frags {
    bf16x8 a[4][NT];
    bf16x8 b[NT][2];
  };
  auto load_a = [&](Frags& f, const uint32_t* Ak, int s) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const uint32_t* Aq = Ak + q * kWinPart + abase + 210 * (i >> 1) + 56 * (i & 1) -
                             210 * (s >> 2) - 28 * (s & 3);
        u32x4 u;
        u[0] = Aq[0];
        u[1] = Aq[2];
        u[2] = Aq[4];
        u[3] = Aq[6];
        f.a[i][q] = __builtin_bit_cast(bf16x8, u);
      }
  };
  auto load_b = [&](Frags& f, uint16_t (*Bb)[kTN][KCH], int sl) {
    const int slot = (2 * sl) ^ bswz;
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        f.b[q][j] = *reinterpret_cast<const bf16x8*>(&Bb[q][32 * j + l32][8 * slot]);
  };
  // products of terms (a term, b term), smallest first: the last three for
  // NT = 2, all six for NT = 3; an accumulator is revisited only after all 8
  // tiles, so consecutive MFMAs are independent
  constexpr int PA[6] = {2, 0, 1, 1, 0, 0};
  constexpr int PB[6] = {0, 2, 1, 0, 1, 0};
  auto mma = [&](const Frags& f) {
#pragma unroll
    for (int pr = (NT == 3 ? 0 : 3); pr < 6; ++pr)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[i][PA[pr]], f.b[PB[pr]][j],
                                                              acc[i][j], 0, 0, 0);
  };

  // one offset: NCH chunks; copies for the next chunk (and at the last chunk
  // the next offset's window) are issued before this chunk's MFMAs
  auto offset_step = [&](int k, const uint32_t* Ak, uint32_t* Anext) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const bool has_next = !(k == oe - 1 && c == NCH - 1);
      if (has_next) {
        if (c < NCH - 1) copy_B((c & 1) ? Bs0 : Bs1, k, c + 1);
        else copy_B(Bs0, k + 1, 0);  // NCH is even: chunk 0 uses Bs0
        if (c == NCH - 1) copy_A(Anext, k + 1);
      }
      // compiler-only fence (no instruction): memory operations stay on
      // their side, so the copies are issued here and not sunk to the end
      asm volatile("" ::: "memory");
      uint16_t (*Bb)[kTN][KCH] = (c & 1) ? Bs1 : Bs0;
      constexpr int KS = KCH / 16;  // k-steps per chunk
      Frags f[2];
      load_a(f[0], Ak, KS * c);
      load_b(f[0], Bb, 0);
#pragma unroll
      for (int sl = 0; sl < KS; ++sl) {
        if (sl + 1 < KS) {
          load_a(f[(sl + 1) & 1], Ak, KS * c + sl + 1);
          load_b(f[(sl + 1) & 1], Bb, sl + 1);
        }
        mma(f[sl & 1]);
      }
      __syncthreads();  // waits for this wave's copies, then for the others
    }
  };

  if (ob < oe) {
    copy_A(Aw0, ob);
    copy_B(Bs0, ob, 0);
    __syncthreads();
    for (int k = ob; k < oe; k += 2) {  // window buffers alternate by offset
      offset_step(k, Aw0, Aw1);
      if (k + 1 < oe) offset_step(k + 1, Aw1, Aw0);
    }
  }

  // epilogue: lane holds column l32 of each 32x32 tile, rows 8(v/4) + 4h + v%4
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const Tile t = tile_target(tile, nt4, cls, m, 32 * j + l32);
    const size_t node = ((size_t)t.tx * a.n + t.ty) * a.n + t.tz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int I = 4 * w + i;
      const int ax = I >> 1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ay = 4 * (I & 1) + q;
        const int az0 = 4 * h;
        float4 v = make_float4(acc[i][j][4 * q], acc[i][j][4 * q + 1], acc[i][j][4 * q + 2],
                               acc[i][j][4 * q + 3]);
        float* dst;
        if (a.partial) {
          dst = a.partial + ((size_t)g * a.n * a.n * a.n + node) * 512 + ax * 64 + ay * 8 + az0;
        } else if (a.grid_out) {
          const size_t NN = (size_t)a.n * 8;
          dst = a.Y + ((size_t)(t.tx * 8 + ax) * NN + (t.ty * 8 + ay)) * NN + (t.tz * 8 + az0);
        } else {
          dst = a.Y + node * 512 + ax * 64 + ay * 8 + az0;
        }
        float4* d4 = reinterpret_cast<float4*>(dst);
        if (a.accumulate && !a.partial) {
          const float4 o = *d4;
          v.x += o.x;
          v.y += o.y;
          v.z += o.z;
          v.w += o.w;
        }
        *d4 = v;
      }
    }
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(kThreads, 1) void k_toep8_split(ToepMfmaArgs a) {
  PFMM_SPLIT_LDS(NT)
  const int m = a.m;
  const int nt4 = a.n / m / 4;
  const int nblk = nt4 * nt4 * nt4 * m * m * m;
  // XCD-aware order: consecutive dispatch ids go to different XCDs, so give
  // each XCD a contiguous run of tiles (spatially close targets share sources)
  const int b = blockIdx.x;
  const int per = nblk / 8;
  const int lin = (nblk % 8 == 0) ? (b % 8) * per + b / 8 : b;
  split_tile<NT>(a, lin, blockIdx.y, Aw0, Aw1, Bs0, Bs1, Os);
}

// Persistent form for batches: workgroups take (field, tile) items from an
// atomic counter until the list is exhausted (every workgroup leaves through
// the same uniform test).  Items cover all offsets (one group).
template <int NT>
__global__ __launch_bounds__(kThreads, 1) void k_batch_split(const ToepMfmaArgs* __restrict__ args,
                                                             const MmaItem* __restrict__ items,
                                                             int nitems, unsigned* __restrict__ counter) {
  PFMM_SPLIT_LDS(NT)
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int idx = cur;
    __syncthreads();  // every thread has read `cur` before thread 0 overwrites it
    if (idx >= nitems) break;
    const MmaItem it = items[idx];
    const ToepMfmaArgs a = args[it.arg];
    split_tile<NT>(a, it.tile, 0, Aw0, Aw1, Bs0, Bs1, Os);
  }
}

// ---------------------------------------------------------------------------
// FP64 form on v_mfma_f64_16x16x4_f64 for the FP64 coarse levels (q = 8).
// Workgroup tile: 512 outputs x 16 consecutive targets of one class; wave w
// holds outputs [128 w, 128 w + 128) as 8 tiles of 16 rows (a tile: fixed x,
// 2 y, 8 z indices).  A k-step takes 4 consecutive sources a' (fixed x, y,
// 4 z indices).  The A operand is one double per lane from the offset's FP64
// window (15^3, double-buffered in LDS); the B operand one double per lane
// read from the L2-resident sources with a register prefetch of 8 k-steps.
// ---------------------------------------------------------------------------
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kW64 = 15 * 15 * 15;

// One workgroup's share: tile `blk` (= class * tiles + tile) over offset
// group g.  Ends with a barrier, so the caller may reuse the LDS at once.
__device__ __forceinline__ void f64_tile(const ToepF64Args& a, int blk, int g, double (*Wd)[kW64]) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int l16 = l & 15, kq = l >> 4;  // row / column within a tile, k lane group
  const int m = a.m, nk = a.n / m, ntarg = nk * nk * nk;
  const int tiles = (ntarg + 15) / 16;
  const int cls = blk / tiles, tile = blk % tiles;
  const int cx = cls / (m * m), cy = (cls / m) % m, cz = cls % m;
  const int ob = (a.noff * g) / a.groups, oe = (a.noff * (g + 1)) / a.groups;
  const int* offs = a.offs + (size_t)cls * a.noff;
  const int E = 2 * a.C + 1, nmask = a.n - 1;

  // this lane's target (B column / C column)
  const int tk = tile * 16 + l16;
  const bool tvalid = tk < ntarg;
  const int tkk = tvalid ? tk : 0;
  const int tx = cx + m * (tkk / (nk * nk)), ty = cy + m * ((tkk / nk) % nk), tz = cz + m * (tkk % nk);

  double rw[14];
  auto load_W = [&](int k) {
    const int pk = offs[k];
    const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
#pragma unroll
    for (int r = 0; r < 14; ++r) {
      const int i = tid + 256 * r;
      double v = 0.0;
      if (i < kW64) {
        const int jx = i / 225, jy = (i / 15) % 15, jz = i % 15;
        v = a.tab[((size_t)(jx - 7 - 8 * dx + a.C) * E + (jy - 7 - 8 * dy + a.C)) * E +
                  (jz - 7 - 8 * dz + a.C)];
      }
      rw[r] = v;
    }
  };
  auto store_W = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 14; ++r) {
      const int i = tid + 256 * r;
      if (i < kW64) Wd[buf][i] = rw[r];
    }
  };

  doublex4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = doublex4{0.0, 0.0, 0.0, 0.0};

  // A rows of tile i: ax = 2w + i/4, ay = 2(i%4) + l16/8, az = l16%8
  const int azl = l16 & 7, ayl = l16 >> 3;
  if (ob < oe) {
    load_W(ob);
    store_W(0);
    __syncthreads();
    for (int k = ob; k < oe; ++k) {
      const double* W = &Wd[(k - ob) & 1][0];
      const int pk = offs[k];
      const int dx = ((pk >> 16) & 255) - 128, dy = ((pk >> 8) & 255) - 128, dz = (pk & 255) - 128;
      const int ux0 = tx + dx, uy0 = ty + dy, uz0 = tz + dz;
      // a source outside an isolated box contributes nothing
      const bool use = tvalid && (!a.isolated || ((unsigned)ux0 < (unsigned)a.n &&
                                                  (unsigned)uy0 < (unsigned)a.n &&
                                                  (unsigned)uz0 < (unsigned)a.n));
      const int ux = ux0 & nmask, uy = uy0 & nmask, uz = uz0 & nmask;
      const double* X = a.X + (((size_t)ux * a.n + uy) * a.n + uz) * 512;
      const bool has_next = k + 1 < oe;
      if (has_next) load_W(k + 1);
      double b[8], bn[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = use ? X[4 * u + kq] : 0.0;
      for (int blk = 0; blk < 16; ++blk) {  // 16 blocks of 8 k-steps
        if (blk + 1 < 16) {
#pragma unroll
          for (int u = 0; u < 8; ++u) bn[u] = use ? X[32 * (blk + 1) + 4 * u + kq] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int s = 8 * blk + u;           // k-step: sources 4s .. 4s+3
          const int bx = s >> 4, by = (s >> 1) & 7, bz = 4 * (s & 1) + kq;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int ax = 2 * w + (i >> 2), ay = 2 * (i & 3) + ayl;
            const double av = W[((ax - bx + 7) * 15 + (ay - by + 7)) * 15 + (azl - bz + 7)];
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[u], acc[i], 0, 0, 0);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = bn[u];
      }
      if (has_next) store_W((k + 1 - ob) & 1);
      __syncthreads();
    }
  }
  // epilogue: lane holds rows kq + 4 v of each tile, column l16
  if (tvalid) {
    const size_t node = ((size_t)tx * a.n + ty) * a.n + tz;
    double* Y = a.partial ? a.partial + (size_t)g * a.n * a.n * a.n * 512 : a.Y;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double* d = Y + node * 512 + 128 * w + 16 * i + kq;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        d[4 * v] = (a.accumulate && !a.partial) ? d[4 * v] + acc[i][v] : acc[i][v];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256, 2) void k_toep8_f64(ToepF64Args a) {
  __shared__ double Wd[2][kW64];
  f64_tile(a, blockIdx.x, blockIdx.y, Wd);
}

// Persistent form for batches (as k_batch_split): items cover all offsets.
__global__ __launch_bounds__(256, 2) void k_batch_f64(const ToepF64Args* __restrict__ args,
                                                      const MmaItem* __restrict__ items, int nitems,
                                                      unsigned* __restrict__ counter) {
  __shared__ double Wd[2][kW64];
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int idx = cur;
    __syncthreads();  // every thread has read `cur` before thread 0 overwrites it
    if (idx >= nitems) break;
    const MmaItem it = items[idx];
    const ToepF64Args a = args[it.arg];
    f64_tile(a, it.tile, 0, Wd);
  }
}

__global__ void k_reset_counter(unsigned* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

template <class K>
int resident(K kernel) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

__global__ void k_reduce_f64(const double* __restrict__ part, int groups, int64_t n,
                             double* __restrict__ Y, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = accumulate ? Y[i] : 0.0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * n + i];
  Y[i] = s;
}

}  // namespace

int toep8_f64_tiles(int n, int m) {
  const int nk = n / m;
  return ((nk * nk * nk + 15) / 16) * m * m * m;
}

hipError_t launch_toep8_f64(const ToepF64Args& a, hipStream_t st) {
  if (a.groups < 1 || (a.groups > 1 && !a.partial) || a.C < 31) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_toep8_f64, dim3(toep8_f64_tiles(a.n, a.m), a.groups), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.partial) return e;
  const int64_t n = (int64_t)a.n * a.n * a.n * 512;
  hipLaunchKernelGGL(k_reduce_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a.partial,
                     a.groups, n, a.Y, a.accumulate);
  return hipGetLastError();
}

bool toep8_supported(int n, int m) {
  const int nk = n / m;
  return nk >= 4 && nk % 4 == 0;
}

hipError_t make_windows(const double* tab64, int C, int nt, uint32_t* win, hipStream_t st) {
  if (nt < 2 || nt > 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_make_windows, dim3(343), dim3(256), 0, st, tab64, C, nt, win);
  return hipGetLastError();
}

// (padded by 1 KB: the last window's staging copies whole 1 KB pieces)
size_t window_dwords(int nt) { return (size_t)343 * nt * kWinPart + 256; }

hipError_t split_blocks(const float* X, uint16_t* out, int nt, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_split_blocks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, out,
                     nt, n);
  return hipGetLastError();
}

hipError_t split_mesh(const float* rho, float scale, int N, int nt, uint16_t* out,
                      hipStream_t st) {
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_split_mesh, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, rho,
                     scale, N, nt, out);
  return hipGetLastError();
}

int toep8_split_tiles(int n, int m) {
  const int nt4 = n / m / 4;
  return nt4 * nt4 * nt4 * m * m * m;
}

int batch_mma_grid(int kind) {
  return kind == 2 ? resident(k_batch_split<2>) : kind == 3 ? resident(k_batch_split<3>)
                                                          : resident(k_batch_f64);
}

hipError_t launch_batch_mma(int kind, const void* args, const MmaItem* items, int nitems,
                            unsigned* counter, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grid > nitems) grid = nitems;
  if (grid <= 0) return hipSuccess;
  switch (kind) {
    case 2:
      hipLaunchKernelGGL(k_batch_split<2>, dim3(grid), dim3(kThreads), 0, st,
                         (const ToepMfmaArgs*)args, items, nitems, counter);
      break;
    case 3:
      hipLaunchKernelGGL(k_batch_split<3>, dim3(grid), dim3(kThreads), 0, st,
                         (const ToepMfmaArgs*)args, items, nitems, counter);
      break;
    case 64:
      hipLaunchKernelGGL(k_batch_f64, dim3(grid), dim3(kThreads), 0, st, (const ToepF64Args*)args,
                         items, nitems, counter);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_toep8_split(const ToepMfmaArgs& a, int nt, hipStream_t st) {
  if (!toep8_supported(a.n, a.m) || a.groups < 1 || nt < 2 || nt > 3 || a.noff > kSplitMaxOffs ||
      (a.isolated && !a.zero))
    return hipErrorInvalidValue;
  const int nt4 = a.n / a.m / 4;
  const int nblk = nt4 * nt4 * nt4 * a.m * a.m * a.m;
  if (nt == 2)
    hipLaunchKernelGGL(k_toep8_split<2>, dim3(nblk, a.groups), dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_toep8_split<3>, dim3(nblk, a.groups), dim3(kThreads), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.partial) return e;
  const int64_t n = (int64_t)a.n * a.n * a.n * 512;
  hipLaunchKernelGGL(k_reduce_groups, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     a.partial, a.groups, n, a.Y, a.accumulate);
  return hipGetLastError();
}

}  // namespace pfmm
