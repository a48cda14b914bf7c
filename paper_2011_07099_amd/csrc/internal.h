// Internal declarations of libpfmm: plan layout, kernel argument blocks and
// the host-side launchers of every device stage.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace pfmm {

// Workgroup index -> leaf, for kernels with one workgroup per leaf of the
// mesh.  Dispatch deals workgroups to the 8 XCDs in turn; this gives each XCD
// a contiguous range of leaves, so the leaves it runs one after another are
// neighbours along z, whose mesh rows (s floats each) share 128-byte lines:
// the second half of a line then comes from that XCD's L2 instead of HBM.
__device__ __forceinline__ int64_t xcd_leaf(int64_t i, int64_t n) {
  return (n & 7) ? i : (i & 7) * (n >> 3) + (i >> 3);
}

// Optional timing of a routine's kernels: begin() before and end(part) after
// its part-th kernel (or group of kernels), on the stream it launches on.
// A null timer times nothing.
struct KernelTimer {
  virtual hipError_t begin(hipStream_t s) = 0;
  virtual hipError_t end(hipStream_t s, int part) = 0;
  virtual ~KernelTimer() = default;
};

// ---------------------------------------------------------------------------
// Green's function tabulation (FP64, plan time)
// ---------------------------------------------------------------------------
enum GreenKind {
  GK_X = 0, GK_K = 1, GK_S1 = 2, GK_S = 3, GK_E = 4,  // as pfmm_green
  GK_N = 5                                             // free space, no wrap (isolated twin)
};

// A Green's function and its parameters: a1, a2 of G_S; the splitting radius
// rs of G_E.
struct GreenSpec {
  int kind;
  double a1, a2, rs;
};

// Tabulate G(eta * j) for j in [-C, C]^3 into dst[(2C+1)^3] (FP64, C order),
// eta = 1 / den.  `self_h` > 0 gives the value at j = 0 for the real-space
// kinds (potential at the centre of a uniform cube cell of side self_h);
// self_h == 0 leaves 0 there.  `N` is the mesh size (frequency range of G_K
// and of the Fourier part of G_E).  G_K and G_E allocate and free their own
// temporaries and synchronise `st`.
hipError_t tabulate_green(const GreenSpec& g, int N, int C, int64_t den, double self_h,
                          double* dst, hipStream_t st);
// The same without allocating or synchronising: the Fourier kinds (G_K, G_E)
// keep their partial sums in the caller's workspace `ws` of
// tabulate_workspace_doubles(kind, N, C) doubles (0 for the real-space kinds).
size_t tabulate_workspace_doubles(int kind, int N, int C);
hipError_t tabulate_green_ws(const GreenSpec& g, int N, int C, int64_t den, double self_h,
                             double* dst, double* ws, hipStream_t st);

// Near-zone acceleration tables d[i][j] = -(4th-order central difference of the
// lattice G along axis i at j) for j in [-C, C]^3, i = x, y, z (FP64, device).
// Allocates and frees a temporary table; synchronises `st`.
hipError_t tabulate_accel(const GreenSpec& g, int N, int C, double* d[3], hipStream_t st);
// FP64 -> FP32 copy.
hipError_t cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// Block-Toeplitz operator: Y[t] (+)= sum_{d in D(class(t))} K_d X[(t+d) mod n]
// with K_d[a, a'] = tab[a - a' - q d] (target minus source), blocks of q^3 points.  Used for the
// interaction-zone convolution (Eq. 6; blocks = gridlets) and for the near
// zone (blocks = leaf cells or sub-blocks of them).
// ---------------------------------------------------------------------------
struct ToepArgs {
  int n;            // nodes per axis at this level (power of two)
  int m;            // classes per axis: targets with t mod m == c share D(c)
  int q;            // block edge
  int noff;         // offsets per class
  const int* offs;  // [m^3][noff] packed offsets (see pack_offset)
  const void* tab;  // table (float or double), extent E = 2C+1 per axis, centre C
  int C;
  const void* X;    // sources: blocks [n^3][q^3] or (grid_in) mesh [nq]^3
  void* Y;          // outputs: blocks or (grid_out) mesh
  int grid_in, grid_out;
  double xscale;    // sources are multiplied by this (h^3: density -> mass)
  int accumulate;   // 0: overwrite Y, 1: add to Y
  int fp64;         // 0: FP32 tab/X/Y, 1: FP64 tab/X/Y
  int groups;       // >1: offsets split over workgroups writing `partial`
  void* partial;    // [groups][n^3][q^3] (block layout only), summed in order
  int isolated;     // 1: no periodic images, sources outside [0, n)^3 are zero
  int mesh64;       // grid_in / grid_out mesh arrays hold doubles (fp64 only); else floats
};

// Workgroups of one launch of the portable kernel (before offset groups).
int toeplitz_workgroups(int q, int fp64, int n, int m);

inline int pack_offset(int dx, int dy, int dz) {
  return ((dx + 128) & 255) << 16 | ((dy + 128) & 255) << 8 | ((dz + 128) & 255);
}

hipError_t launch_toeplitz(const ToepArgs& a, hipStream_t st);

// ---------------------------------------------------------------------------
// Split-precision block-Toeplitz operator on the BF16 matrix cores for 8^3
// blocks (toeplitz_mfma.hip).  Operands are held as nt in {2, 3} bf16 terms.
// Windows of a table are precomputed per offset in [-3, 3]^3
// (window_dwords(nt) uint32 per table); sources are nt term arrays
// [n^3][512] laid out one after another in X.  `groups` > 1 splits each
// class's offsets over workgroups that write `partial` [groups][n^3][512],
// summed in order into Y.
// ---------------------------------------------------------------------------
struct ToepMfmaArgs {
  int n, m, noff;
  const int* offs;
  const uint32_t* win;
  const uint16_t* X;
  float* Y;
  int grid_out;
  int accumulate;
  int groups;
  float* partial;
  int isolated;          // 1: sources outside the box are zero (read from `zero`)
  const uint16_t* zero;  // >= 512 zero bf16 values (isolated only)
};
// Most offsets per class the split kernel stages (the near zone at m = 2).
constexpr int kSplitMaxOffs = 216;
bool toep8_supported(int n, int m);
size_t window_dwords(int nt);
hipError_t make_windows(const double* tab64, int C, int nt, uint32_t* win, hipStream_t st);
hipError_t split_blocks(const float* X, uint16_t* out, int nt, int64_t n, hipStream_t st);
hipError_t split_mesh(const float* rho, float scale, int N, int nt, uint16_t* out,
                      hipStream_t st);
hipError_t launch_toep8_split(const ToepMfmaArgs& a, int nt, hipStream_t st);

// FP64 form on the matrix cores for the FP64 coarse levels (q = 8): FP64
// table (centre C >= 31), FP64 sources and outputs [n^3][512].
struct ToepF64Args {
  int n, m, noff;
  const int* offs;
  const double* tab;
  int C;
  const double* X;
  double* Y;
  int accumulate;
  int groups;
  double* partial;  // [groups][n^3][512] when groups > 1
  int isolated;     // 1: sources outside the box are zero
};
int toep8_f64_tiles(int n, int m);
hipError_t launch_toep8_f64(const ToepF64Args& a, hipStream_t st);

// ---------------------------------------------------------------------------
// Batches of independent fields (batch.hip): one work item = one tile of
// targets of one class of one interaction-zone level or near zone of one
// field, all offsets of its zone, FP32 or FP64 operands (block edge q <= 8).
// ---------------------------------------------------------------------------
struct BatchItem {
  const void* tab;  // float or (fp64) double table
  const void* X;    // float or (fp64) double sources
  void* Y;          // float or (fp64) double outputs
  const int* offs;
  int n, m, q, C, noff, cls, t0, grid;
  float xscale;
  int fp64;         // FP64 operands: tile width 1, FP64 sums
  int tpt;          // FP32 tile width (targets per thread): 1, 2 or 4
};
int batch_targets_per_item(int q, int tpt, int fp64);

// Matrix-core items of a batch (toeplitz_mfma.hip): one item = one workgroup
// tile of one contraction, all offsets; `arg` indexes a device array of
// ToepMfmaArgs (kind 2: split near zone, 3: split interaction zone) or
// ToepF64Args (kind 64).  Groups and partial sums are not used (groups = 1).
struct MmaItem {
  int arg, tile;
};
int toep8_split_tiles(int n, int m);  // tiles (workgroups) of one split launch
int batch_mma_grid(int kind);         // resident workgroups of a persistent kind
hipError_t launch_batch_mma(int kind, const void* args, const MmaItem* items, int nitems,
                            unsigned* counter, int grid, hipStream_t st);
int batch_resident_grid();
hipError_t launch_batch_toeplitz(const BatchItem* items, int nitems, unsigned* counter, int grid,
                                 hipStream_t st);

// ---------------------------------------------------------------------------
// Learned correction of the interaction-zone tables (learned.hip)
// ---------------------------------------------------------------------------
constexpr int kMlpIn = 8;          // network inputs per table entry
constexpr int kMlpParams = 4801;  // 8 -> 64 -> 64 -> 1
hipError_t mlp_forward(const float* theta, const float* feats, int n, int bf16, float* delta,
                       hipStream_t st);
hipError_t apply_correction(const double* g0, const float* delta, const int* uidx, int64_t n,
                            double* t64, float* t32, hipStream_t st);
hipError_t residual(const float* phi, const float* t, int64_t n, double* part, double* stats,
                    float* r, hipStream_t st);
size_t table_grad_partial_doubles(int m, int q, int noff);
hipError_t table_grad(int n, int m, int q, int noff, const int* offs, const void* lam,
                      const void* M, int fp64, int C, double* part, double* g, hipStream_t st);
hipError_t orbit_gather(const double* g, const double* g0, const int* ptr, const int* pos, int nu,
                        float* ddelta, hipStream_t st);
size_t mlp_backward_partial_floats(int n);
hipError_t mlp_backward(const float* theta, const float* feats, const float* ddelta, int n,
                        float* part, float* grad, hipStream_t st);
hipError_t adam_step(float* theta, float* m1, float* m2, float* grad, int n, float count,
                     float lr, int step, hipStream_t st);
// dst[i] += src[i], i < n
hipError_t add_into(float* dst, const float* src, int n, hipStream_t st);

// ---------------------------------------------------------------------------
// G_* as one grid-valued function on the whole mesh (gstar.hip)
// ---------------------------------------------------------------------------
int gstar_orbit(int x, int y, int z, int N);  // orbit of a mesh separation
int gstar_orbits(int N);                      // number of orbits
struct GStarFft;
hipError_t gstar_fft_create(int N, GStarFft** out);
void gstar_fft_destroy(GStarFft* f);
// near-zone table gradient (FP64 per entry of the (4s-1)^3 table)
hipError_t gstar_near_grad(const float* r, const float* rho, int N, int s, double h3, double* g,
                           hipStream_t st);
// N^3 sum_t q_t rho(t - x) with q = r + 2 (loss / B)(t - mean t), stats as residual()'s
hipError_t gstar_pm_corr(GStarFft* f, const float* r, const float* t, const float* rho,
                         const double* stats, double* corr, hipStream_t st);
// scale times a centred table (extent C >= N/2) at every mesh point, FP64
hipError_t gstar_mesh_values(const double* tab, int C, int N, double scale, double* out,
                             hipStream_t st);

// ---------------------------------------------------------------------------
// Upward / downward passes (tensor products of 1D Lagrange operators).
// Gridlet buffers are FP32 or FP64 per level; `*64` flags give the type of
// each operand (0 = float, 1 = double).  Weights are passed in both types.
// ---------------------------------------------------------------------------
struct Weights {
  const float* f;
  const double* d;
};
// P2M: M[b][a] = h3 * sum_c A[ax][cx] A[ay][cy] A[az][cz] rho[b s + c]
hipError_t launch_p2m(const float* rho, void* M, int m64, Weights A, int N, int s, int p,
                      double h3, hipStream_t st);
// M2M (Eq. 5): Mp[B][a] = sum_o sum_a' T_o(x)T_o(x)T_o [a][a'] Mc[2B+o][a']
hipError_t launch_m2m(const void* Mc, int c64, void* Mp, int p64, Weights T, int nparent, int p,
                      hipStream_t st);
// L2L (Eq. 7): Pc[2B+o][a'] (+)= sum_a T_o[ax][a'x] T_o[ay][a'y] T_o[az][a'z] Pp[B][a]
hipError_t launch_l2l(const void* Pp, int p64, void* Pc, int c64, Weights T, int nparent, int p,
                      hipStream_t st, int accumulate = 0);
// L2P: phi[b s + c] (+)= sum_a A[ax][cx] A[ay][cy] A[az][cz] P[b][a]
hipError_t launch_l2p(const void* P, int p64, float* phi, Weights A, int N, int s, int p,
                      hipStream_t st, int accumulate = 0);
// acc[c][b s + cell] += scale sum_a (A or Ad per axis) P[b][a], c = x, y, z:
// the gradient of the leaf's local expansion times `scale`, with Ad the
// derivative of the 1D interpolation weights, on axis c.
hipError_t launch_l2p_grad(const void* P, int p64, float* acc, Weights A, Weights Ad,
                           double scale, int N, int s, int p, hipStream_t st);
// a = -grad(phi), periodic 4th-order central differences.
hipError_t launch_fd4(const float* phi, float* acc, int N, hipStream_t st);
// The same three steps with an FP64 mesh (density in, or potential and
// accelerations out) and FP64 gridlets: the PFMM_PREC_FP64 solve with FP64
// buffers.
hipError_t launch_p2m_f64in(const double* rho, void* M, Weights A, int N, int s, int p, double h3,
                            hipStream_t st);
hipError_t launch_l2p_f64out(const void* P, double* phi, Weights A, int N, int s, int p,
                             hipStream_t st, int accumulate = 0);
hipError_t launch_l2p_grad_f64out(const void* P, double* acc, Weights A, Weights Ad, double scale,
                                  int N, int s, int p, hipStream_t st);
hipError_t launch_fd4_f64(const double* phi, double* acc, int N, hipStream_t st);
// ---------------------------------------------------------------------------
// Interaction zones by FFT convolution (the HPM comparator)
// ---------------------------------------------------------------------------
struct M2LFft;
// Plans for levels 2 .. L at gridlet size p, batches of targets sized so that
// their grids take at most `budget_bytes`; allocates.
hipError_t m2l_fft_create(int L, int p, size_t budget_bytes, M2LFft** out);
void m2l_fft_destroy(M2LFft* f);
// Transform the kernels G(eta_l w) of every level from the FP64 level tables;
// synchronises `st`.
hipError_t m2l_fft_tables(M2LFft* f, const std::vector<double*>& tab64, hipStream_t st);
// Pl (+)= the level-l interaction-zone sums of the masses Ml (FP64 buffers
// and transforms when fp64, else FP32).
hipError_t m2l_fft_level(M2LFft* f, int l, const void* Ml, void* Pl, int fp64, int accumulate,
                         hipStream_t st);

// ---------------------------------------------------------------------------
// Leaf near zone by FFT convolution on the doubled grid (Sec. 2-3)
// ---------------------------------------------------------------------------
struct NearFft;
// P2M and L2P folded into the leaf transforms of the potential (library
// kernels, FP32 leaf gridlets of p^3 values in leaf order, p = 4 or 8): the
// forward transform writes M = P2M(rho), the inverse adds L2P(Pl).  A null
// M or Pl leaves that step out.
struct LeafTree {
  float* M = nullptr;         // leaf gridlet masses out (P2M, times h3)
  const float* Pl = nullptr;  // leaf locals in (L2P)
  const float* A = nullptr;   // weights A[a][c], p x s (gridlet node a, cell c)
  float h3 = 0.0f;            // cell volume
  int p = 0;                  // gridlet size
};
// Plans and buffers for N^3 cells in leaves of s^3 (about 100 bytes per cell);
// allocates.
hipError_t near_fft_create(int N, int s, NearFft** out);
void near_fft_destroy(NearFft* f);
// Transform the near-zone kernels of `ntabs` (1 .. 4) FP64 tables (centred,
// edge 4s - 1, indexed by target minus source cell) times `scale`; allocates
// the kernels on first use and synchronises `st`.
hipError_t near_fft_tables(NearFft* f, const double* const* tabs, int ntabs, double scale,
                           hipStream_t st);
// Kernels transformed so far.
int near_fft_kernels(const NearFft* f);
// 1 when the leaf transforms are the library's own kernels (s = 4, 8, 16),
// 0 when they go through rocFFT.
int near_fft_fused(const NearFft* f);
// out[t] = the near zone of rho with kernel t, t < nout (written, not added);
// isolated: sources outside the box are absent instead of periodic images.
// Parts for a timer: 0 the forward transforms, then per kernel t the
// stencil (1 + 2t) and the inverse transform (2 + 2t).
hipError_t near_fft_run(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                        hipStream_t st, KernelTimer* kt = nullptr);
// 1 when the transforms can fold the P2M and L2P of gridlet size p.
int near_fft_folds(const NearFft* f, int p);
// near_fft_run in two halves around the tree, P2M and L2P folded in (see
// LeafTree): near_fft_begin runs the forward transforms with P2M into
// tree.M (then records `after_fwd` when given: the leaf masses are ready),
// the stencils and inverses of outputs 1 .. nout - 1, and the stencil of
// output 0; near_fft_end, once tree.Pl holds the leaf locals, the inverse
// transform of output 0 with L2P added.  Timer parts as near_fft_run.
hipError_t near_fft_begin(NearFft* f, const float* rho, float* const* out, int nout, int isolated,
                          const LeafTree& tree, hipEvent_t after_fwd, hipStream_t st,
                          KernelTimer* kt = nullptr);
hipError_t near_fft_end(NearFft* f, float* out0, const LeafTree& tree, hipStream_t st,
                        KernelTimer* kt = nullptr);

// ---------------------------------------------------------------------------
// Interaction zones as spectral stencils (per-node transforms, FP64)
// ---------------------------------------------------------------------------
struct M2LSpectral;
// Buffers for levels 2 .. L at gridlet size p (4 or 8); allocates.
hipError_t m2l_spectral_create(int L, int p, M2LSpectral** out);
void m2l_spectral_destroy(M2LSpectral* f);
// Transform the kernels of every offset in [-3, 3]^3 from the FP64 level
// tables; synchronises `st`.
hipError_t m2l_spectral_tables(M2LSpectral* f, const std::vector<double*>& tab64, hipStream_t st);
// on = 1: the 16^3 leaf level's stencil (L = 4) sums each zone column in
// FP32 (FP32 sources and kernel values) and the column sums in FP64.
void m2l_spectral_set_f32(M2LSpectral* f, int on);
// Pl (+)= the level-l zone sums of Ml over `offs` (noff per class: 8 classes
// at levels >= 3, one at level 2); m64 / p64: the buffers hold doubles.
// Parts for a timer: 0 the node transforms, 1 the stencil, 2 the inverse.
hipError_t m2l_spectral_level(M2LSpectral* f, int l, const void* Ml, int m64, void* Pl, int p64,
                              int accumulate, const int* offs, int noff, int isolated, hipStream_t st,
                              KernelTimer* kt = nullptr);

// FP64 -> FP32 copy of n elements.
hipError_t launch_cast_d2f(const double* src, float* dst, int64_t n, hipStream_t st);

// What the direct periodic convolution of a plan needs (plan.hip): mesh
// size, G and stream.  Returns 0 (PFMM_OK), or a status with the message set.
struct DirectSpec {
  int N;
  int isolated;
  GreenSpec green;
  hipStream_t stream;
};
int plan_direct_spec(const void* plan, DirectSpec* out);
// Set the calling thread's message for pfmm_last_error and return `status`.
int set_error(int status, const std::string& msg);
void clear_error();

}  // namespace pfmm
