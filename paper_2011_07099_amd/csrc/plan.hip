// C ABI of libpfmm (declared in include/pfmm.h): plan creation, options and
// the solve sequence of the natively periodic FMM (Sec. 2, Eqs. 5-7).
//
// Solve sequence, all on the plan's stream, nothing allocated:
//   1. P2M at the leaves (level L): cell masses -> leaf gridlets.
//   2. M2M (Eq. 5) for levels L-1 .. 2.
//   3. Level 2: interaction zone = the 37 non-neighbour nodes of the periodic
//      4^3 level, each once, with the periodic G (Eq. 6).
//   4. Levels 3 .. L: L2L (Eq. 7) of the parent's field, then the 189-node
//      interaction zone of the node's parity class (Sec. 2, Fig. 2).
//   5. L2P at the leaves, then the direct near zone (27 leaves) added on the
//      mesh.  A leaf wider than 8 cells is cut into sub-blocks of 8^3 cells;
//      the 27 neighbouring leaves of a sub-block are then the (3m)^3
//      sub-blocks around its leaf, m = s/8, and depend on the sub-block's
//      position in its leaf.
//   6. Optionally a = -grad(phi) by 4th-order differences (Sec. 3).
#include "../../include/pfmm.h"
#include "internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

using namespace pfmm;

struct pfmm_plan_s {
  int N = 0, L = 0, p = 0, s = 0, green = 0, prec = PFMM_PREC_FP32;
  double a1 = -0.125;
  double a2 = 0.0;
  double rs = 0.1;  // G_E splitting radius
  hipStream_t stream = nullptr;
  // The near zone runs on `side` while the tree runs on `stream` (fork and
  // join by events), except when profiling
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // with P2M and L2P folded into the near zone's leaf transforms: the leaf
  // masses are ready (side -> stream), the leaf locals are ready (stream -> side)
  hipEvent_t ev_mass = nullptr, ev_local = nullptr;
  int qn = 0, mn = 0;  // near-zone block edge and classes per axis
  float* dA = nullptr;  // [p][s] P2M / L2P weights
  float* dT = nullptr;  // [2][p][p] M2M / L2L weights
  double* dA64 = nullptr;
  double* dT64 = nullptr;
  float* dAd = nullptr;   // [p][s] derivative of the L2P weights
  double* dAd64 = nullptr;
  int fp64_levels = 2;            // levels 2 .. 1+fp64_levels kept in FP64 (default max(2, L-2))
  int learned_kind = 0;           // created as PFMM_GREEN_LEARNED (G_S1 tables plus a network)
  int batch_refs = 0;             // live batches bound to this plan (its buffers are in their graphs)
  std::vector<void*> M, P;        // gridlet masses / potentials per level
  std::vector<double*> tab64;     // per level, (8p-1)^3
  std::vector<float*> tab32;
  double* ntab64 = nullptr;       // near, (4s-1)^3
  float* ntab32 = nullptr;
  int* offs_l2 = nullptr;         // [37] periodic, [316] isolated (capacity 316)
  int nl2 = 37;                   // level-2 offsets in use
  int isolated = 0;               // no periodic images (PFMM_OPT_ISOLATED)
  int m2l_fft = 0;                // interaction zones by FFT convolution (PFMM_OPT_M2L)
  M2LFft* fft = nullptr;          // its plans, grids and transformed kernels
  int m2l_spectral = 0;           // interaction zones as spectral stencils (PFMM_OPT_M2L)
  M2LSpectral* mspec = nullptr;   // its spectra and transformed kernels
  int near_fft = 0;               // leaf near zone by FFT convolution (PFMM_OPT_NEAR)
  int fold = 0;                   // P2M and L2P inside its leaf transforms (PFMM_OPT_FOLD)
  int zones_f32 = 0;              // FP32 columns in the 16^3 spectral stencil (PFMM_OPT_ZONES_FP32)
  NearFft* nfft = nullptr;        // its plans, buffers and transformed kernels
  uint16_t* zero = nullptr;       // 512 zero bf16 values: the source outside an isolated box
  // accelerations from the expansion (PFMM_OPT_ACCEL; tables on first use)
  int accel_mode = 0;
  double* ndtab64[3] = {nullptr, nullptr, nullptr};  // near acceleration kernels, (4s-1)^3
  float* ndtab32[3] = {nullptr, nullptr, nullptr};
  uint32_t* ndwin[3] = {nullptr, nullptr, nullptr};  // their windows (split near zone)
  int* offs_iz = nullptr;         // [8][189]
  int* offs_near = nullptr;       // [mn^3][(3 mn)^3]
  // split-precision matrix-core path (8^3 blocks)
  std::vector<uint32_t*> win;     // per level: table windows (p == 8)
  uint32_t* nwin = nullptr;       // near-table windows (8^3-cell sub-blocks)
  uint16_t* xs = nullptr;         // bf16 gridlet-mass terms (3 arrays of xwords)
  size_t xwords = 0;
  uint16_t* xsn = nullptr;        // bf16 density terms in sub-blocks (2 arrays of N^3)
  float* part = nullptr;          // split-offset partial sums (matrix-core path)
  size_t part_floats = 0;
  void* spart = nullptr;          // split-offset partial sums (portable kernel)
  // learned correction of the interaction-zone tables (allocated on first use)
  int learned = 0;                // 0 none, 1 network inference, 2 network training,
                                  // 3 grid-valued tables (parameters = delta)
  int nu = 0;                     // unique (|j| sorted) entries per level
  std::vector<double*> g0;        // uncorrected FP64 level tables
  std::vector<int*> uidx, optr, opos;
  float* feats = nullptr;         // [(L-1) nu][kMlpIn]
  float* delta = nullptr;         // [(L-1) nu]
  float* theta = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* wgrad = nullptr;
  float* ddelta = nullptr;
  float* mlp_part = nullptr;
  float* gm = nullptr;            // Adam state and gradient of the grid-valued tables
  float* gv = nullptr;
  float* ggrad = nullptr;
  float* resid = nullptr;         // mesh scratch: d loss / d phi
  float* tphi = nullptr;          // mesh scratch: forward potential
  double* rpart = nullptr;
  double* rstats = nullptr;
  std::vector<void*> lam;         // adjoint per level
  double* tgpart = nullptr;
  std::vector<double*> tgrad;     // table gradient per level (last accumulate)
  int adam_t = 0, accumulated = 0;
  double lr = 1e-3;
  // G_* on the whole mesh (pfmm_gstar_*, allocated on first use): one relative
  // correction per orbit of mesh separations, applied to the near table, every
  // level's table and the direct solve's table
  int gstar = 0;                  // 1 while the correction is set
  int nug = 0;                    // orbits of mesh separations
  float* gdelta = nullptr;        // [nug]
  float* gdd = nullptr;           // gradient of one field [nug]
  float* gacc = nullptr;          // accumulated gradient [nug]
  std::vector<double*> gl0;       // uncorrected level tables
  std::vector<int*> gluidx, glptr, glpos;  // per level: entry -> orbit, orbit -> entries
  double* gn0 = nullptr;          // uncorrected near table
  int *gnuidx = nullptr, *gnptr = nullptr, *gnpos = nullptr;
  double* gd0 = nullptr;          // uncorrected direct table
  int* gduidx = nullptr;
  double* gmesh0 = nullptr;       // -G(x) / N^6 at every mesh point (PM-side gather weights)
  int *gmptr = nullptr, *gmpos = nullptr;
  double* gnear = nullptr;        // near-table gradient of one field
  double* gcorr = nullptr;        // PM-side correlation (N^3)
  float* gtarget = nullptr;       // PM potential with G_*
  GStarFft* gfft = nullptr;
  int gacc_n = 0;                 // fields accumulated
  // direct periodic convolution over the whole box (allocated on first use)
  double* dtab64 = nullptr;
  float* dtab32 = nullptr;
  int* doffs = nullptr;
  int dq = 0, dC = 0, dnoff = 0;
  std::vector<void*> owned;
  // stage timing (PFMM_OPT_PROFILE): a ring of event sets, one per solve;
  // each timed launch (or group of launches) has a start and an end event
  int profile = 0;             // 0 off, 1 serial stages, 2 live (near zone beside the tree)
  std::vector<hipEvent_t> ev;  // [kSlots][2 kMaxIntervals], created when profiling is first on
  std::vector<int> ev_tag;     // [kSlots][kMaxIntervals]: stage | level << 8 | part << 16
  std::vector<int> ev_used;    // intervals recorded per slot
  int nprof = 0;               // profiled solves since profiling was enabled
};

namespace {
// bf16 terms per operand on the matrix-core path: interaction zones (gridlet
// masses cancel strongly) and near zone (cell masses)
constexpr int kM2LTerms = 3;
constexpr int kNearTerms = 2;
constexpr int kMaxIntervals = 64;  // timed launch groups per solve
constexpr int kSlots = 16;         // most recent profiled solves kept
}

namespace {

thread_local std::string g_err;

pfmm_status fail(pfmm_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

pfmm_status hip_fail(hipError_t e, const char* where) {
  return fail(PFMM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Handles are tokens, not addresses: a tag byte, a generation count and a
// slot index.  Destroying an object bumps its slot's generation, so a stale
// handle is refused even after the slot has been reused by a new object.
template <class T, uintptr_t Tag>
class Registry {
 public:
  void* add(T* obj) {
    std::lock_guard<std::mutex> lk(mu_);
    uint32_t slot;
    if (!free_.empty()) {
      slot = free_.back();
      free_.pop_back();
    } else {
      slot = (uint32_t)obj_.size();
      obj_.push_back(nullptr);
      gen_.push_back(1);
    }
    obj_[slot] = obj;
    return reinterpret_cast<void*>(Tag << 56 | (uintptr_t)gen_[slot] << 24 | slot);
  }
  T* get(const void* h) {
    std::lock_guard<std::mutex> lk(mu_);
    uint32_t slot;
    return find(h, slot);
  }
  // Remove and return the object of a live handle (nullptr for any other).
  T* remove(const void* h) {
    std::lock_guard<std::mutex> lk(mu_);
    uint32_t slot;
    T* obj = find(h, slot);
    if (!obj) return nullptr;
    obj_[slot] = nullptr;
    gen_[slot] = (gen_[slot] + 1) & 0xffffffffu;
    if (!gen_[slot]) gen_[slot] = 1;
    free_.push_back(slot);
    return obj;
  }

 private:
  T* find(const void* h, uint32_t& slot) {
    const uintptr_t v = reinterpret_cast<uintptr_t>(h);
    if ((v >> 56) != Tag) return nullptr;
    slot = (uint32_t)(v & 0xffffff);
    const uint32_t gen = (uint32_t)((v >> 24) & 0xffffffffu);
    if (slot >= obj_.size() || gen_[slot] != gen) return nullptr;
    return obj_[slot];
  }
  std::mutex mu_;
  std::vector<T*> obj_;
  std::vector<uint32_t> gen_;
  std::vector<uint32_t> free_;
};

Registry<pfmm_plan_s, 0x70> g_plans;

pfmm_plan_s* plan_of(pfmm_plan_t h) { return g_plans.get(h); }
pfmm_status bad_plan() { return fail(PFMM_ERR_BAD_HANDLE, "not a live plan handle"); }

// Is work on `st` being captured into a graph?  Calls that allocate or
// synchronise must not run then.
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e == hipErrorStreamCaptureImplicit) return true;
  return e == hipSuccess && cs == hipStreamCaptureStatusActive;
}
pfmm_status capture_fail(const char* what) {
  return fail(PFMM_ERR_CAPTURE, std::string(what) + " allocates or synchronises: not while the "
                                "plan's stream is being captured");
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t cube(int64_t v) { return v * v * v; }

// 1D Lagrange basis of the gridlet nodes t_a = a + 1/2 - p/2 (units of the
// gridlet spacing) evaluated at x: the solution of the moment-matching
// (Vandermonde) system of Sec. 2, one axis at a time.
double lagrange(int p, int a, double x) {
  double v = 1.0;
  const double ta = a + 0.5 - 0.5 * p;
  for (int b = 0; b < p; ++b) {
    if (b == a) continue;
    const double tb = b + 0.5 - 0.5 * p;
    v *= (x - tb) / (ta - tb);
  }
  return v;
}

// Derivative of that basis polynomial: the sum over b != a of the product of
// the other factors, with 1/(t_a - t_b) in place of the factor of b.
double lagrange_deriv(int p, int a, double x) {
  const double ta = a + 0.5 - 0.5 * p;
  double sum = 0.0;
  for (int b = 0; b < p; ++b) {
    if (b == a) continue;
    const double tb = b + 0.5 - 0.5 * p;
    double v = 1.0 / (ta - tb);
    for (int c = 0; c < p; ++c) {
      if (c == a || c == b) continue;
      const double tc = c + 0.5 - 0.5 * p;
      v *= (x - tc) / (ta - tc);
    }
    sum += v;
  }
  return sum;
}

template <class T>
hipError_t dalloc(pfmm_plan_s* pl, T** ptr, size_t count) {
  void* raw = nullptr;
  hipError_t e = hipMalloc(&raw, count * sizeof(T));
  if (e != hipSuccess) return e;
  pl->owned.push_back(raw);
  *ptr = static_cast<T*>(raw);
  return hipSuccess;
}

void release(pfmm_plan_s* pl) {
  if (pl->fft) m2l_fft_destroy(pl->fft);
  pl->fft = nullptr;
  if (pl->nfft) near_fft_destroy(pl->nfft);
  pl->nfft = nullptr;
  if (pl->mspec) m2l_spectral_destroy(pl->mspec);
  pl->mspec = nullptr;
  if (pl->gfft) gstar_fft_destroy(pl->gfft);
  pl->gfft = nullptr;
  for (hipEvent_t e : pl->ev)
    if (e) (void)hipEventDestroy(e);
  pl->ev.clear();
  if (pl->side) {
    (void)hipStreamSynchronize(pl->side);
    (void)hipStreamDestroy(pl->side);
  }
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  if (pl->ev_mass) (void)hipEventDestroy(pl->ev_mass);
  if (pl->ev_local) (void)hipEventDestroy(pl->ev_local);
  for (void* q : pl->owned) (void)hipFree(q);
  pl->owned.clear();
  delete pl;
}

// Is level l kept in FP64?  Levels 2 .. 1 + fp64_levels are, except a leaf
// whose FP64 P2M / L2P staging would not fit in 64 KiB of LDS.
bool level64(const pfmm_plan_s* pl, int l) {
  const int top = pl->prec == PFMM_PREC_FP64 ? pl->L : 1 + pl->fp64_levels;
  if (l < 2 || l > top) return false;
  if (l == pl->L) {
    const int p = pl->p, s = pl->s;
    const size_t w1 = (size_t)(p * (s + 1) + s * s * (s + 1) + s * s * p + s * p * p);
    const size_t w2 = (size_t)(3 * p * s + p * p * p + p * p * s + p * s * s);
    if ((w1 > w2 ? w1 : w2) * sizeof(double) > 65536) return false;
  }
  return true;
}

Weights wts(const float* f, const double* d) {
  Weights w;
  w.f = f;
  w.d = d;
  return w;
}

GreenSpec green_spec(const pfmm_plan_s* pl) {
  GreenSpec g;
  g.kind = pl->isolated ? GK_N : pl->green;
  g.a1 = pl->a1;
  g.a2 = pl->a2;
  g.rs = pl->rs;
  return g;
}

// Transformed kernels of the FFT near zone: G, and the three acceleration
// kernels when accelerations come from the expansion
pfmm_status refresh_near_fft(pfmm_plan_s* pl) {
  if (!pl->nfft) return PFMM_OK;
  const double* tabs[4] = {pl->ntab64, pl->ndtab64[0], pl->ndtab64[1], pl->ndtab64[2]};
  const int n = pl->accel_mode ? 4 : 1;
  const double h3 = 1.0 / ((double)pl->N * pl->N * pl->N);
  const hipError_t e = near_fft_tables(pl->nfft, tabs, n, h3, pl->stream);
  if (e == hipErrorOutOfMemory) return fail(PFMM_ERR_OUT_OF_MEMORY, "FFT near-zone kernels");
  if (e != hipSuccess) return hip_fail(e, "FFT near-zone kernels");
  return PFMM_OK;
}

// Near-zone acceleration kernels of the plan's G (allocated on first use)
pfmm_status tabulate_accel_tables(pfmm_plan_s* pl) {
  const int Cn = 2 * pl->s - 1;
  const int64_t n = cube(2 * Cn + 1);
  hipError_t e = hipSuccess;
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    if (!pl->ndtab64[c]) e = dalloc(pl, &pl->ndtab64[c], n);
    if (e == hipSuccess && !pl->ndtab32[c]) e = dalloc(pl, &pl->ndtab32[c], n);
    if (e == hipSuccess && pl->nwin && !pl->ndwin[c])
      e = dalloc(pl, &pl->ndwin[c], window_dwords(kNearTerms));
  }
  if (e == hipErrorOutOfMemory) return fail(PFMM_ERR_OUT_OF_MEMORY, "acceleration tables");
  if (e == hipSuccess)
    e = tabulate_accel(green_spec(pl), pl->N, Cn, pl->ndtab64, pl->stream);
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    e = cast_f64_f32(pl->ndtab64[c], pl->ndtab32[c], n, pl->stream);
    if (e == hipSuccess && pl->nwin) e = make_windows(pl->ndtab64[c], Cn, kNearTerms, pl->ndwin[c], pl->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(e, "acceleration tables");
  return refresh_near_fft(pl);
}

hipError_t gstar_base(pfmm_plan_s* pl);
pfmm_status gstar_apply(pfmm_plan_s* pl);

pfmm_status tabulate_all(pfmm_plan_s* pl) {
  const int p = pl->p;
  const int C = 4 * p - 1;
  const int64_t nlev = cube(2 * C + 1);
  for (int l = 2; l <= pl->L; ++l) {
    hipError_t e = tabulate_green(green_spec(pl), pl->N, C,
                                  (int64_t(1) << l) * p, 0.0, pl->tab64[l], pl->stream);
    if (e == hipSuccess) e = cast_f64_f32(pl->tab64[l], pl->tab32[l], nlev, pl->stream);
    if (e != hipSuccess) return hip_fail(e, "tabulate level table");
  }
  const int Cn = 2 * pl->s - 1;
  hipError_t e = tabulate_green(green_spec(pl), pl->N, Cn, pl->N,
                                1.0 / pl->N, pl->ntab64, pl->stream);
  if (e == hipSuccess) e = cast_f64_f32(pl->ntab64, pl->ntab32, cube(2 * Cn + 1), pl->stream);
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l)
    if (pl->win[l]) e = make_windows(pl->tab64[l], C, kM2LTerms, pl->win[l], pl->stream);
  if (e == hipSuccess && pl->nwin)
    e = make_windows(pl->ntab64, Cn, kNearTerms, pl->nwin, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(e, "tabulate near table");
  if (pl->dtab64) {  // the direct solve's table, once it exists, follows G too
    e = tabulate_green(green_spec(pl), pl->N, pl->dC, pl->N, 1.0 / pl->N, pl->dtab64, pl->stream);
    if (e == hipSuccess) e = cast_f64_f32(pl->dtab64, pl->dtab32, cube(2 * pl->dC + 1), pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) return hip_fail(e, "direct solve tables");
  }
  if (pl->fft) {  // transformed kernels of the FFT interaction zones follow G
    e = m2l_fft_tables(pl->fft, pl->tab64, pl->stream);
    if (e != hipSuccess) return hip_fail(e, "FFT kernels");
  }
  if (pl->mspec) {  // and those of the spectral stencils
    e = m2l_spectral_tables(pl->mspec, pl->tab64, pl->stream);
    if (e != hipSuccess) return hip_fail(e, "spectral zone kernels");
  }
  pfmm_status s0 = pl->accel_mode ? tabulate_accel_tables(pl) : refresh_near_fft(pl);
  if (s0 != PFMM_OK || !pl->gdelta) return s0;
  // G_* follows the new G: new uncorrected copies, the correction applied again
  e = gstar_base(pl);
  if (e != hipSuccess) return hip_fail(e, "G_* tables");
  return pl->gstar ? gstar_apply(pl) : PFMM_OK;
}

// Offset groups of a level's matrix-core launch: enough workgroups to give
// the 256 compute units two rounds (a level-l launch has 8^(l-2) tiles).
// Offset groups of a portable-kernel launch: at least 1024 workgroups.
int scalar_groups(int q, int fp64, int n, int m, int noff) {
  const int wg = toeplitz_workgroups(q, fp64, n, m);
  if (wg <= 0) return 1;
  const int g = (1024 + wg - 1) / wg;
  return g < noff ? g : noff;
}

// Offset groups of an FP64 matrix-core launch: at least 512 workgroups.
int f64_groups(int n, int m, int noff) {
  const int tiles = toep8_f64_tiles(n, m);
  const int g = (512 + tiles - 1) / tiles;
  return g < noff ? g : noff;
}

// Order one class's offsets for cache reuse and append them packed.  The
// targets of a class lie on a lattice of step m (here 2 for the zones that
// are split into classes), so the sources of offsets d and d + 2e overlap in
// all but one layer of a workgroup's tile.  Offsets are grouped by parity and
// each group is walked as a serpentine (boustrophedon) path, so consecutive
// offsets differ by one lattice step and share most of their sources while
// those are still in L2.  The order changes rounding only.
void append_in_reuse_order(std::vector<std::array<int, 3>> ds, std::vector<int>& out) {
  auto rank = [](std::vector<int> v, int x) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return (int)(std::lower_bound(v.begin(), v.end(), x) - v.begin());
  };
  for (int par = 0; par < 8; ++par) {
    std::vector<std::array<int, 3>> g;
    for (const auto& d : ds)
      if (((d[0] & 1) << 2 | (d[1] & 1) << 1 | (d[2] & 1)) == par) g.push_back(d);
    std::vector<int> xs, ys, zs;
    for (const auto& d : g) {
      xs.push_back(d[0]);
      ys.push_back(d[1]);
      zs.push_back(d[2]);
    }
    const int ny = (int)std::set<int>(ys.begin(), ys.end()).size();
    auto key = [&](const std::array<int, 3>& d) {
      const int ix = rank(xs, d[0]);
      const int iy0 = rank(ys, d[1]);
      const int iy = (ix & 1) ? ny - 1 - iy0 : iy0;
      const int iz0 = rank(zs, d[2]);
      const int iz = ((ix * ny + iy) & 1) ? -iz0 : iz0;
      return std::array<int, 3>{ix, iy, iz};
    };
    std::stable_sort(g.begin(), g.end(),
                     [&](const std::array<int, 3>& a, const std::array<int, 3>& b) {
                       return key(a) < key(b);
                     });
    for (const auto& d : g) out.push_back(pack_offset(d[0], d[1], d[2]));
  }
}

// Offset groups of a level's matrix-core launch.  Each group sums its share
// of the offsets in the FP32 matrix-core accumulators and writes a partial;
// the partials are added in FP64.  The zone sums cancel 10^2-10^3 fold, so
// shorter FP32 accumulations matter: 32 groups (about 6 offsets each) cut the
// leaf's accumulation error about 2.5-fold at no measurable cost.  At least
// enough groups to give the 256 compute units two rounds (a level-l launch has
// 8^(l-2) tiles); the partials of a level stay within 1 GiB.
int m2l_groups(int l) {
  const int64_t tiles = (int64_t)1 << (3 * (l - 2));
  const int64_t level_bytes = ((int64_t)1 << (3 * l)) * 512 * 4;
  int64_t g = (512 + tiles - 1) / tiles;
  const int64_t fit = ((int64_t)1 << 30) / level_bytes;
  g = std::max(g, std::min<int64_t>(32, fit));
  return (int)std::min<int64_t>(g, 37);
}

pfmm_status build(pfmm_plan_s* pl) {
  const int N = pl->N, L = pl->L, p = pl->p, s = pl->s;
  const int p3 = p * p * p;
  hipError_t e = hipSuccess;
  auto chk = [&](const char* what) -> pfmm_status {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return fail(PFMM_ERR_OUT_OF_MEMORY, std::string("allocation failed: ") + what);
    if (e != hipSuccess) return hip_fail(e, what);
    return PFMM_OK;
  };
  pfmm_status st;

  // 1D operators in FP64 on the host, stored as FP32
  std::vector<float> A(p * s), T(2 * p * p);
  for (int a = 0; a < p; ++a)
    for (int c = 0; c < s; ++c)
      A[a * s + c] = (float)lagrange(p, a, (c + 0.5 - 0.5 * s) * ((double)p / s));
  for (int o = 0; o < 2; ++o)
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        const double tb = b + 0.5 - 0.5 * p;
        T[(o * p + a) * p + b] = (float)lagrange(p, a, (o - 0.5) * 0.5 * p + 0.5 * tb);
      }
  e = dalloc(pl, &pl->dA, A.size());
  if ((st = chk("P2M weights"))) return st;
  e = dalloc(pl, &pl->dT, T.size());
  if ((st = chk("M2M weights"))) return st;
  e = hipMemcpy(pl->dA, A.data(), A.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pl->dT, T.data(), T.size() * sizeof(float), hipMemcpyHostToDevice);
  if ((st = chk("upload weights"))) return st;

  std::vector<double> A64(A.begin(), A.end()), T64(T.begin(), T.end());
  for (int a = 0; a < p; ++a)
    for (int c = 0; c < s; ++c) A64[a * s + c] = lagrange(p, a, (c + 0.5 - 0.5 * s) * ((double)p / s));
  for (int o = 0; o < 2; ++o)
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b)
        T64[(o * p + a) * p + b] = lagrange(p, a, (o - 0.5) * 0.5 * p + 0.5 * (b + 0.5 - 0.5 * p));
  e = dalloc(pl, &pl->dA64, A64.size());
  if (e == hipSuccess) e = dalloc(pl, &pl->dT64, T64.size());
  if (e == hipSuccess)
    e = hipMemcpy(pl->dA64, A64.data(), A64.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pl->dT64, T64.data(), T64.size() * sizeof(double), hipMemcpyHostToDevice);
  if ((st = chk("FP64 weights"))) return st;
  {
    std::vector<double> D64(p * s);
    for (int a = 0; a < p; ++a)
      for (int c = 0; c < s; ++c) D64[a * s + c] = lagrange_deriv(p, a, (c + 0.5 - 0.5 * s) * ((double)p / s));
    std::vector<float> D(D64.begin(), D64.end());
    e = dalloc(pl, &pl->dAd, D.size());
    if (e == hipSuccess) e = dalloc(pl, &pl->dAd64, D64.size());
    if (e == hipSuccess) e = hipMemcpy(pl->dAd, D.data(), D.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(pl->dAd64, D64.data(), D64.size() * sizeof(double), hipMemcpyHostToDevice);
    if ((st = chk("derivative weights"))) return st;
  }

  // per-level gridlet buffers (levels 2 and 3 sized for FP64) and tables
  pl->M.assign(L + 1, nullptr);
  pl->P.assign(L + 1, nullptr);
  pl->tab64.assign(L + 1, nullptr);
  pl->tab32.assign(L + 1, nullptr);
  const int64_t nlev = cube(8 * p - 1);
  for (int l = 2; l <= L; ++l) {
    const size_t nodes = (size_t)1 << (3 * l);
    const size_t wbytes = sizeof(double);  // any level may be kept in FP64
    char* mb = nullptr;
    e = dalloc(pl, &mb, nodes * p3 * wbytes);
    pl->M[l] = mb;
    if ((st = chk("multipole buffer"))) return st;
    e = dalloc(pl, &mb, nodes * p3 * wbytes);
    pl->P[l] = mb;
    if ((st = chk("local buffer"))) return st;
    e = dalloc(pl, &pl->tab64[l], nlev);
    if ((st = chk("level table"))) return st;
    e = dalloc(pl, &pl->tab32[l], nlev);
    if ((st = chk("level table"))) return st;
  }
  const int64_t nnear = cube(4 * s - 1);
  e = dalloc(pl, &pl->ntab64, nnear);
  if ((st = chk("near table"))) return st;
  e = dalloc(pl, &pl->ntab32, nnear);
  if ((st = chk("near table"))) return st;

  // matrix-core path: windows, split sources and partial sums, sized for
  // every level / near zone it can serve
  pl->win.assign(L + 1, nullptr);
  size_t xwords = 0;
  if (p == 8) {
    for (int l = 2; l <= L; ++l) {
      if (!toep8_supported(1 << l, l == 2 ? 1 : 2)) continue;
      e = dalloc(pl, &pl->win[l], window_dwords(kM2LTerms));
      if ((st = chk("level windows"))) return st;
      const size_t nodes = (size_t)1 << (3 * l);
      xwords = std::max(xwords, nodes * 512);
      const int G = m2l_groups(l);
      pl->part_floats = std::max(pl->part_floats, G > 1 ? (size_t)G * nodes * 512 : (size_t)0);
    }
  }
  {
    const int qn = s <= 8 ? s : 8, mn = s / qn;
    if (qn == 8 && toep8_supported(N / 8, mn)) {
      e = dalloc(pl, &pl->nwin, window_dwords(kNearTerms));
      if ((st = chk("near windows"))) return st;
      e = dalloc(pl, &pl->xsn, (size_t)kNearTerms * N * N * N);
      if ((st = chk("split density"))) return st;
    }
  }
  if (xwords) {
    pl->xwords = xwords;
    e = dalloc(pl, &pl->xs, 3 * xwords);
    if ((st = chk("split sources"))) return st;
  }
  if (pl->part_floats) {
    e = dalloc(pl, &pl->part, pl->part_floats);
    if ((st = chk("partial sums"))) return st;
  }
  {
    // portable-kernel partial sums: any level may run there (FP64 for the
    // coarse levels), block layout only
    size_t bytes = 0;
    for (int l = 2; l <= L; ++l) {
      const int n = 1 << l, m = l == 2 ? 1 : 2, noff = l == 2 ? 316 : 189;  // 316: isolated level 2
      for (int f64 = 0; f64 <= 1; ++f64) {  // the FP64 level count is an option
        int G = scalar_groups(p, f64, n, m, noff);
        if (f64 && p == 8) G = std::max(G, f64_groups(n, m, noff));
        const size_t w = f64 ? sizeof(double) : sizeof(float);
        if (G > 1) bytes = std::max(bytes, (size_t)G * ((size_t)1 << (3 * l)) * p3 * w);
      }
    }
    if (bytes) {
      char* sp = nullptr;
      e = dalloc(pl, &sp, bytes);
      pl->spart = sp;
      if ((st = chk("partial sums"))) return st;
    }
  }

  // zones (Sec. 2, Fig. 2); the offsets of a class are listed in reuse order
  std::vector<int> l2, iz, nz;
  for (int dx = -2; dx <= 1; ++dx)
    for (int dy = -2; dy <= 1; ++dy)
      for (int dz = -2; dz <= 1; ++dz)
        if (dx == -2 || dy == -2 || dz == -2) l2.push_back(pack_offset(dx, dy, dz));
  for (int c = 0; c < 8; ++c) {
    const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
    std::vector<std::array<int, 3>> cls;
    for (int dx = -2 - cx; dx <= 3 - cx; ++dx)
      for (int dy = -2 - cy; dy <= 3 - cy; ++dy)
        for (int dz = -2 - cz; dz <= 3 - cz; ++dz)
          if (std::abs(dx) > 1 || std::abs(dy) > 1 || std::abs(dz) > 1)
            cls.push_back({dx, dy, dz});
    append_in_reuse_order(cls, iz);
  }
  pl->qn = s <= 8 ? s : 8;
  pl->mn = s / pl->qn;
  const int mn = pl->mn;
  for (int c = 0; c < mn * mn * mn; ++c) {
    const int cx = c / (mn * mn), cy = (c / mn) % mn, cz = c % mn;
    std::vector<std::array<int, 3>> cls;
    for (int dx = -mn - cx; dx <= 2 * mn - 1 - cx; ++dx)
      for (int dy = -mn - cy; dy <= 2 * mn - 1 - cy; ++dy)
        for (int dz = -mn - cz; dz <= 2 * mn - 1 - cz; ++dz) cls.push_back({dx, dy, dz});
    append_in_reuse_order(cls, nz);
  }
  if (l2.size() != 37 || iz.size() != 8 * 189 || nz.size() != (size_t)cube(3 * mn) * cube(mn))
    return fail(PFMM_ERR_HIP, "internal: zone sizes");
  e = dalloc(pl, &pl->offs_l2, (size_t)316);
  if (e == hipSuccess) e = dalloc(pl, &pl->zero, (size_t)512);
  if (e == hipSuccess) e = hipMemset(pl->zero, 0, 512 * sizeof(uint16_t));
  if (e == hipSuccess) e = dalloc(pl, &pl->offs_iz, iz.size());
  if (e == hipSuccess) e = dalloc(pl, &pl->offs_near, nz.size());
  if ((st = chk("zone lists"))) return st;
  e = hipMemcpy(pl->offs_l2, l2.data(), l2.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pl->offs_iz, iz.data(), iz.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(pl->offs_near, nz.data(), nz.size() * sizeof(int), hipMemcpyHostToDevice);
  if ((st = chk("upload zone lists"))) return st;
  (void)N;
  // default priority (no priority streams anywhere in this library)
  e = hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking);
  if ((st = chk("side stream"))) return st;
  e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_mass, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_local, hipEventDisableTiming);
  if ((st = chk("fork events"))) return st;
  return tabulate_all(pl);
}

}  // namespace

namespace {
pfmm_status learned_apply(pfmm_plan_s* pl, int bf16);
}
void drop_cached_batches(pfmm_plan_s* pl);

extern "C" {

pfmm_status pfmm_plan_create(int N, int L, int p, int green_kind, pfmm_plan_t* out) {
  g_err.clear();
  if (!out) return fail(PFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!is_pow2(N) || N < 8 || N > 1024)
    return fail(PFMM_ERR_INVALID_ARG, "N must be a power of two in [8, 1024]");
  if (L < 2 || (1 << L) > N) return fail(PFMM_ERR_INVALID_ARG, "need 2 <= L and 2^L <= N");
  if (p < 1 || p > 10) return fail(PFMM_ERR_INVALID_ARG, "p must be in [1, 10]");
  if (green_kind < PFMM_GREEN_X || green_kind > PFMM_GREEN_LEARNED)
    return fail(PFMM_ERR_INVALID_ARG, "unknown green_kind");
  const int s = N >> L;
  if (s > 16)
    return fail(PFMM_ERR_UNSUPPORTED, "leaf width N/2^L must be <= 16 (one leaf is staged in 64 KiB "
                                      "of LDS by the mesh transfers)");
  pfmm_plan_s* pl = new (std::nothrow) pfmm_plan_s;
  if (!pl) return fail(PFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  pl->N = N;
  pl->L = L;
  pl->p = p;
  pl->s = s;
  // a learned G is G_S1's tables with the network's correction on top
  pl->learned_kind = green_kind == PFMM_GREEN_LEARNED;
  pl->green = pl->learned_kind ? PFMM_GREEN_S1 : green_kind;
  // deeper trees keep every level down to L - 1 in FP64: the downward
  // interpolation (Eq. 7) amplifies a coarse level's rounding on its way to
  // the mesh, once per level it passes
  pl->fp64_levels = std::max(2, L - 2);
  pfmm_status st = build(pl);
  if (st != PFMM_OK) {
    (void)hipDeviceSynchronize();
    release(pl);
    return st;
  }
  *out = static_cast<pfmm_plan_t>(g_plans.add(pl));
  return PFMM_OK;
}

pfmm_status pfmm_plan_set(pfmm_plan_t h, int option, const void* value, size_t bytes) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (!value) return fail(PFMM_ERR_INVALID_ARG, "value is NULL");
  if (option != PFMM_OPT_STREAM && option != PFMM_OPT_PROFILE && capturing(pl->stream))
    return capture_fail("pfmm_plan_set");
  // a live batch holds this plan's buffers, zone lists and routes in its graph
  if (pl->batch_refs > 0 &&
      (option == PFMM_OPT_PRECISION || option == PFMM_OPT_ISOLATED || option == PFMM_OPT_FP64_LEVELS ||
       option == PFMM_OPT_M2L || option == PFMM_OPT_NEAR || option == PFMM_OPT_ZONES_FP32))
    return fail(PFMM_ERR_INVALID_ARG, "the plan is bound to a live batch: this option would change "
                                      "what the batch's graph uses");
  switch (option) {
    case PFMM_OPT_PRECISION: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "precision is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != PFMM_PREC_FP32 && v != PFMM_PREC_BF16X3 && v != PFMM_PREC_FP64)
        return fail(PFMM_ERR_INVALID_ARG, "unknown precision");
      if (v == PFMM_PREC_FP64) {
        const int keep = pl->fp64_levels;
        pl->fp64_levels = 30;
        const bool leaf = level64(pl, pl->L);
        pl->fp64_levels = keep;
        if (!leaf)
          return fail(PFMM_ERR_UNSUPPORTED, "PFMM_PREC_FP64: the leaf's FP64 mesh transfers do not fit "
                                            "in 64 KiB of LDS at this leaf width and p");
      }
      pl->prec = v;
      return PFMM_OK;
    }
    case PFMM_OPT_ZONES_FP32: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "zones_fp32 is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != 0 && v != 1) return fail(PFMM_ERR_INVALID_ARG, "zones_fp32 is 0 or 1");
      pl->zones_f32 = v;
      if (pl->mspec) m2l_spectral_set_f32(pl->mspec, v);
      return PFMM_OK;
    }
    case PFMM_OPT_FOLD: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "fold is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != 0 && v != 1) return fail(PFMM_ERR_INVALID_ARG, "fold is 0 or 1");
      pl->fold = v;
      return PFMM_OK;
    }
    case PFMM_OPT_LEARNED_WEIGHTS: {
      if (bytes != (size_t)kMlpParams * sizeof(float))
        return fail(PFMM_ERR_INVALID_ARG, "learned weights are PFMM_MLP_PARAMS floats");
      return pfmm_learned_set(h, static_cast<const float*>(value), 1);
    }
    case PFMM_OPT_STREAM: {
      if (bytes != sizeof(hipStream_t)) return fail(PFMM_ERR_INVALID_ARG, "stream is a hipStream_t");
      std::memcpy(&pl->stream, value, sizeof(hipStream_t));
      return PFMM_OK;
    }
    case PFMM_OPT_ISOLATED: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "isolated is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != 0 && v != 1) return fail(PFMM_ERR_INVALID_ARG, "isolated must be 0 or 1");
      if (v && pl->green != PFMM_GREEN_X)
        return fail(PFMM_ERR_UNSUPPORTED, "the isolated twin uses G_X without images: PFMM_GREEN_X");
      if (!pl->g0.empty()) return fail(PFMM_ERR_UNSUPPORTED, "plan has learned tables");
      if (v && pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "the FFT interaction zones are periodic only");
      // level-2 zone: 37 periodic representatives, or every non-neighbour
      // node of the 4^3 level, d in [-3, 3]^3 \ [-1, 1]^3 (316)
      std::vector<int> l2;
      const int lo = v ? -3 : -2, hi = v ? 3 : 1;
      for (int dx = lo; dx <= hi; ++dx)
        for (int dy = lo; dy <= hi; ++dy)
          for (int dz = lo; dz <= hi; ++dz)
            if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) > 1)
              l2.push_back(pack_offset(dx, dy, dz));
      if (l2.size() != (v ? 316u : 37u)) return fail(PFMM_ERR_HIP, "internal: level-2 zone size");
      hipError_t e = hipMemcpy(pl->offs_l2, l2.data(), l2.size() * sizeof(int), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "level-2 zone");
      pl->isolated = v;
      pl->nl2 = (int)l2.size();
      return tabulate_all(pl);
    }
    case PFMM_OPT_GS_A1:
    case PFMM_OPT_GS_A2:
    case PFMM_OPT_EWALD_RS: {
      const bool ewald = option == PFMM_OPT_EWALD_RS;
      const std::string name = ewald ? "r_S" : option == PFMM_OPT_GS_A1 ? "a1" : "a2";
      if (bytes != sizeof(double)) return fail(PFMM_ERR_INVALID_ARG, name + " is a double");
      if (pl->green != (ewald ? PFMM_GREEN_E : PFMM_GREEN_S))
        return fail(PFMM_ERR_INVALID_ARG,
                    name + (ewald ? " needs PFMM_GREEN_E" : " needs PFMM_GREEN_S"));
      double v;
      std::memcpy(&v, value, sizeof v);
      if (!std::isfinite(v)) return fail(PFMM_ERR_INVALID_ARG, name + " must be finite");
      if (ewald && !(v > 0.0 && v <= 0.25))
        return fail(PFMM_ERR_INVALID_ARG, "r_S must be in (0, 1/4] of the box");
      (ewald ? pl->rs : option == PFMM_OPT_GS_A1 ? pl->a1 : pl->a2) = v;
      pfmm_status r = tabulate_all(pl);
      if (r != PFMM_OK || pl->g0.empty()) return r;
      // new uncorrected tables; keep the plan's correction on top of them
      const int64_t ntab = cube(8 * pl->p - 1);
      for (int l = 2; l <= pl->L; ++l) {
        const hipError_t e = hipMemcpy(pl->g0[l], pl->tab64[l], ntab * sizeof(double),
                                       hipMemcpyDeviceToDevice);
        if (e != hipSuccess) return hip_fail(e, "refresh tables");
      }
      return pl->learned ? learned_apply(pl, 0) : PFMM_OK;
    }
    case PFMM_OPT_ACCEL: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "accel mode is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != PFMM_ACCEL_FD4 && v != PFMM_ACCEL_EXPANSION)
        return fail(PFMM_ERR_INVALID_ARG, "unknown acceleration mode");
      pl->accel_mode = v;
      if (!v) return PFMM_OK;
      const pfmm_status r = tabulate_accel_tables(pl);
      if (r != PFMM_OK) pl->accel_mode = 0;
      return r;
    }
    case PFMM_OPT_M2L: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "M2L mode is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != PFMM_M2L_GEMM && v != PFMM_M2L_FFT && v != PFMM_M2L_SPECTRAL)
        return fail(PFMM_ERR_INVALID_ARG, "unknown M2L mode");
      if (v == PFMM_M2L_SPECTRAL) {
        if (pl->p != 4 && pl->p != 6 && pl->p != 8)
          return fail(PFMM_ERR_UNSUPPORTED, "the spectral interaction zones need p = 4, 6 or 8");
        if (!pl->mspec) {
          M2LSpectral* f = nullptr;
          hipError_t e = m2l_spectral_create(pl->L, pl->p, &f);
          if (e == hipErrorOutOfMemory) return fail(PFMM_ERR_OUT_OF_MEMORY, "spectral zone buffers");
          if (e != hipSuccess) return hip_fail(e, "spectral zone buffers");
          m2l_spectral_set_f32(f, pl->zones_f32);
          pl->mspec = f;
          e = m2l_spectral_tables(pl->mspec, pl->tab64, pl->stream);
          if (e != hipSuccess) return hip_fail(e, "spectral zone kernels");
        }
        pl->m2l_fft = 0;
        pl->m2l_spectral = 1;
        return PFMM_OK;
      }
      if (v == PFMM_M2L_FFT) {
        if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "the FFT interaction zones are periodic only");
        if (!pl->g0.empty()) return fail(PFMM_ERR_UNSUPPORTED, "plan has learned tables");
        if (!pl->fft) {
          M2LFft* f = nullptr;
          hipError_t e = m2l_fft_create(pl->L, pl->p, (size_t)1 << 30, &f);
          if (e == hipErrorOutOfMemory) return fail(PFMM_ERR_OUT_OF_MEMORY, "FFT workspace");
          if (e != hipSuccess) return hip_fail(e, "FFT plans");
          pl->fft = f;
          e = m2l_fft_tables(pl->fft, pl->tab64, pl->stream);
          if (e != hipSuccess) return hip_fail(e, "FFT kernels");
        }
      }
      pl->m2l_fft = v;
      pl->m2l_spectral = 0;
      return PFMM_OK;
    }
    case PFMM_OPT_NEAR: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "near-zone mode is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v != PFMM_NEAR_DIRECT && v != PFMM_NEAR_FFT)
        return fail(PFMM_ERR_INVALID_ARG, "unknown near-zone mode");
      if (v == PFMM_NEAR_FFT && !pl->nfft) {
        NearFft* f = nullptr;
        const hipError_t e = near_fft_create(pl->N, pl->s, &f);
        if (e == hipErrorOutOfMemory) return fail(PFMM_ERR_OUT_OF_MEMORY, "FFT near-zone buffers");
        if (e != hipSuccess) return hip_fail(e, "FFT near-zone plans");
        pl->nfft = f;
        const pfmm_status r = refresh_near_fft(pl);
        if (r != PFMM_OK) {
          near_fft_destroy(pl->nfft);
          pl->nfft = nullptr;
          return r;
        }
      }
      pl->near_fft = v;
      return PFMM_OK;
    }
    case PFMM_OPT_FP64_LEVELS: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "fp64 levels is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v < 0 || v > 30) return fail(PFMM_ERR_INVALID_ARG, "fp64 levels must be in [0, 30]");
      pl->fp64_levels = v;
      return PFMM_OK;
    }
    case PFMM_OPT_PROFILE: {
      if (bytes != sizeof(int32_t)) return fail(PFMM_ERR_INVALID_ARG, "profile is an int32");
      int32_t v;
      std::memcpy(&v, value, sizeof v);
      if (v < 0 || v > 2) return fail(PFMM_ERR_INVALID_ARG, "profile must be 0, 1 or 2");
      if (v && pl->ev.empty()) {  // the ring of timing events, on first use
        pl->ev.assign((size_t)kSlots * 2 * kMaxIntervals, nullptr);
        for (auto& ev : pl->ev) {
          const hipError_t e = hipEventCreate(&ev);
          if (e != hipSuccess) return hip_fail(e, "timing events");
        }
        pl->ev_tag.assign((size_t)kSlots * kMaxIntervals, 0);
        pl->ev_used.assign(kSlots, 0);
      }
      pl->profile = v;
      pl->nprof = 0;
      return PFMM_OK;
    }
    default:
      return fail(PFMM_ERR_INVALID_ARG, "unknown option");
  }
}

}  // extern "C"

namespace {

// Records a start and an end event around each timed launch group of one
// solve, into the plan's ring slot; the tag holds the stage, the tree level
// and the part (kernel) within the stage.
struct SolveTimer final : KernelTimer {
  bool on = false;
  hipEvent_t* ev = nullptr;
  int* tag = nullptr;
  int n = 0, stage = 0, level = 0;
  void at(int st, int lv) {
    stage = st;
    level = lv;
  }
  hipError_t begin(hipStream_t s) override {
    if (!on || n >= kMaxIntervals) return hipSuccess;
    return hipEventRecord(ev[2 * n], s);
  }
  hipError_t end(hipStream_t s, int part) override {
    if (!on || n >= kMaxIntervals) return hipSuccess;
    tag[n] = stage | level << 8 | part << 16;
    const hipError_t e = hipEventRecord(ev[2 * n + 1], s);
    ++n;
    return e;
  }
};

// The whole solve (see pfmm_solve).  io64: density, potential and accel are
// doubles (pfmm_solve_f64, PFMM_PREC_FP64 plans only), else floats.
pfmm_status solve_impl(pfmm_plan_s* pl, const void* rho_in, void* phi_out, void* accel_out,
                       int io64 = 0) {
  if (!rho_in || !phi_out) return fail(PFMM_ERR_INVALID_ARG, "density and potential are required");
  if (rho_in == (const void*)phi_out || rho_in == (const void*)accel_out ||
      (accel_out && accel_out == phi_out))
    return fail(PFMM_ERR_INVALID_ARG, "buffers must not alias");
  const bool f64 = pl->prec == PFMM_PREC_FP64;
  if (io64 && !f64) return fail(PFMM_ERR_INVALID_ARG, "FP64 buffers need a PFMM_PREC_FP64 plan");
  // FP64 precision sums the near zone directly in FP64, whatever PFMM_OPT_NEAR says
  const bool near_fft = pl->near_fft && !f64;
  if (near_fft && (((uintptr_t)rho_in | (uintptr_t)phi_out | (uintptr_t)accel_out) & 15))
    return fail(PFMM_ERR_INVALID_ARG, "the FFT near zone needs 16-byte aligned density and outputs");
  const float* rho = static_cast<const float*>(rho_in);
  float* phi = static_cast<float*>(phi_out);
  float* accel = static_cast<float*>(accel_out);
  const int N = pl->N, L = pl->L, p = pl->p, s = pl->s;
  const size_t n3 = (size_t)N * N * N;
  // component c of the accelerations, in the caller's type
  auto acc_c = [&](int c) -> void* {
    return io64 ? (void*)(static_cast<double*>(accel_out) + c * n3) : (void*)(accel + c * n3);
  };
  const double h3 = 1.0 / ((double)N * N * N);
  hipStream_t st = pl->stream;
  hipError_t e;
  const int slot = pl->nprof % kSlots;
  SolveTimer tm;
  tm.on = pl->profile != 0;
  if (tm.on) {
    tm.ev = pl->ev.data() + (size_t)slot * 2 * kMaxIntervals;
    tm.tag = pl->ev_tag.data() + (size_t)slot * kMaxIntervals;
  }
  // one stage's launches as one timed interval (profiling only)
  auto timed = [&](int stage, int level, hipStream_t s, auto&& launch) -> hipError_t {
    tm.at(stage, level);
    hipError_t r = tm.begin(s);
    if (r == hipSuccess) r = launch();
    if (r == hipSuccess) r = tm.end(s, 0);
    return r;
  };

  const Weights A = wts(pl->dA, pl->dA64), T = wts(pl->dT, pl->dT64);
  auto is64 = [&](int l) { return (int)level64(pl, l); };
  const bool mx = pl->prec == PFMM_PREC_BF16X3;
  // interaction zone of one level: matrix cores for FP32 levels with windows
  auto m2l = [&](const ToepArgs& ta0, int l) -> hipError_t {
    ToepArgs ta = ta0;
    if (pl->m2l_fft)  // the FFT-convolution comparator, in the level's precision
      return m2l_fft_level(pl->fft, l, ta.X, ta.Y, ta.fp64, ta.accumulate, st);
    if (pl->m2l_spectral)  // spectral stencils, FP64 throughout; each kernel timed
      return m2l_spectral_level(pl->mspec, l, ta.X, ta.fp64, ta.Y, ta.fp64, ta.accumulate, ta.offs,
                                ta.noff, ta.isolated, st, tm.on ? &tm : nullptr);
    if (ta.fp64 && ta.q == 8 && ta.C >= 31) {  // FP64 coarse level on the matrix cores
      ToepF64Args fa{};
      fa.n = ta.n;
      fa.m = ta.m;
      fa.noff = ta.noff;
      fa.offs = ta.offs;
      fa.tab = (const double*)ta.tab;
      fa.C = ta.C;
      fa.X = (const double*)ta.X;
      fa.Y = (double*)ta.Y;
      fa.accumulate = ta.accumulate;
      fa.groups = f64_groups(ta.n, ta.m, ta.noff);
      fa.isolated = ta.isolated;
      fa.partial = fa.groups > 1 ? (double*)pl->spart : nullptr;
      if (fa.groups > 1 && !fa.partial) fa.groups = 1;
      return launch_toep8_f64(fa, st);
    }
    if (!mx || ta.fp64 || !pl->win[l] || ta.noff > kSplitMaxOffs) {
      ta.groups = scalar_groups(ta.q, ta.fp64, ta.n, ta.m, ta.noff);
      ta.partial = ta.groups > 1 ? pl->spart : nullptr;
      if (ta.groups > 1 && !ta.partial) ta.groups = 1;
      return launch_toeplitz(ta, st);
    }
    const size_t nodes = (size_t)1 << (3 * l);
    hipError_t r = split_blocks((const float*)ta.X, pl->xs, kM2LTerms, (int64_t)(nodes * 512), st);
    if (r != hipSuccess) return r;
    ToepMfmaArgs ma{};
    ma.n = ta.n;
    ma.m = ta.m;
    ma.noff = ta.noff;
    ma.offs = ta.offs;
    ma.win = pl->win[l];
    ma.X = pl->xs;
    ma.Y = (float*)ta.Y;
    ma.accumulate = ta.accumulate;
    ma.groups = std::min(m2l_groups(l), ta.noff);
    ma.isolated = ta.isolated;
    ma.zero = pl->zero;
    ma.partial = ma.groups > 1 ? pl->part : nullptr;
    return launch_toep8_split(ma, kM2LTerms, st);
  };

  // near zone (reads only the density): writes phi; on the side stream, so
  // that it runs beside the tree, unless stages are timed one after another
  const bool overlap = pl->profile != 1;
  hipStream_t sn = overlap ? pl->side : st;
  if (overlap) {
    e = hipEventRecord(pl->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->side, pl->ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "fork");
  }
  ToepArgs nb{};
  nb.q = pl->qn;
  nb.m = pl->mn;
  nb.n = N / pl->qn;
  nb.noff = (int)cube(3 * pl->mn);
  nb.offs = pl->offs_near;
  nb.fp64 = f64;
  nb.mesh64 = io64;
  nb.tab = f64 ? (const void*)pl->ntab64 : (const void*)pl->ntab32;
  nb.C = 2 * s - 1;
  nb.X = rho_in;
  nb.Y = phi_out;
  nb.grid_in = 1;
  nb.grid_out = 1;
  nb.xscale = 1.0 / ((double)N * N * N);
  nb.accumulate = 0;
  nb.groups = 1;
  nb.isolated = pl->isolated;
  // P2M and L2P folded into the FFT near zone's leaf transforms of the
  // potential (FP32 leaf gridlets): the tree waits for the forward
  // transforms, the potential's inverse transform for the leaf locals
  const bool fold = pl->fold && near_fft && !io64 && !is64(L) && near_fft_folds(pl->nfft, p);
  LeafTree lt{};
  if (fold) {
    lt.M = static_cast<float*>(pl->M[L]);
    lt.Pl = static_cast<const float*>(pl->P[L]);
    lt.A = pl->dA;
    lt.h3 = (float)h3;
    lt.p = p;
  }
  tm.at(PFMM_STAGE_NEAR, 0);
  if (near_fft) {  // each of its kernels timed
    float* outs[4] = {phi, nullptr, nullptr, nullptr};
    int nout = 1;
    if (accel && pl->accel_mode)
      for (int c = 0; c < 3; ++c) outs[nout++] = accel + (size_t)c * N * N * N;
    e = fold ? near_fft_begin(pl->nfft, rho, outs, nout, pl->isolated, lt,
                              overlap ? pl->ev_mass : nullptr, sn, tm.on ? &tm : nullptr)
             : near_fft_run(pl->nfft, rho, outs, nout, pl->isolated, sn, tm.on ? &tm : nullptr);
  } else if (mx && pl->nwin) {
    e = tm.begin(sn);
    if (e == hipSuccess) e = split_mesh(rho, (float)h3, N, kNearTerms, pl->xsn, sn);
    if (e == hipSuccess) {
      ToepMfmaArgs ma{};
      ma.n = nb.n;
      ma.m = nb.m;
      ma.noff = nb.noff;
      ma.offs = nb.offs;
      ma.win = pl->nwin;
      ma.X = pl->xsn;
      ma.Y = phi;
      ma.grid_out = 1;
      ma.accumulate = 0;
      ma.groups = 1;
      ma.isolated = pl->isolated;
      ma.zero = pl->zero;
      e = launch_toep8_split(ma, kNearTerms, sn);
      // accelerations from the expansion: the near zone with the three
      // acceleration kernels, into the three components
      for (int c = 0; c < 3 && e == hipSuccess && accel && pl->accel_mode; ++c) {
        ma.win = pl->ndwin[c];
        ma.Y = accel + (size_t)c * N * N * N;
        e = launch_toep8_split(ma, kNearTerms, sn);
      }
    }
    if (e == hipSuccess) e = tm.end(sn, 0);
  } else {
    e = tm.begin(sn);
    if (e == hipSuccess) e = launch_toeplitz(nb, sn);
    for (int c = 0; c < 3 && e == hipSuccess && accel && pl->accel_mode; ++c) {
      nb.tab = f64 ? (const void*)pl->ndtab64[c] : (const void*)pl->ndtab32[c];
      nb.Y = acc_c(c);
      e = launch_toeplitz(nb, sn);
    }
    if (e == hipSuccess) e = tm.end(sn, 0);
  }
  if (e == hipSuccess && overlap && !fold) e = hipEventRecord(pl->ev_join, pl->side);
  if (e != hipSuccess) return hip_fail(e, "near zone");

  // upward pass
  if (fold) {
    if (overlap) {
      e = hipStreamWaitEvent(st, pl->ev_mass, 0);
      if (e != hipSuccess) return hip_fail(e, "leaf masses");
    }
  } else {
    e = timed(PFMM_STAGE_P2M, 0, st, [&] {
      return io64 ? launch_p2m_f64in(static_cast<const double*>(rho_in), pl->M[L], A, N, s, p, h3, st)
                  : launch_p2m(rho, pl->M[L], is64(L), A, N, s, p, (double)h3, st);
    });
    if (e != hipSuccess) return hip_fail(e, "P2M");
  }
  for (int l = L - 1; l >= 2; --l) {
    e = timed(PFMM_STAGE_M2M, l, st, [&] {
      return launch_m2m(pl->M[l + 1], is64(l + 1), pl->M[l], is64(l), T, 1 << l, p, st);
    });
    if (e != hipSuccess) return hip_fail(e, "M2M");
  }

  // interaction zones, level 2 (periodic) then 3 .. L with L2L first
  ToepArgs a{};
  a.q = p;
  a.C = 4 * p - 1;
  a.xscale = 1.0;
  a.n = 4;
  a.m = 1;
  a.noff = pl->nl2;
  a.offs = pl->offs_l2;
  a.isolated = pl->isolated;
  a.fp64 = is64(2);
  a.tab = a.fp64 ? (const void*)pl->tab64[2] : (const void*)pl->tab32[2];
  a.X = pl->M[2];
  a.Y = pl->P[2];
  a.accumulate = 0;
  // the spectral zones time each of their kernels themselves
  auto m2l_timed = [&](const ToepArgs& ta, int l) -> hipError_t {
    if (pl->m2l_spectral && !pl->m2l_fft) {
      tm.at(PFMM_STAGE_M2L, l);
      return m2l(ta, l);
    }
    return timed(PFMM_STAGE_M2L, l, st, [&] { return m2l(ta, l); });
  };
  e = m2l_timed(a, 2);
  if (e != hipSuccess) return hip_fail(e, "M2L level 2");
  for (int l = 3; l <= L; ++l) {
    e = timed(PFMM_STAGE_L2L, l, st, [&] {
      return launch_l2l(pl->P[l - 1], is64(l - 1), pl->P[l], is64(l), T, 1 << (l - 1), p, st);
    });
    if (e != hipSuccess) return hip_fail(e, "L2L");
    a.n = 1 << l;
    a.m = 2;
    a.noff = 189;
    a.offs = pl->offs_iz;
    a.fp64 = is64(l);
    a.tab = a.fp64 ? (const void*)pl->tab64[l] : (const void*)pl->tab32[l];
    a.X = pl->M[l];
    a.Y = pl->P[l];
    a.accumulate = 1;
    e = m2l_timed(a, l);
    if (e != hipSuccess) return hip_fail(e, "M2L");
  }

  // downward to the mesh, added to the near zone
  if (fold) {
    if (overlap) {
      e = hipEventRecord(pl->ev_local, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(sn, pl->ev_local, 0);
    }
    tm.at(PFMM_STAGE_NEAR, 0);
    if (e == hipSuccess) e = near_fft_end(pl->nfft, phi, lt, sn, tm.on ? &tm : nullptr);
    if (e == hipSuccess && overlap) e = hipEventRecord(pl->ev_join, sn);
    if (e != hipSuccess) return hip_fail(e, "near zone");
  }
  if (overlap) {
    e = hipStreamWaitEvent(st, pl->ev_join, 0);
    if (e != hipSuccess) return hip_fail(e, "join");
  }
  if (!fold) {
    e = timed(PFMM_STAGE_L2P, 0, st, [&] {
      return io64 ? launch_l2p_f64out(pl->P[L], static_cast<double*>(phi_out), A, N, s, p, st, 1)
                  : launch_l2p(pl->P[L], is64(L), phi, A, N, s, p, st, 1);
    });
    if (e != hipSuccess) return hip_fail(e, "L2P");
  }

  if (accel && pl->accel_mode) {
    // far part: gradient of the leaf's local expansion, -d/dx = -(1/eta_L) d/dv
    const Weights Ad = wts(pl->dAd, pl->dAd64);
    const double sc = -(double)(1 << L) * p;
    e = timed(PFMM_STAGE_FD4, 0, st, [&] {
      return io64 ? launch_l2p_grad_f64out(pl->P[L], static_cast<double*>(accel_out), A, Ad, sc, N, s,
                                           p, st)
                  : launch_l2p_grad(pl->P[L], is64(L), accel, A, Ad, sc, N, s, p, st);
    });
    if (e != hipSuccess) return hip_fail(e, "expansion gradient");
  } else if (accel) {
    e = timed(PFMM_STAGE_FD4, 0, st, [&] {
      return io64 ? launch_fd4_f64(static_cast<const double*>(phi_out), static_cast<double*>(accel_out),
                                   N, st)
                  : launch_fd4(phi, accel, N, st);
    });
    if (e != hipSuccess) return hip_fail(e, "FD4");
  }
  if (pl->profile) {
    pl->ev_used[slot] = tm.n;
    ++pl->nprof;
  }
  return PFMM_OK;
}

// A learned-G plan without weights solves with its G_S1 tables: say so.
pfmm_status note_fallback(const pfmm_plan_s* pl, pfmm_status st) {
  if (st == PFMM_OK && pl->learned_kind && !pl->learned)
    g_err = "PFMM_GREEN_LEARNED: no network weights set, solved with the G_S1 fallback";
  return st;
}

}  // namespace

extern "C" {

pfmm_status pfmm_solve(pfmm_plan_t h, const float* rho, float* phi, float* accel) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  return note_fallback(pl, solve_impl(pl, rho, phi, accel, 0));
}

pfmm_status pfmm_solve_f64(pfmm_plan_t h, const double* rho, double* phi, double* accel) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  return note_fallback(pl, solve_impl(pl, rho, phi, accel, 1));
}

pfmm_status pfmm_plan_read(pfmm_plan_t h, int buffer, int level, void* dst) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (!dst) return fail(PFMM_ERR_INVALID_ARG, "dst is NULL");
  const void* src = nullptr;
  size_t bytes = 0;
  const size_t p3 = (size_t)pl->p * pl->p * pl->p;
  if (buffer == PFMM_BUF_TABLE_NEAR) {
    src = pl->ntab64;
    bytes = (size_t)cube(4 * pl->s - 1) * sizeof(double);
  } else {
    if (level < 2 || level > pl->L) return fail(PFMM_ERR_INVALID_ARG, "level out of range");
    const size_t nodes = (size_t)1 << (3 * level);
    switch (buffer) {
      case PFMM_BUF_MULTIPOLE:
      case PFMM_BUF_LOCAL: {
        const void* b = buffer == PFMM_BUF_MULTIPOLE ? pl->M[level] : pl->P[level];
        hipError_t e = level64(pl, level)
                           ? launch_cast_d2f((const double*)b, (float*)dst, (int64_t)(nodes * p3),
                                             pl->stream)
                           : hipMemcpyAsync(dst, b, nodes * p3 * sizeof(float),
                                            hipMemcpyDeviceToDevice, pl->stream);
        if (e != hipSuccess) return hip_fail(e, "read buffer");
        return PFMM_OK;
      }
      case PFMM_BUF_TABLE_LEVEL:
        src = pl->tab64[level];
        bytes = (size_t)cube(8 * pl->p - 1) * sizeof(double);
        break;
      default: return fail(PFMM_ERR_INVALID_ARG, "unknown buffer");
    }
  }
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, pl->stream);
  if (e != hipSuccess) return hip_fail(e, "read buffer");
  return PFMM_OK;
}

}  // extern "C"

namespace {

// Visit every timed interval of the recent profiled solves (newest first):
// f(solve index, interval index within the solve, tag, ms).  Waits for them.
template <class F>
pfmm_status each_interval(pfmm_plan_s* pl, F f) {
  if (pl->nprof == 0) return fail(PFMM_ERR_INVALID_ARG, "no profiled solve");
  const int nsol = pl->nprof < kSlots ? pl->nprof : kSlots;
  for (int j = 0; j < nsol; ++j) {
    const int slot = (pl->nprof - 1 - j) % kSlots;
    const hipEvent_t* ev = pl->ev.data() + (size_t)slot * 2 * kMaxIntervals;
    const int* tag = pl->ev_tag.data() + (size_t)slot * kMaxIntervals;
    for (int k = 0; k < pl->ev_used[slot]; ++k) {
      hipError_t e = hipEventSynchronize(ev[2 * k + 1]);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
      if (e != hipSuccess) return hip_fail(e, "profile events");
      f(j, k, tag[k], (double)t);
    }
  }
  return PFMM_OK;
}

int solves_kept(const pfmm_plan_s* pl) { return pl->nprof < kSlots ? pl->nprof : kSlots; }

}  // namespace

extern "C" {

pfmm_status pfmm_plan_stage_times(pfmm_plan_t h, double* ms, int* launches) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_plan_stage_times");
  if (!ms) return fail(PFMM_ERR_INVALID_ARG, "ms is NULL");
  for (int k = 0; k < PFMM_STAGE_COUNT; ++k) {
    ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  const double w = pl->nprof ? 1.0 / solves_kept(pl) : 0.0;
  return each_interval(pl, [&](int j, int, int tag, double t) {
    const int stg = tag & 255;
    if (stg >= PFMM_STAGE_COUNT) return;
    ms[stg] += t * w;
    if (launches && j == 0) launches[stg] += 1;
  });
}

pfmm_status pfmm_plan_level_times(pfmm_plan_t h, int stage, double* ms) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_plan_level_times");
  if (!ms) return fail(PFMM_ERR_INVALID_ARG, "ms is NULL");
  if (stage != PFMM_STAGE_M2M && stage != PFMM_STAGE_M2L && stage != PFMM_STAGE_L2L)
    return fail(PFMM_ERR_INVALID_ARG, "stage has no per-level launches");
  for (int l = 0; l <= pl->L; ++l) ms[l] = 0.0;
  const double w = pl->nprof ? 1.0 / solves_kept(pl) : 0.0;
  return each_interval(pl, [&](int, int, int tag, double t) {
    const int l = (tag >> 8) & 255;
    if ((tag & 255) == stage && l <= pl->L) ms[l] += t * w;
  });
}

pfmm_status pfmm_plan_kernel_times(pfmm_plan_t h, int stage, int level, double* ms, int* count) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_plan_kernel_times");
  if (!ms || !count) return fail(PFMM_ERR_INVALID_ARG, "ms and count are required");
  if (stage < 0 || stage >= PFMM_STAGE_COUNT) return fail(PFMM_ERR_INVALID_ARG, "unknown stage");
  for (int k = 0; k < 8; ++k) ms[k] = 0.0;
  *count = 0;
  const double w = pl->nprof ? 1.0 / solves_kept(pl) : 0.0;
  return each_interval(pl, [&](int, int, int tag, double t) {
    const int part = (tag >> 16) & 255;
    if ((tag & 255) != stage || ((tag >> 8) & 255) != level || part >= 8) return;
    ms[part] += t * w;
    if (part + 1 > *count) *count = part + 1;
  });
}

pfmm_status pfmm_plan_info(pfmm_plan_t h, int* s, int64_t* table_entries) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (s) *s = pl->s;
  if (table_entries) *table_entries = cube(8 * pl->p - 1);
  return PFMM_OK;
}

pfmm_status pfmm_plan_destroy(pfmm_plan_t h) {
  g_err.clear();
  if (!h) return PFMM_OK;
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_plan_destroy");
  drop_cached_batches(pl);
  if (pl->batch_refs > 0)
    return fail(PFMM_ERR_INVALID_ARG, "the plan is bound to a live batch: destroy the batch first");
  if (!g_plans.remove(h)) return bad_plan();
  hipError_t e = hipStreamSynchronize(pl->stream);
  release(pl);
  if (e != hipSuccess) return hip_fail(e, "destroy");
  return PFMM_OK;
}

const char* pfmm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent fields
// ---------------------------------------------------------------------------
struct pfmm_batch_s {
  std::vector<pfmm_plan_s*> plans;
  std::vector<pfmm_plan_t> handles;  // the plans' handles (checked live before every launch)
  bool cached = false;               // made by pfmm_solve_batch, owned by its cache
  std::vector<const float*> rho;
  std::vector<float*> phi;
  hipStream_t caller = nullptr;  // stream of plans[0]; solves are ordered with it
  hipStream_t stream = nullptr;  // the batch's own stream (captured into the graph)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // the matrix-core persistent kernels run beside the portable one (their
  // outputs are disjoint): two more streams, forked and joined by events
  hipStream_t s_split = nullptr, s_f64 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_split = nullptr, ev_f64 = nullptr;
  // fields whose every contraction is one of their plan's own transform
  // kernels (FFT near zone, spectral zones) need no work list: each runs its
  // whole solve as one chain, the chains spread over kChains forked streams
  static constexpr int kChains = 4;
  hipStream_t s_chain[kChains] = {};
  hipEvent_t ev_chain[kChains] = {};
  BatchItem* items = nullptr;  // device work list (portable kernel)
  unsigned* counter = nullptr;  // [0] portable, [1] split, [2] FP64 matrix-core list
  int nitems = 0, grid = 0;
  // matrix-core work lists: split near zones (plans in split precision) and
  // the FP64 levels at p = 8
  ToepMfmaArgs* sargs = nullptr;
  ToepF64Args* fargs = nullptr;
  MmaItem* sitems = nullptr;
  MmaItem* fitems = nullptr;
  int nsplit = 0, nf64 = 0, sgrid = 0, fgrid = 0;
  // portable item groups (block edge, FP64, near zone): tuned tile width and
  // the timed launch of the group's items at widths 1, 2, 4 (-1: not timed)
  struct Group {
    std::string key;
    int q, fp64, near, width;
    double ms[3];
  };
  std::vector<Group> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

Registry<pfmm_batch_s, 0x71> g_batches;

pfmm_batch_s* batch_of(pfmm_batch_t h) { return g_batches.get(h); }
pfmm_status bad_batch() { return fail(PFMM_ERR_BAD_HANDLE, "not a live batch handle"); }

// Batches made by pfmm_solve_batch, one per set of (plan, density,
// potential), reused while that set is solved again.
struct CachedBatch {
  std::vector<pfmm_plan_t> plans;
  std::vector<const float*> rho;
  std::vector<float*> phi;
  pfmm_batch_t handle;
};
std::mutex g_cmu;
std::vector<CachedBatch> g_cache;

void brelease(pfmm_batch_s* b) {
  for (pfmm_plan_s* pl : b->plans) --pl->batch_refs;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->items) (void)hipFree(b->items);
  if (b->counter) (void)hipFree(b->counter);
  if (b->sargs) (void)hipFree(b->sargs);
  if (b->fargs) (void)hipFree(b->fargs);
  if (b->sitems) (void)hipFree(b->sitems);
  if (b->fitems) (void)hipFree(b->fitems);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (hipEvent_t ev : {b->ev_fork, b->ev_split, b->ev_f64})
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t s : {b->s_split, b->s_f64})
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (int c = 0; c < pfmm_batch_s::kChains; ++c) {
    if (b->ev_chain[c]) (void)hipEventDestroy(b->ev_chain[c]);
    if (b->s_chain[c]) {
      (void)hipStreamSynchronize(b->s_chain[c]);
      (void)hipStreamDestroy(b->s_chain[c]);
    }
  }
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Contractions that go to the matrix-core persistent kernels: the near zone
// of a plan in split precision with 8^3-cell sub-blocks, and FP64 levels at
// p = 8 (the same kernels as a single solve, so the same results).
bool batch_split_near(const pfmm_plan_s* pl) {
  return !pl->near_fft && pl->prec == PFMM_PREC_BF16X3 && pl->nwin;
}
bool batch_f64_level(const pfmm_plan_s* pl, int l) { return level64(pl, l) && pl->p == 8; }
// A field solved as one chain of its own kernels (no work items).
bool batch_chain(const pfmm_plan_s* pl) {
  return pl->near_fft && pl->m2l_spectral && near_fft_fused(pl->nfft);
}

// Tuning group of a portable item: block edge, FP64 or FP32, near zone or
// interaction zone (in the terms of the method: p or the leaf width s, and the
// precision).
std::string group_key(const BatchItem& it) {
  return "q" + std::to_string(it.q) + (it.fp64 ? "-f64" : "-f32") + (it.grid ? "-near" : "-zone");
}

// Work items of every other contraction of every field, largest first; the
// FP32 tile width of each group from `widths` (default 2), only the items of
// group `only` when it is given.
std::vector<BatchItem> batch_items(const pfmm_batch_s* b, const std::map<std::string, int>& widths,
                                   const std::string* only = nullptr) {
  struct Keyed {
    double cost;
    BatchItem it;
  };
  std::vector<Keyed> all;
  auto add = [&](BatchItem proto) {
    const std::string key = group_key(proto);
    if (only && key != *only) return;
    const auto wi = widths.find(key);
    proto.tpt = proto.fp64 ? 1 : (wi != widths.end() ? wi->second : 2);
    const int TT = batch_targets_per_item(proto.q, proto.tpt, proto.fp64);
    const int nk = proto.n / proto.m;
    const int ntarg = nk * nk * nk;
    const double cost = (double)proto.noff * std::min(TT, ntarg) * std::pow((double)proto.q, 6.0);
    for (int c = 0; c < proto.m * proto.m * proto.m; ++c)
      for (int t0 = 0; t0 < ntarg; t0 += TT) {
        BatchItem it = proto;
        it.cls = c;
        it.t0 = t0;
        all.push_back({cost, it});
      }
  };
  for (size_t f = 0; f < b->plans.size(); ++f) {
    const pfmm_plan_s* pl = b->plans[f];
    const int p = pl->p;
    for (int l = 2; l <= pl->L; ++l) {
      if (batch_f64_level(pl, l) || pl->m2l_spectral) continue;  // other lists / own launches
      BatchItem it{};
      it.fp64 = level64(pl, l);
      it.tab = it.fp64 ? (const void*)pl->tab64[l] : (const void*)pl->tab32[l];
      it.X = pl->M[l];
      it.Y = pl->P[l];
      it.offs = l == 2 ? pl->offs_l2 : pl->offs_iz;
      it.n = 1 << l;
      it.m = l == 2 ? 1 : 2;
      it.q = p;
      it.C = 4 * p - 1;
      it.noff = l == 2 ? 37 : 189;
      it.grid = 0;
      it.xscale = 1.0f;
      add(it);
    }
    BatchItem nb{};
    nb.fp64 = 0;
    nb.tab = pl->ntab32;
    nb.X = b->rho[f];
    nb.Y = b->phi[f];
    nb.offs = pl->offs_near;
    nb.n = pl->N / pl->qn;
    nb.m = pl->mn;
    nb.q = pl->qn;
    nb.C = 2 * pl->s - 1;
    nb.noff = (int)cube(3 * pl->mn);
    nb.grid = 1;
    nb.xscale = (float)(1.0 / ((double)pl->N * pl->N * pl->N));
    if (!batch_split_near(pl) && !pl->near_fft) add(nb);  // FFT near zones run on their own
  }
  std::stable_sort(all.begin(), all.end(),
                   [](const Keyed& a, const Keyed& c) { return a.cost > c.cost; });
  std::vector<BatchItem> out;
  out.reserve(all.size());
  for (auto& k : all) out.push_back(k.it);
  return out;
}

// Argument arrays and item lists of the matrix-core kernels (one item per
// workgroup tile, all offsets; FP64 items of the larger zone first).
hipError_t batch_mma_upload(pfmm_batch_s* b) {
  std::vector<ToepMfmaArgs> sa;
  std::vector<ToepF64Args> fa;
  std::vector<MmaItem> si, fi;
  for (size_t f = 0; f < b->plans.size(); ++f) {
    const pfmm_plan_s* pl = b->plans[f];
    for (int l = 3; l >= 2; --l) {
      if (l > pl->L || !batch_f64_level(pl, l) || pl->m2l_spectral) continue;
      ToepF64Args x{};
      x.n = 1 << l;
      x.m = l == 2 ? 1 : 2;
      x.noff = l == 2 ? 37 : 189;
      x.offs = l == 2 ? pl->offs_l2 : pl->offs_iz;
      x.tab = pl->tab64[l];
      x.C = 4 * pl->p - 1;
      x.X = (const double*)pl->M[l];
      x.Y = (double*)pl->P[l];
      x.accumulate = 0;
      x.groups = 1;
      x.partial = nullptr;
      const int arg = (int)fa.size();
      fa.push_back(x);
      for (int t = 0; t < toep8_f64_tiles(x.n, x.m); ++t) fi.push_back({arg, t});
    }
    if (batch_split_near(pl)) {
      ToepMfmaArgs y{};
      y.n = pl->N / pl->qn;
      y.m = pl->mn;
      y.noff = (int)cube(3 * pl->mn);
      y.offs = pl->offs_near;
      y.win = pl->nwin;
      y.X = pl->xsn;
      y.Y = b->phi[f];
      y.grid_out = 1;
      y.accumulate = 0;
      y.groups = 1;
      y.partial = nullptr;
      const int arg = (int)sa.size();
      sa.push_back(y);
      for (int t = 0; t < toep8_split_tiles(y.n, y.m); ++t) si.push_back({arg, t});
    }
  }
  // level-3 items (189 offsets) before level-2 items (37)
  std::stable_sort(fi.begin(), fi.end(), [&](const MmaItem& a, const MmaItem& c) {
    return fa[a.arg].noff > fa[c.arg].noff;
  });
  hipError_t e = hipSuccess;
  auto up = [&](auto** dst, const auto& v) {
    if (e != hipSuccess || v.empty()) return;
    e = hipMalloc(dst, v.size() * sizeof(v[0]));
    if (e == hipSuccess)
      e = hipMemcpy(*dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
  };
  up(&b->sargs, sa);
  up(&b->fargs, fa);
  up(&b->sitems, si);
  up(&b->fitems, fi);
  b->nsplit = (int)si.size();
  b->nf64 = (int)fi.size();
  b->sgrid = batch_mma_grid(2);
  b->fgrid = batch_mma_grid(64);
  return e;
}

hipError_t batch_upload(pfmm_batch_s* b, const std::map<std::string, int>& widths,
                        const std::string* only = nullptr) {
  const std::vector<BatchItem> v = batch_items(b, widths, only);
  if (b->items) (void)hipFree(b->items);
  b->items = nullptr;
  hipError_t e = hipMalloc(&b->items, std::max<size_t>(1, v.size()) * sizeof(BatchItem));
  if (e != hipSuccess) return e;
  e = hipMemcpy(b->items, v.data(), v.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  b->nitems = (int)v.size();
  b->grid = batch_resident_grid();
  return e;
}

// The whole batch solve, enqueued on the batch stream.  `part`: 0 = all,
// 1 = upward passes only, 2 = the persistent contractions only, 3 = downward,
// 4 = the portable persistent kernel only.
// One chain field's whole solve on stream `st`, in the order of a single
// solve: near zone (writes the potential), upward pass, level 2, then per
// level L2L and the zones, and L2P added to the potential.
hipError_t batch_chain_solve(pfmm_batch_s* b, size_t f, hipStream_t st) {
  pfmm_plan_s* pl = b->plans[f];
  const Weights T = wts(pl->dT, pl->dT64);
  float* out[1] = {b->phi[f]};
  hipError_t e = near_fft_run(pl->nfft, b->rho[f], out, 1, 0, st);
  if (e == hipSuccess)
    e = launch_p2m(b->rho[f], pl->M[pl->L], level64(pl, pl->L), wts(pl->dA, pl->dA64), pl->N, pl->s,
                   pl->p, 1.0 / ((double)pl->N * pl->N * pl->N), st);
  for (int l = pl->L - 1; l >= 2 && e == hipSuccess; --l)
    e = launch_m2m(pl->M[l + 1], level64(pl, l + 1), pl->M[l], level64(pl, l), T, 1 << l, pl->p, st);
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l) {
    if (l > 2)
      e = launch_l2l(pl->P[l - 1], level64(pl, l - 1), pl->P[l], level64(pl, l), T, 1 << (l - 1),
                     pl->p, st);
    if (e == hipSuccess)
      e = m2l_spectral_level(pl->mspec, l, pl->M[l], level64(pl, l), pl->P[l], level64(pl, l), l > 2,
                             l == 2 ? pl->offs_l2 : pl->offs_iz, l == 2 ? pl->nl2 : 189, 0, st);
  }
  if (e == hipSuccess)
    e = launch_l2p(pl->P[pl->L], level64(pl, pl->L), b->phi[f], wts(pl->dA, pl->dA64), pl->N, pl->s,
                   pl->p, st, 1);
  return e;
}

hipError_t batch_enqueue(pfmm_batch_s* b, int part) {
  hipStream_t st = b->stream;
  hipError_t e = hipSuccess;
  if (part == 0) {  // chain fields, spread over the forked chain streams
    bool any = false;
    for (pfmm_plan_s* pl : b->plans) any = any || batch_chain(pl);
    if (any) {
      e = hipEventRecord(b->ev_fork, st);
      for (int c = 0; c < pfmm_batch_s::kChains && e == hipSuccess; ++c)
        e = hipStreamWaitEvent(b->s_chain[c], b->ev_fork, 0);
      int next = 0;
      for (size_t f = 0; f < b->plans.size() && e == hipSuccess; ++f)
        if (batch_chain(b->plans[f])) {
          e = batch_chain_solve(b, f, b->s_chain[next]);
          next = (next + 1) % pfmm_batch_s::kChains;
        }
    }
  }
  if (e == hipSuccess && (part == 0 || part == 1)) {
    for (size_t f = 0; f < b->plans.size() && e == hipSuccess; ++f) {
      pfmm_plan_s* pl = b->plans[f];
      if (batch_chain(pl)) continue;
      const Weights T = wts(pl->dT, pl->dT64);
      e = launch_p2m(b->rho[f], pl->M[pl->L], level64(pl, pl->L), wts(pl->dA, pl->dA64), pl->N,
                     pl->s, pl->p, 1.0 / ((double)pl->N * pl->N * pl->N), st);
      for (int l = pl->L - 1; l >= 2 && e == hipSuccess; --l)
        e = launch_m2m(pl->M[l + 1], level64(pl, l + 1), pl->M[l], level64(pl, l), T, 1 << l,
                       pl->p, st);
      if (e == hipSuccess && batch_split_near(pl))
        e = split_mesh(b->rho[f], (float)(1.0 / ((double)pl->N * pl->N * pl->N)), pl->N,
                       kNearTerms, pl->xsn, st);
    }
  }
  if (e == hipSuccess && (part == 0 || part == 2)) {
    // the three persistent kernels read only the upward passes' outputs and
    // write disjoint buffers (a field's near zone and each level go to exactly
    // one list), so they run side by side: the tail of one fills with the
    // others' workgroups
    e = hipEventRecord(b->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->s_split, b->ev_fork, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->s_f64, b->ev_fork, 0);
    if (e == hipSuccess)
      e = launch_batch_mma(2, b->sargs, b->sitems, b->nsplit, b->counter + 1, b->sgrid, b->s_split);
    if (e == hipSuccess)
      e = launch_batch_mma(64, b->fargs, b->fitems, b->nf64, b->counter + 2, b->fgrid, b->s_f64);
    // FFT near zones and spectral interaction zones (their own kernels, no
    // work items): they write the potential and each level's zone sums
    // before the downward passes add to them
    for (size_t f = 0; f < b->plans.size() && e == hipSuccess; ++f) {
      pfmm_plan_s* pl = b->plans[f];
      if (batch_chain(pl)) continue;
      if (pl->near_fft) {
        float* out[1] = {b->phi[f]};
        e = near_fft_run(pl->nfft, b->rho[f], out, 1, 0, st);
      }
      for (int l = 2; l <= pl->L && e == hipSuccess && pl->m2l_spectral; ++l)
        e = m2l_spectral_level(pl->mspec, l, pl->M[l], level64(pl, l), pl->P[l], level64(pl, l), 0,
                               l == 2 ? pl->offs_l2 : pl->offs_iz, l == 2 ? pl->nl2 : 189, 0, st);
    }
    if (e == hipSuccess) e = launch_batch_toeplitz(b->items, b->nitems, b->counter, b->grid, st);
    if (e == hipSuccess) e = hipEventRecord(b->ev_split, b->s_split);
    if (e == hipSuccess) e = hipEventRecord(b->ev_f64, b->s_f64);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_split, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_f64, 0);
  } else if (e == hipSuccess && part == 4) {
    e = launch_batch_toeplitz(b->items, b->nitems, b->counter, b->grid, st);
  }
  if (e == hipSuccess && (part == 0 || part == 3)) {
    for (size_t f = 0; f < b->plans.size() && e == hipSuccess; ++f) {
      pfmm_plan_s* pl = b->plans[f];
      if (batch_chain(pl)) continue;
      const Weights T = wts(pl->dT, pl->dT64);
      for (int l = 3; l <= pl->L && e == hipSuccess; ++l)
        e = launch_l2l(pl->P[l - 1], level64(pl, l - 1), pl->P[l], level64(pl, l), T,
                       1 << (l - 1), pl->p, st, 1);
      if (e == hipSuccess)
        e = launch_l2p(pl->P[pl->L], level64(pl, pl->L), b->phi[f], wts(pl->dA, pl->dA64),
                       pl->N, pl->s, pl->p, st, 1);
    }
  }
  if (e == hipSuccess && part == 0) {  // join the chains
    bool any = false;
    for (pfmm_plan_s* pl : b->plans) any = any || batch_chain(pl);
    for (int c = 0; c < pfmm_batch_s::kChains && e == hipSuccess && any; ++c) {
      e = hipEventRecord(b->ev_chain[c], b->s_chain[c]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_chain[c], 0);
    }
  }
  return e;
}


// Cache: a flat JSON object {"<signature>": tile_width, ...}.
int cache_lookup(const char* path, const std::string& key) {
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  std::fclose(f);
  const std::string pat = "\"" + key + "\":";
  const size_t at = txt.find(pat);
  if (at == std::string::npos) return 0;
  const int v = std::atoi(txt.c_str() + at + pat.size());
  return (v == 1 || v == 2 || v == 4) ? v : 0;
}

void cache_store(const char* path, const std::string& key, int tpt) {
  std::string txt;
  if (FILE* f = std::fopen(path, "r")) {
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
  }
  const size_t close = txt.rfind('}');
  std::string body = close == std::string::npos ? std::string() : txt.substr(0, close);
  const size_t open = body.find('{');
  body = open == std::string::npos ? std::string() : body.substr(open + 1);
  while (!body.empty() && (body.back() == ' ' || body.back() == '\n')) body.pop_back();
  std::string out = "{" + body + (body.empty() ? "" : ",") + "\n  \"" + key + "\": " +
                    std::to_string(tpt) + "\n}\n";
  if (FILE* f = std::fopen(path, "w")) {
    std::fwrite(out.data(), 1, out.size(), f);
    std::fclose(f);
  }
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

pfmm_status batch_create_impl(int n, const pfmm_plan_t* handles, const float* const* density,
                              float* const* potential, bool cached, pfmm_batch_t* out) {
  if (!out) return fail(PFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > 4096 || !handles || !density || !potential)
    return fail(PFMM_ERR_INVALID_ARG, "need 1 <= n <= 4096 and non-NULL arrays");
  std::vector<pfmm_plan_s*> plans(n);
  for (int i = 0; i < n; ++i) {
    plans[i] = plan_of(handles[i]);
    if (!plans[i]) return bad_plan();
    if (!density[i] || !potential[i]) return fail(PFMM_ERR_INVALID_ARG, "NULL buffer in batch");
  }
  if (capturing(plans[0]->stream)) return capture_fail("creating a batch");
  pfmm_batch_s* b = new (std::nothrow) pfmm_batch_s;
  if (!b) return fail(PFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->cached = cached;
  for (int i = 0; i < n; ++i) {
    if (plans[i]->prec == PFMM_PREC_FP64) {
      delete b;
      return fail(PFMM_ERR_UNSUPPORTED, "batches of PFMM_PREC_FP64 plans");
    }
    if (plans[i]->p > 8) {
      delete b;
      return fail(PFMM_ERR_UNSUPPORTED, "batches need p <= 8");
    }
    if (plans[i]->isolated) {
      delete b;
      return fail(PFMM_ERR_UNSUPPORTED, "batches of isolated plans");
    }
    if (plans[i]->m2l_fft) {
      delete b;
      return fail(PFMM_ERR_UNSUPPORTED, "batches of plans with FFT interaction zones");
    }
    if (plans[i]->near_fft && !near_fft_fused(plans[i]->nfft)) {
      delete b;
      return fail(PFMM_ERR_UNSUPPORTED,
                  "batches take the FFT near zone for leaf edges 4, 8 and 16 only");
    }
    if (plans[i]->near_fft && (((uintptr_t)density[i] | (uintptr_t)potential[i]) & 15)) {
      delete b;
      return fail(PFMM_ERR_INVALID_ARG, "the FFT near zone needs 16-byte aligned density and outputs");
    }
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) {
        delete b;
        return fail(PFMM_ERR_INVALID_ARG, "a plan appears twice in a batch");
      }
    b->plans.push_back(plans[i]);
    b->handles.push_back(handles[i]);
    b->rho.push_back(density[i]);
    b->phi.push_back(potential[i]);
  }
  // from here on the plans know the batch holds them (brelease undoes this)
  for (pfmm_plan_s* pl : b->plans) ++pl->batch_refs;
  b->caller = plans[0]->stream;
  // default priority (no priority streams anywhere in this library)
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->s_split, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->s_f64, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&b->ev_fork, &b->ev_split, &b->ev_f64})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  for (int c = 0; c < pfmm_batch_s::kChains && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&b->s_chain[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_chain[c], hipEventDisableTiming);
  }
  // inputs written on the caller's stream must be visible to the tuning runs
  if (e == hipSuccess) e = hipStreamSynchronize(b->caller);
  if (e == hipSuccess) e = hipMalloc(&b->counter, 3 * sizeof(unsigned));
  if (e == hipSuccess) e = batch_mma_upload(b);
  if (e != hipSuccess) {
    brelease(b);
    return hip_fail(e, "batch work lists");
  }
  // tile width per group of portable items: cache, else time each candidate
  // on the group's own items (after one full solve makes every input valid)
  std::map<std::string, int> widths;
  {
    std::map<std::string, pfmm_batch_s::Group> found;
    for (const BatchItem& it : batch_items(b, widths)) {
      const std::string key = group_key(it);
      if (!found.count(key))
        found[key] = {key, it.q, it.fp64, it.grid, it.fp64 ? 1 : 2, {-1.0, -1.0, -1.0}};
    }
    for (auto& kv : found) b->groups.push_back(kv.second);
  }
  const char* cache = std::getenv("PFMM_TUNE_CACHE");
  e = batch_upload(b, widths);
  if (e == hipSuccess) e = batch_enqueue(b, 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int cand[3] = {1, 2, 4};
  for (auto& g : b->groups) {
    if (e != hipSuccess) break;
    if (g.fp64) continue;  // FP64 items have tile width 1
    const std::string ckey = "batch-" + g.key;
    int w = cache ? cache_lookup(cache, ckey) : 0;
    if (!w) {
      double best = 1e300;
      for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        std::map<std::string, int> trial = widths;
        trial[g.key] = cand[c];
        e = batch_upload(b, trial, &g.key);
        float ms = 0.f, msmin = 1e30f;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) {  // first run warms up
          e = hipEventRecord(e0, b->stream);
          if (e == hipSuccess) e = batch_enqueue(b, 4);
          if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (r > 0) msmin = std::min(msmin, ms);
        }
        if (e != hipSuccess) break;
        g.ms[c] = msmin;
        if (msmin < best) {
          best = msmin;
          w = cand[c];
        }
      }
      if (e == hipSuccess && cache) cache_store(cache, ckey, w);
    }
    g.width = w;
    widths[g.key] = w;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e == hipSuccess) e = batch_upload(b, widths);
  if (e != hipSuccess) {
    (void)hipDeviceSynchronize();
    brelease(b);
    return hip_fail(e, "batch tuning");
  }
  // capture the whole batch solve
  if (e == hipSuccess) e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t ee = batch_enqueue(b, 0);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (ee != hipSuccess) e = ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipDeviceSynchronize();
    brelease(b);
    return hip_fail(e, "batch graph");
  }
  *out = static_cast<pfmm_batch_t>(g_batches.add(b));
  return PFMM_OK;
}

pfmm_status batch_launch(pfmm_batch_s* b) {
  for (pfmm_plan_t ph : b->handles)
    if (!plan_of(ph)) return fail(PFMM_ERR_BAD_HANDLE, "a plan of the batch is no longer live");
  hipError_t e = hipEventRecord(b->ev_in, b->caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->caller, b->ev_out, 0);
  if (e != hipSuccess) return hip_fail(e, "batch solve");
  return PFMM_OK;
}

pfmm_status batch_destroy_impl(pfmm_batch_t h) {
  pfmm_batch_s* b = g_batches.remove(h);
  if (!b) return bad_batch();
  const hipError_t e = hipStreamSynchronize(b->stream);
  brelease(b);
  if (e != hipSuccess) return hip_fail(e, "batch destroy");
  return PFMM_OK;
}

}  // namespace

// Release the batches pfmm_solve_batch made for sets that hold `pl`.
void drop_cached_batches(pfmm_plan_s* pl) {
  std::vector<pfmm_batch_t> drop;
  {
    std::lock_guard<std::mutex> lk(g_cmu);
    for (size_t i = 0; i < g_cache.size();) {
      bool uses = false;
      for (pfmm_plan_t ph : g_cache[i].plans) uses = uses || plan_of(ph) == pl;
      if (uses) {
        drop.push_back(g_cache[i].handle);
        g_cache.erase(g_cache.begin() + i);
      } else {
        ++i;
      }
    }
  }
  for (pfmm_batch_t bh : drop) (void)batch_destroy_impl(bh);
}

extern "C" {

pfmm_status pfmm_batch_create(int n, const pfmm_plan_t* plans, const float* const* density,
                              float* const* potential, pfmm_batch_t* out) {
  g_err.clear();
  return batch_create_impl(n, plans, density, potential, false, out);
}

pfmm_status pfmm_batch_solve(pfmm_batch_t h) {
  g_err.clear();
  pfmm_batch_s* b = batch_of(h);
  if (!b || b->cached) return bad_batch();
  return batch_launch(b);
}

pfmm_status pfmm_solve_batch(int n, const pfmm_plan_t* plans, const float* const* density,
                             float* const* potential) {
  g_err.clear();
  if (n < 1 || n > 4096 || !plans || !density || !potential)
    return fail(PFMM_ERR_INVALID_ARG, "need 1 <= n <= 4096 and non-NULL arrays");
  pfmm_batch_t hit = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cmu);
    for (const CachedBatch& c : g_cache) {
      if ((int)c.plans.size() != n) continue;
      bool same = true;
      for (int i = 0; i < n && same; ++i)
        same = c.plans[i] == plans[i] && c.rho[i] == density[i] && c.phi[i] == potential[i];
      if (same) {
        hit = c.handle;
        break;
      }
    }
  }
  if (!hit) {  // first solve of this set: build and capture its batch (plan time)
    pfmm_status st = batch_create_impl(n, plans, density, potential, true, &hit);
    if (st != PFMM_OK) return st;
    CachedBatch c;
    c.plans.assign(plans, plans + n);
    c.rho.assign(density, density + n);
    c.phi.assign(potential, potential + n);
    c.handle = hit;
    std::lock_guard<std::mutex> lk(g_cmu);
    g_cache.push_back(std::move(c));
  }
  pfmm_batch_s* b = batch_of(hit);
  if (!b) return bad_batch();
  return batch_launch(b);
}
pfmm_status pfmm_batch_info(pfmm_batch_t h, int* items, int* groups) {
  g_err.clear();
  pfmm_batch_s* b = batch_of(h);
  if (!b) return bad_batch();
  if (items) *items = b->nitems + b->nsplit + b->nf64;
  if (groups) *groups = (int)b->groups.size();
  return PFMM_OK;
}

pfmm_status pfmm_batch_group(pfmm_batch_t h, int group, int* desc, double* ms) {
  g_err.clear();
  pfmm_batch_s* b = batch_of(h);
  if (!b) return bad_batch();
  if (group < 0 || group >= (int)b->groups.size())
    return fail(PFMM_ERR_INVALID_ARG, "group out of range");
  const auto& g = b->groups[group];
  if (desc) {
    desc[0] = g.q;
    desc[1] = g.fp64;
    desc[2] = g.near;
    desc[3] = g.width;
  }
  if (ms)
    for (int i = 0; i < 3; ++i) ms[i] = g.ms[i];
  return PFMM_OK;
}

pfmm_status pfmm_batch_destroy(pfmm_batch_t h) {
  g_err.clear();
  if (!h) return PFMM_OK;
  pfmm_batch_s* b = batch_of(h);
  if (!b || b->cached) return bad_batch();
  if (capturing(b->caller)) return capture_fail("pfmm_batch_destroy");
  return batch_destroy_impl(h);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned correction of the interaction-zone tables, and the direct solve
// ---------------------------------------------------------------------------
namespace {

int unique_count(int p) {  // sorted triples 4p-1 >= u1 >= u2 >= u3 >= 0
  const int K = 4 * p;
  return K * (K + 1) * (K + 2) / 6;
}

// Allocate the correction's index maps, features and network buffers.
pfmm_status learned_prepare(pfmm_plan_s* pl) {
  if (pl->gstar)  // its base tables would be G_*'s
    return fail(PFMM_ERR_INVALID_ARG,
                "G_* is set on the whole mesh; clear it with pfmm_gstar_set first");
  if (!pl->g0.empty()) return PFMM_OK;
  const int p = pl->p, L = pl->L, C = 4 * p - 1, E = 2 * C + 1, K = 4 * p;
  const int64_t ntab = cube(E);
  const int nu = unique_count(p);
  pl->nu = nu;
  // unique index of a sorted triple
  std::vector<int> uid((size_t)K * K * K, -1);
  std::vector<float> fl;
  int c = 0;
  for (int u1 = 0; u1 < K; ++u1)
    for (int u2 = 0; u2 <= u1; ++u2)
      for (int u3 = 0; u3 <= u2; ++u3) uid[((size_t)u1 * K + u2) * K + u3] = c++;
  std::vector<int> uidx((size_t)ntab);
  std::vector<std::vector<int>> orbit(nu);
  for (int jx = -C; jx <= C; ++jx)
    for (int jy = -C; jy <= C; ++jy)
      for (int jz = -C; jz <= C; ++jz) {
        int a[3] = {std::abs(jx), std::abs(jy), std::abs(jz)};
        std::sort(a, a + 3);
        const int u = uid[((size_t)a[2] * K + a[1]) * K + a[0]];
        const int64_t pos = ((int64_t)(jx + C) * E + (jy + C)) * E + (jz + C);
        uidx[pos] = u;
        orbit[u].push_back((int)pos);
      }
  std::vector<int> ptr(nu + 1, 0), pos;
  for (int u = 0; u < nu; ++u) {
    ptr[u + 1] = ptr[u] + (int)orbit[u].size();
    pos.insert(pos.end(), orbit[u].begin(), orbit[u].end());
  }
  for (int l = 2; l <= L; ++l)
    for (int u1 = 0; u1 < K; ++u1)
      for (int u2 = 0; u2 <= u1; ++u2)
        for (int u3 = 0; u3 <= u2; ++u3) {
          fl.push_back((float)u1 / K);
          fl.push_back((float)u2 / K);
          fl.push_back((float)u3 / K);
          fl.push_back((float)(u1 % p) / p);
          fl.push_back((float)(u2 % p) / p);
          fl.push_back((float)(u3 % p) / p);
          fl.push_back((float)l / 8.f);
          fl.push_back((float)p / 10.f);
        }
  const int nent = (L - 1) * nu;
  hipError_t e = hipSuccess;
  pl->g0.assign(L + 1, nullptr);
  pl->uidx.assign(L + 1, nullptr);
  pl->optr.assign(L + 1, nullptr);
  pl->opos.assign(L + 1, nullptr);
  int* d_uidx = nullptr;
  int* d_ptr = nullptr;
  int* d_pos = nullptr;
  e = dalloc(pl, &d_uidx, (size_t)ntab);
  if (e == hipSuccess) e = dalloc(pl, &d_ptr, ptr.size());
  if (e == hipSuccess) e = dalloc(pl, &d_pos, pos.size());
  if (e == hipSuccess) e = hipMemcpy(d_uidx, uidx.data(), uidx.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice);
  for (int l = 2; l <= L && e == hipSuccess; ++l) {
    pl->uidx[l] = d_uidx;
    pl->optr[l] = d_ptr;
    pl->opos[l] = d_pos;
    e = dalloc(pl, &pl->g0[l], (size_t)ntab);
    if (e == hipSuccess)
      e = hipMemcpy(pl->g0[l], pl->tab64[l], ntab * sizeof(double), hipMemcpyDeviceToDevice);
  }
  if (e == hipSuccess) e = dalloc(pl, &pl->feats, fl.size());
  if (e == hipSuccess) e = hipMemcpy(pl->feats, fl.data(), fl.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = dalloc(pl, &pl->delta, (size_t)nent);
  if (e == hipSuccess) e = dalloc(pl, &pl->theta, (size_t)kMlpParams);
  if (e != hipSuccess) {
    pl->g0.clear();
    return hip_fail(e, "learned correction buffers");
  }
  return PFMM_OK;
}

// Tables from the current network (or the uncorrected ones when learned == 0).
pfmm_status learned_apply(pfmm_plan_s* pl, int bf16) {
  const int p = pl->p, C = 4 * p - 1;
  const int64_t ntab = cube(2 * C + 1);
  hipStream_t st = pl->stream;
  hipError_t e = hipSuccess;
  if (pl->learned == 1 || pl->learned == 2)
    e = mlp_forward(pl->theta, pl->feats, (pl->L - 1) * pl->nu, bf16, pl->delta, st);
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l) {
    if (pl->learned) {
      e = apply_correction(pl->g0[l], pl->delta + (size_t)(l - 2) * pl->nu, pl->uidx[l], ntab,
                           pl->tab64[l], pl->tab32[l], st);
    } else {
      e = hipMemcpyAsync(pl->tab64[l], pl->g0[l], ntab * sizeof(double), hipMemcpyDeviceToDevice,
                         st);
      if (e == hipSuccess) e = cast_f64_f32(pl->tab64[l], pl->tab32[l], ntab, st);
    }
    if (e == hipSuccess && pl->win[l])
      e = make_windows(pl->tab64[l], C, kM2LTerms, pl->win[l], st);
  }
  // the spectral zones' transformed kernels follow the corrected tables
  if (e == hipSuccess && pl->mspec) e = m2l_spectral_tables(pl->mspec, pl->tab64, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "apply learned correction");
  return PFMM_OK;
}

// Buffers of the adjoint sweep shared by every table-gradient mode: mesh
// scratch, residual statistics, the adjoint per level and the table gradients.
pfmm_status adjoint_alloc(pfmm_plan_s* pl) {
  if (pl->resid) return PFMM_OK;
  const int N = pl->N, L = pl->L, p = pl->p;
  const size_t n3 = (size_t)N * N * N, p3 = (size_t)p * p * p;
  const int64_t ntab = cube(8 * p - 1);
  pl->lam.assign(L + 1, nullptr);
  pl->tgrad.assign(L + 1, nullptr);
  hipError_t e = dalloc(pl, &pl->resid, n3);
  if (e == hipSuccess) e = dalloc(pl, &pl->tphi, n3);
  if (e == hipSuccess) e = dalloc(pl, &pl->rpart, (size_t)4 * 1024);
  if (e == hipSuccess) e = dalloc(pl, &pl->rstats, (size_t)4);
  size_t tg = 0;
  for (int l = 2; l <= L && e == hipSuccess; ++l) {
    char* b = nullptr;
    e = dalloc(pl, &b, ((size_t)1 << (3 * l)) * p3 * sizeof(double));
    pl->lam[l] = b;
    if (e == hipSuccess) e = dalloc(pl, &pl->tgrad[l], (size_t)ntab);
    tg = std::max(tg, table_grad_partial_doubles(l == 2 ? 1 : 2, p, l == 2 ? 37 : 189));
  }
  if (e == hipSuccess) e = dalloc(pl, &pl->tgpart, tg);
  if (e != hipSuccess) {
    pl->resid = nullptr;
    return hip_fail(e, "adjoint buffers");
  }
  return PFMM_OK;
}

pfmm_status learned_train_alloc(pfmm_plan_s* pl) {
  if (pl->adam_m) return PFMM_OK;
  pfmm_status s0 = adjoint_alloc(pl);
  if (s0 != PFMM_OK) return s0;
  const int nent = (pl->L - 1) * pl->nu;
  hipError_t e = dalloc(pl, &pl->adam_m, (size_t)kMlpParams);
  if (e == hipSuccess) e = dalloc(pl, &pl->adam_v, (size_t)kMlpParams);
  if (e == hipSuccess) e = dalloc(pl, &pl->wgrad, (size_t)kMlpParams);
  if (e == hipSuccess) e = dalloc(pl, &pl->ddelta, (size_t)nent);
  if (e == hipSuccess) e = dalloc(pl, &pl->mlp_part, mlp_backward_partial_floats(nent));
  if (e == hipSuccess) e = hipMemset(pl->adam_m, 0, kMlpParams * 4);
  if (e == hipSuccess) e = hipMemset(pl->adam_v, 0, kMlpParams * 4);
  if (e == hipSuccess) e = hipMemset(pl->wgrad, 0, kMlpParams * 4);
  if (e != hipSuccess) {
    pl->adam_m = nullptr;
    return hip_fail(e, "training buffers");
  }
  return PFMM_OK;
}

// Residual of the last forward solve (pl->tphi) against `target` into
// pl->resid / pl->rstats, then the adjoint sweep (transposes of L2P and L2L)
// and the gradient of the loss with respect to every entry of every level's
// interaction-zone table into pl->tgrad.
hipError_t adjoint_tables(pfmm_plan_s* pl, const float* target) {
  const int N = pl->N, L = pl->L, p = pl->p;
  const int64_t n3 = (int64_t)N * N * N;
  hipStream_t st = pl->stream;
  hipError_t e = residual(pl->tphi, target, n3, pl->rpart, pl->rstats, pl->resid, st);
  if (e == hipSuccess)
    e = launch_p2m(pl->resid, pl->lam[L], level64(pl, L), wts(pl->dA, pl->dA64), N, pl->s, p, 1.0,
                   st);
  for (int l = L - 1; l >= 2 && e == hipSuccess; --l)
    e = launch_m2m(pl->lam[l + 1], level64(pl, l + 1), pl->lam[l], level64(pl, l),
                   wts(pl->dT, pl->dT64), 1 << l, p, st);
  for (int l = 2; l <= L && e == hipSuccess; ++l) {
    const int m = l == 2 ? 1 : 2, noff = l == 2 ? 37 : 189;
    e = table_grad(1 << l, m, p, noff, l == 2 ? pl->offs_l2 : pl->offs_iz, pl->lam[l], pl->M[l],
                   level64(pl, l), 4 * p - 1, pl->tgpart, pl->tgrad[l], st);
  }
  return e;
}

pfmm_status direct_prepare(pfmm_plan_s* pl) {
  if (pl->dtab64) return PFMM_OK;
  const int N = pl->N;
  const int q = N >= 16 ? 8 : N / 2, n = N / q;
  const int C = N / 2 + q - 1;
  std::vector<int> offs;
  for (int dx = -n / 2; dx < n / 2; ++dx)
    for (int dy = -n / 2; dy < n / 2; ++dy)
      for (int dz = -n / 2; dz < n / 2; ++dz) offs.push_back(pack_offset(dx, dy, dz));
  const int64_t ntab = cube(2 * C + 1);
  hipError_t e = dalloc(pl, &pl->dtab64, (size_t)ntab);
  if (e == hipSuccess) e = dalloc(pl, &pl->dtab32, (size_t)ntab);
  if (e == hipSuccess) e = dalloc(pl, &pl->doffs, offs.size());
  if (e == hipSuccess)
    e = hipMemcpy(pl->doffs, offs.data(), offs.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = tabulate_green(green_spec(pl), N, C, N, 1.0 / N, pl->dtab64, pl->stream);
  if (e == hipSuccess) e = cast_f64_f32(pl->dtab64, pl->dtab32, ntab, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) {
    pl->dtab64 = nullptr;
    return hip_fail(e, "direct solve tables");
  }
  pl->dq = q;
  pl->dC = C;
  pl->dnoff = (int)offs.size();
  return PFMM_OK;
}

// The exact periodic convolution with the plan's direct table (prepared).
hipError_t direct_launch(pfmm_plan_s* pl, const float* rho, float* phi) {
  ToepArgs a{};
  a.n = pl->N / pl->dq;
  a.m = 1;
  a.q = pl->dq;
  a.noff = pl->dnoff;
  a.offs = pl->doffs;
  a.tab = pl->dtab32;
  a.C = pl->dC;
  a.X = rho;
  a.Y = phi;
  a.grid_in = 1;
  a.grid_out = 1;
  a.xscale = 1.0 / ((double)pl->N * pl->N * pl->N);
  a.accumulate = 0;
  a.groups = 1;
  return launch_toeplitz(a, pl->stream);
}

// --- G_* on the whole mesh -------------------------------------------------

pfmm_status gstar_check(pfmm_plan_s* pl) {
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "G_* of an isolated plan");
  if (pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "G_* with FFT interaction zones");
  if (pl->accel_mode)
    return fail(PFMM_ERR_UNSUPPORTED, "G_* with accelerations from the expansion");
  if (pl->s % pl->p)
    return fail(PFMM_ERR_UNSUPPORTED, "G_* on the mesh needs p to divide the leaf width");
  if (pl->learned)
    return fail(PFMM_ERR_INVALID_ARG,
                "the interaction-zone tables carry a learned correction; clear it first");
  return PFMM_OK;
}

// orbit -> entries (CSR) of an entry -> orbit map
void orbit_csr(const std::vector<int>& uidx, int nu, std::vector<int>& ptr, std::vector<int>& pos) {
  ptr.assign(nu + 1, 0);
  for (int u : uidx) ++ptr[u + 1];
  for (int u = 0; u < nu; ++u) ptr[u + 1] += ptr[u];
  pos.assign(uidx.size(), 0);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (size_t i = 0; i < uidx.size(); ++i) pos[fill[uidx[i]]++] = (int)i;
}

template <class T>
hipError_t upload(pfmm_plan_s* pl, T** dst, const std::vector<T>& v) {
  hipError_t e = dalloc(pl, dst, v.size());
  if (e == hipSuccess) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Uncorrected copies of every table G_* replaces, from the current tables.
hipError_t gstar_base(pfmm_plan_s* pl) {
  const int p = pl->p, N = pl->N;
  const int64_t nlev = cube(8 * p - 1), nnear = cube(4 * pl->s - 1), ndir = cube(2 * pl->dC + 1);
  hipStream_t st = pl->stream;
  hipError_t e = hipSuccess;
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l)
    e = hipMemcpyAsync(pl->gl0[l], pl->tab64[l], nlev * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pl->gn0, pl->ntab64, nnear * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pl->gd0, pl->dtab64, ndir * sizeof(double), hipMemcpyDeviceToDevice, st);
  const double n6 = (double)N * N * N * (double)N * N * N;
  if (e == hipSuccess) e = gstar_mesh_values(pl->gd0, pl->dC, N, -1.0 / n6, pl->gmesh0, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

pfmm_status gstar_prepare(pfmm_plan_s* pl) {
  if (pl->gdelta) return PFMM_OK;
  pfmm_status s0 = direct_prepare(pl);
  if (s0 == PFMM_OK) s0 = adjoint_alloc(pl);
  if (s0 != PFMM_OK) return s0;
  const int N = pl->N, L = pl->L, p = pl->p, s = pl->s;
  const int nu = gstar_orbits(N);
  std::vector<int> ptr, pos;
  hipError_t e = hipSuccess;
  pl->gl0.assign(L + 1, nullptr);
  pl->gluidx.assign(L + 1, nullptr);
  pl->glptr.assign(L + 1, nullptr);
  pl->glpos.assign(L + 1, nullptr);
  // level tables: entry j is the mesh separation j (N / 2^l) / p
  for (int l = 2; l <= L && e == hipSuccess; ++l) {
    const int C = 4 * p - 1, E = 2 * C + 1, w = (N >> l) / p;
    std::vector<int> u((size_t)E * E * E);
    for (int x = 0; x < E; ++x)
      for (int y = 0; y < E; ++y)
        for (int z = 0; z < E; ++z)
          u[((size_t)x * E + y) * E + z] = gstar_orbit((x - C) * w, (y - C) * w, (z - C) * w, N);
    orbit_csr(u, nu, ptr, pos);
    e = upload(pl, &pl->gluidx[l], u);
    if (e == hipSuccess) e = upload(pl, &pl->glptr[l], ptr);
    if (e == hipSuccess) e = upload(pl, &pl->glpos[l], pos);
    if (e == hipSuccess) e = dalloc(pl, &pl->gl0[l], u.size());
  }
  // near table: entry m is the mesh separation m
  if (e == hipSuccess) {
    const int C = 2 * s - 1, E = 2 * C + 1;
    std::vector<int> u((size_t)E * E * E);
    for (int x = 0; x < E; ++x)
      for (int y = 0; y < E; ++y)
        for (int z = 0; z < E; ++z)
          u[((size_t)x * E + y) * E + z] = gstar_orbit(x - C, y - C, z - C, N);
    orbit_csr(u, nu, ptr, pos);
    e = upload(pl, &pl->gnuidx, u);
    if (e == hipSuccess) e = upload(pl, &pl->gnptr, ptr);
    if (e == hipSuccess) e = upload(pl, &pl->gnpos, pos);
    if (e == hipSuccess) e = dalloc(pl, &pl->gn0, u.size());
    if (e == hipSuccess) e = dalloc(pl, &pl->gnear, u.size());
  }
  // direct table (periodic images of the same separations share an orbit)
  if (e == hipSuccess) {
    const int C = pl->dC, E = 2 * C + 1;
    std::vector<int> u((size_t)E * E * E);
    for (int x = 0; x < E; ++x)
      for (int y = 0; y < E; ++y)
        for (int z = 0; z < E; ++z)
          u[((size_t)x * E + y) * E + z] = gstar_orbit(x - C, y - C, z - C, N);
    e = upload(pl, &pl->gduidx, u);
    if (e == hipSuccess) e = dalloc(pl, &pl->gd0, u.size());
  }
  // every mesh point, for the PM side of the gradient
  if (e == hipSuccess) {
    std::vector<int> u((size_t)N * N * N);
    for (int x = 0; x < N; ++x)
      for (int y = 0; y < N; ++y)
        for (int z = 0; z < N; ++z) u[((size_t)x * N + y) * N + z] = gstar_orbit(x, y, z, N);
    orbit_csr(u, nu, ptr, pos);
    e = upload(pl, &pl->gmptr, ptr);
    if (e == hipSuccess) e = upload(pl, &pl->gmpos, pos);
    if (e == hipSuccess) e = dalloc(pl, &pl->gmesh0, u.size());
    if (e == hipSuccess) e = dalloc(pl, &pl->gcorr, u.size());
    if (e == hipSuccess) e = dalloc(pl, &pl->gtarget, u.size());
  }
  if (e == hipSuccess) e = dalloc(pl, &pl->gdd, (size_t)nu);
  if (e == hipSuccess) e = dalloc(pl, &pl->gacc, (size_t)nu);
  if (e == hipSuccess) e = hipMemset(pl->gacc, 0, (size_t)nu * sizeof(float));
  if (e == hipSuccess) e = gstar_fft_create(N, &pl->gfft);
  if (e == hipSuccess) e = gstar_base(pl);
  float* d = nullptr;
  if (e == hipSuccess) e = dalloc(pl, &d, (size_t)nu);
  if (e == hipSuccess) e = hipMemset(d, 0, (size_t)nu * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "G_* buffers");
  pl->nug = nu;
  pl->gdelta = d;  // set last: marks the state complete
  return PFMM_OK;
}

// Every table from G_* = G (1 + delta[orbit]), and what is derived from them.
pfmm_status gstar_apply(pfmm_plan_s* pl) {
  const int p = pl->p, C = 4 * p - 1;
  const int64_t nlev = cube(2 * C + 1), nnear = cube(4 * pl->s - 1), ndir = cube(2 * pl->dC + 1);
  hipStream_t st = pl->stream;
  hipError_t e = hipSuccess;
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l) {
    e = apply_correction(pl->gl0[l], pl->gdelta, pl->gluidx[l], nlev, pl->tab64[l], pl->tab32[l],
                         st);
    if (e == hipSuccess && pl->win[l]) e = make_windows(pl->tab64[l], C, kM2LTerms, pl->win[l], st);
  }
  if (e == hipSuccess)
    e = apply_correction(pl->gn0, pl->gdelta, pl->gnuidx, nnear, pl->ntab64, pl->ntab32, st);
  if (e == hipSuccess && pl->nwin)
    e = make_windows(pl->ntab64, 2 * pl->s - 1, kNearTerms, pl->nwin, st);
  if (e == hipSuccess)
    e = apply_correction(pl->gd0, pl->gdelta, pl->gduidx, ndir, pl->dtab64, pl->dtab32, st);
  if (e == hipSuccess && pl->mspec) e = m2l_spectral_tables(pl->mspec, pl->tab64, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "apply G_*");
  return refresh_near_fft(pl);
}

// Forward solve with G_*, its PM potential, and the residual statistics.
pfmm_status gstar_forward(pfmm_plan_s* pl, const float* rho) {
  pfmm_status s0 = solve_impl(pl, rho, pl->tphi, nullptr);
  if (s0 != PFMM_OK) return s0;
  const hipError_t e = direct_launch(pl, rho, pl->gtarget);
  if (e != hipSuccess) return hip_fail(e, "PM potential with G_*");
  return PFMM_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace pfmm {
int plan_direct_spec(const void* h, DirectSpec* out) {
  pfmm_plan_s* pl = plan_of(static_cast<pfmm_plan_t>(const_cast<void*>(h)));
  if (!pl) return bad_plan();
  out->N = pl->N;
  out->isolated = pl->isolated;
  out->green = green_spec(pl);
  out->stream = pl->stream;
  return PFMM_OK;
}
int set_error(int status, const std::string& msg) { return fail((pfmm_status)status, msg); }
void clear_error() { g_err.clear(); }
}  // namespace pfmm

extern "C" {

pfmm_status pfmm_plan_direct(pfmm_plan_t h, const float* rho, float* phi) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "direct solve of an isolated plan");
  if (!rho || !phi || (const void*)rho == (const void*)phi)
    return fail(PFMM_ERR_INVALID_ARG, "density and potential must be distinct device arrays");
  if (!pl->dtab64 && capturing(pl->stream)) return capture_fail("the first pfmm_plan_direct");
  pfmm_status s0 = direct_prepare(pl);
  if (s0 != PFMM_OK) return s0;
  const hipError_t e = direct_launch(pl, rho, phi);
  if (e != hipSuccess) return hip_fail(e, "direct solve");
  return PFMM_OK;
}


pfmm_status pfmm_learned_set(pfmm_plan_t h, const float* weights, int bf16) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (pl->gstar)
    return fail(PFMM_ERR_INVALID_ARG,
                "G_* is set on the whole mesh; clear it with pfmm_gstar_set first");
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_set");
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "learned tables of an isolated plan");
  if (pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "learned tables with FFT interaction zones");
  if (!weights) {
    if (pl->g0.empty()) return PFMM_OK;  // never corrected
    pl->learned = 0;
    return learned_apply(pl, 0);
  }
  pfmm_status s0 = learned_prepare(pl);
  if (s0 != PFMM_OK) return s0;
  hipError_t e = hipMemcpy(pl->theta, weights, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload weights");
  pl->learned = 1;
  return learned_apply(pl, bf16 ? 1 : 0);
}

pfmm_status pfmm_learned_train_begin(pfmm_plan_t h, const float* weights, double lr) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (pl->gstar)
    return fail(PFMM_ERR_INVALID_ARG,
                "G_* is set on the whole mesh; clear it with pfmm_gstar_set first");
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_train_begin");
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "learned tables of an isolated plan");
  if (pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "learned tables with FFT interaction zones");
  if (!weights || !(lr > 0.0)) return fail(PFMM_ERR_INVALID_ARG, "need weights and lr > 0");
  pfmm_status s0 = learned_prepare(pl);
  if (s0 == PFMM_OK) s0 = learned_train_alloc(pl);
  if (s0 != PFMM_OK) return s0;
  hipError_t e = hipMemcpy(pl->theta, weights, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(pl->adam_m, 0, kMlpParams * 4);
  if (e == hipSuccess) e = hipMemset(pl->adam_v, 0, kMlpParams * 4);
  if (e == hipSuccess) e = hipMemset(pl->wgrad, 0, kMlpParams * 4);
  if (e != hipSuccess) return hip_fail(e, "training state");
  pl->learned = 2;
  pl->adam_t = 0;
  pl->accumulated = 0;
  pl->lr = lr;
  return learned_apply(pl, 0);
}

pfmm_status pfmm_learned_accumulate(pfmm_plan_t h, const float* rho, const float* target,
                                    double* loss) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_accumulate");
  if (pl->learned != 2 && pl->learned != 3)
    return fail(PFMM_ERR_INVALID_ARG, "call pfmm_learned_train_begin or pfmm_table_train_begin first");
  if (!rho || !target) return fail(PFMM_ERR_INVALID_ARG, "density and target are required");
  const int N = pl->N, L = pl->L, p = pl->p;
  const int64_t n3 = (int64_t)N * N * N;
  hipStream_t st = pl->stream;
  pfmm_status s0 = solve_impl(pl, rho, pl->tphi, nullptr);
  if (s0 != PFMM_OK) return s0;
  hipError_t e = adjoint_tables(pl, target);
  const int nent = (L - 1) * pl->nu;
  if (e == hipSuccess) e = hipMemsetAsync(pl->ddelta, 0, nent * sizeof(float), st);
  for (int l = 2; l <= L && e == hipSuccess; ++l)
    e = orbit_gather(pl->tgrad[l], pl->g0[l], pl->optr[l], pl->opos[l], pl->nu,
                     pl->ddelta + (size_t)(l - 2) * pl->nu, st);
  if (e == hipSuccess) {
    if (pl->learned == 3)  // grid-valued tables: ddelta is the parameters' gradient
      e = add_into(pl->ggrad, pl->ddelta, nent, st);
    else
      e = mlp_backward(pl->theta, pl->feats, pl->ddelta, nent, pl->mlp_part, pl->wgrad, st);
  }
  double stats[3] = {0, 0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(stats, pl->rstats, sizeof stats, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "learned gradient");
  ++pl->accumulated;
  if (loss) *loss = stats[1];
  return PFMM_OK;
}

pfmm_status pfmm_learned_loss(pfmm_plan_t h, const float* rho, const float* target,
                              double* loss) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_loss");
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "learned tables of an isolated plan");
  if (pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "learned tables with FFT interaction zones");
  if (!rho || !target || !loss) return fail(PFMM_ERR_INVALID_ARG, "NULL argument");
  pfmm_status s0 = learned_prepare(pl);
  if (s0 == PFMM_OK) s0 = learned_train_alloc(pl);
  if (s0 == PFMM_OK) s0 = solve_impl(pl, rho, pl->tphi, nullptr);
  if (s0 != PFMM_OK) return s0;
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  double stats[3] = {0, 0, 0};
  hipError_t e = residual(pl->tphi, target, n3, pl->rpart, pl->rstats, pl->resid, pl->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(stats, pl->rstats, sizeof stats, hipMemcpyDeviceToHost, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(e, "loss");
  *loss = stats[1];
  return PFMM_OK;
}

pfmm_status pfmm_learned_step(pfmm_plan_t h) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_step");
  if ((pl->learned != 2 && pl->learned != 3) || pl->accumulated == 0)
    return fail(PFMM_ERR_INVALID_ARG, "no accumulated gradient");
  const hipError_t e =
      pl->learned == 3
          ? adam_step(pl->delta, pl->gm, pl->gv, pl->ggrad, (pl->L - 1) * pl->nu,
                      (float)pl->accumulated, (float)pl->lr, ++pl->adam_t, pl->stream)
          : adam_step(pl->theta, pl->adam_m, pl->adam_v, pl->wgrad, kMlpParams,
                      (float)pl->accumulated, (float)pl->lr, ++pl->adam_t, pl->stream);
  if (e != hipSuccess) return hip_fail(e, "adam");
  pl->accumulated = 0;
  return learned_apply(pl, 0);
}

pfmm_status pfmm_table_params(pfmm_plan_t h, int* count) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_table_params");
  if (!count) return fail(PFMM_ERR_INVALID_ARG, "count is NULL");
  if (pl->isolated) return fail(PFMM_ERR_UNSUPPORTED, "learned tables of an isolated plan");
  if (pl->m2l_fft) return fail(PFMM_ERR_UNSUPPORTED, "learned tables with FFT interaction zones");
  const pfmm_status s0 = learned_prepare(pl);
  if (s0 != PFMM_OK) return s0;
  *count = (pl->L - 1) * pl->nu;
  return PFMM_OK;
}

pfmm_status pfmm_table_set(pfmm_plan_t h, const float* delta) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (pl->gstar)
    return fail(PFMM_ERR_INVALID_ARG,
                "G_* is set on the whole mesh; clear it with pfmm_gstar_set first");
  if (capturing(pl->stream)) return capture_fail("pfmm_table_set");
  if (!delta) return pfmm_learned_set(h, nullptr, 0);
  int n = 0;
  pfmm_status s0 = pfmm_table_params(h, &n);
  if (s0 != PFMM_OK) return s0;
  const hipError_t e = hipMemcpy(pl->delta, delta, (size_t)n * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload table parameters");
  pl->learned = 3;
  pl->accumulated = 0;
  return learned_apply(pl, 0);
}

pfmm_status pfmm_table_get(pfmm_plan_t h, float* delta) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_table_get");
  if (!delta) return fail(PFMM_ERR_INVALID_ARG, "delta is NULL");
  if (pl->learned != 3) return fail(PFMM_ERR_INVALID_ARG, "the plan has no grid-valued tables");
  const hipError_t e = hipMemcpy(delta, pl->delta, (size_t)(pl->L - 1) * pl->nu * sizeof(float),
                                 hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "download table parameters");
  return PFMM_OK;
}

pfmm_status pfmm_table_grad(pfmm_plan_t h, float* grad) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_table_grad");
  if (!grad) return fail(PFMM_ERR_INVALID_ARG, "grad is NULL");
  if (pl->learned != 3 || !pl->ggrad)
    return fail(PFMM_ERR_INVALID_ARG, "call pfmm_table_train_begin first");
  const size_t n = (size_t)(pl->L - 1) * pl->nu;
  hipError_t e = hipMemcpy(grad, pl->ggrad, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(pl->ggrad, 0, n * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "table gradient");
  pl->accumulated = 0;
  return PFMM_OK;
}

pfmm_status pfmm_table_train_begin(pfmm_plan_t h, double lr) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (pl->gstar)
    return fail(PFMM_ERR_INVALID_ARG,
                "G_* is set on the whole mesh; clear it with pfmm_gstar_set first");
  if (capturing(pl->stream)) return capture_fail("pfmm_table_train_begin");
  if (!(lr > 0.0)) return fail(PFMM_ERR_INVALID_ARG, "need lr > 0");
  int n = 0;
  pfmm_status s0 = pfmm_table_params(h, &n);
  if (s0 == PFMM_OK) s0 = learned_train_alloc(pl);
  if (s0 != PFMM_OK) return s0;
  hipError_t e = hipSuccess;
  if (!pl->gm) e = dalloc(pl, &pl->gm, (size_t)n);
  if (e == hipSuccess && !pl->gv) e = dalloc(pl, &pl->gv, (size_t)n);
  if (e == hipSuccess && !pl->ggrad) e = dalloc(pl, &pl->ggrad, (size_t)n);
  if (e == hipSuccess) e = hipMemset(pl->delta, 0, (size_t)n * 4);
  if (e == hipSuccess) e = hipMemset(pl->gm, 0, (size_t)n * 4);
  if (e == hipSuccess) e = hipMemset(pl->gv, 0, (size_t)n * 4);
  if (e == hipSuccess) e = hipMemset(pl->ggrad, 0, (size_t)n * 4);
  if (e != hipSuccess) return hip_fail(e, "table training state");
  pl->learned = 3;
  pl->adam_t = 0;
  pl->accumulated = 0;
  pl->lr = lr;
  return learned_apply(pl, 0);
}

pfmm_status pfmm_learned_get(pfmm_plan_t h, float* weights) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_get");
  if (!weights || !pl->learned) return fail(PFMM_ERR_INVALID_ARG, "no network on this plan");
  const hipError_t e =
      hipMemcpy(weights, pl->theta, kMlpParams * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "download weights");
  return PFMM_OK;
}

pfmm_status pfmm_learned_read_grad(pfmm_plan_t h, int level, double* table_grad,
                                   float* weight_grad) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_learned_read_grad");
  if (pl->learned != 2) return fail(PFMM_ERR_INVALID_ARG, "not training");
  if (level < 2 || level > pl->L) return fail(PFMM_ERR_INVALID_ARG, "level out of range");
  hipError_t e = hipSuccess;
  if (table_grad)
    e = hipMemcpy(table_grad, pl->tgrad[level], cube(8 * pl->p - 1) * sizeof(double),
                  hipMemcpyDeviceToHost);
  if (e == hipSuccess && weight_grad)
    e = hipMemcpy(weight_grad, pl->wgrad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "read gradient");
  return PFMM_OK;
}

pfmm_status pfmm_gstar_params(pfmm_plan_t h, int* count) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (!count) return fail(PFMM_ERR_INVALID_ARG, "count is NULL");
  const pfmm_status s0 = gstar_check(pl);
  if (s0 != PFMM_OK) return s0;
  *count = gstar_orbits(pl->N);
  return PFMM_OK;
}

pfmm_status pfmm_gstar_set(pfmm_plan_t h, const float* delta) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_gstar_set");
  if (!delta) {  // back to G everywhere
    if (!pl->gstar) return PFMM_OK;
    const hipError_t e = hipMemset(pl->gdelta, 0, (size_t)pl->nug * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "clear G_*");
    pl->gstar = 0;
    return gstar_apply(pl);
  }
  pfmm_status s0 = gstar_check(pl);
  if (s0 == PFMM_OK) s0 = gstar_prepare(pl);
  if (s0 != PFMM_OK) return s0;
  const hipError_t e =
      hipMemcpy(pl->gdelta, delta, (size_t)pl->nug * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "upload G_*");
  pl->gstar = 1;
  return gstar_apply(pl);
}

pfmm_status pfmm_gstar_get(pfmm_plan_t h, float* delta) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_gstar_get");
  if (!delta) return fail(PFMM_ERR_INVALID_ARG, "delta is NULL");
  if (!pl->gdelta) return fail(PFMM_ERR_INVALID_ARG, "the plan has no G_* values");
  const hipError_t e =
      hipMemcpy(delta, pl->gdelta, (size_t)pl->nug * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "download G_*");
  return PFMM_OK;
}

pfmm_status pfmm_gstar_loss(pfmm_plan_t h, const float* rho, double* loss) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_gstar_loss");
  if (!rho || !loss) return fail(PFMM_ERR_INVALID_ARG, "NULL argument");
  pfmm_status s0 = gstar_check(pl);
  if (s0 == PFMM_OK) s0 = gstar_prepare(pl);
  if (s0 == PFMM_OK) s0 = gstar_forward(pl, rho);
  if (s0 != PFMM_OK) return s0;
  const int64_t n3 = (int64_t)pl->N * pl->N * pl->N;
  double stats[4] = {0, 0, 0, 0};
  hipError_t e = residual(pl->tphi, pl->gtarget, n3, pl->rpart, pl->rstats, pl->resid, pl->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(stats, pl->rstats, sizeof stats, hipMemcpyDeviceToHost, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(e, "G_* loss");
  *loss = stats[1];
  return PFMM_OK;
}

pfmm_status pfmm_gstar_accumulate(pfmm_plan_t h, const float* rho, double* loss) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_gstar_accumulate");
  if (!rho) return fail(PFMM_ERR_INVALID_ARG, "density is NULL");
  pfmm_status s0 = gstar_check(pl);
  if (s0 == PFMM_OK) s0 = gstar_prepare(pl);
  if (s0 == PFMM_OK) s0 = gstar_forward(pl, rho);
  if (s0 != PFMM_OK) return s0;
  const int N = pl->N, nu = pl->nug;
  hipStream_t st = pl->stream;
  // the FMM side: adjoint sweep and level-table gradients, then the near table
  hipError_t e = adjoint_tables(pl, pl->gtarget);
  if (e == hipSuccess) e = hipMemsetAsync(pl->gdd, 0, (size_t)nu * sizeof(float), st);
  for (int l = 2; l <= pl->L && e == hipSuccess; ++l)
    e = orbit_gather(pl->tgrad[l], pl->gl0[l], pl->glptr[l], pl->glpos[l], nu, pl->gdd, st);
  const double h3 = 1.0 / ((double)N * N * N);
  if (e == hipSuccess) e = gstar_near_grad(pl->resid, rho, N, pl->s, h3, pl->gnear, st);
  if (e == hipSuccess) e = orbit_gather(pl->gnear, pl->gn0, pl->gnptr, pl->gnpos, nu, pl->gdd, st);
  // the PM side (its weights carry -1 / N^6: h^3 and the unnormalised FFT)
  if (e == hipSuccess)
    e = gstar_pm_corr(pl->gfft, pl->resid, pl->gtarget, rho, pl->rstats, pl->gcorr, st);
  if (e == hipSuccess)
    e = orbit_gather(pl->gcorr, pl->gmesh0, pl->gmptr, pl->gmpos, nu, pl->gdd, st);
  if (e == hipSuccess) e = add_into(pl->gacc, pl->gdd, nu, st);
  double stats[4] = {0, 0, 0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(stats, pl->rstats, sizeof stats, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "G_* gradient");
  ++pl->gacc_n;
  if (loss) *loss = stats[1];
  return PFMM_OK;
}

pfmm_status pfmm_gstar_grad(pfmm_plan_t h, float* grad) {
  g_err.clear();
  pfmm_plan_s* pl = plan_of(h);
  if (!pl) return bad_plan();
  if (capturing(pl->stream)) return capture_fail("pfmm_gstar_grad");
  if (!grad) return fail(PFMM_ERR_INVALID_ARG, "grad is NULL");
  if (!pl->gdelta || pl->gacc_n == 0) return fail(PFMM_ERR_INVALID_ARG, "no accumulated gradient");
  hipError_t e = hipMemcpy(grad, pl->gacc, (size_t)pl->nug * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(pl->gacc, 0, (size_t)pl->nug * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "G_* gradient");
  pl->gacc_n = 0;
  return PFMM_OK;
}

}  // extern "C"
