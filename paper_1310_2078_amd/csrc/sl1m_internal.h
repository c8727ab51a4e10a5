// Internal declarations of the SL1M HIP library (gfx950).
//
// Data layout in HBM (all inside the caller's workspace):
//   pixels are regrouped into segments of equal (kind, sigma) and stored in
//   that permuted order twice: as 48/64-byte records read through the scalar
//   unit by the forward kernels (one record per loop step, uniform across the
//   wavefront) and as structure-of-arrays read per lane by the adjoint kernels.
//   Visibilities keep the caller's order; their static per-visibility data and
//   the per-call residual travel in 32..88-byte records that the adjoint
//   kernels read through the scalar unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sl1m.h"

namespace sl1m {

constexpr int kBlock = 256;           // threads per block (4 wavefronts)
constexpr int kMaxLayers = 16;        // distinct (kind, sigma) groups per plan
constexpr double kMagic = 805306368.0;  // 1.5 * 2^29: ulp 2^-23 turn; low 23 bits = fraction

// Pixel record for the forward kernels (read via scalar loads).
//   delta:    c3 = n - 1 (stable form), c4 unused
//   gaussian: c3 = l^2 + m^2,            c4 = n - 1 + r^2/2 (0 for paraxial)
// scale = (1/n) * per-pixel beam (separable gains) ; r2r = l^2+m^2 in R.
template <typename R>
struct PixRec {
  double l, m, c3, c4;
  R lr, mr, scale, r2r;
};

// Per-visibility coordinates for delta adjoint kernels (read via scalar
// loads); the per-call residual lives in a separate array.
template <typename R>
struct VisRecD {
  double u, v, w, pad;
};

// Float32 hi/lo splits of three coordinates, a = a_hi + a_lo with a_hi the
// float32 rounding of a (SL1M_PREC_FP32_HILO): (l, m, n - 1) per pixel and
// (u, v, w) per visibility, read via scalar loads.
struct HLRec {
  float ah, al, bh, bl, ch, cl, pad0, pad1;
};

// Delta residual record of the square-grid adjoint in polar form: the
// residual's phase folded into the phase origin of the per-cell phasor,
// org = kMagic + arg(r) / (2 pi) (turns), and mag = |r|.
struct ResPolar {
  double org;
  float mag, pad;
};

// Per-(layer, visibility) record for Gaussian adjoint kernels.  The phase is
// psi = A l + B m + C r^2 + NW kappa + E0 (turns, E0 carries kMagic in FP32
// mode); the taper is exp(c1 * ((u - w l)^2 + (v - w m)^2)).
template <typename R>
struct VisRecG {
  double A, B, C, NW, E0;
  R ur, vr, wr, c1;
};

struct Segment {
  int64_t start, count;  // in permuted pixel order
  int kind;              // sl1m_pixel_kind
  double sigma;
  int layer;             // index among Gaussian layers, -1 for delta
};

struct Chunk {           // a contiguous pixel range inside one segment
  int64_t j0, j1;
  double sigma;          // Gaussian scale of the segment (0 for delta)
  int32_t seg, layer;
};

// Grid evaluation.  A segment of pixels (the delta pixels, or one Gaussian
// (kind, sigma) layer) whose positions lie on a product set of |l| and |m|
// values symmetric under l -> -l and m -> -m is evaluated per grid cell: cell
// (ia, ib) stands for the four positions (+-|l|_ia, +-|m|_ib).  Cells are
// numbered
//   q = ((ib / kGridNB) * n_a + ia) * kGridNB + ib % kGridNB
// so the kGridNB cells of one |l| value and one group of |m| values are
// adjacent.  Sign slots: 0 = (+l, +m), 1 = (-l, +m), 2 = (+l, -m), 3 = (-l, -m);
// a zero coordinate takes the + slot.
constexpr int kGridVPL = 1;      // visibilities per lane of the grid forward
constexpr int kGridNB = 8;       // |m| values per forward group
constexpr int kGridNBA = 4;      // |m| values per adjoint lane
constexpr int kGridKB = 32;      // visibilities per adjoint LDS batch (delta)
constexpr int kGridKBG = 16;     // visibilities per adjoint LDS batch (Gaussian)
constexpr int kGridMaxGL = 18;   // |m| groups one adjoint block touches (n_a >= 16)
constexpr int kGridMinA = 16;

// Per-call forward record of one delta cell: n - 1 of the cell and the sign
// combinations of the four amplitudes x_s (x times 1/n and beam factor):
//   e1 = x0 + x1 + x2 + x3, e2 = x1 + x2 - x0 - x3,
//   e3 = x0 + x1 - x2 - x3, e4 = x0 - x1 + x2 - x3;
// `empty` = 1 when no pixel sits in the cell.
struct GridRec {
  double nu;
  float e1, e2, e3, e4;
  int32_t empty, pad;
};

// Per-call forward record of one Gaussian cell: l^2 + m^2, kappa = n - 1 +
// r^2/2 (0 for paraxial pixels) and the amplitudes of the four sign slots.
struct GridRecG {
  double r2, kappa;
  float x[4];
};
static_assert(sizeof(GridRec) == sizeof(GridRecG), "grid records share one buffer");

// Per-call forward record of a mirrored pair (square delta grids), for |l|
// index ia and |m| index bb = kGridNB g + b: bb < ia: cell (ia, bb) (e) and
// its mirror (bb, ia) (f), which share n - 1; bb == ia: the cell alone (f = 0);
// bb > ia: nothing (zero record; the mirror's own record covers the cell).
// Records are ordered as the forward sweeps them: group g, then ia from
// kGridNB g to n_a - 1, then b; group g starts at record
// kGridNB (g n_a - (kGridNB / 2) g (g - 1)).
struct GridPairRec {
  double nu;
  float e1, e2, e3, e4;
  float f1, f2, f3, f4;
  int32_t empty, pad;
};

// The same for a square Gaussian grid: l^2 + m^2 and kappa of the pair, the
// amplitudes of the cell's (x) and the mirror's (y) sign slots.
struct GridPairRecG {
  double r2, kappa;
  float x[4], y[4];
};
static_assert(sizeof(GridPairRecG) == sizeof(GridPairRec), "pair records share one buffer");

__host__ __device__ inline int64_t pair_rec_base(int g, int na) {
  return static_cast<int64_t>(kGridNB) *
         (static_cast<int64_t>(g) * na - (kGridNB / 2) * static_cast<int64_t>(g) * (g - 1));
}

struct GridChunk {       // forward: one |m| group times an |l| range
  int32_t g, ia0, ia1, pad;
};

// Square delta grids (the |l| values equal the |m| values): cells (a, b) and
// (b, a) have the same l^2 + m^2 and share C, so every cell off the diagonal
// is evaluated as half of a pair (a, b) + (b, a) with a > b, and each
// diagonal cell alone.  Adjoint pair blocks: lane-sets (g4, ia) with
// ia >= kGridNBA g4, row-major, at most kBlock lane-sets and kGridMaxGL
// groups per block; lane-set (g4, ia) writes cell (ia, b) when b <= ia and the
// mirror (b, ia) when b < ia, b = kGridNBA g4 + bi.
struct GridPairBlock {
  int32_t g4, ia;        // first lane-set of the block
  int32_t count;         // lane-sets in the block
  int32_t n_gl;          // groups the block touches
};

// One segment on the grid path and where its tables live in the plan's
// concatenated grid arrays.
struct GridSeg {
  int32_t seg;           // index into the plan's segments
  int32_t kind;          // sl1m_pixel_kind
  int32_t layer;         // Gaussian layer (-1 for delta)
  int32_t na, nb, ng;    // distinct |l|, distinct |m|, |m| groups of kGridNB
  int64_t cells;         // ng * kGridNB * na
  int64_t la_off, mb_off, cell_off;
  int32_t fc0, nfc;      // forward chunks [fc0, fc0 + nfc) = partial rows
  int32_t nfs;           // chunks taking cells one by one (all, unless square)
  int32_t square;        // 1: square delta grid (pairs)
  int32_t ablocks;       // adjoint blocks of lane-sets (not square)
  int32_t pblocks, pb0;  // square: pair blocks, first entry in the pair-block table
  int64_t pr_off, n_pairs;  // square: pair records [pr_off, pr_off + n_pairs)
};

}  // namespace sl1m

namespace sl1m {
// timing kinds (sl1m_timing): 0 forward, 1 adjoint, 2 FISTA update, then the
// grid kernels by launch: 3 delta forward, 4 delta adjoint, 5 Gaussian
// forward (one launch per layer), 6 Gaussian adjoint (all layers)
constexpr int kTimingKinds = 8;
enum TimingKind { T_FWD = 0, T_ADJ = 1, T_UPDATE = 2, T_GRID_FWD_DELTA = 3,
                  T_GRID_ADJ_DELTA = 4, T_GRID_FWD_GAUSS = 5, T_GRID_ADJ_GAUSS = 6 };
}  // namespace sl1m

struct sl1m_plan {
  int device = 0;
  int64_t n_pix = 0, n_vis = 0;
  int precision = SL1M_PREC_FP32;
  int max_rhs = 1;            // right-hand sides the workspace is sized for
  size_t real_bytes = 4;      // 4 or 8
  bool has_gain = false;      // per-visibility complex gain constants present
  bool beam_pair = false;     // per-pair (non-separable) beam factors
  bool any_gauss = false, any_delta = false;
  int n_layers = 0;           // Gaussian layers
  std::vector<sl1m::Segment> segs;
  std::vector<double> layer_sigma;

  // forward tiling: lanes own visibilities
  int fwd_vpl = 4;            // visibilities per lane
  int64_t fwd_vtiles = 0;
  std::vector<sl1m::Chunk> fchunks_delta, fchunks_gauss;
  int n_fchunks = 0;
  // adjoint tiling: lanes own pixels
  int adj_ppl = 4;            // pixels per lane
  std::vector<sl1m::Chunk> ptiles_delta, ptiles_gauss;
  int64_t adj_kchunk = 0;     // visibilities per chunk
  int n_achunks = 0;
  // matrix-core plans (SL1M_PREC_MFMA_*): forward chunks of mf_chunk pixels and
  // adjoint chunks of adj_kchunk visibilities (multiples of 32); images and
  // residual records are packed into the operand type on every call
  int mfma = 0;               // 0, or the plan's MFMA precision
  int n_mfchunks = 0;
  int64_t mf_chunk = 0;
  int64_t mf_np4 = 0, mf_nv4 = 0;  // pixels, visibilities padded to 32, over 4
  uint16_t* mx = nullptr;     // packed images [NG][np4][4 sides][4 pixels]
  uint16_t* mr = nullptr;     // packed residuals [NG][nv4][4 sides][re, -im][4 visibilities]
  float* mred = nullptr;      // block maxima [2][256], then inverse scales [2]
  // matrix-core plans whose pixels are one square delta grid: the forward on
  // the grid evaluation (per-call packed amplitude combinations of every pair
  // [NG][n_pairs][4 sides][8 words], each pair's nu)
  bool grid_mfma = false;
  void* grid_mfma_b = nullptr;
  double* grid_mfma_nu = nullptr;
  // FP32 hi/lo phase plans (SL1M_PREC_FP32_HILO): the coordinates' float32
  // splits, per pixel (permuted order) and per visibility
  bool hilo = false;
  sl1m::HLRec* phl = nullptr;
  sl1m::HLRec* vhl = nullptr;

  // grid evaluation (single right-hand side, FP32): segments on the grid path
  // and the direct chunks of the other segments
  bool grid = false;
  int grid_multi = 0;             // 2, 4 or 8: multi-RHS calls of up to this many sides on the grid
  std::vector<sl1m::GridSeg> grid_segs;
  int64_t grid_cells = 0;         // all grid segments
  int grid_vtiles = 0;            // forward visibility tiles (kGridVPL per lane)
  int grid_frows = 0;             // forward partial rows of the grid segments
  std::vector<sl1m::GridChunk> grid_fchunks;
  std::vector<sl1m::Chunk> fd1, fg1, pd1, pg1;
  double* grid_la = nullptr;      // |l| values of every grid segment
  double* grid_mb = nullptr;      // |m| values (0 padded to groups of kGridNB)
  double* grid_c3 = nullptr;      // per cell: n - 1 (delta) or l^2 + m^2 (Gaussian)
  double* grid_c4 = nullptr;      // per cell: kappa (wide-field Gaussian) or 0
  int32_t* grid_slot = nullptr;   // [4 * cells] permuted pixel index or -1
  void* grid_rec = nullptr;       // [cells] per-call GridRec / GridRecG records
  sl1m::GridPairRec* grid_prec = nullptr;   // per-call pair records (square grids)
  float* grid_precm = nullptr;               // multi-RHS pair records (square delta grids)
  sl1m::GridChunk* d_grid_fchunks = nullptr;
  sl1m::GridPairBlock* d_grid_pblocks = nullptr;
  sl1m::GridSeg* d_grid_segs = nullptr;     // device copy of grid_segs
  int2* d_grid_gblocks = nullptr;           // Gaussian adjoint blocks: (segment, block)
  int grid_gblocks = 0;
  sl1m::Chunk* d_chunks1 = nullptr;         // fd1 | fg1 | pd1 | pg1

  // device buffers (carved from the workspace)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t* perm = nullptr;          // permuted index -> caller index
  void* pixrec = nullptr;           // PixRec<R>[n_pix]
  double *pl = nullptr, *pm = nullptr, *pc3 = nullptr, *pc4 = nullptr;  // SoA
  void* pscale = nullptr;           // R[n_pix]
  void* pr2 = nullptr;              // R[n_pix]
  double *vu = nullptr, *vv = nullptr, *vw = nullptr;  // visibility coordinates
  void* vgain = nullptr;            // R[2*n_vis] complex gain G_k (or null)
  void* vbeta = nullptr;            // R[n_vis] pair beam exponent (or null)
  void* visrecD = nullptr;          // VisRecD<R>[n_vis]
  void* visrecG = nullptr;          // VisRecG<R>[n_layers*n_vis]
  void* rres = nullptr;             // C2<R>[(1+n_layers)][n_vis][max_rhs] adjoint residuals
  sl1m::ResPolar* rpol = nullptr;   // [n_vis] delta residuals in polar form (grid plans)
  void* layerDs = nullptr;          // R[2*n_layers*n_vis]: D and s
  sl1m::Chunk* d_fchunks = nullptr; // device copies of the chunk tables
  sl1m::Chunk* d_ptiles = nullptr;
  void* fpart = nullptr;            // R2[n_fchunks][n_vis]
  void* apart = nullptr;            // R[n_achunks][n_pix]
  void* xperm = nullptr;            // R[n_pix] permuted input / iterate y
  void* img = nullptr;              // R[n_pix] iterate I
  void* zbuf = nullptr;             // R[n_pix] MFISTA proximal point z_k
  void* res = nullptr;              // R[2*n_vis] residual
  double* red = nullptr;            // reduction scratch [kRedSlots]
  double* red_out = nullptr;        // [8] final reduction results
  int* flag = nullptr;              // domain-check counter
  double* scal = nullptr;           // solver scalars on the device: t_k, 1/L, lambda/L,
                                    // lambda, F(x_{k-1}) (MFISTA)

  // captured FISTA iteration (replayed with hipGraphLaunch)
  hipGraph_t iter_graph = nullptr;
  hipGraphExec_t iter_exec = nullptr;
  const void* iter_vis = nullptr;   // data pointer the captured graph reads
  int iter_method = 0;              // sl1m_method the captured graph runs

  // kernel timing (sl1m_timing_begin/end)
  bool timing = false;
  int timing_cap = 0;
  std::vector<hipEvent_t> tev[sl1m::kTimingKinds];   // pairs (start, stop) per kind
  int tcount[sl1m::kTimingKinds] = {};
};

namespace sl1m {

constexpr int kRedBlocks = 256;

// Records a timing event pair around `launch` when timing is enabled.
template <typename F>
hipError_t timed(sl1m_plan* p, int kind, hipStream_t st, F&& launch) {
  const bool on = p->timing && p->tcount[kind] < p->timing_cap;
  if (on) {
    hipError_t e = hipEventRecord(p->tev[kind][2 * p->tcount[kind]], st);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch();
  if (on && e == hipSuccess) {
    e = hipEventRecord(p->tev[kind][2 * p->tcount[kind] + 1], st);
    ++p->tcount[kind];
  }
  return e;
}

// status helpers (sl1m_api.hip)
sl1m_status set_error(sl1m_status s, const std::string& msg);
sl1m_status hip_error(hipError_t e, const char* what);

// kernels and launchers (sl1m_kernels.hip)
hipError_t launch_prep_pixels(sl1m_plan* p, const double* l, const double* m,
                              const double* ant_fwhm_dev_unused, double beam_coef,
                              hipStream_t st);
// float32 hi/lo splits of the pixel and visibility coordinates (hi/lo plans)
hipError_t launch_prep_hilo(sl1m_plan* p, hipStream_t st);
hipError_t launch_prep_vis(sl1m_plan* p, const double* u, const double* v, const double* w,
                           const int32_t* ap, const int32_t* aq, const double* gain,
                           const double* fwhm, int32_t n_ant, hipStream_t st);
// nr = number of right-hand sides (1, 2, 4 or 8); vectors are [nr][n].
hipError_t launch_gather(sl1m_plan* p, const void* x, void* xp, int nr, hipStream_t st);
hipError_t launch_forward(sl1m_plan* p, const void* xp, int nr, hipStream_t st);
// Partial rows a forward with nr right-hand sides writes (grid or direct split).
int forward_rows(const sl1m_plan* p, int nr);
hipError_t launch_forward_reduce(sl1m_plan* p, const void* data, void* out, bool adj_records,
                                 int nr, hipStream_t st);
hipError_t launch_adjoint_prep(sl1m_plan* p, const void* r, int nr, hipStream_t st);
hipError_t launch_adjoint(sl1m_plan* p, int nr, hipStream_t st);
hipError_t launch_adjoint_reduce(sl1m_plan* p, void* g_out, bool unpermute, int nr,
                                 hipStream_t st);
// FISTA update from device scalars p->scal = {t_k, 1/L, lambda/L}, then t_k -> t_{k+1}.
hipError_t launch_fista_update(sl1m_plan* p, hipStream_t st);
hipError_t launch_fill(void* dst, size_t n_elems, size_t elem_bytes, hipStream_t st);
hipError_t launch_splitmix_start(sl1m_plan* p, uint64_t seed, void* dst, hipStream_t st);
hipError_t launch_scale(sl1m_plan* p, void* x, int64_t n, double a, hipStream_t st);
hipError_t launch_unpermute(sl1m_plan* p, const void* src, void* dst, hipStream_t st);
hipError_t launch_copy_real(sl1m_plan* p, const void* src, void* dst, int64_t n, hipStream_t st);
// dst[perm[j]] = max(0, a * src[j]) (src permuted, dst in the caller's order)
hipError_t launch_dirty_out(sl1m_plan* p, const void* src, void* dst, double a, hipStream_t st);
// MFISTA: z = T(y - g / L) (zbuf); selection and extrapolation from the
// objective reduction of z in red_out (then F(x_k) and t_{k+1} in scal);
// F(x_0) from the objective reduction of x_0.
hipError_t launch_prox(sl1m_plan* p, hipStream_t st);
hipError_t launch_mfista_select(sl1m_plan* p, hipStream_t st);
hipError_t launch_mfista_init(sl1m_plan* p, hipStream_t st);
// Fixed-order FP64 reductions; results land in p->red_out.
//   dot_norm: red_out[0] = <a, b>, red_out[1] = <b, b>            (real [n_pix])
//   objective: red_out[0] = 1/2 |res|^2, red_out[1] = sum I, red_out[2] = nnz
hipError_t launch_dot_norm(sl1m_plan* p, const void* a, const void* b, hipStream_t st);
hipError_t launch_objective_terms(sl1m_plan* p, const void* res, const void* img,
                                  hipStream_t st);
// grid evaluation (sl1m_grid.hip): the grid segments' forward partial rows
// [0, grid_frows) and every pixel of the grid segments in the adjoint partials.
hipError_t launch_grid_forward(sl1m_plan* p, const void* xp, hipStream_t st);
hipError_t launch_grid_adjoint(sl1m_plan* p, hipStream_t st);
// Several right-hand sides (nr = 2 or 4; plans whose grid segments are all
// square delta grids): forward partial rows [r][forward_rows][n_vis] of the
// grid segments, adjoint partials [r][n_achunks][n_pix] from the polar
// residual records [r][n_vis].
bool grid_multi_ok(const sl1m_plan* p, int nr);
// matrix-core operator launches (packing included); partial rows as the
// direct kernels'
hipError_t launch_mfma_forward(sl1m_plan* p, const void* xp, int nr, hipStream_t st);
hipError_t launch_mfma_adjoint(sl1m_plan* p, int nr, hipStream_t st);
hipError_t launch_grid_forward_multi(sl1m_plan* p, const void* xp, int nr, hipStream_t st);
hipError_t launch_grid_adjoint_multi(sl1m_plan* p, int nr, hipStream_t st);
hipError_t launch_domain_check(sl1m_plan* p, const double* l, const double* m,
                               const double* sigma, const double* u, const double* v,
                               const double* w, hipStream_t st);

}  // namespace sl1m
