// Continuous-batching server for SL1M solves on one GPU.
//
// Many FISTA solves of different sizes share the GPU.  Each admitted request
// owns a plan and solver state carved from one caller-provided HBM arena
// (admission by footprint).  Work advances in rounds; a round is one launch of
// each batched kernel (forward delta/Gaussian, reduce, adjoint
// delta/Gaussian, update, final), each with a fixed grid whose blocks stride
// over a table listing every active request's work items for that round.  The
// item decomposition and every reduction order depend only on the request's
// own plan, so a request's result is bitwise the same alone and in any mix.
// Requests submitted while others run join a round once a host thread of
// the server has built their plans (on a stream of its own, off the step
// loop).
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sl1m_grid.h"
#include "sl1m_sched.h"
#include "sl1m_trace.h"

namespace sl1m {
namespace {

using namespace dev;
using sched::Segment;

constexpr int kSrvMaxSlots = 64;
constexpr int kSrvRing = 4;              // rounds in flight (table buffers)
// A round runs as two lanes on two streams: requests with Gaussian pixels in
// one, the others in the second.  Lanes share no request, so their launches
// may overlap: the tail of one lane's kernel is filled by the other's blocks.
constexpr int kSrvLanes = 2;
constexpr int kSrvTileBlocks = 2048;     // per-request operator split target (work-item count)
constexpr double kSrvMaxRound = 4.0;     // OLDEST_FIRST rounds: at most this many budgets
// item tables per round: 4 operator kinds x 6 variants (4 direct tile shapes,
// the grid evaluation, the square-grid evaluation), then reduce, update, final
// and the grid prep (delta, Gaussian).  Square grid requests use the
// square variant: a delta one files its pair chunks and pair blocks under the
// Gaussian kinds, a Gaussian one under the delta kinds.
constexpr int kOpVariants = 6;
constexpr int kGridVariant = 4, kSquareVariant = 5;
constexpr int kTabReduce = 4 * kOpVariants, kTabUpdate = kTabReduce + 1,
              kTabFinal = kTabReduce + 2, kTabPrepD = kTabReduce + 3, kTabPrepG = kTabReduce + 4,
              kTabs = kTabReduce + 5;

struct SegDev {
  int32_t slot, flags;
  int64_t begin, end, prefix;
};

struct TabDev {
  int64_t total;
  int32_t n_seg, pad;
  SegDev seg[kSrvMaxSlots];
};

// Per-slot device descriptor: pointers into the request's plan and state, plus
// solver scalars updated by the batched kernels.
struct ReqDev {
  const PixRec<float>* pix;
  const double *vu, *vv, *vw;
  const float* vgain;
  const float* vbeta;
  const VisRecD<float>* visrecD;
  const VisRecG<float>* visrecG;
  const float* layerDs;
  float2* rres;
  ResPolar* rpol;        // delta residuals in polar form (square delta grids)
  const double *pl, *pm, *pc3, *pc4;
  const float* pscale;
  const float* pr2;
  const int32_t* perm;
  const Chunk* fchunks;  // delta chunks, then Gaussian chunks
  const Chunk* ptiles;   // delta tiles, then Gaussian tiles
  float2* fpart;
  float* apart;
  float* x;              // power-iteration vector (unnormalised; true x = xscale * x)
  float* y;              // FISTA extrapolated point
  float* img;            // FISTA iterate
  const float2* data;    // caller's visibilities
  float* out;            // caller's image
  double* red;           // partial sums: [vis_blocks] then [2 * pix_blocks]
  int* flag;             // non-finite values seen
  int64_t n_pix, n_vis, kchunk, vtiles, vis_blocks, pix_blocks;
  int32_t n_fchunks, n_fd, n_achunks, n_pd, n_pg, vpl, ppl, n_layers, beam_pair;
  double t, inv_L, thr, lam, L, L_safety, rq, xscale, l2, l1, nnz;
  // grid evaluation (requests whose pixels form one grid segment)
  const double *g_la, *g_mb, *g_c3, *g_c4;
  const int32_t* g_slot;
  void* g_rec;                     // GridRec / GridRecG per cell
  const GridChunk* g_fchunks;
  const VisRecG<float>* g_vrec;    // the layer's records (Gaussian)
  const float* g_Ds;               // the layer's (D, s) pairs (Gaussian)
  const float2* g_lres;            // the layer's residual records
  const GridPairBlock* g_pblocks;  // square grids: adjoint pair blocks
  GridPairRec* g_prec;             // square grids: forward pair records
  int64_t g_npairs;
  int64_t g_cells;
  int32_t g_na, g_ng, g_vtiles, g_nfs;
  int32_t g_ablk, g_pad;           // adjoint blocks (lane-set or pair blocks)
};

// Segment of work item w: lane i of each wavefront tests segment i (a table
// has at most kSrvMaxSlots = 64 of them, their prefixes non-decreasing), and
// the number of segments starting at or before w, less one, is the index --
// one vector load per block instead of a chain of dependent scalar loads.
static_assert(kSrvMaxSlots <= 64, "one segment per lane of a wavefront");
__device__ __forceinline__ int find_seg(const TabDev* __restrict__ tab, int64_t w) {
  const int lane = threadIdx.x % 64;
  const bool hit = lane < tab->n_seg && tab->seg[lane].prefix <= w;
  return __popcll(__ballot(hit)) - 1;
}

__device__ __forceinline__ double srv_block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Work-item variants of the operator kernels (one instantiation each, so a
// kernel's register allocation is that of its own tile shape):
//   0: 1 visibility/pixel per lane, 1: 2, 2: 4, 3: 4 with per-pair beams.
template <bool GAUSS, int VPL, bool BEAM>
__global__ __launch_bounds__(kBlock) void k_srv_fwd(const TabDev* __restrict__ tab,
                                                    const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  // item counts stay far below 2^31: decode with 32-bit division; the results
  // are wavefront-uniform and are moved to scalar registers so that the chunk
  // and everything indexed by it are read through the scalar unit
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nvt = static_cast<uint32_t>(q.vtiles);
  const int64_t c = __builtin_amdgcn_readfirstlane(static_cast<int>((GAUSS ? q.n_fd : 0) + item / nvt));
  const int64_t vt = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nvt));
  const Chunk ch = load_chunk(q.fchunks, c);
  const float* xp = (sg.flags & sched::F_POWER) ? q.x : (sg.flags & sched::F_OBJECTIVE) ? q.img : q.y;
  const float xs = (sg.flags & sched::F_POWER) ? static_cast<float>(q.xscale) : 1.0f;
  float2* row = q.fpart + c * q.n_vis;
  if (GAUSS)
    fwd_gauss_tile<float, VPL, BEAM, 1>(q.pix, xp, q.n_pix, q.vu, q.vv, q.vw, q.vbeta, ch, vt,
                                        q.n_vis, row, 0, xs);
  else
    fwd_delta_tile<float, VPL, BEAM, 1>(q.pix, xp, q.n_pix, q.vu, q.vv, q.vw, q.vbeta, ch, vt,
                                        q.n_vis, row, 0, xs);
}

// Sum of forward partial rows, gain, residual; adjoint residual records, or
// (objective phase) per-block partials of |V - M I|^2.
__global__ __launch_bounds__(kBlock) void k_srv_reduce(const TabDev* __restrict__ tab,
                                                       ReqDev* __restrict__ reqs) {
  __shared__ double sh[kBlock];
  {
    const int64_t w = blockIdx.x;
    const SegDev sg = tab->seg[find_seg(tab, w)];
    ReqDev& q = reqs[sg.slot];
    const int64_t blk = sg.begin + (w - sg.prefix);
    const int64_t k = blk * kBlock + threadIdx.x;
    double l2 = 0.0;
    if (k < q.n_vis) {
      float2 acc = make_float2(0.f, 0.f);
      strided_sum<float2>(q.fpart + k, q.n_fchunks, q.n_vis, acc);
      float re = acc.x, im = acc.y;
      const float gr = q.vgain ? q.vgain[2 * k] : 1.f, gi = q.vgain ? q.vgain[2 * k + 1] : 0.f;
      if (q.vgain) {
        const float tr = gr * re - gi * im;
        im = gr * im + gi * re;
        re = tr;
      }
      if (sg.flags & (sched::F_FISTA | sched::F_OBJECTIVE)) {
        re -= q.data[k].x;
        im -= q.data[k].y;
      }
      if (sg.flags & sched::F_OBJECTIVE)
        l2 = static_cast<double>(re) * re + static_cast<double>(im) * im;
      else
        write_res<float>(q.rres, q.layerDs, q.n_layers, q.n_vis, 1, k, 0, gr, gi, re, im, q.rpol);
    }
    if (sg.flags & sched::F_OBJECTIVE) {
      l2 = srv_block_sum(l2, sh);
      if (threadIdx.x == 0) q.red[blk] = l2;
    }
  }
}

template <bool GAUSS, int PPL, bool BEAM>
__global__ __launch_bounds__(kBlock) void k_srv_adj(const TabDev* __restrict__ tab,
                                                    const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  // pixel tiles fastest: the blocks running together share a visibility chunk
  const uint32_t nt = static_cast<uint32_t>(GAUSS ? q.n_pg : q.n_pd);
  const int64_t kc = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nt));
  const int64_t tile = __builtin_amdgcn_readfirstlane(static_cast<int>((GAUSS ? q.n_pd : 0) + item % nt));
  const Chunk tl = load_chunk(q.ptiles, tile);
  float* row = q.apart + kc * q.n_pix;
  if (GAUSS)
    adj_gauss_tile<float, PPL, BEAM, 1>(q.visrecG, q.rres, q.vbeta, q.pl, q.pm, q.pc3, q.pc4,
                                        q.pr2, tl, 0, kc, q.kchunk, q.n_vis, row, 0);
  else
    adj_delta_tile<float, PPL, BEAM, 1>(q.visrecD, q.rres, q.vbeta, q.pl, q.pm, q.pc3, q.pr2, tl,
                                        0, kc, q.kchunk, q.n_vis, row, 0);
}

// Per pixel block: FISTA step (threshold + momentum), power-iteration update
// (x <- g with partial <x, g> and |g|^2), or the objective pass (partial sum
// and non-zero count, copy of the image to the caller's order).
// The adjoint partial rows are summed for the block's kBlock pixels by its
// four wavefronts: wavefront w adds rows c = w, w + 4, ... for four pixels per
// lane (64 apart, so every load is one contiguous 256-byte line per
// wavefront), and the four partial sums of a pixel meet in LDS as
// (s0 + s1) + (s2 + s3) -- the order of the per-plan FISTA kernel.
__global__ __launch_bounds__(kBlock) void k_srv_update(const TabDev* __restrict__ tab,
                                                       ReqDev* __restrict__ reqs) {
  static_assert(kBlock == 256, "four wavefronts of 64 lanes");
  __shared__ double sh[kBlock];
  __shared__ float srow[4][kBlock];
  {
    const int64_t w = blockIdx.x;
    const SegDev sg = tab->seg[find_seg(tab, w)];
    ReqDev& q = reqs[sg.slot];
    const int64_t blk = sg.begin + (w - sg.prefix);
    const int64_t j0 = blk * kBlock;
    const int64_t j = j0 + threadIdx.x;
    if (!(sg.flags & sched::F_OBJECTIVE)) {  // uniform over the block
      const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
      float g4[4] = {0.f, 0.f, 0.f, 0.f};
      const int nr = q.n_achunks;
      if (wv < nr) {
        // rows wv, wv + 4, ...: four rows of the four pixels are loaded
        // before they are added (sixteen loads per round trip); every pixel
        // still adds its rows in order
        const int cnt = (nr - wv + 3) / 4;
        const int64_t stride = 4 * q.n_pix;
        const float* base = q.apart + static_cast<int64_t>(wv) * q.n_pix + j0 + ln;
        bool ok[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) ok[s4] = j0 + ln + 64 * s4 < q.n_pix;
        int c = 0;
        for (; c + 4 <= cnt; c += 4) {
          float a[4][4];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
              a[r][s4] = ok[s4] ? base[(c + r) * stride + 64 * s4] : 0.f;
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) g4[s4] += a[r][s4];
        }
        for (; c < cnt; ++c)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
            if (ok[s4]) g4[s4] += base[c * stride + 64 * s4];
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) srow[wv][ln + 64 * s4] = g4[s4];
    }
    __syncthreads();
    double p0 = 0.0, p1 = 0.0;
    if (j < q.n_pix) {
      if (sg.flags & sched::F_OBJECTIVE) {
        const float v = q.img[j];
        p0 = v;
        p1 = v != 0.f ? 1.0 : 0.0;
        q.out[q.perm[j]] = v;
      } else {
        const int t = threadIdx.x;
        float g = (srow[0][t] + srow[1][t]) + (srow[2][t] + srow[3][t]);
        g *= q.pscale[j];
        if (sg.flags & sched::F_POWER) {
          const float xo = q.x[j] * static_cast<float>(q.xscale);
          p0 = static_cast<double>(xo) * g;
          p1 = static_cast<double>(g) * g;
          q.x[j] = g;
        } else {
          const double t = q.t;
          const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
          const float beta = static_cast<float>((t - 1.0) / tn);
          const float z = q.y[j] - g * static_cast<float>(q.inv_L);
          if (!isfinite(z)) atomicOr(q.flag, 1);
          const float thr = static_cast<float>(q.thr);
          const float in = z > thr ? z - thr : 0.f;
          const float io = q.img[j];
          q.y[j] = in + beta * (in - io);
          q.img[j] = in;
        }
      }
    }
    if (sg.flags & (sched::F_POWER | sched::F_OBJECTIVE)) {
      p0 = srv_block_sum(p0, sh);
      p1 = srv_block_sum(p1, sh);
      if (threadIdx.x == 0) {
        q.red[q.vis_blocks + 2 * blk] = p0;
        q.red[q.vis_blocks + 2 * blk + 1] = p1;
      }
    }
  }
}

// One block per request: fixed-order sums of the partials and the scalar
// state updates (power step, FISTA momentum, objective terms).
__global__ __launch_bounds__(kBlock) void k_srv_final(const TabDev* __restrict__ tab,
                                                      ReqDev* __restrict__ reqs) {
  __shared__ double sh[kBlock];
  {
    const int64_t w = blockIdx.x;
    const SegDev sg = tab->seg[find_seg(tab, w)];
    ReqDev& q = reqs[sg.slot];
    if (sg.flags & sched::F_FISTA) {
      if (threadIdx.x == 0) q.t = 0.5 * (1.0 + sqrt(1.0 + 4.0 * q.t * q.t));
      return;
    }
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < q.pix_blocks; i += blockDim.x) {
      a += q.red[q.vis_blocks + 2 * i];
      b += q.red[q.vis_blocks + 2 * i + 1];
    }
    if (sg.flags & sched::F_OBJECTIVE)
      for (int64_t i = threadIdx.x; i < q.vis_blocks; i += blockDim.x) c += q.red[i];
    a = srv_block_sum(a, sh);
    b = srv_block_sum(b, sh);
    c = srv_block_sum(c, sh);
    if (threadIdx.x == 0) {
      if (sg.flags & sched::F_POWER) {
        q.rq = a;
        q.xscale = b > 0.0 ? 1.0 / sqrt(b) : 0.0;
        if (sg.flags & sched::F_LAST_POWER) {
          q.L = q.L_safety * a;
          q.inv_L = 1.0 / q.L;
          q.thr = q.lam / q.L;
          q.t = 1.0;
        }
      } else {
        q.l2 = 0.5 * c;
        q.l1 = a;
        q.nnz = b;
      }
    }
  }
}

// Grid evaluation.  Prep: the per-call cell records of the phase's input
// vector (power step: x scaled by xscale; FISTA: y; objective: I), one block
// per kBlock cells.
template <bool GAUSS>
__global__ __launch_bounds__(kBlock) void k_srv_gprep(const TabDev* __restrict__ tab,
                                                      const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const int64_t c = (sg.begin + (w - sg.prefix)) * kBlock + threadIdx.x;
  const float* xp = (sg.flags & sched::F_POWER) ? q.x : (sg.flags & sched::F_OBJECTIVE) ? q.img : q.y;
  const float xs = (sg.flags & sched::F_POWER) ? static_cast<float>(q.xscale) : 1.0f;
  if (c < q.g_npairs) {  // square grids: pair records too
    if (GAUSS)
      grid_write_pair_rec_gauss(c, q.g_na, q.g_slot, q.g_c3, q.g_c4, xp, q.pscale, xs,
                                reinterpret_cast<GridPairRecG*>(q.g_prec));
    else
      grid_write_pair_rec(c, q.g_na, q.g_slot, q.g_c3, xp, q.pscale, xs, q.g_prec);
  }
  if (c >= q.g_cells) return;
  float x[4];
  int32_t empty = 1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t j = q.g_slot[4 * c + s];
    x[s] = j >= 0 ? q.pscale[j] * xs * xp[j] : 0.0f;
    if (j >= 0) empty = 0;
  }
  if (GAUSS) {
    GridRecG r;
    r.r2 = q.g_c3[c];
    r.kappa = q.g_c4[c];
#pragma unroll
    for (int s = 0; s < 4; ++s) r.x[s] = x[s];
    static_cast<GridRecG*>(q.g_rec)[c] = r;
  } else {
    GridRec r;
    r.nu = q.g_c3[c];
    r.e1 = (x[0] + x[1]) + (x[2] + x[3]);
    r.e2 = (x[1] + x[2]) - (x[0] + x[3]);
    r.e3 = (x[0] + x[1]) - (x[2] + x[3]);
    r.e4 = (x[0] - x[1]) + (x[2] - x[3]);
    r.empty = empty;
    r.pad = 0;
    static_cast<GridRec*>(q.g_rec)[c] = r;
  }
}

// Forward items (grid chunk, visibility tile); partial row = grid chunk.
template <bool GAUSS>
__global__ __launch_bounds__(kBlock) void k_srv_gfwd(const TabDev* __restrict__ tab,
                                                     const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nvt = static_cast<uint32_t>(q.g_vtiles);
  const int64_t c = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nvt));
  const int64_t vt = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nvt));
  const ConstPtr<GridChunk> cc = as_const(q.g_fchunks) + c;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  float2* row = q.fpart + c * q.n_vis;
  if (GAUSS)
    grid_fwd_gauss_tile(static_cast<const GridRecG*>(q.g_rec), q.g_la, q.g_mb, ch, q.g_na,
                        q.g_vrec, q.g_Ds, vt, q.n_vis, row);
  else
    grid_fwd_delta_tile(static_cast<const GridRec*>(q.g_rec), q.g_la, q.g_mb, ch, q.g_na, q.vu,
                        q.vv, q.vw, vt, q.n_vis, row);
}

// Adjoint items (lane-set block, visibility chunk); partial row = chunk.
template <bool GAUSS>
__global__ __launch_bounds__(kBlock) void k_srv_gadj(const TabDev* __restrict__ tab,
                                                     const ReqDev* __restrict__ reqs) {
  __shared__ float4 lds[kGridKBG * kGridMaxGL * kGridNBA];
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nb = static_cast<uint32_t>(q.g_ablk);  // blocks fastest
  const int64_t kc = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nb));
  const int64_t blk = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nb));
  float* row = q.apart + kc * q.n_pix;
  if (GAUSS)
    grid_adj_gauss_tile(q.g_vrec, q.g_lres, q.g_la, q.g_mb, q.g_c3, q.g_c4, q.g_slot, q.g_na,
                        2 * q.g_ng, blk, kc, q.kchunk, q.n_vis, row,
                        reinterpret_cast<float4(*)[kGridMaxGL][kGridNBA]>(lds));
  else
    grid_adj_delta_tile(q.visrecD, q.rres, q.vv, q.g_la, q.g_mb, q.g_c3, q.g_slot, q.g_na,
                        2 * q.g_ng, blk, kc, q.kchunk, q.n_vis, row,
                        reinterpret_cast<float2(*)[kGridMaxGL][kGridNBA]>(lds));
}

// Square delta grids: pair forward chunks (items over chunks nfs.., rows
// nfs..) and pair adjoint blocks.
__global__ __launch_bounds__(kBlock) void k_srv_gfwd_pairs(const TabDev* __restrict__ tab,
                                                           const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nvt = static_cast<uint32_t>(q.g_vtiles);
  const int64_t c = __builtin_amdgcn_readfirstlane(static_cast<int>(q.g_nfs + item / nvt));
  const int64_t vt = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nvt));
  const ConstPtr<GridChunk> cc = as_const(q.g_fchunks) + c;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_delta_pairs_tile(q.g_prec, q.g_la, q.g_mb, ch, q.g_na, q.vu, q.vv, q.vw, vt, q.n_vis,
                            q.fpart + c * q.n_vis);
}

__global__ __launch_bounds__(kBlock) void k_srv_gadj_pairs(const TabDev* __restrict__ tab,
                                                           const ReqDev* __restrict__ reqs) {
  __shared__ float4 lds[kGridKBG][kGridMaxGL][kGridNBA];
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nb = static_cast<uint32_t>(q.g_ablk);  // blocks fastest
  const int64_t kc = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nb));
  const int64_t bi = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nb));
  const ConstPtr<GridPairBlock> cb = as_const(q.g_pblocks) + bi;
  GridPairBlock pb;
  pb.g4 = cb->g4;
  pb.ia = cb->ia;
  pb.count = cb->count;
  pb.n_gl = cb->n_gl;
  grid_adj_delta_pairs_tile(q.visrecD, q.rpol, q.vu, q.vv, q.g_la, q.g_mb, q.g_c3, q.g_slot,
                            q.g_na, pb, kc, q.kchunk, q.n_vis, q.apart + kc * q.n_pix, lds);
}

// Square Gaussian grids: pair forward chunks (one visibility per lane) and
// pair adjoint blocks.
__global__ __launch_bounds__(kBlock) void k_srv_ggfwd_pairs(const TabDev* __restrict__ tab,
                                                            const ReqDev* __restrict__ reqs) {
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nvt = static_cast<uint32_t>(q.g_vtiles);
  const int64_t c = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nvt));
  const int64_t vt = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nvt));
  const ConstPtr<GridChunk> cc = as_const(q.g_fchunks) + c;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_gauss_pairs_tile(reinterpret_cast<const GridPairRecG*>(q.g_prec), q.g_la, q.g_mb, ch,
                            q.g_na, q.g_vrec, q.g_Ds, vt, q.n_vis, q.fpart + c * q.n_vis);
}

__global__ __launch_bounds__(kBlock) void k_srv_ggadj_pairs(const TabDev* __restrict__ tab,
                                                            const ReqDev* __restrict__ reqs) {
  __shared__ float4 lds[kGridKBG][kGridMaxGL][kGridNBA][2];
  const int64_t w = blockIdx.x;
  const SegDev sg = tab->seg[find_seg(tab, w)];
  const ReqDev& q = reqs[sg.slot];
  const uint32_t item = static_cast<uint32_t>(sg.begin + (w - sg.prefix));
  const uint32_t nb = static_cast<uint32_t>(q.g_ablk);  // blocks fastest
  const int64_t kc = __builtin_amdgcn_readfirstlane(static_cast<int>(item / nb));
  const int64_t bi = __builtin_amdgcn_readfirstlane(static_cast<int>(item % nb));
  const ConstPtr<GridPairBlock> cb = as_const(q.g_pblocks) + bi;
  GridPairBlock pb;
  pb.g4 = cb->g4;
  pb.ia = cb->ia;
  pb.count = cb->count;
  pb.n_gl = cb->n_gl;
  grid_adj_gauss_pairs_tile(q.g_vrec, q.g_lres, q.g_la, q.g_mb, q.g_c3, q.g_c4, q.g_slot, q.g_na,
                            pb, kc, q.kchunk, q.n_vis, q.apart + kc * q.n_pix, lds);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// A request moves PENDING -> ADMITTING (arena and slot reserved by the step
// loop, plan built by the admission thread) -> ACTIVE (in the rounds) -> DONE,
// or to CANCELLED from any state before DONE.
struct Ticket {
  sched::Request req;
  sl1m_problem problem;
  const void* vis = nullptr;
  void* img_out = nullptr;
  sl1m_solve_params params{};
  enum State { PENDING, ADMITTING, ACTIVE, DONE, CANCELLED } state = PENDING;
  sl1m_plan* plan = nullptr;
  size_t arena_off = 0;
  size_t footprint = 0;
  sl1m_solve_info info{};
  double submit_s = 0, admit_s = 0, finish_s = 0;
  bool freed = true;
  bool grid_allowed = false;
  // written by the admission thread, read by the step loop once `built` is set
  std::atomic<int> built{0};
  sl1m_status build_status = SL1M_OK;
  int8_t fwd_variant = 0, adj_variant = 0, grid_kind = 0, lane = 0;
};

}  // namespace
}  // namespace sl1m

struct sl1m_server {
  std::mutex mu;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  sl1m::sched::Arena alloc;
  int max_slots = 0;
  double budget = 3e10;                // evals per round (OLDEST_FIRST: the least), shared by the active requests
  int policy = SL1M_SERVE_OLDEST_FIRST;  // how the round budget is shared
  hipStream_t stream = nullptr;        // rounds (non-blocking, default priority)
  hipStream_t lane_stream = nullptr;   // the second lane of each round
  hipEvent_t lane_event[sl1m::kSrvRing] = {};  // end of the second lane's round
  hipStream_t admit_stream = nullptr;  // plan creation of admitted requests (admission thread)
  hipStream_t read_stream = nullptr;   // results of finished requests (step loop)
  int device = 0;
  // admission thread: builds the plans of reserved requests in submission order
  std::thread admitter;
  std::mutex wq_mu;
  std::condition_variable wq_cv;
  std::deque<sl1m::Ticket*> wq;
  bool wq_stop = false;
  std::deque<uint64_t> admitting;       // reserved requests, in submission order
  sl1m::ReqDev* d_reqs = nullptr;
  sl1m::TabDev* d_tabs = nullptr;      // [kSrvRing][kSrvLanes][kTabs]
  sl1m::TabDev* h_tabs = nullptr;      // pinned mirror
  int8_t fwd_variant[sl1m::kSrvMaxSlots] = {};  // tile variant of each slot's request
  int8_t adj_variant[sl1m::kSrvMaxSlots] = {};
  int8_t grid_kind[sl1m::kSrvMaxSlots] = {};    // 0 direct, 1 grid delta, 2 grid Gaussian
  int8_t lane[sl1m::kSrvMaxSlots] = {};         // lane of each slot's request
  hipEvent_t ring_event[sl1m::kSrvRing] = {};
  int64_t ring_round[sl1m::kSrvRing] = {-1, -1, -1, -1};
  std::vector<int> free_slots;
  std::map<uint64_t, std::unique_ptr<sl1m::Ticket>> tickets;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;         // tickets in slot order of admission
  std::deque<std::pair<int64_t, std::vector<uint64_t>>> finishing;  // round -> tickets
  uint64_t next_ticket = 1;
  int64_t round = 0;
  int64_t completed_round = -1;
  double evals_scheduled = 0;
  std::chrono::steady_clock::time_point t0;
};

namespace sl1m {
namespace {

double now_s(const sl1m_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

#define SRV_HIP(call, what)                           \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

size_t extra_bytes(const sl1m_problem& p) {
  const size_t np = static_cast<size_t>(p.n_pix), nv = static_cast<size_t>(p.n_vis);
  const size_t vb = (nv + kBlock - 1) / kBlock, pb = (np + kBlock - 1) / kBlock;
  return sched::Arena::round_up(4 * np) + sched::Arena::round_up(8 * (vb + 2 * pb + 2)) +
         sched::Arena::round_up(sizeof(int));
}

// State of ring slot i's round: hipSuccess once it has ended on both lanes.
// Both events are recorded every round, also by a lane without work in it,
// and each lane's stream runs its rounds in order, so every earlier round has
// ended too.
hipError_t ring_query(sl1m_server* s, int i) {
  hipError_t q = hipEventQuery(s->ring_event[i]);
  if (q == hipSuccess) q = hipEventQuery(s->lane_event[i]);
  return q;
}

// Releases memory and slot of requests whose last round has completed.
void harvest(sl1m_server* s) {
  for (int i = 0; i < kSrvRing; ++i) {
    if (s->ring_round[i] < 0) continue;
    const hipError_t q = ring_query(s, i);
    if (q == hipSuccess) {
      s->completed_round = std::max(s->completed_round, s->ring_round[i]);
      s->ring_round[i] = -1;
    } else if (q == hipErrorNotReady) {
      (void)hipGetLastError();  // "not ready" is not an error; keep launch checks clean
    }
  }
  // rounds complete in order on each lane: everything up to completed_round is done
  while (!s->finishing.empty() && s->finishing.front().first <= s->completed_round) {
    for (uint64_t id : s->finishing.front().second) {
      Ticket& t = *s->tickets[id];
      if (t.state != Ticket::ACTIVE) continue;
      // the round has completed; read through a stream of its own so that
      // neither rounds in flight nor admissions are waited for
      ReqDev q;
      int nonfinite = 0;
      hipError_t e = hipMemcpyAsync(&q, s->d_reqs + t.req.slot, sizeof(ReqDev),
                                    hipMemcpyDeviceToHost, s->read_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->read_stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&nonfinite, q.flag, sizeof(int), hipMemcpyDeviceToHost,
                           s->read_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->read_stream);
      if (e != hipSuccess) {
        t.info.status = SL1M_EHIP;
      } else {
        t.info.iters = t.params.max_iter;
        t.info.L = q.L;
        t.info.l2_term = q.l2;
        t.info.l1_term = q.l1;
        t.info.F = q.l2 + t.params.lambda * q.l1;
        t.info.nnz = static_cast<int64_t>(q.nnz);
        t.info.status = (nonfinite || !std::isfinite(t.info.F)) ? SL1M_EDIVERGED : SL1M_OK;
      }
      t.finish_s = now_s(s);
      t.state = Ticket::DONE;
    }
    s->finishing.pop_front();
  }
  // free memory of finished or cancelled requests once no in-flight round uses it
  for (auto it = s->active.begin(); it != s->active.end();) {
    Ticket& t = *s->tickets[*it];
    const bool over = t.state == Ticket::DONE || t.state == Ticket::CANCELLED;
    if (over && t.req.last_round <= s->completed_round) {
      if (t.plan) sl1m_plan_destroy(t.plan);
      t.plan = nullptr;
      s->alloc.release(t.arena_off);
      s->free_slots.push_back(t.req.slot);
      t.freed = true;
      it = s->active.erase(it);
    } else {
      ++it;
    }
  }
}

sl1m_status admit(sl1m_server* s, Ticket& t) {
  const sl1m_problem& pr = t.problem;
  const size_t ws_al = t.footprint - extra_bytes(pr);
  char* base = s->arena + t.arena_off;
  sl1m_plan* plan = nullptr;
  int gkind = 0;
  if (t.grid_allowed) {
    sl1m_problem pg = pr;
    pg.grid_mode = SL1M_GRID_AUTO;
    if (sl1m_status st = sl1m_plan_create(&pg, base, ws_al, s->admit_stream, &plan)) return st;
    const bool pure = plan->grid_segs.size() == 1 && plan->fd1.empty() && plan->fg1.empty() &&
                      plan->pd1.empty() && plan->pg1.empty();
    if (pure) {
      gkind = plan->grid_segs[0].kind == SL1M_PIX_DELTA ? 1 : 2;
    } else {
      sl1m_plan_destroy(plan);
      plan = nullptr;
    }
  }
  if (!plan) {
    if (sl1m_status st = sl1m_plan_create(&pr, base, ws_al, s->admit_stream, &plan)) return st;
  }
  t.plan = plan;
  char* extra = base + ws_al;
  float* y = reinterpret_cast<float*>(extra);
  double* red = reinterpret_cast<double*>(extra + sched::Arena::round_up(4 * pr.n_pix));
  const size_t vb = (pr.n_vis + kBlock - 1) / kBlock, pb = (pr.n_pix + kBlock - 1) / kBlock;
  int* flag = reinterpret_cast<int*>(reinterpret_cast<char*>(red) +
                                     sched::Arena::round_up(8 * (vb + 2 * pb + 2)));
  hipStream_t st = s->admit_stream;
  SRV_HIP(launch_fill(y, pr.n_pix, 4, st), "zero y");
  SRV_HIP(launch_fill(plan->img, pr.n_pix, 4, st), "zero I");
  SRV_HIP(launch_fill(flag, 1, sizeof(int), st), "zero flag");
  const bool power = !(t.params.L > 0.0);
  double xscale = 1.0;
  if (power && pr.n_pix > 0) {
    SRV_HIP(launch_splitmix_start(plan, t.params.seed, plan->xperm, st), "start vector");
    SRV_HIP(launch_dot_norm(plan, plan->xperm, plan->xperm, st), "start norm");
    double h[2];
    SRV_HIP(hipMemcpyAsync(h, plan->red_out, sizeof(h), hipMemcpyDeviceToHost, st), "read norm");
    SRV_HIP(hipStreamSynchronize(st), "admission sync");
    if (!(h[1] > 0.0)) return set_error(SL1M_EINVAL, "power iteration start vector is zero");
    xscale = 1.0 / std::sqrt(h[1]);
  }
  ReqDev q{};
  q.pix = static_cast<const PixRec<float>*>(plan->pixrec);
  q.vu = plan->vu;
  q.vv = plan->vv;
  q.vw = plan->vw;
  q.vgain = static_cast<const float*>(plan->vgain);
  q.vbeta = static_cast<const float*>(plan->vbeta);
  q.visrecD = static_cast<const VisRecD<float>*>(plan->visrecD);
  q.visrecG = static_cast<const VisRecG<float>*>(plan->visrecG);
  q.layerDs = static_cast<const float*>(plan->layerDs);
  q.rres = static_cast<float2*>(plan->rres);
  q.rpol = plan->rpol;
  q.pl = plan->pl;
  q.pm = plan->pm;
  q.pc3 = plan->pc3;
  q.pc4 = plan->pc4;
  q.pscale = static_cast<const float*>(plan->pscale);
  q.pr2 = static_cast<const float*>(plan->pr2);
  q.perm = plan->perm;
  q.fchunks = plan->d_fchunks;
  q.ptiles = plan->d_ptiles;
  q.fpart = static_cast<float2*>(plan->fpart);
  q.apart = static_cast<float*>(plan->apart);
  q.x = static_cast<float*>(plan->xperm);
  q.y = y;
  q.img = static_cast<float*>(plan->img);
  q.data = static_cast<const float2*>(t.vis);
  q.out = static_cast<float*>(t.img_out);
  q.red = red;
  q.flag = flag;
  q.n_pix = plan->n_pix;
  q.n_vis = plan->n_vis;
  q.kchunk = plan->adj_kchunk;
  q.vpl = plan->beam_pair ? 4 : plan->fwd_vpl;
  q.ppl = plan->beam_pair ? 4 : plan->adj_ppl;
  q.vtiles = (plan->n_vis + kBlock * q.vpl - 1) / (kBlock * q.vpl);
  q.vis_blocks = static_cast<int64_t>(vb);
  q.pix_blocks = static_cast<int64_t>(pb);
  q.n_fchunks = forward_rows(plan, 1);
  q.n_fd = static_cast<int32_t>(plan->fchunks_delta.size());
  if (gkind) {
    const GridSeg& g = plan->grid_segs[0];
    q.g_la = plan->grid_la + g.la_off;
    q.g_mb = plan->grid_mb + g.mb_off;
    q.g_c3 = plan->grid_c3 + g.cell_off;
    q.g_c4 = plan->grid_c4 + g.cell_off;
    q.g_slot = plan->grid_slot + 4 * g.cell_off;
    q.g_rec = static_cast<char*>(plan->grid_rec) + sizeof(GridRec) * g.cell_off;
    q.g_fchunks = plan->d_grid_fchunks + g.fc0;
    if (gkind == 2) {
      q.g_vrec = static_cast<const VisRecG<float>*>(plan->visrecG) +
                 static_cast<int64_t>(g.layer) * plan->n_vis;
      q.g_Ds = static_cast<const float*>(plan->layerDs) + static_cast<int64_t>(g.layer) * 2 * plan->n_vis;
      q.g_lres = static_cast<const float2*>(plan->rres) + static_cast<int64_t>(1 + g.layer) * plan->n_vis;
    }
    q.g_pblocks = plan->d_grid_pblocks + g.pb0;
    q.g_prec = g.square ? plan->grid_prec + g.pr_off : nullptr;
    q.g_npairs = g.square ? g.n_pairs : 0;
    q.g_cells = g.cells;
    q.g_na = g.na;
    q.g_ng = g.ng;
    q.g_vtiles = plan->grid_vtiles;
    q.g_nfs = g.nfs;
    q.g_ablk = static_cast<int32_t>(g.square ? g.pblocks : g.ablocks);
    if (g.square) {
      gkind = gkind == 1 ? 3 : 4;  // square delta, square Gaussian
      if (gkind == 4) q.g_vtiles = static_cast<int32_t>((plan->n_vis + kBlock - 1) / kBlock);
    }
  }
  q.n_achunks = plan->n_achunks;
  q.n_pd = static_cast<int32_t>(plan->ptiles_delta.size());
  q.n_pg = static_cast<int32_t>(plan->ptiles_gauss.size());
  q.n_layers = plan->n_layers;
  q.beam_pair = plan->beam_pair ? 1 : 0;
  q.t = 1.0;
  q.lam = t.params.lambda;
  q.L_safety = t.params.L_safety > 0.0 ? t.params.L_safety : 1.01;
  q.L = power ? 0.0 : t.params.L;
  q.inv_L = power ? 0.0 : 1.0 / t.params.L;
  q.thr = power ? 0.0 : t.params.lambda / t.params.L;
  q.xscale = xscale;
  auto variant = [&](int per_lane) { return plan->beam_pair ? 3 : (per_lane == 4 ? 2 : per_lane == 2 ? 1 : 0); };
  const int gvar = gkind >= 3 ? kSquareVariant : kGridVariant;
  t.fwd_variant = static_cast<int8_t>(gkind ? gvar : variant(q.vpl));
  t.adj_variant = static_cast<int8_t>(gkind ? gvar : variant(q.ppl));
  t.grid_kind = static_cast<int8_t>(gkind == 3 ? 1 : gkind == 4 ? 2 : gkind);
  t.lane = static_cast<int8_t>(t.grid_kind == 2 || (gkind == 0 && !plan->ptiles_gauss.empty()) ? 1 : 0);
  SRV_HIP(hipMemcpyAsync(s->d_reqs + t.req.slot, &q, sizeof(ReqDev), hipMemcpyHostToDevice, st),
          "upload request descriptor");
  SRV_HIP(hipStreamSynchronize(st), "admission sync");
  // work-item counts
  sched::Shape& sh = t.req.shape;
  if (gkind >= 3) {
    // square grid: pair items only, under the Gaussian kinds for a delta grid
    // and under the delta kinds for a Gaussian grid (routed to the square
    // variant's kernels)
    const GridSeg& g = plan->grid_segs[0];
    const int64_t nf = static_cast<int64_t>(g.nfc) * q.g_vtiles;
    const int64_t na = static_cast<int64_t>(g.pblocks) * q.n_achunks;
    sh.fwd_delta = gkind == 4 ? nf : 0;
    sh.fwd_gauss = gkind == 3 ? nf : 0;
    sh.adj_delta = gkind == 4 ? na : 0;
    sh.adj_gauss = gkind == 3 ? na : 0;
    sh.prep_blocks = (std::max(g.cells, g.n_pairs) + kBlock - 1) / kBlock;
  } else if (gkind) {
    // one grid segment: all items are of its kind
    const GridSeg& g = plan->grid_segs[0];
    const int64_t nf = static_cast<int64_t>(g.nfc) * q.g_vtiles;
    const int64_t na = static_cast<int64_t>(g.ablocks) * q.n_achunks;
    sh.fwd_delta = gkind == 1 ? nf : 0;
    sh.fwd_gauss = gkind == 2 ? nf : 0;
    sh.adj_delta = gkind == 1 ? na : 0;
    sh.adj_gauss = gkind == 2 ? na : 0;
    sh.prep_blocks = (g.cells + kBlock - 1) / kBlock;
  } else {
    sh.fwd_delta = q.vtiles * q.n_fd;
    sh.fwd_gauss = q.vtiles * (q.n_fchunks - q.n_fd);
    const int64_t n_pt = static_cast<int64_t>(plan->ptiles_delta.size() + plan->ptiles_gauss.size());
    sh.adj_delta = static_cast<int64_t>(q.n_pd) * q.n_achunks;
    sh.adj_gauss = (n_pt - q.n_pd) * q.n_achunks;
    sh.prep_blocks = 0;
  }
  sh.vis_blocks = q.vis_blocks;
  sh.pix_blocks = q.pix_blocks;
  sh.evals_per_op = static_cast<double>(pr.n_pix) * static_cast<double>(pr.n_vis);
  sh.power_iters = power ? (t.params.power_iters > 0 ? t.params.power_iters : 30) : 0;
  sh.max_iter = t.params.max_iter;
  sched::start_request(t.req);
  return SL1M_OK;
}

// The admission thread: builds the plan, start vector and device descriptor
// of each reserved request (admit()) on the admission stream, in submission
// order, without the server lock, so the step loop keeps launching rounds
// meanwhile.  It touches only the ticket's own fields, the request's arena
// range and its reserved slot of the descriptor table, none of which a round
// in flight reads.
void admission_thread(sl1m_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Ticket* t = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->wq_mu);
      s->wq_cv.wait(lk, [&] { return s->wq_stop || !s->wq.empty(); });
      if (s->wq_stop) return;
      t = s->wq.front();
      s->wq.pop_front();
    }
    sl1m_status st;
    try {
      const TraceRange range("sl1m server admission build");
      st = admit(s, *t);
    } catch (...) {
      st = set_error(SL1M_ENOMEM, "host allocation failed");
    }
    t->build_status = st;
    t->built.store(1, std::memory_order_release);
  }
}

// Returns a reserved request's plan, arena range and slot.
void release_reserved(sl1m_server* s, Ticket& t) {
  if (t.plan) sl1m_plan_destroy(t.plan);
  t.plan = nullptr;
  s->alloc.release(t.arena_off);
  s->free_slots.push_back(t.req.slot);
  t.freed = true;
}

// Moves built requests into the rounds, in submission order (the admission
// thread builds in that order, so the first unbuilt one ends the pass).
void integrate_admitted(sl1m_server* s) {
  while (!s->admitting.empty()) {
    Ticket& t = *s->tickets[s->admitting.front()];
    if (!t.built.load(std::memory_order_acquire)) break;
    s->admitting.pop_front();
    if (t.state == Ticket::CANCELLED) {
      release_reserved(s, t);
    } else if (t.build_status != SL1M_OK) {
      release_reserved(s, t);
      t.state = Ticket::DONE;
      t.info.status = t.build_status;
    } else {
      const int slot = t.req.slot;
      s->fwd_variant[slot] = t.fwd_variant;
      s->adj_variant[slot] = t.adj_variant;
      s->grid_kind[slot] = t.grid_kind;
      s->lane[slot] = t.lane;
      t.admit_s = now_s(s);
      t.state = Ticket::ACTIVE;
      s->active.push_back(t.req.ticket);
    }
  }
}

sl1m_status launch_round(sl1m_server* s) {
  std::vector<sched::Request*> act;
  for (uint64_t id : s->active) {
    Ticket& t = *s->tickets[id];
    if (t.state == Ticket::ACTIVE) act.push_back(&t.req);
  }
  if (act.empty()) return SL1M_OK;
  const int ring = static_cast<int>(s->round % kSrvRing);
  if (s->ring_round[ring] >= 0) {  // the buffers are still in use by an older round
    SRV_HIP(hipEventSynchronize(s->ring_event[ring]), "round sync");
    SRV_HIP(hipEventSynchronize(s->lane_event[ring]), "round sync");
    s->completed_round = std::max(s->completed_round, s->ring_round[ring]);
    s->ring_round[ring] = -1;
  }
  // each request's share of the round.  FAIR: equal shares with a floor so
  // that a crowded round still moves every request by a useful amount.
  // OLDEST_FIRST: the earliest admitted request takes the whole round (act
  // is in admission order); the small requests (at most 128 budgets of work
  // in total) share a quarter of it between them, so that however many of
  // them run alongside, the oldest keeps at least four fifths of each round;
  // the other large ones get a floor of 1/1024 of the round (close to
  // first-come-first-served among the large ones).
  // OLDEST_FIRST rounds hold at least one FISTA iteration (two operator
  // applications) of the oldest request, between the budget and kSrvMaxRound
  // times it: a large request then runs in rounds of enough blocks to fill
  // the GPU past the launch tails, while a queue of small requests keeps
  // short rounds (each round advances a small request by one step).
  double B = s->budget;
  if (s->policy == SL1M_SERVE_OLDEST_FIRST)
    B = std::min(kSrvMaxRound * s->budget, std::max(s->budget, 2.0 * act[0]->shape.evals_per_op));
  const double fair = std::max(B / static_cast<double>(act.size()), B / 32.0);
  auto is_small = [&](const sched::Request* r) {
    const sched::Shape& sh = r->shape;
    return sh.evals_per_op * (2.0 * (sh.power_iters + sh.max_iter) + 1.0) <= 128.0 * s->budget;
  };
  int n_small = 0;
  for (size_t i = 1; i < act.size(); ++i) n_small += is_small(act[i]) ? 1 : 0;
  const double small_share =
      std::max(B / 1024.0, B / 4.0 / static_cast<double>(std::max(n_small, 1)));
  for (size_t i = 0; i < act.size(); ++i) {
    if (s->policy == SL1M_SERVE_OLDEST_FIRST)
      act[i]->share = i == 0 ? B : is_small(act[i]) ? small_share : B / 1024.0;
    else
      act[i]->share = fair;
  }
  sched::RoundPlan rp;
  sched::plan_round(act, fair, s->round, rp);
  // split the planner's segments into per-(lane, kernel, variant) tables
  std::vector<Segment> tabs[kSrvLanes][kTabs];
  auto route = [&](int kind, int base, const int8_t* var) {
    for (const Segment& g : rp.seg[kind]) tabs[s->lane[g.slot]][base + var[g.slot]].push_back(g);
  };
  auto route1 = [&](int kind, int tab) {
    for (const Segment& g : rp.seg[kind]) tabs[s->lane[g.slot]][tab].push_back(g);
  };
  route(sched::K_FWD_DELTA, 0 * kOpVariants, s->fwd_variant);
  route(sched::K_FWD_GAUSS, 1 * kOpVariants, s->fwd_variant);
  route(sched::K_ADJ_DELTA, 2 * kOpVariants, s->adj_variant);
  route(sched::K_ADJ_GAUSS, 3 * kOpVariants, s->adj_variant);
  route1(sched::K_REDUCE, kTabReduce);
  route1(sched::K_UPDATE, kTabUpdate);
  route1(sched::K_FINAL, kTabFinal);
  for (const Segment& g : rp.seg[sched::K_PREP])
    tabs[s->lane[g.slot]][s->grid_kind[g.slot] == 2 ? kTabPrepG : kTabPrepD].push_back(g);
  for (int ln = 0; ln < kSrvLanes; ++ln) {
    TabDev* ht = s->h_tabs + (ring * kSrvLanes + ln) * kTabs;
    int64_t items = 0;
    for (int k = 0; k < kTabs; ++k) {
      TabDev& tb = ht[k];
      tb.n_seg = static_cast<int32_t>(tabs[ln][k].size());
      int64_t pre = 0;
      for (int i = 0; i < tb.n_seg; ++i) {
        const Segment& g = tabs[ln][k][i];
        tb.seg[i] = SegDev{g.slot, g.flags, g.begin, g.end, pre};
        pre += g.end - g.begin;
      }
      tb.total = pre;
      items += pre;
    }
    if (items == 0) continue;
    hipStream_t st = ln == 0 ? s->stream : s->lane_stream;
    TabDev* dt = s->d_tabs + (ring * kSrvLanes + ln) * kTabs;
    SRV_HIP(hipMemcpyAsync(dt, ht, sizeof(TabDev) * kTabs, hipMemcpyHostToDevice, st),
            "upload round tables");
    auto go = [&](int k, auto kernel, auto* reqs) -> hipError_t {
      if (ht[k].total == 0) return hipSuccess;
      const unsigned g = static_cast<unsigned>(ht[k].total);  // one block per item
      hipLaunchKernelGGL(kernel, dim3(g), dim3(kBlock), 0, st, dt + k, reqs);
      return hipGetLastError();
    };
    const ReqDev* cr = s->d_reqs;
    ReqDev* r = s->d_reqs;
    hipError_t e = hipSuccess;
    // kernel order within a lane: prep, forward, reduce, adjoint, update, final
    if (e == hipSuccess) e = go(kTabPrepD, k_srv_gprep<false>, cr);
    if (e == hipSuccess) e = go(kTabPrepG, k_srv_gprep<true>, cr);
    if (e == hipSuccess) e = go(0, k_srv_fwd<false, 1, false>, cr);
    if (e == hipSuccess) e = go(1, k_srv_fwd<false, 2, false>, cr);
    if (e == hipSuccess) e = go(2, k_srv_fwd<false, 4, false>, cr);
    if (e == hipSuccess) e = go(3, k_srv_fwd<false, 4, true>, cr);
    if (e == hipSuccess) e = go(kGridVariant, k_srv_gfwd<false>, cr);
    if (e == hipSuccess) e = go(kSquareVariant, k_srv_ggfwd_pairs, cr);
    if (e == hipSuccess) e = go(kOpVariants + 0, k_srv_fwd<true, 1, false>, cr);
    if (e == hipSuccess) e = go(kOpVariants + 1, k_srv_fwd<true, 2, false>, cr);
    if (e == hipSuccess) e = go(kOpVariants + 2, k_srv_fwd<true, 4, false>, cr);
    if (e == hipSuccess) e = go(kOpVariants + 3, k_srv_fwd<true, 4, true>, cr);
    if (e == hipSuccess) e = go(kOpVariants + kGridVariant, k_srv_gfwd<true>, cr);
    if (e == hipSuccess) e = go(kOpVariants + kSquareVariant, k_srv_gfwd_pairs, cr);
    if (e == hipSuccess) e = go(kTabReduce, k_srv_reduce, r);
    if (e == hipSuccess) e = go(2 * kOpVariants + 0, k_srv_adj<false, 1, false>, cr);
    if (e == hipSuccess) e = go(2 * kOpVariants + 1, k_srv_adj<false, 2, false>, cr);
    if (e == hipSuccess) e = go(2 * kOpVariants + 2, k_srv_adj<false, 4, false>, cr);
    if (e == hipSuccess) e = go(2 * kOpVariants + 3, k_srv_adj<false, 4, true>, cr);
    if (e == hipSuccess) e = go(2 * kOpVariants + kGridVariant, k_srv_gadj<false>, cr);
    if (e == hipSuccess) e = go(2 * kOpVariants + kSquareVariant, k_srv_ggadj_pairs, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + 0, k_srv_adj<true, 1, false>, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + 1, k_srv_adj<true, 2, false>, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + 2, k_srv_adj<true, 4, false>, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + 3, k_srv_adj<true, 4, true>, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + kGridVariant, k_srv_gadj<true>, cr);
    if (e == hipSuccess) e = go(3 * kOpVariants + kSquareVariant, k_srv_gadj_pairs, cr);
    if (e == hipSuccess) e = go(kTabUpdate, k_srv_update, r);
    if (e == hipSuccess) e = go(kTabFinal, k_srv_final, r);
    if (e != hipSuccess) return hip_error(e, "batched round launch");
  }
  // the lanes do not wait for each other: the round has ended once both of
  // its events have (recorded also on a lane without work in this round, so
  // that they cover that lane's earlier rounds)
  SRV_HIP(hipEventRecord(s->lane_event[ring], s->lane_stream), "record lane event");
  SRV_HIP(hipEventRecord(s->ring_event[ring], s->stream), "record round event");
  s->ring_round[ring] = s->round;
  if (!rp.finishing.empty()) s->finishing.emplace_back(s->round, rp.finishing);
  s->evals_scheduled += rp.evals;  // forward and adjoint item evals
  ++s->round;
  return SL1M_OK;
}

}  // namespace
}  // namespace sl1m

using namespace sl1m;

extern "C" {

sl1m_status sl1m_server_create(void* arena, size_t arena_bytes, int32_t max_slots,
                               double round_budget_evals, sl1m_server** out) {
  try {
    if (!out) return set_error(SL1M_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena || reinterpret_cast<uintptr_t>(arena) % 256 != 0)
      return set_error(SL1M_EINVAL, "arena must be a 256-byte aligned device pointer");
    if (max_slots < 1 || max_slots > kSrvMaxSlots)
      return set_error(SL1M_EINVAL, "max_slots must be in [1, 64]");
    const size_t hdr = sched::Arena::round_up(sizeof(ReqDev) * kSrvMaxSlots) +
                       sched::Arena::round_up(sizeof(TabDev) * kSrvRing * kSrvLanes * kTabs);
    if (arena_bytes < hdr + (1u << 20)) return set_error(SL1M_ENOMEM, "arena too small");
    auto s = std::make_unique<sl1m_server>();
    s->t0 = std::chrono::steady_clock::now();
    s->d_reqs = reinterpret_cast<ReqDev*>(arena);
    s->d_tabs = reinterpret_cast<TabDev*>(static_cast<char*>(arena) +
                                          sched::Arena::round_up(sizeof(ReqDev) * kSrvMaxSlots));
    s->arena = static_cast<char*>(arena) + hdr;
    s->arena_bytes = arena_bytes - hdr;
    s->alloc.reset(s->arena_bytes);
    s->max_slots = max_slots;
    s->budget = round_budget_evals > 0 ? round_budget_evals : 3e10;
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    SRV_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->h_tabs),
                          sizeof(TabDev) * kSrvRing * kSrvLanes * kTabs, hipHostMallocDefault),
            "pinned round tables");
    SRV_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "round stream");
    SRV_HIP(hipStreamCreateWithFlags(&s->lane_stream, hipStreamNonBlocking), "lane stream");
    SRV_HIP(hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking), "admission stream");
    SRV_HIP(hipStreamCreateWithFlags(&s->read_stream, hipStreamNonBlocking), "result stream");
    SRV_HIP(hipGetDevice(&s->device), "current device");
    for (auto& e : s->ring_event) SRV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    for (auto& e : s->lane_event) SRV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    sl1m_server* srv = s.get();
    s->admitter = std::thread(admission_thread, srv);
    *out = s.release();
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  }
}

sl1m_status sl1m_server_submit(sl1m_server* s, const sl1m_problem* problem, const void* vis,
                               const sl1m_solve_params* params, void* img_out,
                               uint64_t* ticket) {
  try {
    if (!s || !problem || !params || !ticket) return set_error(SL1M_EINVAL, "NULL argument");
    if (problem->precision != SL1M_PREC_FP32)
      return set_error(SL1M_EINVAL, "the server runs FP32 plans only");
    if (params->method != SL1M_FISTA)
      return set_error(SL1M_EINVAL, "the server runs FISTA only");
    if (problem->max_rhs > 1) return set_error(SL1M_EINVAL, "the server solves one image each");
    if ((problem->n_vis > 0 && !vis) || (problem->n_pix > 0 && !img_out))
      return set_error(SL1M_EINVAL, "vis or img_out is NULL");
    if (!(params->lambda >= 0.0) || params->max_iter < 0)
      return set_error(SL1M_EINVAL, "lambda must be >= 0 and max_iter >= 0");
    auto t = std::make_unique<Ticket>();
    t->problem = *problem;
    t->problem.tile_blocks = problem->tile_blocks > 0 ? problem->tile_blocks : kSrvTileBlocks;
    // the batched kernels take the grid evaluation for a request whose pixels
    // form one qualifying grid segment and the direct one otherwise; the
    // footprint covers either plan (decided at admission)
    size_t ws = 0, ws_off = 0;
    if (problem->grid_mode != SL1M_GRID_OFF) {
      if (sl1m_status st = sl1m_plan_workspace_bytes(&t->problem, &ws)) return st;
    }
    t->problem.grid_mode = SL1M_GRID_OFF;
    if (sl1m_status st = sl1m_plan_workspace_bytes(&t->problem, &ws_off)) return st;
    t->grid_allowed = problem->grid_mode != SL1M_GRID_OFF;
    t->footprint = sched::Arena::round_up(std::max(ws, ws_off)) + extra_bytes(t->problem);
    t->vis = vis;
    t->img_out = img_out;
    t->params = *params;
    std::lock_guard<std::mutex> lk(s->mu);
    if (t->footprint > s->alloc.size())
      return set_error(SL1M_ENOMEM, "request footprint exceeds the server arena");
    t->submit_s = now_s(s);
    const uint64_t id = s->next_ticket++;
    t->req.ticket = id;
    s->tickets[id] = std::move(t);
    s->pending.push_back(id);
    *ticket = id;
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  }
}

sl1m_status sl1m_server_set_policy(sl1m_server* s, int32_t policy) {
  if (!s) return set_error(SL1M_EINVAL, "server is NULL");
  if (policy != SL1M_SERVE_FAIR && policy != SL1M_SERVE_OLDEST_FIRST)
    return set_error(SL1M_EINVAL, "unknown serving policy");
  std::lock_guard<std::mutex> lk(s->mu);
  s->policy = policy;
  return SL1M_OK;
}

sl1m_status sl1m_server_step(sl1m_server* s, int32_t* n_active, int32_t* n_pending) {
  const TraceRange range("sl1m_server_step");
  try {
    if (!s) return set_error(SL1M_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    harvest(s);
    integrate_admitted(s);
    // reserve memory and a slot for pending requests (in submission order)
    // while both allow, and hand them to the admission thread
    for (auto it = s->pending.begin(); it != s->pending.end() && !s->free_slots.empty();) {
      Ticket& t = *s->tickets[*it];
      size_t off = 0;
      if (!s->alloc.alloc(t.footprint, &off)) {
        ++it;
        continue;
      }
      t.arena_off = off;
      t.req.slot = s->free_slots.back();
      s->free_slots.pop_back();
      t.freed = false;
      t.state = Ticket::ADMITTING;
      s->admitting.push_back(t.req.ticket);
      {
        std::lock_guard<std::mutex> wl(s->wq_mu);
        s->wq.push_back(&t);
      }
      s->wq_cv.notify_one();
      it = s->pending.erase(it);
    }
    sl1m_status st = launch_round(s);
    if (n_active) {
      int32_t a = 0;
      for (uint64_t id : s->active)
        if (s->tickets[id]->state == Ticket::ACTIVE) ++a;
      *n_active = a;
    }
    if (n_pending) *n_pending = static_cast<int32_t>(s->pending.size() + s->admitting.size());
    return st;
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

sl1m_status sl1m_server_poll(sl1m_server* s, uint64_t ticket, sl1m_solve_info* info,
                             int32_t* done, double* times) {
  if (!s || !done) return set_error(SL1M_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return set_error(SL1M_EINVAL, "unknown ticket");
  // rounds already launched may still read a cancelled request's data and
  // write its image, and the admission thread may still be building it: it is
  // done only once all of them have ended and its memory has been released
  // (harvest, integrate_admitted), so the caller may then free vis and img_out
  harvest(s);
  integrate_admitted(s);
  Ticket& t = *it->second;
  *done = t.state == Ticket::DONE || (t.state == Ticket::CANCELLED && t.freed);
  if (info) *info = t.info;
  if (t.state == Ticket::CANCELLED && info) info->status = SL1M_ECANCELLED;
  if (times) {
    times[0] = t.submit_s;
    times[1] = t.admit_s;
    times[2] = t.finish_s;
  }
  return SL1M_OK;
}

sl1m_status sl1m_server_cancel(sl1m_server* s, uint64_t ticket) {
  if (!s) return set_error(SL1M_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return set_error(SL1M_EINVAL, "unknown ticket");
  Ticket& t = *it->second;
  if (t.state == Ticket::PENDING) {
    for (auto p = s->pending.begin(); p != s->pending.end(); ++p)
      if (*p == ticket) {
        s->pending.erase(p);
        break;
      }
    t.state = Ticket::CANCELLED;
  } else if (t.state == Ticket::ADMITTING) {
    t.state = Ticket::CANCELLED;  // released once its build has ended (integrate_admitted)
  } else if (t.state == Ticket::ACTIVE) {
    t.req.cancelled = true;
    t.state = Ticket::CANCELLED;
  }
  return SL1M_OK;
}

sl1m_status sl1m_server_stats(sl1m_server* s, sl1m_server_stats_t* out) {
  if (!s || !out) return set_error(SL1M_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->rounds = s->round;
  out->completed_rounds = s->completed_round + 1;
  out->evals_scheduled = s->evals_scheduled;
  out->arena_bytes = s->alloc.size();
  out->arena_used = s->alloc.used_bytes();
  int32_t a = 0;
  for (uint64_t id : s->active)
    if (s->tickets[id]->state == Ticket::ACTIVE) ++a;
  out->active = a;
  out->pending = static_cast<int32_t>(s->pending.size() + s->admitting.size());
  return SL1M_OK;
}

sl1m_status sl1m_server_destroy(sl1m_server* s) {
  if (!s) return SL1M_OK;
  if (s->admitter.joinable()) {  // ends after the build in progress, if any
    {
      std::lock_guard<std::mutex> wl(s->wq_mu);
      s->wq_stop = true;
    }
    s->wq_cv.notify_all();
    s->admitter.join();
  }
  (void)hipStreamSynchronize(s->stream);
  if (s->lane_stream) (void)hipStreamSynchronize(s->lane_stream);
  (void)hipStreamSynchronize(s->admit_stream);
  if (s->read_stream) (void)hipStreamSynchronize(s->read_stream);
  for (auto& kv : s->tickets)
    if (kv.second->plan) sl1m_plan_destroy(kv.second->plan);
  for (auto& e : s->ring_event)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : s->lane_event)
    if (e) (void)hipEventDestroy(e);
  if (s->lane_stream) (void)hipStreamDestroy(s->lane_stream);
  if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
  if (s->read_stream) (void)hipStreamDestroy(s->read_stream);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->h_tabs) (void)hipHostFree(s->h_tabs);
  delete s;
  return SL1M_OK;
}

}  // extern "C"
