// Grid evaluation of the operators (gfx950, float32 plans): kernels and
// launchers.  The factorisation and the tiles are in sl1m_grid.h.  Every
// segment on the grid path gets a prep launch and its forward and adjoint
// launches (two each for a square delta grid: single cells and pairs); a plan
// has at most 17 segments, the delta pixels and 16 Gaussian layers.
#include "sl1m_grid.h"

namespace sl1m {

namespace {

using namespace dev;

// Per-call forward records of a delta segment: amplitudes a_j = x_j * scale_j
// gathered into the cells' sign slots and combined into e1..e4.
__global__ void k_grid_prep_delta(const float* __restrict__ xp, const float* __restrict__ pscale,
                                  const int32_t* __restrict__ slot, const double* __restrict__ nu,
                                  int64_t cells, GridRec* __restrict__ rec) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= cells) return;
  float x[4];
  int32_t empty = 1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t j = slot[4 * q + s];
    x[s] = j >= 0 ? xp[j] * pscale[j] : 0.0f;
    if (j >= 0) empty = 0;
  }
  GridRec r;
  r.nu = nu[q];
  r.e1 = (x[0] + x[1]) + (x[2] + x[3]);
  r.e2 = (x[1] + x[2]) - (x[0] + x[3]);
  r.e3 = (x[0] + x[1]) - (x[2] + x[3]);
  r.e4 = (x[0] - x[1]) + (x[2] - x[3]);
  r.empty = empty;
  r.pad = 0;
  rec[q] = r;
}

// Per-call pair records of a square delta segment.
__global__ void k_grid_prep_pairs(const float* __restrict__ xp, const float* __restrict__ pscale,
                                  const int32_t* __restrict__ slot, const double* __restrict__ nu,
                                  int na, int64_t n_pairs, GridPairRec* __restrict__ rec) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  grid_write_pair_rec(p, na, slot, nu, xp, pscale, 1.0f, rec);
}

__global__ void k_grid_prep_pairs_gauss(const float* __restrict__ xp,
                                        const float* __restrict__ pscale,
                                        const int32_t* __restrict__ slot,
                                        const double* __restrict__ r2,
                                        const double* __restrict__ kap, int na, int64_t n_pairs,
                                        GridPairRecG* __restrict__ rec) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  grid_write_pair_rec_gauss(p, na, slot, r2, kap, xp, pscale, 1.0f, rec);
}

// Per-call forward records of a Gaussian segment.
__global__ void k_grid_prep_gauss(const float* __restrict__ xp, const float* __restrict__ pscale,
                                  const int32_t* __restrict__ slot, const double* __restrict__ r2,
                                  const double* __restrict__ kap, int64_t cells,
                                  GridRecG* __restrict__ rec) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= cells) return;
  GridRecG r;
  r.r2 = r2[q];
  r.kappa = kap[q];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t j = slot[4 * q + s];
    r.x[s] = j >= 0 ? xp[j] * pscale[j] : 0.0f;
  }
  rec[q] = r;
}

// Forward: block (vtile, chunk of the segment); partial row = blockIdx.y.
__global__ __launch_bounds__(kBlock) void k_grid_fwd_delta(
    const GridRec* __restrict__ rec, const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    float2* __restrict__ part) {
  const ConstPtr<GridChunk> cc = as_const(chunks) + blockIdx.y;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_delta_tile(rec, la, mb, ch, na, vu, vv, vw, blockIdx.x, n_vis,
                      part + static_cast<int64_t>(blockIdx.y) * n_vis);
}

__global__ __launch_bounds__(kBlock) void k_grid_fwd_delta_pairs(
    const GridPairRec* __restrict__ rec, const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    float2* __restrict__ part) {
  const ConstPtr<GridChunk> cc = as_const(chunks) + blockIdx.y;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_delta_pairs_tile(rec, la, mb, ch, na, vu, vv, vw, blockIdx.x, n_vis,
                            part + static_cast<int64_t>(blockIdx.y) * n_vis);
}

__global__ __launch_bounds__(kBlock) void k_grid_fwd_gauss(
    const GridRecG* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk* __restrict__ chunks, int na,
    const VisRecG<float>* __restrict__ vrec, const float* __restrict__ Ds, int64_t n_vis,
    float2* __restrict__ part) {
  const ConstPtr<GridChunk> cc = as_const(chunks) + blockIdx.y;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_gauss_tile(rec, la, mb, ch, na, vrec, Ds, blockIdx.x, n_vis,
                      part + static_cast<int64_t>(blockIdx.y) * n_vis);
}

__global__ __launch_bounds__(kBlock) void k_grid_fwd_gauss_pairs(
    const GridPairRecG* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk* __restrict__ chunks, int na,
    const VisRecG<float>* __restrict__ vrec, const float* __restrict__ Ds, int64_t n_vis,
    float2* __restrict__ part) {
  const ConstPtr<GridChunk> cc = as_const(chunks) + blockIdx.y;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_gauss_pairs_tile(rec, la, mb, ch, na, vrec, Ds, blockIdx.x, n_vis,
                            part + static_cast<int64_t>(blockIdx.y) * n_vis);
}

// Adjoint: block (lane-set block, visibility chunk); partial row = blockIdx.y.
constexpr size_t kGridLds = sizeof(float2) * kGridKB * kGridMaxGL * kGridNBA;
static_assert(kGridLds == sizeof(float4) * kGridKBG * kGridMaxGL * kGridNBA,
              "delta and Gaussian LDS batches have one size");

__global__ __launch_bounds__(kBlock) void k_grid_adj_delta(
    const VisRecD<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ vv, const double* __restrict__ la, const double* __restrict__ mb,
    const double* __restrict__ nu, const int32_t* __restrict__ slot, int na, int ng4,
    int64_t kchunk, int64_t n_vis, float* __restrict__ part, int64_t n_pix) {
  __shared__ float2 bsh[kGridKB][kGridMaxGL][kGridNBA];
  grid_adj_delta_tile(vrec, rres, vv, la, mb, nu, slot, na, ng4, blockIdx.x, blockIdx.y, kchunk,
                      n_vis, part + static_cast<int64_t>(blockIdx.y) * n_pix, bsh);
}

// Square delta grid adjoint: one pair block per block x (GridPairBlock).
__global__ __launch_bounds__(kBlock) void k_grid_adj_delta_square(
    const VisRecD<float>* __restrict__ vrec, const ResPolar* __restrict__ rpol,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ nu,
    const int32_t* __restrict__ slot, int na, const GridPairBlock* __restrict__ blocks,
    int64_t kchunk, int64_t n_vis, float* __restrict__ part, int64_t n_pix) {
  __shared__ float4 bsh[kGridKBG][kGridMaxGL][kGridNBA];
  const ConstPtr<GridPairBlock> cb = as_const(blocks) + blockIdx.x;
  GridPairBlock pb;
  pb.g4 = cb->g4;
  pb.ia = cb->ia;
  pb.count = cb->count;
  pb.n_gl = cb->n_gl;
  grid_adj_delta_pairs_tile(vrec, rpol, vu, vv, la, mb, nu, slot, na, pb, blockIdx.y, kchunk,
                            n_vis, part + static_cast<int64_t>(blockIdx.y) * n_pix, bsh);
}

// Square delta grid, NR right-hand sides sharing the phasors (residual
// records [n_vis][NR] of the delta slot); blockIdx.z picks the NBI cells of
// each lane-set, side r of chunk y goes to part + r rstride + y n_pix.
template <int NR, int NBI>
__global__ __launch_bounds__(kBlock) void k_grid_adj_delta_square_multi(
    const VisRecD<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ nu,
    const int32_t* __restrict__ slot, int na, const GridPairBlock* __restrict__ blocks,
    int64_t kchunk, int64_t n_vis, float* __restrict__ part, int64_t n_pix, int64_t rstride) {
  __shared__ float4 bsh[kGridKBM][kGridMaxGL][NBI];
  const ConstPtr<GridPairBlock> cb = as_const(blocks) + blockIdx.x;
  GridPairBlock pb;
  pb.g4 = cb->g4;
  pb.ia = cb->ia;
  pb.count = cb->count;
  pb.n_gl = cb->n_gl;
  grid_adj_delta_pairs_multi_tile<NR, NBI>(
      vrec, rres, vu, vv, la, mb, nu, slot, na, pb, static_cast<int>(blockIdx.z) * NBI,
      blockIdx.y, kchunk, n_vis, part + static_cast<int64_t>(blockIdx.y) * n_pix, rstride, bsh);
}

// All Gaussian grid segments in one launch: block x of the (block, chunk)
// grid maps to (segment, block within the segment) through `gblocks`, so a
// plan with several small layers still fills the GPU with one launch.  For a
// square segment the block is a pair block (index into `pblocks` from the
// segment's pb0).
__global__ __launch_bounds__(kBlock) void k_grid_adj_gauss_multi(
    const int2* __restrict__ gblocks, const GridSeg* __restrict__ segs,
    const GridPairBlock* __restrict__ pblocks, const VisRecG<float>* __restrict__ vrec,
    const float2* __restrict__ rres, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ c3, const double* __restrict__ c4,
    const int32_t* __restrict__ slot, int64_t kchunk, int64_t n_vis, float* __restrict__ part,
    int64_t n_pix) {
  __shared__ float4 bsh[kGridKBG][kGridMaxGL][kGridNBA][2];
  const ConstPtr<int2> cgb = as_const(gblocks) + blockIdx.x;
  const int si = cgb->x, blk = cgb->y;
  const ConstPtr<GridSeg> cs = as_const(segs) + si;
  const int64_t co = cs->cell_off, layer = cs->layer;
  float* row = part + static_cast<int64_t>(blockIdx.y) * n_pix;
  if (cs->square) {
    const ConstPtr<GridPairBlock> cb = as_const(pblocks) + cs->pb0 + blk;
    GridPairBlock pb;
    pb.g4 = cb->g4;
    pb.ia = cb->ia;
    pb.count = cb->count;
    pb.n_gl = cb->n_gl;
    grid_adj_gauss_pairs_tile(vrec + layer * n_vis, rres + (1 + layer) * n_vis, la + cs->la_off,
                              mb + cs->mb_off, c3 + co, c4 + co, slot + 4 * co, cs->na, pb,
                              blockIdx.y, kchunk, n_vis, row, bsh);
  } else {
    grid_adj_gauss_tile(vrec + layer * n_vis, rres + (1 + layer) * n_vis, la + cs->la_off,
                        mb + cs->mb_off, c3 + co, c4 + co, slot + 4 * co, cs->na, 2 * cs->ng, blk,
                        blockIdx.y, kchunk, n_vis, row,
                        reinterpret_cast<float4(*)[kGridMaxGL][kGridNBA]>(&bsh[0][0][0][0]));
  }
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Multi-RHS pair records of a square delta segment (xp: [r][n_pix]).
template <int NR>
__global__ void k_grid_prep_pairs_multi(const float* __restrict__ xp, int64_t n_pix,
                                        const float* __restrict__ pscale,
                                        const int32_t* __restrict__ slot,
                                        const double* __restrict__ nu, int na, int64_t n_pairs,
                                        float* __restrict__ rec) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  grid_write_pair_rec_multi<NR>(p, na, slot, nu, xp, n_pix, pscale, rec);
}

// Multi-RHS forward: block (visibility tile of kBlock, pair chunk); partial
// row blockIdx.y of right-hand side r at rows + r rhs_stride.
template <int NR>
__global__ __launch_bounds__(kBlock) void k_grid_fwd_delta_pairs_multi(
    const float* __restrict__ rec, const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    float2* __restrict__ rows, int64_t rhs_stride) {
  const ConstPtr<GridChunk> cc = as_const(chunks) + blockIdx.y;
  GridChunk ch;
  ch.g = cc->g;
  ch.ia0 = cc->ia0;
  ch.ia1 = cc->ia1;
  grid_fwd_delta_pairs_multi_tile<NR>(rec, la, mb, ch, na, vu, vv, vw, blockIdx.x, n_vis,
                                      rows + static_cast<int64_t>(blockIdx.y) * n_vis,
                                      rhs_stride);
}

}  // namespace

hipError_t launch_grid_forward(sl1m_plan* p, const void* xp, hipStream_t st) {
  if (p->n_vis == 0) return hipSuccess;
  const float* x = static_cast<const float*>(xp);
  const float* scale = static_cast<const float*>(p->pscale);
  float2* part = static_cast<float2*>(p->fpart);
  for (const GridSeg& g : p->grid_segs) {
    const int64_t co = g.cell_off;
    const double* la = p->grid_la + g.la_off;
    const double* mb = p->grid_mb + g.mb_off;
    const int32_t* slot = p->grid_slot + 4 * co;
    const GridChunk* ch = p->d_grid_fchunks + g.fc0;
    float2* rows = part + static_cast<int64_t>(g.fc0) * p->n_vis;
    const dim3 grid(static_cast<unsigned>(p->grid_vtiles), static_cast<unsigned>(g.nfc));
    if (g.kind == SL1M_PIX_DELTA) {
      GridRec* rec = static_cast<GridRec*>(p->grid_rec) + co;
      if (g.nfs > 0)  // cell records (a square grid's forward reads pair records only)
        hipLaunchKernelGGL(k_grid_prep_delta, dim3(blocks_for(g.cells)), dim3(kBlock), 0, st, x,
                           scale, slot, p->grid_c3 + co, g.cells, rec);
      // single-cell chunks, then (square grids) pair chunks
      const unsigned vt = static_cast<unsigned>(p->grid_vtiles);
      if (g.nfs > 0) {
        hipError_t e = timed(p, T_GRID_FWD_DELTA, st, [&] {
          hipLaunchKernelGGL(k_grid_fwd_delta, dim3(vt, static_cast<unsigned>(g.nfs)),
                             dim3(kBlock), 0, st, rec, la, mb, ch, g.na, p->vu, p->vv, p->vw,
                             p->n_vis, rows);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
      }
      if (g.nfc > g.nfs) {
        GridPairRec* prec = p->grid_prec + g.pr_off;
        hipLaunchKernelGGL(k_grid_prep_pairs, dim3(blocks_for(g.n_pairs)), dim3(kBlock), 0, st, x,
                           scale, slot, p->grid_c3 + co, g.na, g.n_pairs, prec);
        hipError_t e = timed(p, T_GRID_FWD_DELTA, st, [&] {
          hipLaunchKernelGGL(k_grid_fwd_delta_pairs,
                             dim3(vt, static_cast<unsigned>(g.nfc - g.nfs)), dim3(kBlock), 0, st,
                             prec, la, mb, ch + g.nfs, g.na, p->vu, p->vv, p->vw, p->n_vis,
                             rows + static_cast<int64_t>(g.nfs) * p->n_vis);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
      }
    } else {
      const VisRecG<float>* vrec =
          static_cast<const VisRecG<float>*>(p->visrecG) + static_cast<int64_t>(g.layer) * p->n_vis;
      const float* Ds = static_cast<const float*>(p->layerDs) + static_cast<int64_t>(g.layer) * 2 * p->n_vis;
      if (g.square) {
        // mirrored pairs, one visibility per lane
        GridPairRecG* prec = reinterpret_cast<GridPairRecG*>(p->grid_prec + g.pr_off);
        hipLaunchKernelGGL(k_grid_prep_pairs_gauss, dim3(blocks_for(g.n_pairs)), dim3(kBlock), 0,
                           st, x, scale, slot, p->grid_c3 + co, p->grid_c4 + co, g.na, g.n_pairs,
                           prec);
        hipError_t e = timed(p, T_GRID_FWD_GAUSS, st, [&] {
          hipLaunchKernelGGL(k_grid_fwd_gauss_pairs,
                             dim3(static_cast<unsigned>(blocks_for(p->n_vis)),
                                  static_cast<unsigned>(g.nfc)),
                             dim3(kBlock), 0, st, prec, la, mb, ch, g.na, vrec, Ds, p->n_vis, rows);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
      } else {
        GridRecG* rec = static_cast<GridRecG*>(p->grid_rec) + co;
        hipLaunchKernelGGL(k_grid_prep_gauss, dim3(blocks_for(g.cells)), dim3(kBlock), 0, st, x,
                           scale, slot, p->grid_c3 + co, p->grid_c4 + co, g.cells, rec);
        hipError_t e = timed(p, T_GRID_FWD_GAUSS, st, [&] {
          hipLaunchKernelGGL(k_grid_fwd_gauss, grid, dim3(kBlock), 0, st, rec, la, mb, ch, g.na,
                             vrec, Ds, p->n_vis, rows);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipGetLastError();
}

hipError_t launch_grid_adjoint(sl1m_plan* p, hipStream_t st) {
  if (p->n_achunks == 0) return hipSuccess;
  float* part = static_cast<float*>(p->apart);
  const float2* rres = static_cast<const float2*>(p->rres);
  for (const GridSeg& g : p->grid_segs) {
    const int64_t co = g.cell_off;
    const double* la = p->grid_la + g.la_off;
    const double* mb = p->grid_mb + g.mb_off;
    const int32_t* slot = p->grid_slot + 4 * co;
    const dim3 grid(static_cast<unsigned>(g.ablocks), static_cast<unsigned>(p->n_achunks));
    if (g.kind == SL1M_PIX_DELTA && g.square) {
      if (g.pblocks > 0) {
        hipError_t e = timed(p, T_GRID_ADJ_DELTA, st, [&] {
          hipLaunchKernelGGL(k_grid_adj_delta_square,
                             dim3(static_cast<unsigned>(g.pblocks),
                                  static_cast<unsigned>(p->n_achunks)),
                             dim3(kBlock), 0, st, static_cast<const VisRecD<float>*>(p->visrecD),
                             p->rpol, p->vu, p->vv, la, mb, p->grid_c3 + co, slot, g.na,
                             p->d_grid_pblocks + g.pb0, p->adj_kchunk, p->n_vis, part, p->n_pix);
          return hipGetLastError();
        });
        if (e != hipSuccess) return e;
      }
    } else if (g.kind == SL1M_PIX_DELTA) {
      hipError_t e = timed(p, T_GRID_ADJ_DELTA, st, [&] {
        hipLaunchKernelGGL(k_grid_adj_delta, grid, dim3(kBlock), 0, st,
                           static_cast<const VisRecD<float>*>(p->visrecD), rres, p->vv, la, mb,
                           p->grid_c3 + co, slot, g.na, 2 * g.ng, p->adj_kchunk, p->n_vis, part,
                           p->n_pix);
        return hipGetLastError();
      });
      if (e != hipSuccess) return e;
    }
  }
  // every Gaussian grid segment in one launch (residual records of layer L,
  // single right-hand side: slot 1 + L)
  if (p->grid_gblocks > 0) {
    hipError_t e = timed(p, T_GRID_ADJ_GAUSS, st, [&] {
      hipLaunchKernelGGL(k_grid_adj_gauss_multi,
                         dim3(static_cast<unsigned>(p->grid_gblocks),
                              static_cast<unsigned>(p->n_achunks)),
                         dim3(kBlock), 0, st, p->d_grid_gblocks, p->d_grid_segs,
                         p->d_grid_pblocks, static_cast<const VisRecG<float>*>(p->visrecG), rres,
                         p->grid_la, p->grid_mb, p->grid_c3, p->grid_c4, p->grid_slot,
                         p->adj_kchunk, p->n_vis, part, p->n_pix);
      return hipGetLastError();
    });
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

bool grid_multi_ok(const sl1m_plan* p, int nr) {
  return p->grid && p->grid_multi > 0 && (nr == 2 || nr == 4 || nr == 8) && nr <= p->grid_multi;
}

template <int NR>
static hipError_t grid_forward_multi_t(sl1m_plan* p, const float* x, hipStream_t st) {
  const float* scale = static_cast<const float*>(p->pscale);
  float2* part = static_cast<float2*>(p->fpart);
  const int64_t rhs_stride = static_cast<int64_t>(forward_rows(p, NR)) * p->n_vis;
  const unsigned vt = static_cast<unsigned>(blocks_for(p->n_vis));
  for (const GridSeg& g : p->grid_segs) {
    const int64_t co = g.cell_off;
    float* rec = p->grid_precm + static_cast<int64_t>(pair_rec_floats<NR>()) * g.pr_off;
    hipLaunchKernelGGL(k_grid_prep_pairs_multi<NR>, dim3(blocks_for(g.n_pairs)), dim3(kBlock), 0,
                       st, x, p->n_pix, scale, p->grid_slot + 4 * co, p->grid_c3 + co, g.na,
                       g.n_pairs, rec);
    hipLaunchKernelGGL(k_grid_fwd_delta_pairs_multi<NR>, dim3(vt, static_cast<unsigned>(g.nfc)),
                       dim3(kBlock), 0, st, rec, p->grid_la + g.la_off, p->grid_mb + g.mb_off,
                       p->d_grid_fchunks + g.fc0, g.na, p->vu, p->vv, p->vw, p->n_vis,
                       part + static_cast<int64_t>(g.fc0) * p->n_vis, rhs_stride);
  }
  return hipGetLastError();
}

hipError_t launch_grid_forward_multi(sl1m_plan* p, const void* xp, int nr, hipStream_t st) {
  if (p->n_vis == 0) return hipSuccess;
  if (!grid_multi_ok(p, nr)) return hipErrorInvalidValue;
  const float* x = static_cast<const float*>(xp);
  if (nr == 2) return grid_forward_multi_t<2>(p, x, st);
  return nr == 4 ? grid_forward_multi_t<4>(p, x, st) : grid_forward_multi_t<8>(p, x, st);
}

template <int NR, int NBI>
static hipError_t grid_adjoint_multi_t(sl1m_plan* p, hipStream_t st) {
  const int64_t rstride = static_cast<int64_t>(p->n_achunks) * p->n_pix;
  for (const GridSeg& g : p->grid_segs) {
    if (g.pblocks == 0) continue;
    const int64_t co = g.cell_off;
    hipLaunchKernelGGL((k_grid_adj_delta_square_multi<NR, NBI>),
                       dim3(static_cast<unsigned>(g.pblocks), static_cast<unsigned>(p->n_achunks),
                            static_cast<unsigned>(kGridNBA / NBI)),
                       dim3(kBlock), 0, st, static_cast<const VisRecD<float>*>(p->visrecD),
                       static_cast<const float2*>(p->rres), p->vu, p->vv, p->grid_la + g.la_off,
                       p->grid_mb + g.mb_off, p->grid_c3 + co, p->grid_slot + 4 * co, g.na,
                       p->d_grid_pblocks + g.pb0, p->adj_kchunk, p->n_vis,
                       static_cast<float*>(p->apart), p->n_pix, rstride);
  }
  return hipGetLastError();
}

hipError_t launch_grid_adjoint_multi(sl1m_plan* p, int nr, hipStream_t st) {
  if (p->n_achunks == 0) return hipSuccess;
  if (!grid_multi_ok(p, nr)) return hipErrorInvalidValue;
  if (nr == 2) return grid_adjoint_multi_t<2, 2>(p, st);
  return nr == 4 ? grid_adjoint_multi_t<4, 2>(p, st) : grid_adjoint_multi_t<8, 1>(p, st);
}

}  // namespace sl1m
