// Grid evaluation of the delta-pixel operators (gfx950, float32 plans).
//
// The element of eq. (deltam) without gains is
//   M_kj = exp(-2 pi i (u_k l_j + v_k m_j + w_k nu_j)),  nu_j = n_j - 1,
// and factorises exactly into A_k(l_j) B_k(m_j) C_k(nu_j) with
//   A = exp(-2 pi i u l), B = exp(-2 pi i v m), C = exp(-2 pi i w nu).
// nu depends on l^2 + m^2 only, so the four positions (+-|l|, +-|m|) of one
// grid cell share C, and a sign flip of l or m conjugates A or B.  Writing
// A = ac - i as, B = bc - i bs, C = cc - i cs (cosines and sines of the phases
// in turns) and x_s for the amplitudes of the cell's sign slots
// (0 = (+,+), 1 = (-,+), 2 = (+,-), 3 = (-,-)):
//
// forward   sum_s x_s M_s = C (ReS - i ImS') with
//           ReS  = ac bc e1 + as bs e2,   ImS' = ac bs e3 + as bc e4,
//           e1 = x0+x1+x2+x3, e2 = x1+x2-x0-x3, e3 = x0+x1-x2-x3, e4 = x0-x1+x2-x3;
// adjoint   Re conj(M_s) r for every slot from z = conj(C) r and the four sums
//           G1 = sum bc ac z1, G2 = sum bs as z1, G3 = sum bs ac z2, G4 = sum bc as z2:
//           g0 = G1-G2-G3-G4, g1 = G1+G2-G3+G4, g2 = G1+G2+G3-G4, g3 = G1-G2+G3+G4.
//
// Per cell and visibility that is one phase FMA (FP64), one sincos and 12
// FP32 operations for four matrix entries, against three phase FMAs, one
// sincos and two FMAs per entry in the direct evaluation; the A and B phasors
// are amortised over a row of cells.  Phases use the same exact reduction as
// the direct kernels (FP64 FMAs from kMagic, low 23 mantissa bits).
#include "sl1m_device.h"

namespace sl1m {

namespace {

using namespace dev;

constexpr int kGridVPL = 2;     // forward visibilities per lane
constexpr int kGridSegIA = 8;   // forward: |l| values per inner FP32 sum (64 cells)

// Per-call forward records: amplitudes a_j = x_j * scale_j gathered into the
// cells' sign slots and combined into e1..e4.
__global__ void k_grid_prep(const float* __restrict__ xp, const float* __restrict__ pscale,
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

// Forward: block (vtile, chunk); lanes own kGridVPL visibilities each and sweep
// the chunk's cells (one |m| group of kGridNB values times an |l| range) in a
// wavefront-uniform order, reading the cell records through the scalar unit.
// Partial row `blockIdx.y` of `part` receives sum over the chunk's cells.
__global__ __launch_bounds__(kBlock) void k_grid_fwd(
    const GridRec* __restrict__ rec, const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    float2* __restrict__ part) {
  const ConstPtr<GridChunk> cch = as_const(chunks) + blockIdx.y;
  const int g = cch->g, ia0 = cch->ia0, ia1 = cch->ia1;
  const ConstPtr<GridRec> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int64_t kbase = static_cast<int64_t>(blockIdx.x) * (kBlock * kGridVPL) + threadIdx.x;
  const double origin = kMagic;
  double u[kGridVPL], w[kGridVPL];
  float bc[kGridNB][kGridVPL], bs[kGridNB][kGridVPL];
  float ore[kGridVPL], oim[kGridVPL];
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = k < n_vis;
    u[i] = ok ? vu[k] : 0.0;
    const double v = ok ? vv[k] : 0.0;
    w[i] = ok ? vw[k] : 0.0;
#pragma unroll
    for (int b = 0; b < kGridNB; ++b) phasor(fma(v, cmb[g * kGridNB + b], origin), bc[b][i], bs[b][i]);
    ore[i] = oim[i] = 0.0f;
  }
  for (int s0 = ia0; s0 < ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ia1 ? s0 + kGridSegIA : ia1;
    float re[kGridVPL], imn[kGridVPL];
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) re[i] = imn[i] = 0.0f;
    for (int ia = s0; ia < s1; ++ia) {
      const double l = cla[ia];
      float ac[kGridVPL], as[kGridVPL];
#pragma unroll
      for (int i = 0; i < kGridVPL; ++i) phasor(fma(u[i], l, origin), ac[i], as[i]);
      const int q0 = (g * na + ia) * kGridNB;
#pragma unroll
      for (int b = 0; b < kGridNB; ++b) {
        if (crec[q0 + b].empty) continue;  // wavefront-uniform
        const double nu = crec[q0 + b].nu;
        const float e1 = crec[q0 + b].e1, e2 = crec[q0 + b].e2;
        const float e3 = crec[q0 + b].e3, e4 = crec[q0 + b].e4;
#pragma unroll
        for (int i = 0; i < kGridVPL; ++i) {
          float cc, cs;
          phasor(fma(w[i], nu, origin), cc, cs);
          const float res_ = fmaf(ac[i] * bc[b][i], e1, as[i] * bs[b][i] * e2);
          const float ims = fmaf(ac[i] * bs[b][i], e3, as[i] * bc[b][i] * e4);
          re[i] = fmaf(cc, res_, re[i]);
          re[i] = fmaf(-cs, ims, re[i]);
          imn[i] = fmaf(cc, ims, imn[i]);
          imn[i] = fmaf(cs, res_, imn[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) {
      ore[i] += re[i];
      oim[i] += imn[i];
    }
  }
  float2* out = part + static_cast<int64_t>(blockIdx.y) * n_vis;
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    if (k < n_vis) out[k] = make_float2(ore[i], -oim[i]);
  }
}

// Adjoint: block (lane-set tile, visibility chunk).  Lane-set t = g4 * na + ia
// owns the kGridNBA cells (ia, g4 * kGridNBA + bi) and their 16 sign slots.
// Visibility records and residuals are wavefront-uniform scalar loads; the B
// phasors of the block's |m| groups are computed once per batch of kGridKB
// visibilities by the whole block and read from LDS.  Partial row
// `blockIdx.y` receives Re sum_k conj(M_kj) r_k for every delta pixel j of
// the block's cells (indexed by permuted pixel).
__global__ __launch_bounds__(kBlock) void k_grid_adj(
    const VisRecD<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ vv, const double* __restrict__ la, const double* __restrict__ mb,
    const double* __restrict__ nu, const int32_t* __restrict__ slot, int na, int ng4,
    int64_t kchunk, int64_t n_vis, float* __restrict__ part, int64_t n_pix) {
  __shared__ float2 bsh[kGridKB][kGridMaxGL][kGridNBA];
  const int64_t n_sets = static_cast<int64_t>(ng4) * na;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kBlock;
  const int64_t t = t0 + threadIdx.x;
  const bool active = t < n_sets;
  const int gl0 = static_cast<int>(t0 / na);
  const int64_t tlast = (t0 + kBlock - 1 < n_sets ? t0 + kBlock - 1 : n_sets - 1);
  int n_gl = static_cast<int>(tlast / na) - gl0 + 1;
  if (n_gl > kGridMaxGL) n_gl = kGridMaxGL;  // the plan keeps na >= kGridMinA, so this never binds
  const int g4 = active ? static_cast<int>(t / na) : gl0;
  const int ia = active ? static_cast<int>(t % na) : 0;
  const int gl = g4 - gl0;
  const int qbase = ((g4 / 2) * na + ia) * kGridNB + (g4 % 2) * kGridNBA;
  const double l = la[ia];
  double nuv[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) nuv[bi] = active ? nu[qbase + bi] : 0.0;

  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const ConstPtr<float> cres = as_const(reinterpret_cast<const float*>(rres));
  const double origin = kMagic;
  const int k0 = static_cast<int>(blockIdx.y * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float o1[kGridNBA], o2[kGridNBA], o3[kGridNBA], o4[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) o1[bi] = o2[bi] = o3[bi] = o4[bi] = 0.0f;

  const int fill = kGridKB * n_gl * kGridNBA;
  for (int kb = k0; kb < k1; kb += kGridKB) {
    __syncthreads();  // the previous batch's reads are done
    for (int e = threadIdx.x; e < fill; e += kBlock) {
      const int kk = e / (n_gl * kGridNBA);
      const int rem = e - kk * (n_gl * kGridNBA);
      const int gg = rem / kGridNBA, bi = rem - gg * kGridNBA;
      const int k = kb + kk;
      float c = 0.0f, s = 0.0f;
      if (k < k1) phasor(fma(vv[k], mb[(gl0 + gg) * kGridNBA + bi], origin), c, s);
      bsh[kk][gg][bi] = make_float2(c, s);
    }
    __syncthreads();
    const int ke = kb + kGridKB < k1 ? kb + kGridKB : k1;
    float G1[kGridNBA], G2[kGridNBA], G3[kGridNBA], G4[kGridNBA];
#pragma unroll
    for (int bi = 0; bi < kGridNBA; ++bi) G1[bi] = G2[bi] = G3[bi] = G4[bi] = 0.0f;
    for (int k = kb; k < ke; ++k) {
      const double u = cvrec[k].u, w = cvrec[k].w;
      const float rr = cres[2 * static_cast<int64_t>(k)], ri = cres[2 * static_cast<int64_t>(k) + 1];
      float ac, as;
      phasor(fma(u, l, origin), ac, as);
      const float2* bp = &bsh[k - kb][gl][0];
#pragma unroll
      for (int bi = 0; bi < kGridNBA; ++bi) {
        const float2 bb = bp[bi];
        float cc, cs;
        phasor(fma(w, nuv[bi], origin), cc, cs);
        const float z1 = fmaf(cc, rr, -cs * ri);
        const float z2 = fmaf(cc, ri, cs * rr);
        G1[bi] = fmaf(bb.x, ac * z1, G1[bi]);
        G2[bi] = fmaf(bb.y, as * z1, G2[bi]);
        G3[bi] = fmaf(bb.y, ac * z2, G3[bi]);
        G4[bi] = fmaf(bb.x, as * z2, G4[bi]);
      }
    }
#pragma unroll
    for (int bi = 0; bi < kGridNBA; ++bi) {
      o1[bi] += G1[bi];
      o2[bi] += G2[bi];
      o3[bi] += G3[bi];
      o4[bi] += G4[bi];
    }
  }
  if (!active) return;
  float* out = part + static_cast<int64_t>(blockIdx.y) * n_pix;
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    const int64_t q = qbase + bi;
    const float gs[4] = {o1[bi] - o2[bi] - o3[bi] - o4[bi], o1[bi] + o2[bi] - o3[bi] + o4[bi],
                         o1[bi] + o2[bi] + o3[bi] - o4[bi], o1[bi] - o2[bi] + o3[bi] + o4[bi]};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int32_t j = slot[4 * q + s];
      if (j >= 0) out[j] = gs[s];
    }
  }
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_grid_forward(sl1m_plan* p, const void* xp, hipStream_t st) {
  if (p->grid_cells == 0 || p->n_vis == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid_prep, dim3(blocks_for(p->grid_cells)), dim3(kBlock), 0, st,
                     static_cast<const float*>(xp), static_cast<const float*>(p->pscale),
                     p->grid_slot, p->grid_nu, p->grid_cells, p->grid_rec);
  hipLaunchKernelGGL(k_grid_fwd, dim3(static_cast<unsigned>(p->grid_vtiles),
                                      static_cast<unsigned>(p->grid_fchunks.size())),
                     dim3(kBlock), 0, st, p->grid_rec, p->grid_la, p->grid_mb, p->d_grid_fchunks,
                     p->grid_na, p->vu, p->vv, p->vw, p->n_vis, static_cast<float2*>(p->fpart));
  return hipGetLastError();
}

hipError_t launch_grid_adjoint(sl1m_plan* p, hipStream_t st) {
  if (p->grid_cells == 0 || p->n_achunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid_adj, dim3(static_cast<unsigned>(p->grid_ablocks),
                                      static_cast<unsigned>(p->n_achunks)),
                     dim3(kBlock), 0, st, static_cast<const VisRecD<float>*>(p->visrecD),
                     static_cast<const float2*>(p->rres), p->vv, p->grid_la, p->grid_mb,
                     p->grid_nu, p->grid_slot, p->grid_na, 2 * p->grid_ng, p->adj_kchunk, p->n_vis,
                     static_cast<float*>(p->apart), p->n_pix);
  return hipGetLastError();
}

}  // namespace sl1m
