// Grid evaluation of the operators (gfx950, float32 plans): device tiles
// shared by the per-plan kernels (sl1m_grid.hip).
//
// Delta pixels, eq. (deltam) without gains:
//   M_kj = exp(-2 pi i (u_k l_j + v_k m_j + w_k nu_j)),  nu_j = n_j - 1,
// factorises into A_k(l) B_k(m) C_k(nu) with A = exp(-2 pi i u l),
// B = exp(-2 pi i v m), C = exp(-2 pi i w nu).  nu depends on l^2 + m^2 only,
// so the four positions (+-|l|, +-|m|) of a cell share C, and a sign flip of
// l or m conjugates A or B.  With A = ac - i as, B = bc - i bs, C = cc - i cs
// and x_s the amplitudes of the cell's sign slots (0 = (+,+), 1 = (-,+),
// 2 = (+,-), 3 = (-,-)):
//   forward  sum_s x_s M_s = C (ReS - i ImS'),
//            ReS = ac bc e1 + as bs e2,  ImS' = ac bs e3 + as bc e4
//            (e1..e4 are the sign combinations of GridRec);
//   adjoint  z = conj(C) r, G1 = sum bc ac z1, G2 = sum bs as z1,
//            G3 = sum bs ac z2, G4 = sum bc as z2;
//            g0 = G1-G2-G3-G4, g1 = G1+G2-G3+G4, g2 = G1+G2+G3-G4, g3 = G1-G2+G3+G4.
//
// Gaussian pixels, eq. (samlm4)/(samlm5) in the completed-square form of the
// direct kernels (entry = e exp(2 pi i theta) times D (1 + i s) per visibility
// and layer, theta = A l + B m + C r^2 + NW kappa + E0 with A = -D u,
// B = -D v):  the taper exp(c (u - w l)^2) exp(c (v - w m)^2) separates too, but
// is not even in l or m, so per (visibility, |l|) the pair
//   a+ = T(u - w|l|) exp(2 pi i A|l|),  a- = T(u + w|l|) exp(-2 pi i A|l|)
// and per (visibility, |m|) the pair b+, b- are formed, and per cell
// gamma = exp(2 pi i (C r^2 + NW kappa + E0)):
//   forward  sum_s x_s M_s = gamma (b+ (x0 a+ + x1 a-) + b- (x2 a+ + x3 a-));
//   adjoint  Z = conj(gamma) r', Y+- = conj(b+-) Z,
//            g0 = Re conj(a+) Y+, g1 = Re conj(a-) Y+, g2 = Re conj(a+) Y-,
//            g3 = Re conj(a-) Y-.
//
// Phases use the same exact reduction as the direct kernels (FP64 FMAs from
// kMagic, low 23 mantissa bits into 1.0f).
#pragma once

#include "sl1m_device.h"

namespace sl1m {
namespace dev {

constexpr int kGridKBM = 32;   // visibilities per LDS batch of the multi-RHS pair adjoint
constexpr int kGridSegIA = 8;  // forward: |l| values per inner FP32 sum

// ---------------------------------------------------------------------------
// forward tiles: lanes own kGridVPL visibilities of tile `vtile` and sweep the
// chunk's cells (one |m| group of kGridNB values times an |l| range) in a
// wavefront-uniform order; cell records are read through the scalar unit.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void grid_fwd_delta_tile(
    const GridRec* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk& ch, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t vtile, int64_t n_vis,
    float2* __restrict__ out) {
  const ConstPtr<GridRec> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int g = ch.g;
  const int64_t kbase = vtile * (kBlock * kGridVPL) + threadIdx.x;
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
  for (int s0 = ch.ia0; s0 < ch.ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ch.ia1 ? s0 + kGridSegIA : ch.ia1;
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
        // no test of `empty` here: a branch on it would make every record
        // cost two scalar-load round trips, and an empty cell's amplitudes
        // are zero, so it adds exactly nothing
        const double nu = crec[q0 + b].nu;
        const float e1 = crec[q0 + b].e1, e2 = crec[q0 + b].e2;
        const float e3 = crec[q0 + b].e3, e4 = crec[q0 + b].e4;
#pragma unroll
        for (int i = 0; i < kGridVPL; ++i) {
          float cc, cs;
          phasor(fma(w[i], nu, origin), cc, cs);
          const float rs = fmaf(ac[i] * bc[b][i], e1, as[i] * bs[b][i] * e2);
          const float is = fmaf(ac[i] * bs[b][i], e3, as[i] * bc[b][i] * e4);
          re[i] = fmaf(cc, rs, re[i]);
          re[i] = fmaf(-cs, is, re[i]);
          imn[i] = fmaf(cc, is, imn[i]);
          imn[i] = fmaf(cs, rs, imn[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) {
      ore[i] += re[i];
      oim[i] += imn[i];
    }
  }
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    if (k < n_vis) out[k] = make_float2(ore[i], -oim[i]);
  }
}

// Pair record p of a square grid: its group g, |l| index ia, member b and
// |m| index bb = kGridNB g + b; the amplitudes x_j = xs * scale_j * xp_j of
// the cell's (x) and the mirror's (y) sign slots (zero where the pair rules
// of GridPairRec leave them out); cell index q of (ia, bb).
struct PairSlots {
  int64_t q;
  float x[4], y[4];
  int32_t empty;
};

__device__ __forceinline__ PairSlots grid_pair_slots(int64_t p, int na,
                                                     const int32_t* __restrict__ slot,
                                                     const float* __restrict__ xp,
                                                     const float* __restrict__ pscale, float xs) {
  // groups with records: kGridNB g < na; the record offsets increase over them
  const int ngroups = (na + kGridNB - 1) / kGridNB;
  int g = 0;
  while (g + 1 < ngroups && pair_rec_base(g + 1, na) <= p) ++g;
  const int64_t li = p - pair_rec_base(g, na);
  const int ia = kGridNB * g + static_cast<int>(li / kGridNB);
  const int b = static_cast<int>(li % kGridNB), bb = kGridNB * g + b;
  PairSlots r;
  r.q = (static_cast<int64_t>(g) * na + ia) * kGridNB + b;
  r.empty = 1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int32_t j = bb <= ia ? slot[4 * r.q + s] : -1;
    r.x[s] = j >= 0 ? pscale[j] * xs * xp[j] : 0.0f;
    r.empty &= j < 0 ? 1 : 0;
    r.y[s] = 0.0f;
  }
  if (bb < ia) {
    const int64_t qp = (static_cast<int64_t>(ia / kGridNB) * na + bb) * kGridNB + ia % kGridNB;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int32_t j = slot[4 * qp + s];
      r.y[s] = j >= 0 ? pscale[j] * xs * xp[j] : 0.0f;
      r.empty &= j < 0 ? 1 : 0;
    }
  }
  return r;
}

// Writes pair record p of a square delta grid (GridPairRec).
__device__ __forceinline__ void grid_write_pair_rec(int64_t p, int na,
                                                    const int32_t* __restrict__ slot,
                                                    const double* __restrict__ nu,
                                                    const float* __restrict__ xp,
                                                    const float* __restrict__ pscale, float xs,
                                                    GridPairRec* __restrict__ rec) {
  const PairSlots ps = grid_pair_slots(p, na, slot, xp, pscale, xs);
  const float* x = ps.x;
  const float* y = ps.y;
  const int32_t empty = ps.empty;
  const int64_t q = ps.q;
  GridPairRec r;
  r.nu = nu[q];
  r.e1 = (x[0] + x[1]) + (x[2] + x[3]);
  r.e2 = (x[1] + x[2]) - (x[0] + x[3]);
  r.e3 = (x[0] + x[1]) - (x[2] + x[3]);
  r.e4 = (x[0] - x[1]) + (x[2] - x[3]);
  r.f1 = (y[0] + y[1]) + (y[2] + y[3]);
  r.f2 = (y[1] + y[2]) - (y[0] + y[3]);
  r.f3 = (y[0] + y[1]) - (y[2] + y[3]);
  r.f4 = (y[0] - y[1]) + (y[2] - y[3]);
  r.empty = empty;
  r.pad = 0;
  rec[p] = r;
}

// Writes pair record p of a square Gaussian grid (GridPairRecG).
__device__ __forceinline__ void grid_write_pair_rec_gauss(
    int64_t p, int na, const int32_t* __restrict__ slot, const double* __restrict__ r2c,
    const double* __restrict__ kapc, const float* __restrict__ xp,
    const float* __restrict__ pscale, float xs, GridPairRecG* __restrict__ rec) {
  const PairSlots ps = grid_pair_slots(p, na, slot, xp, pscale, xs);
  GridPairRecG r;
  r.r2 = r2c[ps.q];
  r.kappa = kapc[ps.q];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    r.x[s] = ps.x[s];
    r.y[s] = ps.y[s];
  }
  rec[p] = r;
}

// Square delta grid, pair chunk: for every |l| index ia of the chunk and b of
// the group, the cells (ia, b) and (b, ia) (when b < na) share C; their
// amplitudes come from one pair record (GridPairRec).  The partner
// cell has A at |l|_b = |m|_b and B at |m|_ia = |l|_ia.  `mb` is the padded
// |m| table (equal to |l| where defined).
__device__ __forceinline__ void grid_fwd_delta_pairs_tile(
    const GridPairRec* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk& ch, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t vtile, int64_t n_vis,
    float2* __restrict__ out) {
  const ConstPtr<GridPairRec> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int g = ch.g;
  const int64_t kbase = vtile * (kBlock * kGridVPL) + threadIdx.x;
  const double origin = kMagic;
  double u[kGridVPL], v[kGridVPL], w[kGridVPL];
  float bc[kGridNB][kGridVPL], bs[kGridNB][kGridVPL];   // B at |m|_b
  float pc[kGridNB][kGridVPL], ps[kGridNB][kGridVPL];   // A at |l|_b (partner)
  float ore[kGridVPL], oim[kGridVPL];
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = k < n_vis;
    u[i] = ok ? vu[k] : 0.0;
    v[i] = ok ? vv[k] : 0.0;
    w[i] = ok ? vw[k] : 0.0;
#pragma unroll
    for (int b = 0; b < kGridNB; ++b) {
      const double m = cmb[g * kGridNB + b];
      phasor(fma(v[i], m, origin), bc[b][i], bs[b][i]);
      phasor(fma(u[i], m, origin), pc[b][i], ps[b][i]);
    }
    ore[i] = oim[i] = 0.0f;
  }
  for (int s0 = ch.ia0; s0 < ch.ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ch.ia1 ? s0 + kGridSegIA : ch.ia1;
    float re[kGridVPL], imn[kGridVPL];
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) re[i] = imn[i] = 0.0f;
    for (int ia = s0; ia < s1; ++ia) {
      const double l = cla[ia];
      float ac[kGridVPL], as[kGridVPL], qc[kGridVPL], qs[kGridVPL];  // A at |l|_ia, B at |m|_ia
#pragma unroll
      for (int i = 0; i < kGridVPL; ++i) {
        phasor(fma(u[i], l, origin), ac[i], as[i]);
        phasor(fma(v[i], l, origin), qc[i], qs[i]);
      }
      const int p0 = static_cast<int>(pair_rec_base(g, na)) + (ia - kGridNB * g) * kGridNB;
#pragma unroll
      for (int b = 0; b < kGridNB; ++b) {
        const double nu = crec[p0 + b].nu;
        const float e1 = crec[p0 + b].e1, e2 = crec[p0 + b].e2;
        const float e3 = crec[p0 + b].e3, e4 = crec[p0 + b].e4;
        const float f1 = crec[p0 + b].f1, f2 = crec[p0 + b].f2;
        const float f3 = crec[p0 + b].f3, f4 = crec[p0 + b].f4;  // (no `empty` test, as above)
#pragma unroll
        for (int i = 0; i < kGridVPL; ++i) {
          float cc, cs;
          phasor(fma(w[i], nu, origin), cc, cs);
          const float rs = fmaf(ac[i] * bc[b][i], e1,
                                fmaf(as[i] * bs[b][i], e2,
                                     fmaf(pc[b][i] * qc[i], f1, ps[b][i] * qs[i] * f2)));
          const float is = fmaf(ac[i] * bs[b][i], e3,
                                fmaf(as[i] * bc[b][i], e4,
                                     fmaf(pc[b][i] * qs[i], f3, ps[b][i] * qc[i] * f4)));
          re[i] = fmaf(cc, rs, re[i]);
          re[i] = fmaf(-cs, is, re[i]);
          imn[i] = fmaf(cc, is, imn[i]);
          imn[i] = fmaf(cs, rs, imn[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) {
      ore[i] += re[i];
      oim[i] += imn[i];
    }
  }
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    if (k < n_vis) out[k] = make_float2(ore[i], -oim[i]);
  }
}

// Several right-hand sides on a square delta grid (the paper solves every
// polarisation through the same matrix): pair record p holds nu (FP64) and,
// per right-hand side r, the cell's and the mirror's sign combinations
// e1..e4, f1..f4 -- pair_rec_floats<NR>() floats, 8 + 32 NR bytes.
template <int NR>
__host__ __device__ constexpr int pair_rec_floats() {
  return 2 + 8 * NR;
}

template <int NR>
__device__ __forceinline__ void grid_write_pair_rec_multi(int64_t p, int na,
                                                          const int32_t* __restrict__ slot,
                                                          const double* __restrict__ nu,
                                                          const float* __restrict__ xp,
                                                          int64_t n_pix,
                                                          const float* __restrict__ pscale,
                                                          float* __restrict__ rec) {
  float* o = rec + p * pair_rec_floats<NR>();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const PairSlots ps = grid_pair_slots(p, na, slot, xp + r * n_pix, pscale, 1.0f);
    const float* x = ps.x;
    const float* y = ps.y;
    if (r == 0) *reinterpret_cast<double*>(o) = nu[ps.q];
    float* e = o + 2 + 8 * r;
    e[0] = (x[0] + x[1]) + (x[2] + x[3]);
    e[1] = (x[1] + x[2]) - (x[0] + x[3]);
    e[2] = (x[0] + x[1]) - (x[2] + x[3]);
    e[3] = (x[0] - x[1]) + (x[2] - x[3]);
    e[4] = (y[0] + y[1]) + (y[2] + y[3]);
    e[5] = (y[1] + y[2]) - (y[0] + y[3]);
    e[6] = (y[0] + y[1]) - (y[2] + y[3]);
    e[7] = (y[0] - y[1]) + (y[2] - y[3]);
  }
}

// Forward pair chunk for NR right-hand sides, one visibility per lane: the
// phasors (A, B at |l|_ia and at the group's values, C per pair) and the eight
// products of A and B factors are formed once and shared by every right-hand
// side; right-hand side r adds its amplitude combinations (twelve FP32
// operations per pair).  Partial row of right-hand side r at out + r rhs_stride.
template <int NR>
__device__ __forceinline__ void grid_fwd_delta_pairs_multi_tile(
    const float* __restrict__ rec, const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk& ch, int na, const double* __restrict__ vu, const double* __restrict__ vv,
    const double* __restrict__ vw, int64_t vtile, int64_t n_vis, float2* __restrict__ out,
    int64_t rhs_stride) {
  constexpr int kF = pair_rec_floats<NR>();
  const ConstPtr<float> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int g = ch.g;
  const int64_t k = vtile * kBlock + threadIdx.x;
  const bool ok = k < n_vis;
  const double origin = kMagic;
  const double u = ok ? vu[k] : 0.0, v = ok ? vv[k] : 0.0, w = ok ? vw[k] : 0.0;
  float bc[kGridNB], bs[kGridNB];  // B at |m|_b
  float pc[kGridNB], ps[kGridNB];  // A at |l|_b (partner)
#pragma unroll
  for (int b = 0; b < kGridNB; ++b) {
    const double m = cmb[g * kGridNB + b];
    phasor(fma(v, m, origin), bc[b], bs[b]);
    phasor(fma(u, m, origin), pc[b], ps[b]);
  }
  float ore[NR], oim[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) ore[r] = oim[r] = 0.0f;
  for (int s0 = ch.ia0; s0 < ch.ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ch.ia1 ? s0 + kGridSegIA : ch.ia1;
    float re[NR], imn[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) re[r] = imn[r] = 0.0f;
    for (int ia = s0; ia < s1; ++ia) {
      const double l = cla[ia];
      float ac, as, qc, qs;  // A at |l|_ia, B at |m|_ia
      phasor(fma(u, l, origin), ac, as);
      phasor(fma(v, l, origin), qc, qs);
      const int64_t p0 = pair_rec_base(g, na) + static_cast<int64_t>(ia - kGridNB * g) * kGridNB;
#pragma unroll
      for (int b = 0; b < kGridNB; ++b) {
        const ConstPtr<float> rp = crec + (p0 + b) * kF;
        const double nu = *reinterpret_cast<ConstPtr<double>>(rp);
        float cc, cs;
        phasor(fma(w, nu, origin), cc, cs);
        const float p1 = ac * bc[b], p2 = as * bs[b], p3 = pc[b] * qc, p4 = ps[b] * qs;
        const float q1 = ac * bs[b], q2 = as * bc[b], q3 = pc[b] * qs, q4 = ps[b] * qc;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const ConstPtr<float> e = rp + 2 + 8 * r;
          const float rs = fmaf(p1, e[0], fmaf(p2, e[1], fmaf(p3, e[4], p4 * e[5])));
          const float is = fmaf(q1, e[2], fmaf(q2, e[3], fmaf(q3, e[6], q4 * e[7])));
          re[r] = fmaf(cc, rs, re[r]);
          re[r] = fmaf(-cs, is, re[r]);
          imn[r] = fmaf(cc, is, imn[r]);
          imn[r] = fmaf(cs, rs, imn[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      ore[r] += re[r];
      oim[r] += imn[r];
    }
  }
  if (ok)
#pragma unroll
    for (int r = 0; r < NR; ++r) out[r * rhs_stride + k] = make_float2(ore[r], -oim[r]);
}

// Square Gaussian grid, pair chunk, one visibility per lane: for |l| index
// ia and group member b, the cell (ia, bb) and its mirror (bb, ia) share
// gamma; the cell takes a+- at |l|_ia and b+- at |m|_bb, the mirror a+- at
// |l|_bb = |m|_bb and b+- at |m|_ia = |l|_ia.  Amplitudes from one pair record
// (GridPairRecG).  `vrec` and `Ds` as for grid_fwd_gauss_tile.
__device__ __forceinline__ void grid_fwd_gauss_pairs_tile(
    const GridPairRecG* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk& ch, int na,
    const VisRecG<float>* __restrict__ vrec, const float* __restrict__ Ds, int64_t vtile,
    int64_t n_vis, float2* __restrict__ out) {
  const ConstPtr<GridPairRecG> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int g = ch.g;
  const int64_t k = vtile * kBlock + threadIdx.x;
  const bool ok = k < n_vis;
  const int64_t kk = ok ? k : 0;
  const double origin = kMagic;
  const double A = vrec[kk].A, B = vrec[kk].B, C = vrec[kk].C, NW = vrec[kk].NW, E0 = vrec[kk].E0;
  const float ur = vrec[kk].ur, vr = vrec[kk].vr, wr = vrec[kk].wr, c1 = vrec[kk].c1;
  // per member b: the cell's b+- at |m|_bb and the mirror's a+- at the same value
  float bpr[kGridNB], bpi[kGridNB], bmr[kGridNB], bmi[kGridNB];
  float mpr[kGridNB], mpi[kGridNB], mmr[kGridNB], mmi[kGridNB];
#pragma unroll
  for (int b = 0; b < kGridNB; ++b) {
    const double m = cmb[g * kGridNB + b];
    const float mr = static_cast<float>(m);
    float cb, sb, ca, sa;
    phasor(fma(B, m, origin), cb, sb);
    phasor(fma(A, m, origin), ca, sa);
    const float dvp = fmaf(-wr, mr, vr), dvm = fmaf(wr, mr, vr);
    const float dup = fmaf(-wr, mr, ur), dum = fmaf(wr, mr, ur);
    const float tvp = pow2(c1 * (dvp * dvp)), tvm = pow2(c1 * (dvm * dvm));
    const float tup = pow2(c1 * (dup * dup)), tum = pow2(c1 * (dum * dum));
    bpr[b] = tvp * cb;
    bpi[b] = tvp * sb;
    bmr[b] = tvm * cb;
    bmi[b] = -tvm * sb;
    mpr[b] = tup * ca;
    mpi[b] = tup * sa;
    mmr[b] = tum * ca;
    mmi[b] = -tum * sa;
  }
  float ore = 0.0f, oim = 0.0f;
  for (int s0 = ch.ia0; s0 < ch.ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ch.ia1 ? s0 + kGridSegIA : ch.ia1;
    float re = 0.0f, im = 0.0f;
    for (int ia = s0; ia < s1; ++ia) {
      const double l = cla[ia];
      const float lr = static_cast<float>(l);
      float ca, sa, cb, sb;
      phasor(fma(A, l, origin), ca, sa);
      phasor(fma(B, l, origin), cb, sb);
      const float dup = fmaf(-wr, lr, ur), dum = fmaf(wr, lr, ur);
      const float dvp = fmaf(-wr, lr, vr), dvm = fmaf(wr, lr, vr);
      const float tup = pow2(c1 * (dup * dup)), tum = pow2(c1 * (dum * dum));
      const float tvp = pow2(c1 * (dvp * dvp)), tvm = pow2(c1 * (dvm * dvm));
      const float apr = tup * ca, api = tup * sa, amr = tum * ca, ami = -tum * sa;  // cell a+-
      const float qpr = tvp * cb, qpi = tvp * sb, qmr = tvm * cb, qmi = -tvm * sb;  // mirror b+-
      const int p0 = static_cast<int>(pair_rec_base(g, na)) + (ia - kGridNB * g) * kGridNB;
#pragma unroll
      for (int b = 0; b < kGridNB; ++b) {
        const double r2 = crec[p0 + b].r2, kap = crec[p0 + b].kappa;
        const float x0 = crec[p0 + b].x[0], x1 = crec[p0 + b].x[1];
        const float x2 = crec[p0 + b].x[2], x3 = crec[p0 + b].x[3];
        const float y0 = crec[p0 + b].y[0], y1 = crec[p0 + b].y[1];
        const float y2 = crec[p0 + b].y[2], y3 = crec[p0 + b].y[3];
        float cg, sg;
        phasor(fma(C, r2, fma(NW, kap, E0)), cg, sg);
        // cell: b+ (x0 a+ + x1 a-) + b- (x2 a+ + x3 a-)
        const float Ur = fmaf(x0, apr, x1 * amr), Ui = fmaf(x0, api, x1 * ami);
        const float Wr = fmaf(x2, apr, x3 * amr), Wi = fmaf(x2, api, x3 * ami);
        // mirror: qb+ (y0 ma+ + y1 ma-) + qb- (y2 ma+ + y3 ma-)
        const float Vr = fmaf(y0, mpr[b], y1 * mmr[b]), Vi = fmaf(y0, mpi[b], y1 * mmi[b]);
        const float Xr = fmaf(y2, mpr[b], y3 * mmr[b]), Xi = fmaf(y2, mpi[b], y3 * mmi[b]);
        const float Sr = fmaf(bpr[b], Ur, fmaf(-bpi[b], Ui, fmaf(bmr[b], Wr, fmaf(-bmi[b], Wi,
                         fmaf(qpr, Vr, fmaf(-qpi, Vi, fmaf(qmr, Xr, -qmi * Xi)))))));
        const float Si = fmaf(bpr[b], Ui, fmaf(bpi[b], Ur, fmaf(bmr[b], Wi, fmaf(bmi[b], Wr,
                         fmaf(qpr, Vi, fmaf(qpi, Vr, fmaf(qmr, Xi, qmi * Xr)))))));
        re = fmaf(cg, Sr, re);
        re = fmaf(-sg, Si, re);
        im = fmaf(cg, Si, im);
        im = fmaf(sg, Sr, im);
      }
    }
    ore += re;
    oim += im;
  }
  if (ok) {
    const float D = Ds[2 * k], Dsv = D * Ds[2 * k + 1];
    out[k] = make_float2(D * ore - Dsv * oim, Dsv * ore + D * oim);
  }
}

// `vrec` and `Ds` are the layer's per-visibility records and (D, s) pairs.
__device__ __forceinline__ void grid_fwd_gauss_tile(
    const GridRecG* __restrict__ rec, const double* __restrict__ la,
    const double* __restrict__ mb, const GridChunk& ch, int na,
    const VisRecG<float>* __restrict__ vrec, const float* __restrict__ Ds, int64_t vtile,
    int64_t n_vis, float2* __restrict__ out) {
  const ConstPtr<GridRecG> crec = as_const(rec);
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const int g = ch.g;
  const int64_t kbase = vtile * (kBlock * kGridVPL) + threadIdx.x;
  const double origin = kMagic;
  double A[kGridVPL], C[kGridVPL], NW[kGridVPL], E0[kGridVPL];
  float ur[kGridVPL], wr[kGridVPL], c1[kGridVPL];
  float bpr[kGridNB][kGridVPL], bpi[kGridNB][kGridVPL];
  float bmr[kGridNB][kGridVPL], bmi[kGridNB][kGridVPL];
  float ore[kGridVPL], oim[kGridVPL];
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = k < n_vis;
    const int64_t kk = ok ? k : 0;
    A[i] = vrec[kk].A;
    C[i] = vrec[kk].C;
    NW[i] = vrec[kk].NW;
    E0[i] = vrec[kk].E0;
    ur[i] = vrec[kk].ur;
    wr[i] = vrec[kk].wr;
    c1[i] = vrec[kk].c1;
    const double B = vrec[kk].B;
    const float vr = vrec[kk].vr;
#pragma unroll
    for (int b = 0; b < kGridNB; ++b) {
      const double m = cmb[g * kGridNB + b];
      float cb, sb;
      phasor(fma(B, m, origin), cb, sb);
      const float mr = static_cast<float>(m);
      const float dp = fmaf(-wr[i], mr, vr), dm = fmaf(wr[i], mr, vr);
      const float tp = pow2(c1[i] * (dp * dp)), tm = pow2(c1[i] * (dm * dm));
      bpr[b][i] = tp * cb;
      bpi[b][i] = tp * sb;
      bmr[b][i] = tm * cb;
      bmi[b][i] = -tm * sb;
    }
    ore[i] = oim[i] = 0.0f;
  }
  for (int s0 = ch.ia0; s0 < ch.ia1; s0 += kGridSegIA) {
    const int s1 = s0 + kGridSegIA < ch.ia1 ? s0 + kGridSegIA : ch.ia1;
    float re[kGridVPL], im[kGridVPL];
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) re[i] = im[i] = 0.0f;
    for (int ia = s0; ia < s1; ++ia) {
      const double l = cla[ia];
      const float lr = static_cast<float>(l);
      float apr[kGridVPL], api[kGridVPL], amr[kGridVPL], ami[kGridVPL];
#pragma unroll
      for (int i = 0; i < kGridVPL; ++i) {
        float ca, sa;
        phasor(fma(A[i], l, origin), ca, sa);
        const float dp = fmaf(-wr[i], lr, ur[i]), dm = fmaf(wr[i], lr, ur[i]);
        const float tp = pow2(c1[i] * (dp * dp)), tm = pow2(c1[i] * (dm * dm));
        apr[i] = tp * ca;
        api[i] = tp * sa;
        amr[i] = tm * ca;
        ami[i] = -tm * sa;
      }
      const int q0 = (g * na + ia) * kGridNB;
#pragma unroll
      for (int b = 0; b < kGridNB; ++b) {
        const double r2 = crec[q0 + b].r2, kap = crec[q0 + b].kappa;
        const float x0 = crec[q0 + b].x[0], x1 = crec[q0 + b].x[1];
        const float x2 = crec[q0 + b].x[2], x3 = crec[q0 + b].x[3];
#pragma unroll
        for (int i = 0; i < kGridVPL; ++i) {
          float cg, sg;
          phasor(fma(C[i], r2, fma(NW[i], kap, E0[i])), cg, sg);
          const float Ur = fmaf(x0, apr[i], x1 * amr[i]), Ui = fmaf(x0, api[i], x1 * ami[i]);
          const float Wr = fmaf(x2, apr[i], x3 * amr[i]), Wi = fmaf(x2, api[i], x3 * ami[i]);
          const float Sr = fmaf(bpr[b][i], Ur, fmaf(-bpi[b][i], Ui, fmaf(bmr[b][i], Wr, -bmi[b][i] * Wi)));
          const float Si = fmaf(bpr[b][i], Ui, fmaf(bpi[b][i], Ur, fmaf(bmr[b][i], Wi, bmi[b][i] * Wr)));
          re[i] = fmaf(cg, Sr, re[i]);
          re[i] = fmaf(-sg, Si, re[i]);
          im[i] = fmaf(cg, Si, im[i]);
          im[i] = fmaf(sg, Sr, im[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kGridVPL; ++i) {
      ore[i] += re[i];
      oim[i] += im[i];
    }
  }
#pragma unroll
  for (int i = 0; i < kGridVPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    if (k < n_vis) {
      const float D = Ds[2 * k], Dsv = D * Ds[2 * k + 1];
      out[k] = make_float2(D * ore[i] - Dsv * oim[i], Dsv * ore[i] + D * oim[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint tiles: block `blk` of lane-sets t = g4 * na + ia, each owning the
// kGridNBA cells (ia, g4 * kGridNBA + bi) and their 16 sign slots, against
// visibility chunk kc.  Visibility records and residuals are wavefront-uniform
// scalar loads; the per-|m| factors of the block's |m| groups are formed once
// per batch of visibilities by the whole block and read from LDS.  Writes
// Re sum_k conj(M_kj) r_k into out_row[j] for every pixel j of the cells.
// Every thread of the block must call a tile (it synchronises the block).
// ---------------------------------------------------------------------------

// LDS fill of an adjoint block's per-|m| tables: thread t fills the batch rows
// kk = t / G, t / G + S, ... (S = kBlock / G) of the block's slot t % G, where
// G is the number of |m| slots (at most kGridMaxGL kGridNBA = 72, so S >= 3);
// threads t >= S G take no part.  The slot's |m| value stays in a register
// and no index is divided per entry.
struct FillSlot {
  int slot, row0, step;
  bool on;
};

__device__ __forceinline__ FillSlot fill_slot(int G) {
  FillSlot f;
  f.step = kBlock / G;
  f.slot = static_cast<int>(threadIdx.x) % G;
  f.row0 = static_cast<int>(threadIdx.x) / G;
  f.on = f.row0 < f.step;
  return f;
}

struct LaneSet {
  bool active;
  int gl0, n_gl, gl, ia, qbase;
};

__device__ __forceinline__ LaneSet lane_set(int64_t blk, int na, int ng4) {
  LaneSet r;
  const int64_t n_sets = static_cast<int64_t>(ng4) * na;
  const int64_t t0 = blk * kBlock;
  const int64_t t = t0 + threadIdx.x;
  r.active = t < n_sets;
  r.gl0 = static_cast<int>(t0 / na);
  const int64_t tlast = t0 + kBlock - 1 < n_sets ? t0 + kBlock - 1 : n_sets - 1;
  r.n_gl = static_cast<int>(tlast / na) - r.gl0 + 1;
  if (r.n_gl > kGridMaxGL) r.n_gl = kGridMaxGL;  // plans keep na >= kGridMinA: never binds
  const int g4 = r.active ? static_cast<int>(t / na) : r.gl0;
  r.ia = r.active ? static_cast<int>(t % na) : 0;
  r.gl = g4 - r.gl0;
  r.qbase = ((g4 / 2) * na + r.ia) * kGridNB + (g4 % 2) * kGridNBA;
  return r;
}

__device__ __forceinline__ void grid_write(const LaneSet& ls, const int32_t* __restrict__ slot,
                                           const float (&gs)[kGridNBA][4],
                                           float* __restrict__ out_row) {
  if (!ls.active) return;
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    const int64_t q = ls.qbase + bi;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int32_t j = slot[4 * q + s];
      if (j >= 0) out_row[j] = gs[bi][s];
    }
  }
}

__device__ __forceinline__ void grid_adj_delta_tile(
    const VisRecD<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ vv, const double* __restrict__ la, const double* __restrict__ mb,
    const double* __restrict__ nu, const int32_t* __restrict__ slot, int na, int ng4,
    int64_t blk, int64_t kc, int64_t kchunk, int64_t n_vis, float* __restrict__ out_row,
    float2 (*bsh)[kGridMaxGL][kGridNBA]) {
  const LaneSet ls = lane_set(blk, na, ng4);
  const double l = la[ls.ia];
  double nuv[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) nuv[bi] = ls.active ? nu[ls.qbase + bi] : 0.0;
  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const ConstPtr<float> cres = as_const(reinterpret_cast<const float*>(rres));
  const double origin = kMagic;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float o1[kGridNBA], o2[kGridNBA], o3[kGridNBA], o4[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) o1[bi] = o2[bi] = o3[bi] = o4[bi] = 0.0f;
  const FillSlot fs = fill_slot(ls.n_gl * kGridNBA);
  const int fgg = fs.slot / kGridNBA, fbi = fs.slot % kGridNBA;
  const double fm = fs.on ? mb[(ls.gl0 + fgg) * kGridNBA + fbi] : 0.0;
  for (int kb = k0; kb < k1; kb += kGridKB) {
    __syncthreads();  // the previous batch's reads are done
    if (fs.on) {
      for (int kk = fs.row0; kk < kGridKB; kk += fs.step) {
        const int k = kb + kk;
        float c = 0.0f, s = 0.0f;
        if (k < k1) phasor(fma(vv[k], fm, origin), c, s);
        bsh[kk][fgg][fbi] = make_float2(c, s);
      }
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
      const float2* bp = &bsh[k - kb][ls.gl][0];
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
  float gs[kGridNBA][4];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    gs[bi][0] = o1[bi] - o2[bi] - o3[bi] - o4[bi];
    gs[bi][1] = o1[bi] + o2[bi] - o3[bi] + o4[bi];
    gs[bi][2] = o1[bi] + o2[bi] + o3[bi] - o4[bi];
    gs[bi][3] = o1[bi] - o2[bi] + o3[bi] + o4[bi];
  }
  grid_write(ls, slot, gs, out_row);
}

// Square delta grid, pair blocks: lane-set (g4, ia) with ia >= kGridNBA g4
// owns the cells (ia, b) and their mirrors (b, ia), b = kGridNBA g4 + bi
// (written as GridPairBlock describes).
struct PairLane {
  bool active;
  int g4, ia, gl, qbase;
};

// Position of this thread in the pair block's row-major walk over (g4, ia).
__device__ __forceinline__ PairLane pair_lane(const GridPairBlock& pb, int na) {
  PairLane r;
  r.g4 = pb.g4;
  r.ia = pb.ia + static_cast<int>(threadIdx.x);
  r.active = static_cast<int>(threadIdx.x) < pb.count;
  while (r.active && r.ia >= na) {
    ++r.g4;
    r.ia = r.ia - na + kGridNBA * r.g4;
  }
  if (!r.active) {
    r.g4 = pb.g4;
    r.ia = 0;
  }
  r.gl = r.g4 - pb.g4;
  r.qbase = ((r.g4 / 2) * na + r.ia) * kGridNB + (r.g4 % 2) * kGridNBA;
  return r;
}

// Sign-slot values of cell (ia, b), b = kGridNBA g4 + bi, from G[0..3] and of
// its mirror (b, ia) from G[4..7]: the cell when b <= ia, the mirror when
// b < ia (other cells belong to the lane-set of the mirror).
__device__ __forceinline__ void pair_write(const PairLane& pl, int na, int bi,
                                           const float* G8, const int32_t* __restrict__ slot,
                                           float* __restrict__ out_row) {
  const int64_t q = pl.qbase + bi;
  const int b = kGridNBA * pl.g4 + bi;
  const int64_t qp = (static_cast<int64_t>(pl.ia / kGridNB) * na + b) * kGridNB + pl.ia % kGridNB;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h == 0 ? b > pl.ia : b >= pl.ia) continue;
    const float* G = G8 + 4 * h;
    const float gs[4] = {G[0] - G[1] - G[2] - G[3], G[0] + G[1] - G[2] + G[3],
                         G[0] + G[1] + G[2] - G[3], G[0] - G[1] + G[2] + G[3]};
    const int64_t qq = h ? qp : q;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int32_t j = slot[4 * qq + s2];
      if (j >= 0) out_row[j] = gs[s2];
    }
  }
}

// One right-hand side: the block's per-|m| factors B and the partners' A
// (both at |m|_b = |l|_b, times the visibility's |r|) come from LDS; A and B
// at index ia per lane.  Each
// of the 32 sums runs over the chunk's visibilities in one float32
// accumulator (no per-batch partial sums: 32 fewer registers, a fifth
// wavefront per SIMD); the chunks' sums are added by the reduction.
__device__ __forceinline__ void grid_adj_delta_pairs_tile(
    const VisRecD<float>* __restrict__ vrec, const ResPolar* __restrict__ rpol,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ nu,
    const int32_t* __restrict__ slot, int na, const GridPairBlock& pb, int64_t kc,
    int64_t kchunk, int64_t n_vis, float* __restrict__ out_row,
    float4 (*bsh)[kGridMaxGL][kGridNBA]) {
  const PairLane pl = pair_lane(pb, na);
  const bool active = pl.active;
  const int gl = pl.gl;
  const double l = la[pl.ia];
  double nuv[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) nuv[bi] = active ? nu[pl.qbase + bi] : 0.0;
  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const ConstPtr<ResPolar> cpol = as_const(rpol);
  const double origin = kMagic;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float o[kGridNBA][8];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi)
#pragma unroll
    for (int j = 0; j < 8; ++j) o[bi][j] = 0.0f;
  const FillSlot fs = fill_slot(pb.n_gl * kGridNBA);
  const int fgg = fs.slot / kGridNBA, fbi = fs.slot % kGridNBA;
  const double fm = fs.on ? mb[(pb.g4 + fgg) * kGridNBA + fbi] : 0.0;
  for (int kb = k0; kb < k1; kb += kGridKBG) {
    __syncthreads();  // the previous batch's reads are done
    if (fs.on) {
      for (int kk = fs.row0; kk < kGridKBG; kk += fs.step) {
        const int k = kb + kk;
        float bc = 0.0f, bs = 0.0f, ac = 0.0f, as = 0.0f;
        if (k < k1) {
          phasor(fma(vv[k], fm, origin), bc, bs);
          phasor(fma(vu[k], fm, origin), ac, as);
          const float mag = rpol[k].mag;  // per-lane index: a vector load
          bc *= mag;
          bs *= mag;
          ac *= mag;
          as *= mag;
        }
        bsh[kk][fgg][fbi] = make_float4(bc, bs, ac, as);
      }
    }
    __syncthreads();
    const int ke = kb + kGridKBG < k1 ? kb + kGridKBG : k1;
    float (&G)[kGridNBA][8] = o;  // one running sum per chunk (see above)
    for (int k = kb; k < ke; ++k) {
      // z = C r = |r| e^{2 pi i (w nu + arg r / 2 pi)}: the residual's phase
      // rides in the phasor's origin, its modulus on the block's LDS factors
      // (a real factor, unchanged by the sign flips that conjugate A or B;
      // each of the eight products below holds one LDS factor)
      const double u = cvrec[k].u, v = cvrec[k].v, w = cvrec[k].w;
      const double org = cpol[k].org;
      float ac, as, qc, qs;  // A and B at index ia
      phasor(fma(u, l, origin), ac, as);
      phasor(fma(v, l, origin), qc, qs);
      const float4* bp = &bsh[k - kb][gl][0];
#pragma unroll
      for (int bi = 0; bi < kGridNBA; ++bi) {
        const float4 bb = bp[bi];  // |r| B at b (x, y), |r| A at b (z, w)
        float cc, cs;              // z / |r|
        phasor(fma(w, nuv[bi], org), cc, cs);
        // cell (ia, b): A at ia, B at b
        G[bi][0] = fmaf(bb.x, ac * cc, G[bi][0]);
        G[bi][1] = fmaf(bb.y, as * cc, G[bi][1]);
        G[bi][2] = fmaf(bb.y, ac * cs, G[bi][2]);
        G[bi][3] = fmaf(bb.x, as * cs, G[bi][3]);
        // cell (b, ia): A at b, B at ia
        G[bi][4] = fmaf(qc, bb.z * cc, G[bi][4]);
        G[bi][5] = fmaf(qs, bb.w * cc, G[bi][5]);
        G[bi][6] = fmaf(qs, bb.z * cs, G[bi][6]);
        G[bi][7] = fmaf(qc, bb.w * cs, G[bi][7]);
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) pair_write(pl, na, bi, o[bi], slot, out_row);
}

// NR right-hand sides sharing every phasor: z_r = C r_r in Cartesian form
// (the polar form above puts the residual's phase into C, which one C for
// several sides cannot carry), then the eight products per cell pair are
// formed once and scaled per side.  A block covers the NBI cells
// b = kGridNBA g4 + bo + bi (0 <= bi < NBI) of each lane-set, so the
// accumulators stay at 16 NBI NR per lane; kGridNBA / NBI blocks with
// bo = 0, NBI, ... cover the lane-set.  `rres` holds the residual records
// [n_vis][NR]; side r goes to out + r rstride.
template <int NR, int NBI>
__device__ __forceinline__ void grid_adj_delta_pairs_multi_tile(
    const VisRecD<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ nu,
    const int32_t* __restrict__ slot, int na, const GridPairBlock& pb, int bo, int64_t kc,
    int64_t kchunk, int64_t n_vis, float* __restrict__ out, int64_t rstride,
    float4 (*bsh)[kGridMaxGL][NBI]) {
  static_assert(kGridNBA % NBI == 0, "NBI divides the cells of a lane-set");
  const PairLane pl = pair_lane(pb, na);
  const double l = la[pl.ia];
  double nuv[NBI];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi) nuv[bi] = pl.active ? nu[pl.qbase + bo + bi] : 0.0;
  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const ConstPtr<float> cres = as_const(reinterpret_cast<const float*>(rres));
  const double origin = kMagic;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float o[NBI][NR][8];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) o[bi][r][j] = 0.0f;
  const FillSlot fs = fill_slot(pb.n_gl * NBI);
  const int fgg = fs.slot / NBI, fbi = fs.slot % NBI;
  const double fm = fs.on ? mb[(pb.g4 + fgg) * kGridNBA + bo + fbi] : 0.0;
  for (int kb = k0; kb < k1; kb += kGridKBM) {
    __syncthreads();  // the previous batch's reads are done
    if (fs.on) {
      for (int kk = fs.row0; kk < kGridKBM; kk += fs.step) {
        const int k = kb + kk;
        float bc = 0.0f, bs = 0.0f, ac = 0.0f, as = 0.0f;
        if (k < k1) {
          phasor(fma(vv[k], fm, origin), bc, bs);
          phasor(fma(vu[k], fm, origin), ac, as);
        }
        bsh[kk][fgg][fbi] = make_float4(bc, bs, ac, as);
      }
    }
    __syncthreads();
    const int ke = kb + kGridKBM < k1 ? kb + kGridKBM : k1;
    float (&G)[NBI][NR][8] = o;  // one running sum per chunk, as the single tile
    for (int k = kb; k < ke; ++k) {
      const double u = cvrec[k].u, v = cvrec[k].v, w = cvrec[k].w;
      float rr[NR], ri[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rr[r] = cres[2 * (static_cast<int64_t>(k) * NR + r)];
        ri[r] = cres[2 * (static_cast<int64_t>(k) * NR + r) + 1];
      }
      float ac, as, qc, qs;  // A and B at index ia
      phasor(fma(u, l, origin), ac, as);
      phasor(fma(v, l, origin), qc, qs);
      const float4* bp = &bsh[k - kb][pl.gl][0];
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) {
        const float4 bb = bp[bi];  // B at b (x, y), A at b (z, w)
        float cc, cs;              // C
        phasor(fma(w, nuv[bi], origin), cc, cs);
        // cell (ia, b): A at ia, B at b; cell (b, ia): A at b, B at ia
        const float p0 = bb.x * ac, p1 = bb.y * as, p2 = bb.y * ac, p3 = bb.x * as;
        const float p4 = qc * bb.z, p5 = qs * bb.w, p6 = qs * bb.z, p7 = qc * bb.w;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const float z1 = fmaf(cc, rr[r], -cs * ri[r]);
          const float z2 = fmaf(cc, ri[r], cs * rr[r]);
          float* g = G[bi][r];
          g[0] = fmaf(p0, z1, g[0]);
          g[1] = fmaf(p1, z1, g[1]);
          g[2] = fmaf(p2, z2, g[2]);
          g[3] = fmaf(p3, z2, g[3]);
          g[4] = fmaf(p4, z1, g[4]);
          g[5] = fmaf(p5, z1, g[5]);
          g[6] = fmaf(p6, z2, g[6]);
          g[7] = fmaf(p7, z2, g[7]);
        }
      }
    }
  }
  if (!pl.active) return;
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
    for (int r = 0; r < NR; ++r) pair_write(pl, na, bo + bi, o[bi][r], slot, out + r * rstride);
}

// `vrec` and `rres` are the layer's records and residuals (D (1 - i s) conj(G) r);
// LDS holds conj(b+-) r per visibility of the batch and |m| value.
__device__ __forceinline__ void grid_adj_gauss_tile(
    const VisRecG<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ la, const double* __restrict__ mb, const double* __restrict__ r2c,
    const double* __restrict__ kapc, const int32_t* __restrict__ slot, int na, int ng4,
    int64_t blk, int64_t kc, int64_t kchunk, int64_t n_vis, float* __restrict__ out_row,
    float4 (*bsh)[kGridMaxGL][kGridNBA]) {
  const LaneSet ls = lane_set(blk, na, ng4);
  const double l = la[ls.ia];
  const float lr = static_cast<float>(l);
  double r2[kGridNBA], kap[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    r2[bi] = ls.active ? r2c[ls.qbase + bi] : 0.0;
    kap[bi] = ls.active ? kapc[ls.qbase + bi] : 0.0;
  }
  const ConstPtr<VisRecG<float>> crec = as_const(vrec);
  const double origin = kMagic;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float og[kGridNBA][4];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi)
#pragma unroll
    for (int s = 0; s < 4; ++s) og[bi][s] = 0.0f;
  const FillSlot fs = fill_slot(ls.n_gl * kGridNBA);
  const int fgg = fs.slot / kGridNBA, fbi = fs.slot % kGridNBA;
  const double m = fs.on ? mb[(ls.gl0 + fgg) * kGridNBA + fbi] : 0.0;
  const float mr = static_cast<float>(m);
  for (int kb = k0; kb < k1; kb += kGridKBG) {
    __syncthreads();
    if (fs.on) {
      for (int kk = fs.row0; kk < kGridKBG; kk += fs.step) {
        const int k = kb + kk;
        float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (k < k1) {
          float cb, sb;
          phasor(fma(vrec[k].B, m, origin), cb, sb);
          const float w = vrec[k].wr, v = vrec[k].vr, c = vrec[k].c1;
          const float dp = fmaf(-w, mr, v), dm = fmaf(w, mr, v);
          const float tp = pow2(c * (dp * dp)), tm = pow2(c * (dm * dm));
          // conj(b+-) r: the residual rides on the block's factors
          const float2 rk = rres[k];  // per-lane index: a vector load
          const float rr = rk.x, ri = rk.y;
          const float p = cb * rr, q = sb * ri, s = cb * ri, t = sb * rr;
          val = make_float4(tp * (p + q), tp * (s - t), tm * (p - q), tm * (s + t));
        }
        bsh[kk][fgg][fbi] = val;
      }
    }
    __syncthreads();
    const int ke = kb + kGridKBG < k1 ? kb + kGridKBG : k1;
    float g[kGridNBA][4];
#pragma unroll
    for (int bi = 0; bi < kGridNBA; ++bi)
#pragma unroll
      for (int s = 0; s < 4; ++s) g[bi][s] = 0.0f;
    for (int k = kb; k < ke; ++k) {
      const double A = crec[k].A, C = crec[k].C, NW = crec[k].NW, E0 = crec[k].E0;
      const float ur = crec[k].ur, wr = crec[k].wr, c1 = crec[k].c1;
      float ca, sa;
      phasor(fma(A, l, origin), ca, sa);
      const float dp = fmaf(-wr, lr, ur), dm = fmaf(wr, lr, ur);
      const float tp = pow2(c1 * (dp * dp)), tm = pow2(c1 * (dm * dm));
      const float apr = tp * ca, api = tp * sa, amr = tm * ca, ami = -tm * sa;
      const float4* bp = &bsh[k - kb][ls.gl][0];
#pragma unroll
      for (int bi = 0; bi < kGridNBA; ++bi) {
        const float4 bb = bp[bi];  // conj(b+-) r
        float cg, sg;
        phasor(fma(C, r2[bi], fma(NW, kap[bi], E0)), cg, sg);
        // Y+- = conj(P) conj(b+-) r
        const float ypr = fmaf(cg, bb.x, sg * bb.y), ypi = fmaf(cg, bb.y, -sg * bb.x);
        const float ymr = fmaf(cg, bb.z, sg * bb.w), ymi = fmaf(cg, bb.w, -sg * bb.z);
        g[bi][0] = fmaf(apr, ypr, fmaf(api, ypi, g[bi][0]));
        g[bi][1] = fmaf(amr, ypr, fmaf(ami, ypi, g[bi][1]));
        g[bi][2] = fmaf(apr, ymr, fmaf(api, ymi, g[bi][2]));
        g[bi][3] = fmaf(amr, ymr, fmaf(ami, ymi, g[bi][3]));
      }
    }
#pragma unroll
    for (int bi = 0; bi < kGridNBA; ++bi)
#pragma unroll
      for (int s = 0; s < 4; ++s) og[bi][s] += g[bi][s];
  }
  grid_write(ls, slot, og, out_row);
}

// Square Gaussian grid, pair blocks (GridPairBlock): lane-set (g4, ia) owns
// the cells (ia, b) and mirrors (b, ia), b = kGridNBA g4 + bi.  LDS holds, per
// visibility of the batch and |m| value of the block's groups, the cells'
// conj(b+-) r and the mirrors' conj(a+-) r (both at that value, the residual
// multiplied in once by the block instead of once per cell by every lane);
// the lane forms a+- at |l|_ia for its cells and b+- at |m|_ia for its
// mirrors.  Writes as for the delta pair blocks.  `vrec`, `rres` are the
// layer's.
__device__ __forceinline__ void grid_adj_gauss_pairs_tile(
    const VisRecG<float>* __restrict__ vrec, const float2* __restrict__ rres,
    const double* __restrict__ la, const double* __restrict__ mb, const double* __restrict__ r2c,
    const double* __restrict__ kapc, const int32_t* __restrict__ slot, int na,
    const GridPairBlock& pb, int64_t kc, int64_t kchunk, int64_t n_vis,
    float* __restrict__ out_row, float4 (*bsh)[kGridMaxGL][kGridNBA][2]) {
  const PairLane pl = pair_lane(pb, na);
  const bool active = pl.active;
  const int g4 = pl.g4, ia = pl.ia, gl = pl.gl, qbase = pl.qbase;
  const double l = la[ia];
  const float lr = static_cast<float>(l);
  double r2[kGridNBA], kap[kGridNBA];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    r2[bi] = active ? r2c[qbase + bi] : 0.0;
    kap[bi] = active ? kapc[qbase + bi] : 0.0;
  }
  const ConstPtr<VisRecG<float>> crec = as_const(vrec);
  const double origin = kMagic;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  float o[kGridNBA][8];
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi)
#pragma unroll
    for (int j = 0; j < 8; ++j) o[bi][j] = 0.0f;
  const FillSlot fs = fill_slot(pb.n_gl * kGridNBA);
  const int fgg = fs.slot / kGridNBA, fbi = fs.slot % kGridNBA;
  const double m = fs.on ? mb[(pb.g4 + fgg) * kGridNBA + fbi] : 0.0;
  const float mr = static_cast<float>(m);
  for (int kb = k0; kb < k1; kb += kGridKBG) {
    __syncthreads();
    if (fs.on) {
      for (int kk = fs.row0; kk < kGridKBG; kk += fs.step) {
        const int k = kb + kk;
        float4 bv = make_float4(0.0f, 0.0f, 0.0f, 0.0f), av = bv;
        if (k < k1) {
          const float w = vrec[k].wr, c = vrec[k].c1;
          float cb, sb, ca, sa;
          phasor(fma(vrec[k].B, m, origin), cb, sb);
          phasor(fma(vrec[k].A, m, origin), ca, sa);
          const float dvp = fmaf(-w, mr, vrec[k].vr), dvm = fmaf(w, mr, vrec[k].vr);
          const float dup = fmaf(-w, mr, vrec[k].ur), dum = fmaf(w, mr, vrec[k].ur);
          const float tvp = pow2(c * (dvp * dvp)), tvm = pow2(c * (dvm * dvm));
          const float tup = pow2(c * (dup * dup)), tum = pow2(c * (dum * dum));
          // the residual rides on the block's factors: conj(b+-) r for the
          // cell, conj(a+-) r for the mirror
          const float2 rk = rres[k];  // per-lane index: a vector load
          const float rr = rk.x, ri = rk.y;
          const float bp = cb * rr, bq = sb * ri, bs_ = cb * ri, bt = sb * rr;
          const float ap = ca * rr, aq = sa * ri, as_ = ca * ri, at = sa * rr;
          bv = make_float4(tvp * (bp + bq), tvp * (bs_ - bt), tvm * (bp - bq), tvm * (bs_ + bt));
          av = make_float4(tup * (ap + aq), tup * (as_ - at), tum * (ap - aq), tum * (as_ + at));
        }
        bsh[kk][fgg][fbi][0] = bv;
        bsh[kk][fgg][fbi][1] = av;
      }
    }
    __syncthreads();
    const int ke = kb + kGridKBG < k1 ? kb + kGridKBG : k1;
    float (&G)[kGridNBA][8] = o;  // one running sum per chunk, as the delta pair tile
    for (int k = kb; k < ke; ++k) {
      const double A = crec[k].A, B = crec[k].B, C = crec[k].C, NW = crec[k].NW, E0 = crec[k].E0;
      const float ur = crec[k].ur, vr = crec[k].vr, wr = crec[k].wr, c1 = crec[k].c1;
      float ca, sa, cb, sb;
      phasor(fma(A, l, origin), ca, sa);
      phasor(fma(B, l, origin), cb, sb);
      const float dup = fmaf(-wr, lr, ur), dum = fmaf(wr, lr, ur);
      const float dvp = fmaf(-wr, lr, vr), dvm = fmaf(wr, lr, vr);
      const float tup = pow2(c1 * (dup * dup)), tum = pow2(c1 * (dum * dum));
      const float tvp = pow2(c1 * (dvp * dvp)), tvm = pow2(c1 * (dvm * dvm));
      const float apr = tup * ca, api = tup * sa, amr = tum * ca, ami = -tum * sa;  // cell a+-
      const float qpr = tvp * cb, qpi = tvp * sb, qmr = tvm * cb, qmi = -tvm * sb;  // mirror b+-
#pragma unroll
      for (int bi = 0; bi < kGridNBA; ++bi) {
        const float4 bb = bsh[k - kb][gl][bi][0];  // cell: conj(b+-) r at |m|_b
        const float4 ma = bsh[k - kb][gl][bi][1];  // mirror: conj(a+-) r at |l|_b
        float cg, sg;
        phasor(fma(C, r2[bi], fma(NW, kap[bi], E0)), cg, sg);
        // cell: Y+- = conj(P) conj(b+-) r, g = Re conj(a) Y
        const float ypr = fmaf(cg, bb.x, sg * bb.y), ypi = fmaf(cg, bb.y, -sg * bb.x);
        const float ymr = fmaf(cg, bb.z, sg * bb.w), ymi = fmaf(cg, bb.w, -sg * bb.z);
        G[bi][0] = fmaf(apr, ypr, fmaf(api, ypi, G[bi][0]));
        G[bi][1] = fmaf(amr, ypr, fmaf(ami, ypi, G[bi][1]));
        G[bi][2] = fmaf(apr, ymr, fmaf(api, ymi, G[bi][2]));
        G[bi][3] = fmaf(amr, ymr, fmaf(ami, ymi, G[bi][3]));
        // mirror: T+- = conj(P) conj(a+-) r, g' = Re conj(qb) T
        const float tpr = fmaf(cg, ma.x, sg * ma.y), tpi = fmaf(cg, ma.y, -sg * ma.x);
        const float tmr = fmaf(cg, ma.z, sg * ma.w), tmi = fmaf(cg, ma.w, -sg * ma.z);
        G[bi][4] = fmaf(qpr, tpr, fmaf(qpi, tpi, G[bi][4]));
        G[bi][5] = fmaf(qpr, tmr, fmaf(qpi, tmi, G[bi][5]));
        G[bi][6] = fmaf(qmr, tpr, fmaf(qmi, tpi, G[bi][6]));
        G[bi][7] = fmaf(qmr, tmr, fmaf(qmi, tmi, G[bi][7]));
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int bi = 0; bi < kGridNBA; ++bi) {
    const int64_t q = qbase + bi;
    const int b = kGridNBA * g4 + bi;
    const int64_t qp = (static_cast<int64_t>(ia / kGridNB) * na + b) * kGridNB + ia % kGridNB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 0 ? b > ia : b >= ia) continue;
      const int64_t qq = h ? qp : q;
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int32_t j = slot[4 * qq + s2];
        if (j >= 0) out_row[j] = o[bi][4 * h + s2];
      }
    }
  }
}

}  // namespace dev
}  // namespace sl1m
