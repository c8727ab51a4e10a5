// C ABI of the SL1M library: plans, operator calls, power iteration, FISTA.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "sl1m_internal.h"
#include "sl1m_trace.h"

namespace sl1m {

namespace {
thread_local std::string g_last_error;

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Everything about a problem that the host needs before any device buffer
// exists: the grouping of pixels into (kind, sigma) segments, the permutation
// into that order, gain flags and the tiling of both operators.
struct Analysis {
  int64_t n_pix = 0, n_vis = 0;
  int precision = SL1M_PREC_FP32;
  int max_rhs = 1;
  size_t rb = 4;
  std::vector<int32_t> perm;  // empty = identity
  std::vector<Segment> segs;
  std::vector<double> layer_sigma;
  bool has_gain = false, beam_pair = false;
  double beam_coef = 0.0;     // separable beam: scale *= 2^(beam_coef r^2)
  int fwd_vpl = 4, adj_ppl = 4;
  std::vector<Chunk> fd, fg, pd, pg;
  int64_t kchunk = 0;
  int n_achunks = 0;
  bool grid_mfma = false;     // matrix-core plan on one square delta grid (forward)
  int n_mfchunks = 0;         // matrix-core plans: forward chunks of mf_chunk pixels
  int64_t mf_chunk = 0, mf_np4 = 0, mf_nv4 = 0;
  // grid evaluation: segments on the grid path, their concatenated tables,
  // and the direct chunks of the other segments
  bool grid = false;
  int grid_multi = 0;  // largest multi-RHS count (2, 4 or 8) on the grid path; 0: none
  std::vector<GridSeg> gsegs;
  int64_t grid_cells = 0;
  std::vector<double> grid_la, grid_mb, grid_c3, grid_c4;
  std::vector<int32_t> grid_slot;
  std::vector<GridChunk> grid_fc;
  std::vector<GridPairBlock> grid_pb;
  std::vector<int2> grid_gb;   // Gaussian adjoint blocks (segment, block)
  int64_t grid_pairs = 0;      // pair records of all square segments
  int grid_vtiles = 0, grid_frows = 0;
  std::vector<Chunk> fd1, fg1, pd1, pg1;
};

sl1m_status d2h(void* dst, const void* src, size_t bytes, const char* what) {
  if (bytes == 0) return SL1M_OK;
  hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(e, what);
  return SL1M_OK;
}

size_t pixrec_bytes(size_t rb) { return rb == 8 ? sizeof(PixRec<double>) : sizeof(PixRec<float>); }
size_t visrecD_bytes(size_t rb) {
  return rb == 8 ? sizeof(VisRecD<double>) : sizeof(VisRecD<float>);
}
size_t visrecG_bytes(size_t rb) {
  return rb == 8 ? sizeof(VisRecG<double>) : sizeof(VisRecG<float>);
}

// Decides whether the pixels of segment `si` (in permuted order) qualify for
// the grid evaluation and, if so, appends its tables to the analysis: the
// distinct |l| and |m| values, per cell n - 1 (delta) or l^2 + m^2 and kappa
// (Gaussian), and the permuted pixel index of every occupied sign slot.
// Returns false with a reason when they do not qualify.  L and M hold the
// caller's l and m (host copies).
bool analyze_grid(Analysis& a, int si, const std::vector<double>& L, const std::vector<double>& M,
                  std::string& why) {
  const Segment& sg = a.segs[si];
  if (a.precision == SL1M_PREC_FP64) return why = "the plan is float64", false;
  if (a.precision == SL1M_PREC_FP32_HILO) return why = "the plan's phase is float32 hi/lo", false;
  if (a.beam_pair) return why = "the plan has per-pair beams", false;
  if (sg.count < 1024) return why = "fewer than 1024 pixels in the segment", false;
  const int64_t nd = sg.count;
  std::vector<double> al(nd), am(nd);
  for (int64_t t = 0; t < nd; ++t) {
    const int64_t o = a.perm.empty() ? sg.start + t : a.perm[sg.start + t];
    if (!std::isfinite(L[o]) || !std::isfinite(M[o])) return why = "non-finite position", false;
    al[t] = std::fabs(L[o]);
    am[t] = std::fabs(M[o]);
  }
  std::vector<double> ul(al), um(am);
  std::sort(ul.begin(), ul.end());
  ul.erase(std::unique(ul.begin(), ul.end()), ul.end());
  std::sort(um.begin(), um.end());
  um.erase(std::unique(um.begin(), um.end()), um.end());
  const int64_t na = static_cast<int64_t>(ul.size()), nb = static_cast<int64_t>(um.size());
  if (na < kGridMinA) return why = "fewer than 16 distinct |l| values", false;
  const int64_t ng = (nb + kGridNB - 1) / kGridNB;
  const int64_t cells = ng * kGridNB * na;
  if (2 * 4 * cells > 5 * nd) return why = "the pixels fill less than 40% of their grid", false;
  if (4 * (a.grid_cells + cells) > INT32_MAX) return why = "grid too large", false;
  std::vector<int32_t> slot(4 * cells, -1);
  for (int64_t t = 0; t < nd; ++t) {
    const int64_t j = sg.start + t;  // permuted index
    const int64_t o = a.perm.empty() ? j : a.perm[j];
    const int64_t ia = std::lower_bound(ul.begin(), ul.end(), al[t]) - ul.begin();
    const int64_t ib = std::lower_bound(um.begin(), um.end(), am[t]) - um.begin();
    const int sgn = (L[o] < 0.0 ? 1 : 0) + (M[o] < 0.0 ? 2 : 0);
    const int64_t q = ((ib / kGridNB) * na + ia) * kGridNB + ib % kGridNB;
    int32_t& sl = slot[4 * q + sgn];
    if (sl >= 0) return why = "two pixels of the segment share a position", false;
    sl = static_cast<int32_t>(j);
  }
  GridSeg g{};
  g.seg = si;
  g.square = ul == um ? 1 : 0;
  g.kind = sg.kind;
  g.layer = sg.layer;
  g.na = static_cast<int32_t>(na);
  g.nb = static_cast<int32_t>(nb);
  g.ng = static_cast<int32_t>(ng);
  g.cells = cells;
  g.la_off = static_cast<int64_t>(a.grid_la.size());
  g.mb_off = static_cast<int64_t>(a.grid_mb.size());
  g.cell_off = a.grid_cells;
  a.grid_la.insert(a.grid_la.end(), ul.begin(), ul.end());
  std::vector<double> mbp(ng * kGridNB, 0.0);
  std::copy(um.begin(), um.end(), mbp.begin());
  a.grid_mb.insert(a.grid_mb.end(), mbp.begin(), mbp.end());
  a.grid_c3.resize(a.grid_cells + cells, 0.0);
  a.grid_c4.resize(a.grid_cells + cells, 0.0);
  for (int64_t gi = 0; gi < ng; ++gi)
    for (int64_t ia = 0; ia < na; ++ia)
      for (int b = 0; b < kGridNB; ++b) {
        const double l = ul[ia], m = mbp[gi * kGridNB + b];
        const double r2 = l * l + m * m;
        const int64_t q = a.grid_cells + (gi * na + ia) * kGridNB + b;
        // n - 1 = -r^2 / (1 + n), kappa = n - 1 + r^2/2 = -r^4 / (2 (1 + n)^2);
        // cells outside the unit disk stay 0 (the domain check rejects any
        // pixel there)
        if (!(r2 < 1.0)) continue;
        const double n = std::sqrt(1.0 - r2);
        if (sg.kind == SL1M_PIX_DELTA) {
          a.grid_c3[q] = -r2 / (1.0 + n);
        } else {
          a.grid_c3[q] = r2;
          a.grid_c4[q] = sg.kind == SL1M_PIX_GAUSS_WIDE ? -(r2 * r2) / (2.0 * (1.0 + n) * (1.0 + n)) : 0.0;
        }
      }
  a.grid_slot.insert(a.grid_slot.end(), slot.begin(), slot.end());
  a.grid_cells += cells;
  a.gsegs.push_back(g);
  a.grid = true;
  return true;
}

sl1m_status analyze(const sl1m_problem* pr, Analysis& a) {
  if (!pr) return set_error(SL1M_EINVAL, "problem is NULL");
  if (pr->n_pix < 0 || pr->n_vis < 0) return set_error(SL1M_EINVAL, "negative size");
  if (pr->n_pix > INT32_MAX || pr->n_vis > INT32_MAX)
    return set_error(SL1M_EINVAL, "n_pix and n_vis must be below 2^31");
  if (pr->precision < SL1M_PREC_FP64 || pr->precision > SL1M_PREC_FP32_HILO)
    return set_error(SL1M_EINVAL, "unknown precision");
  const bool mfma = pr->precision == SL1M_PREC_MFMA_F16 || pr->precision == SL1M_PREC_MFMA_BF16;
  if (pr->n_pix > 0 && (!pr->l || !pr->m)) return set_error(SL1M_EINVAL, "l or m is NULL");
  if (pr->n_vis > 0 && (!pr->u || !pr->v || !pr->w))
    return set_error(SL1M_EINVAL, "u, v or w is NULL");
  if (pr->max_rhs != 0 && pr->max_rhs != 1 && pr->max_rhs != 2 && pr->max_rhs != 4 &&
      pr->max_rhs != 8)
    return set_error(SL1M_EINVAL, "max_rhs must be 0, 1, 2, 4 or 8");
  a.n_pix = pr->n_pix;
  a.n_vis = pr->n_vis;
  a.max_rhs = pr->max_rhs > 0 ? pr->max_rhs : 1;
  a.precision = pr->precision;
  a.rb = pr->precision == SL1M_PREC_FP64 ? 8 : 4;
  const int64_t np = pr->n_pix;

  // ---- pixel kinds and scales -> segments
  std::vector<uint8_t> kind;
  std::vector<double> sigma;
  if (np > 0 && (pr->sigma || pr->kind)) {
    if (pr->sigma) {
      sigma.resize(np);
      sl1m_status s = d2h(sigma.data(), pr->sigma, np * sizeof(double), "read sigma");
      if (s) return s;
    }
    if (pr->kind) {
      kind.resize(np);
      sl1m_status s = d2h(kind.data(), pr->kind, np, "read kind");
      if (s) return s;
    }
  }
  a.segs.clear();
  a.layer_sigma.clear();
  if (kind.empty() && sigma.empty()) {
    a.segs.push_back(Segment{0, np, SL1M_PIX_DELTA, 0.0, -1});
  } else {
    // key: (kind, sigma) for Gaussian pixels; all delta pixels share one group
    std::map<std::pair<int, double>, std::vector<int32_t>> groups;
    std::vector<int32_t> deltas;
    for (int64_t j = 0; j < np; ++j) {
      const double s = sigma.empty() ? 0.0 : sigma[j];
      int k;
      if (!kind.empty()) {
        k = kind[j];
        if (k > SL1M_PIX_GAUSS_WIDE) return set_error(SL1M_EINVAL, "pixel kind out of range");
      } else {
        k = s > 0.0 ? SL1M_PIX_GAUSS_WIDE : SL1M_PIX_DELTA;
      }
      if (!(s >= 0.0) || !std::isfinite(s))
        return set_error(SL1M_EDOMAIN, "sigma must be finite and >= 0");
      if (k == SL1M_PIX_DELTA)
        deltas.push_back(static_cast<int32_t>(j));
      else
        groups[{k, s}].push_back(static_cast<int32_t>(j));
    }
    if (static_cast<int>(groups.size()) > kMaxLayers)
      return set_error(SL1M_EINVAL, "more than 16 distinct (kind, sigma) Gaussian pixel groups");
    a.perm.reserve(np);
    a.perm.insert(a.perm.end(), deltas.begin(), deltas.end());
    a.segs.push_back(Segment{0, static_cast<int64_t>(deltas.size()), SL1M_PIX_DELTA, 0.0, -1});
    int layer = 0;
    for (auto& g : groups) {
      Segment s{static_cast<int64_t>(a.perm.size()), static_cast<int64_t>(g.second.size()),
                g.first.first, g.first.second, layer++};
      a.perm.insert(a.perm.end(), g.second.begin(), g.second.end());
      a.segs.push_back(s);
      a.layer_sigma.push_back(g.first.second);
    }
    bool identity = true;
    for (int64_t j = 0; j < np && identity; ++j) identity = a.perm[j] == j;
    if (identity) a.perm.clear();
  }
  const bool hilo = pr->precision == SL1M_PREC_FP32_HILO;
  if (mfma && a.segs.size() != 1)
    return set_error(SL1M_EINVAL, "the MFMA precisions evaluate delta pixels only");
  if (hilo && a.segs.size() != 1)
    return set_error(SL1M_EINVAL, "the FP32 hi/lo phase evaluates delta pixels only");

  // ---- gains
  a.has_gain = pr->ant_p != nullptr && pr->n_vis > 0;
  a.beam_pair = false;
  a.beam_coef = 0.0;
  if (a.has_gain) {
    if (!pr->ant_q) return set_error(SL1M_EINVAL, "ant_p given without ant_q");
    if (pr->n_ant <= 0) return set_error(SL1M_EINVAL, "n_ant must be > 0 with antenna indices");
    std::vector<int32_t> ap(pr->n_vis), aq(pr->n_vis);
    sl1m_status s = d2h(ap.data(), pr->ant_p, pr->n_vis * 4, "read ant_p");
    if (s) return s;
    s = d2h(aq.data(), pr->ant_q, pr->n_vis * 4, "read ant_q");
    if (s) return s;
    for (int64_t k = 0; k < pr->n_vis; ++k)
      if (ap[k] < 0 || ap[k] >= pr->n_ant || aq[k] < 0 || aq[k] >= pr->n_ant)
        return set_error(SL1M_EINVAL, "antenna index out of range");
    if (pr->ant_fwhm) {
      std::vector<double> F(pr->n_ant);
      s = d2h(F.data(), pr->ant_fwhm, pr->n_ant * sizeof(double), "read ant_fwhm");
      if (s) return s;
      bool equal = true;
      for (double f : F) {
        if (!(f > 0.0) || !std::isfinite(f))
          return set_error(SL1M_EDOMAIN, "ant_fwhm must be finite and > 0");
        equal = equal && f == F[0];
      }
      if (equal)
        a.beam_coef = -4.0 / (F[0] * F[0]);  // E_p conj(E_q) beam = 2^(-4 r^2 / F^2)
      else
        a.beam_pair = true;
    }
  }
  if (mfma && a.beam_pair)
    return set_error(SL1M_EINVAL, "the MFMA precisions need one beam width for all antennas");
  if (hilo && a.beam_pair)
    return set_error(SL1M_EINVAL, "the FP32 hi/lo phase needs one beam width for all antennas");

  // ---- tiling
  const int64_t nv = pr->n_vis;
  auto lane_ok = [](int32_t v) { return v == 0 || v == 1 || v == 2 || v == 4; };
  if (!lane_ok(pr->fwd_vpl) || !lane_ok(pr->adj_ppl))
    return set_error(SL1M_EINVAL, "fwd_vpl and adj_ppl must be 0, 1, 2 or 4");
  a.fwd_vpl = nv >= 64LL * kBlock * 4 ? 4 : (nv >= 32LL * kBlock * 2 ? 2 : 1);
  if (pr->fwd_vpl) a.fwd_vpl = pr->fwd_vpl;
  if (a.beam_pair) a.fwd_vpl = 4;  // the per-pair-beam kernels exist for 4 per lane only
  const int64_t vtiles = (nv + kBlock * a.fwd_vpl - 1) / (kBlock * a.fwd_vpl);
  const int64_t target_blocks = pr->tile_blocks > 0 ? pr->tile_blocks : 4096;
  if (pr->tile_blocks < 0) return set_error(SL1M_EINVAL, "tile_blocks must be >= 0");
  int64_t target_chunks = vtiles > 0 ? (target_blocks + vtiles - 1) / vtiles : 1;
  target_chunks = std::max<int64_t>(1, std::min<int64_t>(64, target_chunks));
  const int64_t cp = std::max<int64_t>(64, (np + target_chunks - 1) / std::max<int64_t>(1, target_chunks));
  a.fd.clear();
  a.fg.clear();
  for (size_t si = 0; si < a.segs.size(); ++si) {
    const Segment& s = a.segs[si];
    for (int64_t j = s.start; j < s.start + s.count; j += cp) {
      Chunk c{j, std::min(j + cp, s.start + s.count), s.sigma, static_cast<int32_t>(si), s.layer};
      (s.kind == SL1M_PIX_DELTA ? a.fd : a.fg).push_back(c);
    }
  }
  if (nv == 0) {
    a.fd.clear();
    a.fg.clear();
  }
  a.adj_ppl = np >= 64LL * kBlock * 4 ? 4 : (np >= 32LL * kBlock * 2 ? 2 : 1);
  if (pr->adj_ppl) a.adj_ppl = pr->adj_ppl;
  if (a.beam_pair) a.adj_ppl = 4;
  const int64_t tp = static_cast<int64_t>(kBlock) * a.adj_ppl;
  a.pd.clear();
  a.pg.clear();
  for (size_t si = 0; si < a.segs.size(); ++si) {
    const Segment& s = a.segs[si];
    for (int64_t j = s.start; j < s.start + s.count; j += tp) {
      Chunk c{j, std::min(j + tp, s.start + s.count), s.sigma, static_cast<int32_t>(si), s.layer};
      (s.kind == SL1M_PIX_DELTA ? a.pd : a.pg).push_back(c);
    }
  }
  // ---- grid evaluation, segment by segment
  if (pr->grid_mode < SL1M_GRID_AUTO || pr->grid_mode > SL1M_GRID_REQUIRE)
    return set_error(SL1M_EINVAL, "unknown grid_mode");
  a.grid = false;
  if (pr->grid_mode != SL1M_GRID_OFF && nv > 0 && np > 0) {
    std::string why = "no segment has 1024 pixels";
    if (a.precision == SL1M_PREC_FP64) why = "the plan's precision is SL1M_PREC_FP64";
    else if (a.precision == SL1M_PREC_FP32_HILO) why = "the plan's phase is float32 hi/lo";
    else if (a.beam_pair) why = "the plan has per-pair beams";
    bool any_big = false;
    for (const Segment& sg : a.segs) any_big = any_big || sg.count >= 1024;
    if (any_big && a.precision != SL1M_PREC_FP64 && a.precision != SL1M_PREC_FP32_HILO &&
        !a.beam_pair) {
      std::vector<double> L(np), M(np);
      if (sl1m_status e = d2h(L.data(), pr->l, np * sizeof(double), "read l")) return e;
      if (sl1m_status e = d2h(M.data(), pr->m, np * sizeof(double), "read m")) return e;
      for (int si = 0; si < static_cast<int>(a.segs.size()); ++si) {
        std::string w;
        if (!analyze_grid(a, si, L, M, w) && a.segs[si].count >= 1024) why = w;
      }
    }
    if (!a.grid && pr->grid_mode == SL1M_GRID_REQUIRE)
      return set_error(SL1M_EINVAL, "grid evaluation required but " + why);
  }
  if (a.grid) {
    std::vector<char> on(a.segs.size(), 0);
    for (const GridSeg& g : a.gsegs) on[g.seg] = 1;
    a.fd1.clear();
    a.fg1.clear();
    a.pd1.clear();
    a.pg1.clear();
    for (const Chunk& c : a.fd) if (!on[c.seg]) a.fd1.push_back(c);
    for (const Chunk& c : a.fg) if (!on[c.seg]) a.fg1.push_back(c);
    for (const Chunk& c : a.pd) if (!on[c.seg]) a.pd1.push_back(c);
    for (const Chunk& c : a.pg) if (!on[c.seg]) a.pg1.push_back(c);
    a.grid_vtiles = static_cast<int>((nv + kGridVPL * kBlock - 1) / (kGridVPL * kBlock));
    int64_t ng_total = 0;
    for (const GridSeg& g : a.gsegs) ng_total += g.ng;
    const int64_t per_split = static_cast<int64_t>(a.grid_vtiles) * ng_total;
    a.grid_fc.clear();
    a.grid_pb.clear();
    a.grid_pairs = 0;
    for (GridSeg& g : a.gsegs) {
      int64_t split = (target_blocks + per_split - 1) / per_split;
      split = std::max<int64_t>(1, std::min<int64_t>(split, (g.na + 7) / 8));
      const int ra = static_cast<int>((g.na + split - 1) / split);
      g.fc0 = static_cast<int32_t>(a.grid_fc.size());
      if (!g.square) {
        for (int gi = 0; gi < g.ng; ++gi)
          for (int i0 = 0; i0 < g.na; i0 += ra)
            a.grid_fc.push_back(GridChunk{gi, i0, std::min<int>(g.na, i0 + ra), 0});
        g.nfs = static_cast<int32_t>(a.grid_fc.size()) - g.fc0;
        const int64_t sets = static_cast<int64_t>(2) * g.ng * g.na;
        g.ablocks = static_cast<int32_t>((sets + kBlock - 1) / kBlock);
        g.pblocks = 0;
      } else {
        // forward: pair records of the |l| values from each group's first one
        // on, in ranges of about half the single-cell split (a pair is two
        // cells of work)
        g.nfs = 0;
        const int rp = std::max(8, ra / 2);
        for (int gi = 0; gi < g.ng; ++gi)
          for (int i0 = kGridNB * gi; i0 < g.na; i0 += rp)
            a.grid_fc.push_back(GridChunk{gi, i0, std::min<int>(g.na, i0 + rp), 0});
        // adjoint: pair blocks of the rows g4 (ia from kGridNBA g4 to na), at
        // most kBlock lane-sets and kGridMaxGL groups each
        g.ablocks = 0;
        g.pb0 = static_cast<int32_t>(a.grid_pb.size());
        GridPairBlock cur{0, 0, 0, 0};
        for (int g4 = 0; g4 < 2 * g.ng; ++g4) {
          for (int pos = kGridNBA * g4; pos < g.na;) {
            if (cur.count == kBlock || (cur.count > 0 && g4 - cur.g4 + 1 > kGridMaxGL)) {
              a.grid_pb.push_back(cur);
              cur = GridPairBlock{0, 0, 0, 0};
            }
            if (cur.count == 0) {
              cur.g4 = g4;
              cur.ia = pos;
            }
            const int take = std::min(g.na - pos, kBlock - cur.count);
            cur.count += take;
            cur.n_gl = g4 - cur.g4 + 1;
            pos += take;
          }
        }
        if (cur.count > 0) a.grid_pb.push_back(cur);
        g.pblocks = static_cast<int32_t>(a.grid_pb.size()) - g.pb0;
        // pair records of the forward: groups g with kGridNB g < na
        const int gp = (g.na + kGridNB - 1) / kGridNB;
        g.pr_off = a.grid_pairs;
        g.n_pairs = pair_rec_base(gp, g.na);
        a.grid_pairs += g.n_pairs;
      }
      g.nfc = static_cast<int32_t>(a.grid_fc.size()) - g.fc0;
    }
    a.grid_frows = static_cast<int>(a.grid_fc.size());
    // several right-hand sides take the grid path when every grid segment is
    // a square delta grid (pair records with the amplitudes of each side)
    bool all_square_delta = true;
    for (const GridSeg& g : a.gsegs)
      all_square_delta = all_square_delta && g.square && g.kind == SL1M_PIX_DELTA;
    a.grid_multi = all_square_delta ? (a.max_rhs >= 8 ? 8 : a.max_rhs >= 4 ? 4 : a.max_rhs >= 2 ? 2 : 0) : 0;
    a.grid_gb.clear();
    for (int si = 0; si < static_cast<int>(a.gsegs.size()); ++si) {
      const GridSeg& g = a.gsegs[si];
      if (g.kind == SL1M_PIX_DELTA) continue;
      const int nb = g.square ? g.pblocks : g.ablocks;
      for (int b = 0; b < nb; ++b) a.grid_gb.push_back(int2{si, b});
    }
  }

  // matrix-core plans evaluate the forward on the grid when all their pixels
  // form one square delta grid (the adjoint stays on the direct evaluation)
  a.grid_mfma = mfma && a.grid && a.gsegs.size() == 1 && a.gsegs[0].square &&
                a.gsegs[0].kind == SL1M_PIX_DELTA && a.fd1.empty() && a.fg1.empty() &&
                a.pd1.empty() && a.pg1.empty();

  // ---- visibility chunks of the adjoint (shared by all of its kernels)
  // The launches of one adjoint run one after another, so besides the plan's
  // block target every launch should have enough blocks of its own: the
  // smallest launch gets at least kMinLaunchBlocks (grid plans; within the
  // chunk cap), six to eight times the 1024-1280 blocks an MI355X keeps
  // resident of these kernels (4 or 5 wavefronts per SIMD), so that its last,
  // partly filled round is a small part of it.
  constexpr int64_t kMinLaunchBlocks = 8192;
  int64_t ptiles = static_cast<int64_t>(a.pd.size() + a.pg.size());
  int64_t min_launch = 0;
  if (a.grid) {
    ptiles = static_cast<int64_t>(a.pd1.size() + a.pg1.size());
    std::vector<int64_t> launches = {static_cast<int64_t>(a.pd1.size()),
                                     static_cast<int64_t>(a.pg1.size())};
    int64_t gauss = 0;
    for (const GridSeg& g : a.gsegs) {
      ptiles += g.ablocks + g.pblocks;
      if (g.kind == SL1M_PIX_DELTA)
        launches.push_back(g.ablocks + g.pblocks);
      else
        gauss += g.ablocks + g.pblocks;  // one launch for every Gaussian grid segment
    }
    launches.push_back(gauss);
    for (int64_t b : launches)
      if (b > 0) min_launch = min_launch ? std::min(min_launch, b) : b;
  }
  if (nv > 0 && ptiles > 0) {
    const int64_t cap = a.grid ? 256 : 64;
    int64_t want = (target_blocks + ptiles - 1) / ptiles;
    if (min_launch > 0) want = std::max(want, (kMinLaunchBlocks + min_launch - 1) / min_launch);
    want = std::max<int64_t>(1, std::min<int64_t>(cap, want));
    a.kchunk = std::max<int64_t>(64, (nv + want - 1) / want);
    a.n_achunks = static_cast<int>((nv + a.kchunk - 1) / a.kchunk);
  } else {
    a.kchunk = 0;
    a.n_achunks = 0;
  }
  // matrix-core plans: 32-pixel (forward) and 32-visibility (adjoint) steps
  // of 4 x 4 x 4 blocks, fwd_vpl visibilities / adj_ppl pixels per lane;
  // chunks that give each launch kMinLaunchBlocks blocks
  if (mfma) {
    const int64_t grid_kchunk = a.kchunk;
    // lanes per thread: two entries per scalar record load measured best at
    // config 2's shape for 1 to 4 sides, four pixels per lane for 8 sides'
    // adjoint (float16, 65,536 x 97,536)
    if (!pr->fwd_vpl) a.fwd_vpl = nv >= 2LL * 64 * kBlock ? 2 : 1;
    if (!pr->adj_ppl) a.adj_ppl = np >= 2LL * 64 * kBlock ? (a.max_rhs > 4 ? 4 : 2) : 1;
    auto up32 = [](int64_t x) { return (x + 31) / 32 * 32; };
    const int64_t np32 = up32(np), nv32 = up32(nv);
    a.mf_np4 = np32 / 4;
    a.mf_nv4 = nv32 / 4;
    a.n_mfchunks = 0;
    a.mf_chunk = 0;
    a.kchunk = 0;
    a.n_achunks = 0;
    if (np > 0 && nv > 0) {
      const int64_t vt = (nv + kBlock * a.fwd_vpl - 1) / (kBlock * a.fwd_vpl);
      const int64_t nf = std::max<int64_t>(1, std::min<int64_t>(np32 / 32, (kMinLaunchBlocks + vt - 1) / vt));
      a.mf_chunk = up32((np32 + nf - 1) / nf);
      a.n_mfchunks = static_cast<int>((np32 + a.mf_chunk - 1) / a.mf_chunk);
      if (a.grid_mfma && grid_kchunk > 0) {
        // the grid evaluation's visibility chunks (its FP32 adjoint serves up
        // to 4 sides), rounded to the matrix-core adjoint's 32-visibility steps
        a.kchunk = up32(grid_kchunk);
      } else {
        const int64_t pt = (np + kBlock * a.adj_ppl - 1) / (kBlock * a.adj_ppl);
        const int64_t na = std::max<int64_t>(
            1, std::min<int64_t>({256, nv32 / 32, (kMinLaunchBlocks + pt - 1) / pt}));
        a.kchunk = up32((nv32 + na - 1) / na);
      }
      a.n_achunks = static_cast<int>((nv32 + a.kchunk - 1) / a.kchunk);
    }
  }
  return SL1M_OK;
}

struct Layout {
  size_t perm, pixrec, pl, pm, pc3, pc4, pscale, pr2, vu, vv, vw, vgain, vbeta, visrecD, visrecG,
      rres, rpol, layerDs, chunks, fpart, apart, xperm, img, zbuf, res, red, red_out, flag, scal,
      grid_la,
      grid_mb, grid_c3, grid_c4, grid_slot, grid_rec, grid_fc, grid_pb, grid_segs, grid_gb,
      grid_prec, grid_precm, mx, mr, mred, grid_mfma_b, grid_mfma_nu, phl, vhl, total;
};

Layout layout(const Analysis& a) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t np = static_cast<size_t>(a.n_pix), nv = static_cast<size_t>(a.n_vis), rb = a.rb;
  const size_t nr = static_cast<size_t>(a.max_rhs);
  const size_t nl = a.layer_sigma.size();
  const size_t nfc = a.fd.size() + a.fg.size();
  const size_t npt = a.pd.size() + a.pg.size();
  L.perm = take(4 * np);
  // matrix-core plans read records in steps of 32: padded with zero records
  const bool mf = a.precision == SL1M_PREC_MFMA_F16 || a.precision == SL1M_PREC_MFMA_BF16;
  const bool hl = a.precision == SL1M_PREC_FP32_HILO;
  L.pixrec = take(pixrec_bytes(rb) * (mf ? 4 * static_cast<size_t>(a.mf_np4) : np));
  L.pl = take(8 * np);
  L.pm = take(8 * np);
  L.pc3 = take(8 * np);
  L.pc4 = take(8 * np);
  L.pscale = take(rb * np);
  L.pr2 = take(rb * np);
  L.vu = take(8 * nv);
  L.vv = take(8 * nv);
  L.vw = take(8 * nv);
  L.vgain = take(a.has_gain ? 2 * rb * nv : 0);
  L.vbeta = take(a.beam_pair ? rb * nv : 0);
  L.visrecD = take(visrecD_bytes(rb) * (mf ? 4 * static_cast<size_t>(a.mf_nv4) : nv));
  L.visrecG = take(visrecG_bytes(rb) * nl * nv);
  L.rres = take(2 * rb * (1 + nl) * nv * nr);
  L.rpol = take(a.grid ? sizeof(ResPolar) * nv : 0);
  L.layerDs = take(2 * rb * nl * nv);
  L.chunks = take(sizeof(Chunk) * (nfc + npt + a.fd1.size() + a.fg1.size() + a.pd1.size() +
                                   a.pg1.size()));
  const size_t grid_rows = a.grid ? a.grid_fc.size() + a.fd1.size() + a.fg1.size() : 0;
  L.fpart = take(2 * rb *
                 std::max({nfc * nr, grid_rows * std::max<size_t>(1, a.grid_multi),
                           static_cast<size_t>(a.n_mfchunks) * nr}) *
                 nv);
  L.apart = take(rb * static_cast<size_t>(a.n_achunks) * np * nr);
  L.xperm = take(rb * np * nr);
  L.img = take(rb * np);
  L.zbuf = take(rb * np);
  L.res = take(2 * rb * nv);
  L.red = take(8 * 3 * kRedBlocks + 8 * kMaxLayers);
  L.red_out = take(8 * 8);
  L.flag = take(sizeof(int));
  L.scal = take(8 * sizeof(double));
  const size_t cells = static_cast<size_t>(a.grid_cells);
  L.grid_la = take(8 * a.grid_la.size());
  L.grid_mb = take(8 * a.grid_mb.size());
  L.grid_c3 = take(8 * cells);
  L.grid_c4 = take(8 * cells);
  L.grid_slot = take(4 * 4 * cells);
  L.grid_rec = take(sizeof(GridRec) * cells);
  L.grid_fc = take(sizeof(GridChunk) * a.grid_fc.size());
  L.grid_pb = take(sizeof(GridPairBlock) * a.grid_pb.size());
  L.grid_segs = take(sizeof(GridSeg) * a.gsegs.size());
  L.grid_gb = take(sizeof(int2) * a.grid_gb.size());
  L.grid_prec = take(sizeof(GridPairRec) * static_cast<size_t>(a.grid_pairs));
  L.grid_precm = take(a.grid_multi ? sizeof(float) * static_cast<size_t>(2 + 8 * a.grid_multi) *
                                         static_cast<size_t>(a.grid_pairs)
                                   : 0);
  const size_t ngm = mf ? (nr + 3) / 4 : 0;  // groups of 4 sides
  L.mx = take(2 * 16 * ngm * static_cast<size_t>(a.mf_np4));
  L.mr = take(2 * 32 * ngm * static_cast<size_t>(a.mf_nv4));
  L.mred = take(ngm ? sizeof(float) * (2 * 256 + 4) : 0);
  const size_t pairs = static_cast<size_t>(a.grid_pairs);
  L.grid_mfma_b = take(a.grid_mfma ? 64 * ngm * pairs : 0);
  L.grid_mfma_nu = take(a.grid_mfma ? 8 * pairs : 0);
  L.phl = take(hl ? sizeof(HLRec) * static_cast<size_t>(a.n_pix) : 0);
  L.vhl = take(hl ? sizeof(HLRec) * static_cast<size_t>(a.n_vis) : 0);
  L.total = off;
  return L;
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

#define SL1M_HIP(call, what)                           \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_error(e_, what);  \
  } while (0)

sl1m_status check_plan(sl1m_plan* p) {
  if (!p) return set_error(SL1M_EINVAL, "plan is NULL");
  return SL1M_OK;
}

sl1m_status read_red(sl1m_plan* p, double* host, int n, hipStream_t st) {
  SL1M_HIP(hipMemcpyAsync(host, p->red_out, sizeof(double) * n, hipMemcpyDeviceToHost, st),
           "read reduction");
  SL1M_HIP(hipStreamSynchronize(st), "synchronise");
  return SL1M_OK;
}

// V_hat = M x for x already in permuted order in p->xperm (or `xp`); result
// combined into `out` (caller order) minus `data` if given.
sl1m_status apply_forward(sl1m_plan* p, const void* xp, const void* data, void* out, bool recs,
                          hipStream_t st, int nr = 1) {
  SL1M_HIP(timed(p, T_FWD, st, [&] { return launch_forward(p, xp, nr, st); }), "forward kernel");
  SL1M_HIP(launch_forward_reduce(p, data, out, recs, nr, st), "forward reduce");
  return SL1M_OK;
}

// One iteration (forward at y, residual, adjoint, update, t step); the launch
// sequence is the same every iteration.  MFISTA adds the proximal point z, a
// forward at z and its objective, and the device-side selection.
sl1m_status enqueue_iteration(sl1m_plan* p, const void* vis, hipStream_t st, int method) {
  sl1m_status s = apply_forward(p, p->xperm, vis, p->res, true, st);
  if (s) return s;
  SL1M_HIP(timed(p, T_ADJ, st, [&] { return launch_adjoint(p, 1, st); }), "adjoint kernel");
  if (method == SL1M_MFISTA) {
    SL1M_HIP(timed(p, T_UPDATE, st, [&] { return launch_prox(p, st); }), "proximal step");
    s = apply_forward(p, p->zbuf, vis, p->res, false, st);
    if (s) return s;
    SL1M_HIP(launch_objective_terms(p, p->res, p->zbuf, st), "objective of z");
    SL1M_HIP(launch_mfista_select(p, st), "mfista selection");
    return SL1M_OK;
  }
  SL1M_HIP(timed(p, T_UPDATE, st, [&] { return launch_fista_update(p, st); }), "fista update");
  return SL1M_OK;
}

void release_graph(sl1m_plan* p) {
  if (p->iter_exec) (void)hipGraphExecDestroy(p->iter_exec);
  if (p->iter_graph) (void)hipGraphDestroy(p->iter_graph);
  p->iter_exec = nullptr;
  p->iter_graph = nullptr;
  p->iter_vis = nullptr;
  p->iter_method = 0;
}

// Captures one iteration into a graph (on a private stream: capture records
// launches without running them) unless one for the same data pointer and
// method exists.
sl1m_status ensure_graph(sl1m_plan* p, const void* vis, int method) {
  if (p->iter_exec && p->iter_vis == vis && p->iter_method == method) return SL1M_OK;
  release_graph(p);
  hipStream_t cs = nullptr;
  SL1M_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  sl1m_status s = SL1M_OK;
  if (e == hipSuccess) {
    s = enqueue_iteration(p, vis, cs, method);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (s == SL1M_OK && e2 != hipSuccess) s = hip_error(e2, "end capture");
    if (s == SL1M_OK) {
      p->iter_graph = g;
      const hipError_t e3 = hipGraphInstantiate(&p->iter_exec, g, nullptr, nullptr, 0);
      if (e3 != hipSuccess) s = hip_error(e3, "instantiate graph");
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  } else {
    s = hip_error(e, "begin capture");
  }
  (void)hipStreamDestroy(cs);
  if (s != SL1M_OK) {
    release_graph(p);
    return s;
  }
  p->iter_vis = vis;
  p->iter_method = method;
  return SL1M_OK;
}

sl1m_status power_iteration(sl1m_plan* p, int32_t iters, uint64_t seed, const void* x0,
                            double* rq_out, hipStream_t st) {
  const TraceRange range("sl1m power iteration");
  if (x0)
    SL1M_HIP(launch_gather(p, x0, p->xperm, 1, st), "gather start vector");
  else
    SL1M_HIP(launch_splitmix_start(p, seed, p->xperm, st), "start vector");
  double h[3];
  SL1M_HIP(launch_dot_norm(p, p->xperm, p->xperm, st), "norm");
  sl1m_status s = read_red(p, h, 2, st);
  if (s) return s;
  if (!(h[1] > 0.0)) return set_error(SL1M_EINVAL, "power iteration start vector is zero");
  SL1M_HIP(launch_scale(p, p->xperm, p->n_pix, 1.0 / std::sqrt(h[1]), st), "normalise");
  double rq = 0.0;
  for (int32_t it = 0; it < iters; ++it) {
    s = apply_forward(p, p->xperm, nullptr, p->res, true, st);
    if (s) return s;
    SL1M_HIP(timed(p, T_ADJ, st, [&] { return launch_adjoint(p, 1, st); }), "adjoint kernel");
    SL1M_HIP(launch_adjoint_reduce(p, p->img, false, 1, st), "adjoint reduce");
    SL1M_HIP(launch_dot_norm(p, p->xperm, p->img, st), "rayleigh");
    s = read_red(p, h, 2, st);
    if (s) return s;
    rq = h[0];
    if (!(h[1] > 0.0)) break;
    SL1M_HIP(launch_copy_real(p, p->img, p->xperm, p->n_pix, st), "copy");
    SL1M_HIP(launch_scale(p, p->xperm, p->n_pix, 1.0 / std::sqrt(h[1]), st), "normalise");
  }
  *rq_out = rq;
  return SL1M_OK;
}

}  // namespace

sl1m_status set_error(sl1m_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

sl1m_status hip_error(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return SL1M_EHIP;
}

}  // namespace sl1m

using namespace sl1m;

extern "C" {

const char* sl1m_last_error(void) { return g_last_error.c_str(); }

const char* sl1m_version(void) { return "sl1m-mi355x 0.1 (gfx950)"; }

sl1m_status sl1m_plan_workspace_bytes(const sl1m_problem* problem, size_t* bytes) {
  try {
    if (!bytes) return set_error(SL1M_EINVAL, "bytes is NULL");
    Analysis a;
    sl1m_status s = analyze(problem, a);
    if (s) return s;
    *bytes = layout(a).total;
    return SL1M_OK;
  } catch (const std::bad_alloc&) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

sl1m_status sl1m_plan_create(const sl1m_problem* pr, void* workspace, size_t workspace_bytes,
                             void* stream, sl1m_plan** out) {
  const TraceRange range("sl1m_plan_create");
  try {
    if (!out) return set_error(SL1M_EINVAL, "out is NULL");
    *out = nullptr;
    Analysis a;
    sl1m_status s = analyze(pr, a);
    if (s) return s;
    const Layout L = layout(a);
    if (!workspace) return set_error(SL1M_EINVAL, "workspace is NULL");
    if (workspace_bytes < L.total)
      return set_error(SL1M_ENOMEM, "workspace smaller than sl1m_plan_workspace_bytes()");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return set_error(SL1M_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = S(stream);
    int device = 0;
    SL1M_HIP(hipGetDevice(&device), "get device");
    sl1m_plan* p = new sl1m_plan();
    p->device = device;
    p->n_pix = a.n_pix;
    p->n_vis = a.n_vis;
    p->precision = a.precision;
    p->max_rhs = a.max_rhs;
    p->real_bytes = a.rb;
    p->has_gain = a.has_gain;
    p->beam_pair = a.beam_pair;
    p->segs = a.segs;
    p->layer_sigma = a.layer_sigma;
    p->n_layers = static_cast<int>(a.layer_sigma.size());
    p->fwd_vpl = a.fwd_vpl;
    p->adj_ppl = a.adj_ppl;
    p->fchunks_delta = a.fd;
    p->fchunks_gauss = a.fg;
    p->n_fchunks = static_cast<int>(a.fd.size() + a.fg.size());
    p->ptiles_delta = a.pd;
    p->ptiles_gauss = a.pg;
    p->adj_kchunk = a.kchunk;
    p->n_achunks = a.n_achunks;
    p->mfma = a.precision == SL1M_PREC_MFMA_F16 || a.precision == SL1M_PREC_MFMA_BF16
                  ? a.precision : 0;
    p->hilo = a.precision == SL1M_PREC_FP32_HILO;
    p->n_mfchunks = a.n_mfchunks;
    p->mf_chunk = a.mf_chunk;
    p->mf_np4 = a.mf_np4;
    p->mf_nv4 = a.mf_nv4;
    p->grid = a.grid;
    p->grid_multi = a.grid_multi;
    p->grid_segs = a.gsegs;
    p->grid_cells = a.grid_cells;
    p->grid_vtiles = a.grid_vtiles;
    p->grid_frows = a.grid_frows;
    p->grid_fchunks = a.grid_fc;
    p->fd1 = a.fd1;
    p->fg1 = a.fg1;
    p->pd1 = a.pd1;
    p->pg1 = a.pg1;
    for (const Segment& sg : a.segs) {
      if (sg.count == 0) continue;
      (sg.kind == SL1M_PIX_DELTA ? p->any_delta : p->any_gauss) = true;
    }
    char* w = static_cast<char*>(workspace);
    p->ws = w;
    p->ws_bytes = workspace_bytes;
    p->perm = reinterpret_cast<int32_t*>(w + L.perm);
    p->pixrec = w + L.pixrec;
    p->pl = reinterpret_cast<double*>(w + L.pl);
    p->pm = reinterpret_cast<double*>(w + L.pm);
    p->pc3 = reinterpret_cast<double*>(w + L.pc3);
    p->pc4 = reinterpret_cast<double*>(w + L.pc4);
    p->pscale = w + L.pscale;
    p->pr2 = w + L.pr2;
    p->vu = reinterpret_cast<double*>(w + L.vu);
    p->vv = reinterpret_cast<double*>(w + L.vv);
    p->vw = reinterpret_cast<double*>(w + L.vw);
    p->vgain = a.has_gain ? w + L.vgain : nullptr;
    p->vbeta = a.beam_pair ? w + L.vbeta : nullptr;
    p->visrecD = w + L.visrecD;
    p->visrecG = p->n_layers ? w + L.visrecG : nullptr;
    p->rres = w + L.rres;
    p->rpol = a.grid ? reinterpret_cast<ResPolar*>(w + L.rpol) : nullptr;
    p->layerDs = p->n_layers ? w + L.layerDs : nullptr;
    p->d_fchunks = reinterpret_cast<Chunk*>(w + L.chunks);
    p->d_ptiles = p->d_fchunks + p->n_fchunks;
    p->d_chunks1 = p->d_ptiles + a.pd.size() + a.pg.size();
    p->fpart = w + L.fpart;
    p->apart = w + L.apart;
    p->xperm = w + L.xperm;
    p->img = w + L.img;
    p->zbuf = w + L.zbuf;
    p->res = w + L.res;
    p->red = reinterpret_cast<double*>(w + L.red);
    p->red_out = reinterpret_cast<double*>(w + L.red_out);
    p->flag = reinterpret_cast<int*>(w + L.flag);
    p->scal = reinterpret_cast<double*>(w + L.scal);
    if (p->mfma) {
      p->mx = reinterpret_cast<uint16_t*>(w + L.mx);
      p->mr = reinterpret_cast<uint16_t*>(w + L.mr);
      p->mred = reinterpret_cast<float*>(w + L.mred);
    }
    if (p->hilo) {
      p->phl = reinterpret_cast<HLRec*>(w + L.phl);
      p->vhl = reinterpret_cast<HLRec*>(w + L.vhl);
    }
    p->grid_mfma = a.grid_mfma;
    if (a.grid_mfma) {
      p->grid_mfma_b = w + L.grid_mfma_b;
      p->grid_mfma_nu = reinterpret_cast<double*>(w + L.grid_mfma_nu);
    }
    if (a.grid) {
      p->grid_la = reinterpret_cast<double*>(w + L.grid_la);
      p->grid_mb = reinterpret_cast<double*>(w + L.grid_mb);
      p->grid_c3 = reinterpret_cast<double*>(w + L.grid_c3);
      p->grid_c4 = reinterpret_cast<double*>(w + L.grid_c4);
      p->grid_slot = reinterpret_cast<int32_t*>(w + L.grid_slot);
      p->grid_rec = w + L.grid_rec;
      p->d_grid_fchunks = reinterpret_cast<GridChunk*>(w + L.grid_fc);
      p->d_grid_pblocks = reinterpret_cast<GridPairBlock*>(w + L.grid_pb);
      p->d_grid_segs = reinterpret_cast<GridSeg*>(w + L.grid_segs);
      p->d_grid_gblocks = reinterpret_cast<int2*>(w + L.grid_gb);
      p->grid_gblocks = static_cast<int>(a.grid_gb.size());
      p->grid_prec = reinterpret_cast<GridPairRec*>(w + L.grid_prec);
      p->grid_precm = a.grid_multi ? reinterpret_cast<float*>(w + L.grid_precm) : nullptr;
    }

    auto fail = [&](sl1m_status st_) {
      delete p;
      return st_;
    };
    // permutation, chunk tables, layer sigmas (host -> device)
    std::vector<int32_t> perm = a.perm;
    if (perm.empty()) {
      perm.resize(a.n_pix);
      for (int64_t j = 0; j < a.n_pix; ++j) perm[j] = static_cast<int32_t>(j);
    }
    std::vector<Chunk> chunks;
    chunks.insert(chunks.end(), a.fd.begin(), a.fd.end());
    chunks.insert(chunks.end(), a.fg.begin(), a.fg.end());
    chunks.insert(chunks.end(), a.pd.begin(), a.pd.end());
    chunks.insert(chunks.end(), a.pg.begin(), a.pg.end());
    chunks.insert(chunks.end(), a.fd1.begin(), a.fd1.end());
    chunks.insert(chunks.end(), a.fg1.begin(), a.fg1.end());
    chunks.insert(chunks.end(), a.pd1.begin(), a.pd1.end());
    chunks.insert(chunks.end(), a.pg1.begin(), a.pg1.end());
    hipError_t e = hipSuccess;
    if (!perm.empty())
      e = hipMemcpyAsync(p->perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !chunks.empty())
      e = hipMemcpyAsync(p->d_fchunks, chunks.data(), chunks.size() * sizeof(Chunk),
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess && p->n_layers)
      e = hipMemcpyAsync(p->red, a.layer_sigma.data(), p->n_layers * sizeof(double),
                         hipMemcpyHostToDevice, st);
    if (a.grid) {
      auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes)
          e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
      };
      up(p->grid_la, a.grid_la.data(), 8 * a.grid_la.size());
      up(p->grid_mb, a.grid_mb.data(), 8 * a.grid_mb.size());
      up(p->grid_c3, a.grid_c3.data(), 8 * a.grid_c3.size());
      up(p->grid_c4, a.grid_c4.data(), 8 * a.grid_c4.size());
      up(p->grid_slot, a.grid_slot.data(), 4 * a.grid_slot.size());
      up(p->d_grid_fchunks, a.grid_fc.data(), sizeof(GridChunk) * a.grid_fc.size());
      up(p->d_grid_pblocks, a.grid_pb.data(), sizeof(GridPairBlock) * a.grid_pb.size());
      up(p->d_grid_segs, a.gsegs.data(), sizeof(GridSeg) * a.gsegs.size());
      up(p->d_grid_gblocks, a.grid_gb.data(), sizeof(int2) * a.grid_gb.size());
    }
    if (e == hipSuccess) e = launch_fill(p->flag, 1, sizeof(int), st);
    if (e == hipSuccess)
      e = launch_domain_check(p, pr->l, pr->m, pr->sigma, pr->u, pr->v, pr->w, st);
    if (e == hipSuccess) e = launch_prep_pixels(p, pr->l, pr->m, nullptr, a.beam_coef, st);
    if (e == hipSuccess)
      e = launch_prep_vis(p, pr->u, pr->v, pr->w, pr->ant_p, pr->ant_q, pr->ant_gain,
                          a.beam_pair ? pr->ant_fwhm : nullptr, pr->n_ant, st);
    if (e == hipSuccess) e = launch_prep_hilo(p, st);
    if (e == hipSuccess)
      e = launch_fill(p->apart, static_cast<size_t>(p->n_achunks) * p->n_pix * p->max_rhs, a.rb,
                      st);
    if (p->mfma) {  // zero records past the last pixel / visibility (steps of 32)
      const size_t pr_b = sizeof(PixRec<float>), vr_b = sizeof(VisRecD<float>);
      const size_t pad_p = static_cast<size_t>(4 * a.mf_np4 - a.n_pix) * pr_b;
      const size_t pad_v = static_cast<size_t>(4 * a.mf_nv4 - a.n_vis) * vr_b;
      if (e == hipSuccess && pad_p)
        e = launch_fill(static_cast<char*>(p->pixrec) + a.n_pix * pr_b, pad_p / 4, 4, st);
      if (e == hipSuccess && pad_v)
        e = launch_fill(static_cast<char*>(p->visrecD) + a.n_vis * vr_b, pad_v / 4, 4, st);
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, p->flag, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(hip_error(e, "plan preparation"));
    if (bad) {
      set_error(SL1M_EDOMAIN,
                std::to_string(bad) +
                    " input(s) outside the domain (need l^2+m^2 < 1, finite sigma >= 0, finite u,v,w)");
      return fail(SL1M_EDOMAIN);
    }
    *out = p;
    return SL1M_OK;
  } catch (const std::bad_alloc&) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

static void timing_release(sl1m_plan* p) {
  for (auto& v : p->tev) {
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
    v.clear();
  }
  for (int& c : p->tcount) c = 0;
  p->timing = false;
  p->timing_cap = 0;
}

sl1m_status sl1m_plan_destroy(sl1m_plan* plan) {
  if (plan) {
    timing_release(plan);
    release_graph(plan);
  }
  delete plan;
  return SL1M_OK;
}

}  // extern "C"

namespace {

// Candidate launch shapes for sl1m_tune: (grid mode, split target) with the
// plan's own lane counts, then lane counts for the best direct split.
std::vector<sl1m_problem> tune_stage1(const sl1m_problem& base, bool grid_possible) {
  std::vector<sl1m_problem> c;
  for (int g : {SL1M_GRID_AUTO, SL1M_GRID_OFF}) {
    if (g == SL1M_GRID_AUTO && !grid_possible) continue;
    for (int tb : {1024, 2048, 4096, 8192, 16384}) {
      sl1m_problem p = base;
      p.grid_mode = g;
      p.tile_blocks = tb;
      p.fwd_vpl = 0;
      p.adj_ppl = 0;
      c.push_back(p);
    }
  }
  return c;
}

struct TuneTimes {
  double fwd_ms = 0, adj_ms = 0;
};

double median(std::vector<float> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}

// Builds the plan of `pr` in the workspace and times `reps` forward and
// adjoint applications (after one warm-up of each).
sl1m_status tune_one(const sl1m_problem& pr, void* ws, size_t bytes, int reps, hipStream_t st,
                     TuneTimes& out) {
  sl1m_plan* p = nullptr;
  if (sl1m_status s = sl1m_plan_create(&pr, ws, bytes, st, &p)) return s;
  std::vector<hipEvent_t> ev(2 * (2 * reps + 2), nullptr);
  sl1m_status res = SL1M_OK;
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  if (e == hipSuccess) e = launch_splitmix_start(p, 12345, p->xperm, st);
  std::vector<float> tf, ta;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    hipEvent_t* q = &ev[4 * r];
    e = hipEventRecord(q[0], st);
    if (e == hipSuccess) e = launch_forward(p, p->xperm, 1, st);
    if (e == hipSuccess) e = launch_forward_reduce(p, nullptr, p->res, true, 1, st);
    if (e == hipSuccess) e = hipEventRecord(q[1], st);
    if (e == hipSuccess) e = hipEventRecord(q[2], st);
    if (e == hipSuccess) e = launch_adjoint(p, 1, st);
    if (e == hipSuccess) e = launch_adjoint_reduce(p, p->img, false, 1, st);
    if (e == hipSuccess) e = hipEventRecord(q[3], st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int r = 1; r <= reps && e == hipSuccess; ++r) {  // r = 0 is the warm-up
    float a = 0, b = 0;
    e = hipEventElapsedTime(&a, ev[4 * r], ev[4 * r + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[4 * r + 2], ev[4 * r + 3]);
    tf.push_back(a);
    ta.push_back(b);
  }
  if (e != hipSuccess) res = hip_error(e, "tuning run");
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  sl1m_plan_destroy(p);
  out.fwd_ms = median(tf);
  out.adj_ms = median(ta);
  return res;
}

}  // namespace

extern "C" {

sl1m_status sl1m_tune_workspace_bytes(const sl1m_problem* problem, size_t* bytes) {
  try {
    if (!problem || !bytes) return set_error(SL1M_EINVAL, "NULL argument");
    if (problem->precision == SL1M_PREC_MFMA_F16 || problem->precision == SL1M_PREC_MFMA_BF16)
      return set_error(SL1M_EINVAL, "the MFMA precisions have no tuned launch shapes");
    if (problem->precision == SL1M_PREC_FP32_HILO)
      return set_error(SL1M_EINVAL, "the FP32 hi/lo phase has no tuned launch shapes");
    // every plan sl1m_tune may build: the default, (grid mode, split) with the
    // plan's lane counts, and direct plans with every lane count and split
    size_t mx = 0;
    auto need = [&](int g, int tb, int vpl, int ppl) -> sl1m_status {
      sl1m_problem p = *problem;
      p.max_rhs = 1;
      p.grid_mode = g;
      p.tile_blocks = tb;
      p.fwd_vpl = vpl;
      p.adj_ppl = ppl;
      size_t b = 0;
      if (sl1m_status s = sl1m_plan_workspace_bytes(&p, &b)) return s;
      mx = std::max(mx, b);
      return SL1M_OK;
    };
    if (sl1m_status s = need(SL1M_GRID_AUTO, 0, 0, 0)) return s;
    for (int tb : {1024, 2048, 4096, 8192, 16384}) {
      if (sl1m_status s = need(SL1M_GRID_AUTO, tb, 0, 0)) return s;
      for (int vpl : {0, 1, 2, 4})
        for (int ppl : {0, 1, 2, 4})
          if (sl1m_status s = need(SL1M_GRID_OFF, tb, vpl, ppl)) return s;
    }
    *bytes = mx;
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  }
}

sl1m_status sl1m_tune(const sl1m_problem* problem, void* workspace, size_t workspace_bytes,
                      int32_t reps, void* stream, sl1m_tuning* out) {
  const TraceRange range("sl1m_tune");
  try {
    if (!problem || !out) return set_error(SL1M_EINVAL, "NULL argument");
    if (reps < 1 || reps > 100) return set_error(SL1M_EINVAL, "reps must be in [1, 100]");
    size_t need = 0;
    if (sl1m_status s = sl1m_tune_workspace_bytes(problem, &need)) return s;
    if (workspace_bytes < need)
      return set_error(SL1M_ENOMEM, "workspace smaller than sl1m_tune_workspace_bytes()");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    sl1m_problem base = *problem;
    base.max_rhs = 1;
    // does any segment qualify for the grid evaluation?
    bool grid_possible = false;
    {
      Analysis a;
      sl1m_problem p = base;
      p.grid_mode = SL1M_GRID_AUTO;
      p.tile_blocks = 0;
      p.fwd_vpl = p.adj_ppl = 0;
      if (sl1m_status s = analyze(&p, a)) return s;
      grid_possible = a.grid;
    }
    sl1m_tuning r;
    std::memset(&r, 0, sizeof(r));
    // a candidate replaces the current choice (first the plan's defaults) only
    // when at least 1 % faster, so that timing noise does not move the plan
    constexpr double kMargin = 0.99;
    double best = 1e300;
    auto consider = [&](const sl1m_problem& p, const TuneTimes& t) {
      ++r.candidates;
      if (t.fwd_ms + t.adj_ms < best * kMargin) {
        best = t.fwd_ms + t.adj_ms;
        r.tile_blocks = p.tile_blocks;
        r.grid_mode = p.grid_mode;
        r.fwd_vpl = p.fwd_vpl;
        r.adj_ppl = p.adj_ppl;
        r.forward_ms = t.fwd_ms;
        r.adjoint_ms = t.adj_ms;
      }
    };
    {
      sl1m_problem p = base;
      p.grid_mode = SL1M_GRID_AUTO;
      p.tile_blocks = 0;
      p.fwd_vpl = p.adj_ppl = 0;
      TuneTimes t;
      // the first run brings the GPU to its working clock; it is not counted
      // (measured first, the defaults would otherwise look slower)
      if (sl1m_status s = tune_one(p, workspace, workspace_bytes, reps, st, t)) return s;
      if (sl1m_status s = tune_one(p, workspace, workspace_bytes, reps, st, t)) return s;
      r.default_forward_ms = t.fwd_ms;
      r.default_adjoint_ms = t.adj_ms;
      consider(p, t);
    }
    for (const sl1m_problem& p : tune_stage1(base, grid_possible)) {
      TuneTimes t;
      if (sl1m_status s = tune_one(p, workspace, workspace_bytes, reps, st, t)) return s;
      consider(p, t);
    }
    // lane counts of the direct kernels at the best direct split
    if (r.grid_mode == SL1M_GRID_OFF || !grid_possible) {
      const int tb = r.tile_blocks;
      for (int vpl : {1, 2, 4})
        for (int ppl : {1, 2, 4}) {
          sl1m_problem p = base;
          p.grid_mode = SL1M_GRID_OFF;
          p.tile_blocks = tb;
          p.fwd_vpl = vpl;
          p.adj_ppl = ppl;
          TuneTimes t;
          if (sl1m_status s = tune_one(p, workspace, workspace_bytes, reps, st, t)) return s;
          consider(p, t);
        }
    }
    *out = r;
    return SL1M_OK;
  } catch (const std::bad_alloc&) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

sl1m_status sl1m_plan_query(const sl1m_plan* p, sl1m_plan_info* info) {
  if (!p) return set_error(SL1M_EINVAL, "plan is NULL");
  if (!info) return set_error(SL1M_EINVAL, "info is NULL");
  sl1m_plan_info r;
  std::memset(&r, 0, sizeof(r));
  r.n_pix = p->n_pix;
  r.n_vis = p->n_vis;
  r.precision = p->precision;
  r.max_rhs = p->max_rhs;
  r.grid = static_cast<int32_t>(p->grid_segs.size());
  for (const GridSeg& g : p->grid_segs)
    if (g.kind == SL1M_PIX_DELTA) {
      r.grid_abs_l = g.na;
      r.grid_abs_m = g.nb;
    }
  r.n_layers = p->n_layers;
  r.grid_positions = 4 * p->grid_cells;
  r.fwd_vpl = p->fwd_vpl;
  r.adj_ppl = p->adj_ppl;
  r.n_fchunks = p->n_fchunks;
  r.n_fchunks_grid = p->grid ? forward_rows(p, 1) : 0;
  r.n_achunks = p->n_achunks;
  for (const GridSeg& g : p->grid_segs) r.grid_pairs += g.square ? 1 : 0;
  r.grid_multi = p->grid_multi;
  r.grid_mfma = p->grid_mfma ? 1 : 0;
  *info = r;
  return SL1M_OK;
}

sl1m_status sl1m_timing_begin(sl1m_plan* p, int32_t max_launches) {
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if (max_launches < 1 || max_launches > (1 << 20))
      return set_error(SL1M_EINVAL, "max_launches must be in [1, 2^20]");
    timing_release(p);
    for (auto& v : p->tev) {
      v.resize(2 * static_cast<size_t>(max_launches));
      for (hipEvent_t& e : v) SL1M_HIP(hipEventCreate(&e), "create timing event");
    }
    p->timing_cap = max_launches;
    p->timing = true;
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_ENOMEM, "host allocation failed");
  }
}

sl1m_status sl1m_timing_end(sl1m_plan* p, sl1m_timing* out) {
  if (sl1m_status s = check_plan(p)) return s;
  if (!out) return set_error(SL1M_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  if (!p->timing) return set_error(SL1M_EINVAL, "timing was not started");
  for (int kind = 0; kind < kTimingKinds; ++kind) {
    double total = 0.0;
    for (int i = 0; i < p->tcount[kind]; ++i) {
      hipEvent_t a = p->tev[kind][2 * i], b = p->tev[kind][2 * i + 1];
      SL1M_HIP(hipEventSynchronize(b), "timing sync");
      float ms = 0.f;
      SL1M_HIP(hipEventElapsedTime(&ms, a, b), "timing elapsed");
      total += ms;
    }
    out->launches[kind] = p->tcount[kind];
    out->total_ms[kind] = total;
  }
  timing_release(p);
  return SL1M_OK;
}

static sl1m_status forward_impl(sl1m_plan* p, int32_t nr, const void* x, void* vis,
                                void* stream) {
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if (nr != 1 && nr != 2 && nr != 4 && nr != 8)
      return set_error(SL1M_EINVAL, "n_rhs must be 1, 2, 4 or 8");
    if (nr > p->max_rhs) return set_error(SL1M_EINVAL, "n_rhs exceeds the plan's max_rhs");
    if ((p->n_pix > 0 && !x) || (p->n_vis > 0 && !vis))
      return set_error(SL1M_EINVAL, "x or vis is NULL");
    hipStream_t st = S(stream);
    SL1M_HIP(launch_gather(p, x, p->xperm, nr, st), "gather");
    return apply_forward(p, p->xperm, nullptr, vis, false, st, nr);
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

static sl1m_status adjoint_impl(sl1m_plan* p, int32_t nr, const void* r, void* g, void* stream) {
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if (nr != 1 && nr != 2 && nr != 4 && nr != 8)
      return set_error(SL1M_EINVAL, "n_rhs must be 1, 2, 4 or 8");
    if (nr > p->max_rhs) return set_error(SL1M_EINVAL, "n_rhs exceeds the plan's max_rhs");
    if ((p->n_vis > 0 && !r) || (p->n_pix > 0 && !g))
      return set_error(SL1M_EINVAL, "r or g is NULL");
    hipStream_t st = S(stream);
    SL1M_HIP(launch_adjoint_prep(p, r, nr, st), "adjoint prep");
    SL1M_HIP(timed(p, T_ADJ, st, [&] { return launch_adjoint(p, nr, st); }), "adjoint kernel");
    SL1M_HIP(launch_adjoint_reduce(p, g, true, nr, st), "adjoint reduce");
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

sl1m_status sl1m_forward(sl1m_plan* p, const void* x, void* vis, void* stream) {
  return forward_impl(p, 1, x, vis, stream);
}

sl1m_status sl1m_adjoint(sl1m_plan* p, const void* r, void* g, void* stream) {
  return adjoint_impl(p, 1, r, g, stream);
}

sl1m_status sl1m_forward_multi(sl1m_plan* p, int32_t n_rhs, const void* x, void* vis,
                               void* stream) {
  return forward_impl(p, n_rhs, x, vis, stream);
}

sl1m_status sl1m_adjoint_multi(sl1m_plan* p, int32_t n_rhs, const void* r, void* g,
                               void* stream) {
  return adjoint_impl(p, n_rhs, r, g, stream);
}

sl1m_status sl1m_estimate_L(sl1m_plan* p, int32_t iters, uint64_t seed, const void* x0,
                            double* rayleigh_out, void* stream) {
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if (!rayleigh_out) return set_error(SL1M_EINVAL, "rayleigh_out is NULL");
    if (iters < 1) return set_error(SL1M_EINVAL, "iters must be >= 1");
    if (p->n_pix == 0) return set_error(SL1M_EINVAL, "no pixels");
    return power_iteration(p, iters, seed, x0, rayleigh_out, S(stream));
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

// The FISTA solve from I_0 = x0 (caller order; NULL: I_0 = 0), or, with
// `state`, from an exported iteration state (its image, extrapolated point
// and t), which on return holds the state after the last iteration.
static sl1m_status solve_impl(sl1m_plan* p, const void* vis, const void* x0,
                              const sl1m_solve_params* prm, void* img_out, sl1m_solve_info* info,
                              void* stream, sl1m_fista_state* state = nullptr) {
  const TraceRange range("sl1m solve");
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if (!prm || !info) return set_error(SL1M_EINVAL, "params or info is NULL");
    if ((p->n_vis > 0 && !vis) || (p->n_pix > 0 && !img_out))
      return set_error(SL1M_EINVAL, "vis or img_out is NULL");
    if (!(prm->lambda >= 0.0) || !std::isfinite(prm->lambda))
      return set_error(SL1M_EINVAL, "lambda must be finite and >= 0");
    if (prm->max_iter < 0) return set_error(SL1M_EINVAL, "max_iter must be >= 0");
    if (!(prm->eps >= 0.0)) return set_error(SL1M_EINVAL, "eps must be >= 0");
    if (!(prm->nnz_eps >= 0.0)) return set_error(SL1M_EINVAL, "nnz_eps must be >= 0");
    const bool checks = prm->eps > 0.0 || prm->nnz_eps > 0.0;
    if (checks && prm->check_every < 1)
      return set_error(SL1M_EINVAL, "check_every must be >= 1 when eps or nnz_eps > 0");
    if (prm->method != SL1M_FISTA && prm->method != SL1M_MFISTA)
      return set_error(SL1M_EINVAL, "unknown method");
    const int method = prm->method;
    if (state) {
      if (method != SL1M_FISTA) return set_error(SL1M_EINVAL, "resume supports SL1M_FISTA only");
      if (p->n_pix > 0 && (!state->img || !state->y))
        return set_error(SL1M_EINVAL, "state img or y is NULL");
      if (state->t != 0.0 && !(state->t >= 1.0 && std::isfinite(state->t)))
        return set_error(SL1M_EINVAL, "state t must be 0 (fresh start) or >= 1");
      if (state->k < 0) return set_error(SL1M_EINVAL, "state k must be >= 0");
    }
    std::memset(info, 0, sizeof(*info));
    hipStream_t st = S(stream);
    double L = prm->L;
    if (!(L > 0.0)) {
      const int32_t pit = prm->power_iters > 0 ? prm->power_iters : 30;
      double rq = 0.0;
      sl1m_status s = power_iteration(p, pit, prm->seed, nullptr, &rq, st);
      if (s) return s;
      const double safety = prm->L_safety > 0.0 ? prm->L_safety : 1.01;
      L = safety * rq;
      if (!(L > 0.0)) return set_error(SL1M_EINVAL, "estimated L is not positive (M = 0?)");
    }
    info->L = L;
    const bool resume = state && state->t >= 1.0;
    const double scal_h[5] = {resume ? state->t : 1.0, 1.0 / L, prm->lambda / L, prm->lambda,
                              0.0};
    SL1M_HIP(hipMemcpyAsync(p->scal, scal_h, sizeof(scal_h), hipMemcpyHostToDevice, st),
             "solver scalars");
    if (resume) {
      // the state after iteration k: I_k, y_{k+1} and t_{k+1}
      SL1M_HIP(launch_gather(p, state->img, p->img, 1, st), "resume image");
      SL1M_HIP(launch_gather(p, state->y, p->xperm, 1, st), "resume extrapolated point");
    } else if (state) {
      // a fresh start from the state's image (y_1 = I_0)
      SL1M_HIP(launch_gather(p, state->img, p->xperm, 1, st), "start image");
      SL1M_HIP(launch_copy_real(p, p->xperm, p->img, p->n_pix, st), "start image");
    } else if (x0) {
      // warm start: y_1 = I_0 = x0 (the first momentum coefficient is 0)
      SL1M_HIP(launch_gather(p, x0, p->xperm, 1, st), "start image");
      SL1M_HIP(launch_copy_real(p, p->xperm, p->img, p->n_pix, st), "start image");
    } else {
      SL1M_HIP(launch_fill(p->xperm, p->n_pix, p->real_bytes, st), "zero y");
      SL1M_HIP(launch_fill(p->img, p->n_pix, p->real_bytes, st), "zero I");
    }
    SL1M_HIP(launch_fill(p->flag, 1, sizeof(int), st), "zero divergence flag");
    if (method == SL1M_MFISTA) {  // F(x_0) for the first selection
      sl1m_status s = apply_forward(p, p->img, vis, p->res, false, st);
      if (s) return s;
      SL1M_HIP(launch_objective_terms(p, p->res, p->img, st), "objective of x0");
      SL1M_HIP(launch_mfista_init(p, st), "mfista start");
    }
    // a captured graph replays the iteration with one launch (not while the
    // per-kernel timing facility is recording)
    bool use_graph = !p->timing && prm->max_iter > 1;
    if (use_graph && ensure_graph(p, vis, method) != SL1M_OK) {
      use_graph = false;  // capture unavailable: launch the kernels directly
      set_error(SL1M_OK, "");
      (void)hipGetLastError();
    }
    double F_prev = -1.0, nnz_prev = -1.0;
    double h[3];
    int32_t k = 0;
    for (k = 1; k <= prm->max_iter; ++k) {
      if (use_graph) {
        SL1M_HIP(hipGraphLaunch(p->iter_exec, st), "graph launch");
      } else {
        sl1m_status s = enqueue_iteration(p, vis, st, method);
        if (s) return s;
      }
      if (checks && k % prm->check_every == 0) {
        sl1m_status s = apply_forward(p, p->img, vis, p->res, false, st);
        if (s) return s;
        SL1M_HIP(launch_objective_terms(p, p->res, p->img, st), "objective");
        s = read_red(p, h, 3, st);
        if (s) return s;
        const double F = h[0] + prm->lambda * h[1];
        const double nnz = h[2];
        if (!std::isfinite(F)) break;
        // the two stopping rules of Section "Implementation of SL1M": a small
        // change of the objective, or of the number of non-zero pixels
        if (prm->eps > 0.0 && F_prev >= 0.0 && std::fabs(F - F_prev) <= prm->eps * F_prev) {
          info->converged = 1;
          break;
        }
        if (prm->nnz_eps > 0.0 && nnz_prev >= 0.0 &&
            std::fabs(nnz - nnz_prev) < prm->nnz_eps * std::max(nnz_prev, 1.0)) {
          info->converged = 2;
          break;
        }
        F_prev = F;
        nnz_prev = nnz;
      }
    }
    info->iters = std::min(k, prm->max_iter);
    sl1m_status s = apply_forward(p, p->img, vis, p->res, false, st);
    if (s) return s;
    SL1M_HIP(launch_objective_terms(p, p->res, p->img, st), "objective");
    SL1M_HIP(launch_unpermute(p, p->img, img_out, st), "unpermute image");
    double t_next = 0.0;
    if (state) {
      SL1M_HIP(launch_unpermute(p, p->img, state->img, st), "export image");
      SL1M_HIP(launch_unpermute(p, p->xperm, state->y, st), "export extrapolated point");
      SL1M_HIP(hipMemcpyAsync(&t_next, p->scal, sizeof(double), hipMemcpyDeviceToHost, st),
               "read t");
    }
    int nonfinite = 0;
    SL1M_HIP(hipMemcpyAsync(&nonfinite, p->flag, sizeof(int), hipMemcpyDeviceToHost, st),
             "read divergence flag");
    s = read_red(p, h, 3, st);
    if (s) return s;
    info->l2_term = h[0];
    info->l1_term = h[1];
    info->nnz = static_cast<int64_t>(h[2]);
    info->F = h[0] + prm->lambda * h[1];
    if (state) {
      state->t = t_next;
      state->k += info->iters;
    }
    if (!std::isfinite(info->F) || nonfinite) {
      info->status = SL1M_EDIVERGED;
      return set_error(SL1M_EDIVERGED,
                       "the iteration produced non-finite values (is L too small?)");
    }
    info->status = SL1M_OK;
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

sl1m_status sl1m_solve(sl1m_plan* p, const void* vis, const sl1m_solve_params* prm,
                       void* img_out, sl1m_solve_info* info, void* stream) {
  return solve_impl(p, vis, nullptr, prm, img_out, info, stream);
}

sl1m_status sl1m_solve_from(sl1m_plan* p, const void* vis, const void* x0,
                            const sl1m_solve_params* prm, void* img_out, sl1m_solve_info* info,
                            void* stream) {
  if (p && p->n_pix > 0 && !x0) return set_error(SL1M_EINVAL, "x0 is NULL");
  return solve_impl(p, vis, p && p->n_pix > 0 ? x0 : nullptr, prm, img_out, info, stream);
}

sl1m_status sl1m_solve_resume(sl1m_plan* p, const void* vis, sl1m_fista_state* state,
                              const sl1m_solve_params* prm, void* img_out, sl1m_solve_info* info,
                              void* stream) {
  if (!state) return set_error(SL1M_EINVAL, "state is NULL");
  return solve_impl(p, vis, nullptr, prm, img_out, info, stream, state);
}

sl1m_status sl1m_dirty_image(sl1m_plan* p, const void* vis, void* img_out, void* stream) {
  try {
    if (sl1m_status s = check_plan(p)) return s;
    if ((p->n_vis > 0 && !vis) || (p->n_pix > 0 && !img_out))
      return set_error(SL1M_EINVAL, "vis or img_out is NULL");
    hipStream_t st = S(stream);
    if (p->n_vis == 0) {
      SL1M_HIP(launch_fill(img_out, p->n_pix, p->real_bytes, st), "zero image");
      return SL1M_OK;
    }
    SL1M_HIP(launch_adjoint_prep(p, vis, 1, st), "adjoint prep");
    SL1M_HIP(launch_adjoint(p, 1, st), "adjoint kernel");
    SL1M_HIP(launch_adjoint_reduce(p, p->img, false, 1, st), "adjoint reduce");
    SL1M_HIP(launch_dirty_out(p, p->img, img_out, 1.0 / static_cast<double>(p->n_vis), st),
             "dirty image");
    return SL1M_OK;
  } catch (...) {
    return set_error(SL1M_EINVAL, "unexpected host error");
  }
}

}  // extern "C"
