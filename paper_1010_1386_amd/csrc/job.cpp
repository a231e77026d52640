// Job layout, upload, launch and decode (see job.h).
#include "job.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>

#include "context.h"
#include "kernels.h"

namespace rsl {

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int blocks_of(int n, int b) { return (n + b - 1) / b; }

// Algorithmic work of one (prime, point) pair: Horner multiply-adds over all
// coefficients of f and g, plus m_y n_y multiply-subtracts of the Euclidean
// remainder sequence (inversions not counted).
static int64_t pair_mulmods(const Plan& P) {
  int64_t nf = 0, ng = 0;
  for (int d : P.f.rdeg) nf += d + 1;
  for (int d : P.g.rdeg) ng += d + 1;
  return nf + ng + static_cast<int64_t>(P.my) * P.ny;
}

int job_plan(int n, const rsl_poly* f, const rsl_poly* g, const int* var, const rsl_opts* opts, Job* J,
             std::string* err) {
  J->n = n;
  J->plans.assign(n, Plan());
  J->pstatus.assign(n, 0);
  J->live.clear();
  // planning is independent per problem: spread it over host threads
  std::vector<std::string> perr(n);
  parallel_for(n, 4, [&](int k) {
    std::string& e = perr[k];
    int rc = make_plan(&f[k], &g[k], var[k], opts, &J->plans[k], &e);
    if (!rc && !J->plans[k].zero) {
      const Plan& P = J->plans[k];
      if (P.np > kMaxPrimes) { rc = RSL_EINVAL; e = "more than 4096 primes needed (coefficients too large)"; }
      else if (P.E > 3800) { rc = RSL_EINVAL; e = "more than 3800 evaluation points needed (degree bound too large)"; }
      else if (std::max(P.my, P.ny) > 255) { rc = RSL_EINVAL; e = "degree in the eliminated variable above 255"; }
    }
    J->pstatus[k] = rc;
  });
  J->plan_err.clear();
  for (int k = 0; k < n; ++k) {
    if (J->pstatus[k]) {
      if (J->plan_err.empty()) J->plan_err = "problem " + std::to_string(k) + ": " + perr[k];
      continue;
    }
    if (!J->plans[k].zero) J->live.push_back(k);
  }
  if (err && err->empty()) *err = J->plan_err;
  return RSL_OK;
}

int64_t problem_cost(const Plan& P) {
  return pair_mulmods(P) * P.np * (P.E + 1) + static_cast<int64_t>(P.np) * (P.D + 1) * (P.D + 1);
}

int job_build(rsl_ctx* ctx, int n, const rsl_poly* f, const rsl_poly* g, const int* var, const rsl_opts* opts,
              Job* J, std::string* err, const TuneConfig* tc, bool planned, bool defer_tables) {
  if (!planned || J->n != n) job_plan(n, f, g, var, opts, J, err);
  else if (err->empty()) *err = J->plan_err;
  J->tune = tc ? *tc : TuneConfig();
  const int64_t target = std::max(64, J->tune.chunk_target);
  for (int s = 0; s < kNumStages; ++s) J->items[s].clear();
  int maxg = 0, maxE = 0, maxD = 0;
  {
    // live problems in submission order (the order below is by cost)
    std::vector<int> live;
    for (int k = 0; k < n; ++k)
      if (!J->pstatus[k] && !J->plans[k].zero) live.push_back(k);
    J->live.swap(live);
  }
  for (int k : J->live) {
    const Plan& P = J->plans[k];
    for (int gi : P.pidx) maxg = std::max(maxg, gi + 1);
    maxE = std::max(maxE, P.E);
    maxD = std::max(maxD, P.D);
  }
  // larger problems first: their work starts early and the tail is short
  std::vector<int64_t> cost(n, 0);
  for (int k : J->live) {
    const Plan& P = J->plans[k];
    cost[k] = pair_mulmods(P) * P.np * (P.E + 1);
  }
  // a system eliminated in y directly followed by the same system eliminated in
  // x shares the reduction of their common primes: the y problem writes both
  // residue tiles (pair_of[k] = the y problem of x problem k)
  std::vector<int> pair_of(n, -1);
  auto same_poly = [](const rsl_poly& a, const rsl_poly& b) {
    if (a.dx != b.dx || a.dy != b.dy || a.limbs != b.limbs) return false;
    if (a.coeff == b.coeff) return true;
    const size_t words = static_cast<size_t>(a.dx + 1) * (a.dy + 1) * a.limbs;
    return std::memcmp(a.coeff, b.coeff, words * 4) == 0;
  };
  for (int k = 1; k < n; ++k)
    if (var[k] == RSL_X && var[k - 1] == RSL_Y && !J->pstatus[k] && !J->pstatus[k - 1] &&
        !J->plans[k].zero && !J->plans[k - 1].zero && same_poly(f[k], f[k - 1]) && same_poly(g[k], g[k - 1]))
      pair_of[k] = k - 1;
  std::stable_sort(J->live.begin(), J->live.end(), [&](int a, int b) {
    // a pair ranks by its y problem, the x problem right after it
    const int ra = pair_of[a] >= 0 ? pair_of[a] : a, rb = pair_of[b] >= 0 ? pair_of[b] : b;
    if (ra == rb) return pair_of[b] >= 0 && pair_of[a] < 0;
    return cost[ra] > cost[rb] || (cost[ra] == cost[rb] && ra < rb);
  });
  J->need_g = maxg;
  J->need_E = maxE;
  J->need_D = maxD;
  if (ctx && !defer_tables && !J->live.empty()) {
    int rc = ensure_tables(ctx, maxg, maxE, maxD);
    if (rc) { *err = ctx->err; return rc; }
  }

  const int nl = static_cast<int>(J->live.size());
  J->lay.assign(nl, ProbLayout());
  J->dev.assign(nl, DevProblem());
  J->partner.assign(nl, -1);
  J->pshared.assign(nl, 0);
  J->skip_reduce.assign(nl, 0);
  {
    std::vector<int> li_of(n, -1);
    for (int li = 0; li < nl; ++li) li_of[J->live[li]] = li;
    for (int k = 0; k < n; ++k) {
      if (pair_of[k] < 0) continue;
      const int la = li_of[pair_of[k]], lb = li_of[k];
      const Plan &A = J->plans[pair_of[k]], &B = J->plans[k];
      int ns = 0;
      while (ns < A.np && ns < B.np && A.pidx[ns] == B.pidx[ns]) ++ns;
      if (ns == 0) continue;
      J->partner[la] = lb;
      J->pshared[la] = ns;
      J->skip_reduce[lb] = ns;
    }
  }
  J->pairs = 0;
  J->mulmods = 0;
  J->mm_sums_mfma = J->mm_valu = J->mfma_macs = J->interp_mm = 0;
  // stir chunking: enough blocks in flight to cover HBM latency
  int64_t stir_base = 0;
  for (int k : J->live) {
    const Plan& P = J->plans[k];
    stir_base += static_cast<int64_t>(P.np) * blocks_of(P.D + 1, 256);
  }
  // evaluation: with few (prime, point) pairs one lane per pair leaves most
  // SIMDs with a single wave; split each pair over K lanes until about four
  // waves per SIMD are in flight (problems of degree below 4K stay at one lane)
  int64_t all_pairs = 0;
  for (int k : J->live) all_pairs += static_cast<int64_t>(J->plans[k].np) * (J->plans[k].E + 1);
  int evk = J->tune.evk;
  if (opts && opts->eval_lanes > 0) evk = opts->eval_lanes;
  if (evk != 0 && evk != 1 && evk != 2 && evk != 4) {
    *err = "eval_lanes must be 0, 1, 2 or 4";
    return RSL_EINVAL;
  }
  const bool regs_ok = !(opts && opts->eval_regs < 0);
  // long_ok: shapes with |m_y - n_y| > 1 have a register form only with one
  // lane per pair (ures_regs_long, after Horner or the matrix-core sums)
  auto regn_of = [&](const Plan& P, bool long_ok = false) {
    if (!regs_ok || P.my < 1 || P.ny < 1 || (std::abs(P.my - P.ny) > 1 && !long_ok)) return 0;
    for (int nmax : {8, 16, 24, 32})
      if (std::max(P.my, P.ny) <= nmax) return nmax;
    return 0;
  };
  if (evk <= 0) {
    // the register form needs no cross-lane work: keep one lane per pair for it
    bool all_regs = true;
    for (int k : J->live) all_regs = all_regs && regn_of(J->plans[k]) > 0;
    constexpr int64_t kLanesInFlight = 256LL * 4 * 4 * 64;
    evk = 1;
    if (!all_regs)
      while (evk < 4 && all_pairs * evk < kLanesInFlight) evk *= 2;
    else if (all_pairs < 2LL * 256 * 4 * 64)
      evk = 2;  // one wave can issue only about half a SIMD's rate: give each SIMD two
  }
  // interpolation on the matrix cores (staged schedule; the layout keeps the
  // vector items too, for plain runs of the same job)
  // (degree bounds up to kMmMaxD: the operand of a block stays within 64 KB of LDS)
  int dmax = 0;
  for (int k : J->live) dmax = std::max(dmax, J->plans[k].D + 1);
  const bool mm_req = ((opts && opts->interp_mm > 0) || J->tune.interp_mm != 0) && dmax - 1 <= kMmMaxD;
  J->mm_interp = mm_req;
  // one chunk length K for the basis change of every problem, so that problems
  // sharing a prime can share the checkpoint rows; a multiple of the checkpoint
  // spacing, enough chunks for the target number of blocks in flight
  int Kc = kCkpt;
  {
    int64_t nch = 1;
    if (stir_base < target) nch = (target + stir_base - 1) / std::max<int64_t>(stir_base, 1);
    Kc = std::max<int>(kCkpt, static_cast<int>((dmax + nch - 1) / nch));
    if (mm_req) Kc = dmax;  // the matrix-core interpolation writes each sum whole: one chunk
    Kc = (Kc + kCkpt - 1) / kCkpt * kCkpt;  // chunks start at checkpoint rows
  }
  J->crt_ns = 1;
  J->max_np = 0;
  J->any_schur = false;
  const bool schur_req = (opts && opts->eval_schur > 0) || J->tune.schur != 0;
  const bool newton_req = opts && opts->interp_newton > 0;
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    DevProblem& d = J->dev[li];
    d = DevProblem{};
    d.my = P.my;
    d.ny = P.ny;
    d.rowf = P.rowf;
    d.rowg = P.rowg;
    d.myp = (P.my + kRowGroup) / kRowGroup * kRowGroup;
    d.nyp = (P.ny + kRowGroup) / kRowGroup * kRowGroup;
    d.goff = P.rowf * d.myp;
    d.CS = static_cast<int>(align_up(static_cast<size_t>(d.goff) + static_cast<size_t>(P.rowg) * d.nyp, 4));
    d.ncoef = (P.my + 1) * P.rowf + (P.ny + 1) * P.rowg;
    d.L_in = std::max(P.f.L, P.g.L);
    d.D = P.D;
    d.E = P.E;
    d.origin = P.origin;
    d.formal = P.formal;
    d.np = P.np;
    d.L_out = P.L_out;
    d.kchunk = Kc;
    d.nchunk = (P.D + 1 + d.kchunk - 1) / d.kchunk;
    d.evk = 1;
    while (d.evk < evk && std::min(P.my, P.ny) >= 4 * d.evk * 2) d.evk *= 2;
    d.evpb = 64 / d.evk;
    const bool long_ok = d.evk == 1;
    d.regn = (d.evk <= 2) ? regn_of(P, long_ok) : 0;
    d.schur = (schur_req && P.my >= 1 && P.ny >= 1 && P.my + P.ny <= kSchurMaxR) ? 1 : 0;
    d.newton_all = newton_req ? 1 : 0;
    if (d.schur) {  // one wave per pair, kSchurPts points per block
      d.evk = 1;
      d.evpb = kSchurPts;
      d.regn = 0;
      J->any_schur = true;
    }
    // the Horner sums on the matrix cores: the register form (one lane or a
    // lane pair per (prime, point)), x-powers 0..31 in one K slice of the
    // products and x-power 32, if any, on the vector ALUs
    d.evmf = (d.evk <= 2 && d.regn > 0 && !d.schur && P.rowf <= 33 && P.rowg <= 33 && !(ctx && ctx->eval_horner))
                 ? 1 : 0;
    d.dRTf = d.evmf ? dig_rt(P.my + 1) : 0;
    d.dRTg = d.evmf ? dig_rt(P.ny + 1) : 0;
    d.dfr = kDigits * (d.dRTf + d.dRTg);
    d.crt_garner = (ctx && ctx->crt_garner) ? 1 : 0;
    d.wide = P.wide ? 1 : 0;
    d.Lw = P.Lw;
    d.wide_mfma = (P.wide && !(ctx && ctx->wide_valu)) ? 1 : 0;
    d.wdpad = static_cast<int>(align_up(static_cast<size_t>(P.D + 1), kWideMfmaKT));
    d.wlpad = static_cast<int>(align_up(static_cast<size_t>(P.Lw), kWideMfmaTT));
    d.wnpad = static_cast<int>(align_up(static_cast<size_t>(P.np), kWideMfmaK));
    // the convolution's input range: the basis change's chunking, or whole
    d.cchunk = (J->tune.conv_whole || mm_req) ? P.D + 1 : d.kchunk;
    d.ncchunk = (P.D + 1 + d.cchunk - 1) / d.cchunk;
    if (!P.wide) J->crt_ns = std::max(J->crt_ns, (P.np + 63) / 64);
    J->max_np = std::max(J->max_np, P.np);
    J->pairs += static_cast<int64_t>(P.np) * (P.E + 1);
    J->mulmods += pair_mulmods(P) * P.np * (P.E + 1);
    {
      const int64_t pts = static_cast<int64_t>(P.np) * (P.E + 1);
      const int64_t sums = pair_mulmods(P) - static_cast<int64_t>(P.my) * P.ny;  // N_f + N_g
      if (d.evmf) {
        int64_t top = 0;  // terms of x-power 32 (vector ALUs)
        for (int r : P.f.rdeg) top += (r == 32);
        for (int r : P.g.rdeg) top += (r == 32);
        J->mm_sums_mfma += (sums - top) * pts;
        J->mm_valu += (static_cast<int64_t>(P.my) * P.ny + top) * pts;
        // 25 int8 16x16x32 products per 16-point tile and 16-row tile
        const int64_t tiles = static_cast<int64_t>(P.np) * blocks_of(P.E + 1, d.evpb) * (d.evpb / 16);
        J->mfma_macs += tiles * (d.dRTf + d.dRTg) * kDigits * kDigits * 16 * 16 * 32;
      } else {
        J->mm_valu += pair_mulmods(P) * pts;
      }
      J->interp_mm += static_cast<int64_t>(P.np) * (P.D + 1) * (P.D + 2);
    }
  }

  if (J->crt_ns == 5 || J->crt_ns == 7) ++J->crt_ns;  // CRT kernels exist for 1-4, 6 and 8 slots per lane
  for (int li = 0; li < nl; ++li)
    if (J->partner[li] >= 0) {
      const DevProblem& b = J->dev[J->partner[li]];
      DevProblem& a = J->dev[li];
      a.pshared = J->pshared[li];
      a.pmyp = b.myp;
      a.pnyp = b.nyp;
      a.pgoff = b.goff;
      a.pCS = b.CS;
      a.pdRTf = b.dRTf;
      a.pdRTg = b.dRTg;
      a.pdfr = b.dfr;
    }

  // work items, problem by problem (so that each problem's items are
  // contiguous): each problem's items of each stage are counted, the lists
  // sized, and every problem writes its own ranges (in parallel)
  constexpr int kHsegList = kNumStages;  // the segment polynomials' list after the stage lists
  auto emit = [&](int li, int s, WorkItem* out) -> int {
    const Plan& P = J->plans[J->live[li]];
    const DevProblem& d = J->dev[li];
    int c = 0;
    auto put = [&](int slot, int blk, int sub) {
      if (out) out[c] = WorkItem{li, slot, blk, sub};
      ++c;
    };
    switch (s) {
      case kStageReduce: {
        // slots below skip_reduce are reduced by the partner (the same system
        // in y); item slot 0 of block 0 also clears the statuses, so a problem
        // whose slots are all shared keeps one such item
        const int s0 = J->skip_reduce[li];
        if (d.evmf && d.L_in <= 2 && J->partner[li] < 0 && s0 == 0) {  // digit planes a word at a time
          const int nb = blocks_of(reduce_words(d.my, d.ny, d.rowf, d.rowg), 256);
          for (int sl = 0; sl < P.np; ++sl)
            for (int b = 0; b < nb; ++b) put(sl, b, 2);
        } else if (d.L_in > 2) {  // long limb chains: staged limbs, eight primes per thread
          const int first = (s0 / kReduceMlSlots) * kReduceMlSlots;
          for (int sl = first; sl < P.np; sl += kReduceMlSlots)
            for (int b = 0; b < blocks_of(d.CS, kReduceMlCoeffs); ++b) put(sl, b, 1);
          if (first > 0) put(0, 0, 1);
        } else {
          for (int sl = s0; sl < P.np; ++sl)
            for (int b = 0; b < blocks_of(d.CS, 256); ++b) put(sl, b, 0);
          if (s0 > 0) put(0, 0, 0);
        }
        break;
      }
      case kStageEval:
        for (int sl = 0; sl < P.np; ++sl)
          for (int b = 0; b < blocks_of(P.E + 1, d.evpb); ++b) put(sl, b, 0);
        break;
      case kStageConv:
        for (int sl = 0; sl < P.np; ++sl)
          for (int b = 0; b < blocks_of(P.D + 1, 256); ++b)
            for (int ch = 0; ch < d.ncchunk; ++ch)
              if (ch * d.cchunk <= std::min(P.D, b * 256 + 255)) put(sl, b, ch);
        break;
      case kStageStir:  // basis change: blocks of 256 columns
        for (int sl = 0; sl < P.np; ++sl)
          for (int b = 0; b < blocks_of(P.D + 1, 256); ++b)
            for (int ch = 0; ch < d.nchunk; ++ch)
              if (std::min(P.D, (ch + 1) * d.kchunk - 1) >= b * 256) put(sl, b, ch);
        break;
      case kStageNewton:
        // gapped interpolation is possible only with a non-constant leading
        // coefficient (bad points) or a shifted origin
        if (P.origin != 0 || (!P.formal && P.s > 0) || d.newton_all)
          for (int sl = 0; sl < P.np; ++sl) put(sl, 0, 0);
        break;
      case kStageCrt:
        if (!P.wide)
          for (int b = 0; b < blocks_of(P.D + 1, kCrtWaves); ++b) put(-1, b, 0);
        break;
      case kHsegList:
        for (int sl = 0; sl < P.np; ++sl)
          for (int b = 0; b < blocks_of(P.D + 1, kHsegRows); ++b) put(sl, b, 0);
        break;
    }
    return c;
  };
  {
    constexpr int kLists = kNumStages + 1;
    std::vector<int>& cnt = J->tmp_a;
    cnt.assign(static_cast<size_t>(nl) * kLists, 0);
    parallel_for(nl, 16, [&](int li) {
      for (int s = 0; s < kLists; ++s) cnt[static_cast<size_t>(li) * kLists + s] = emit(li, s, nullptr);
    });
    std::vector<int>& off = J->tmp_b;
    off.assign(cnt.size(), 0);
    // the evaluation items grouped by layout variant (problem order within a
    // variant): each variant is one launch of the staged schedule
    std::vector<int>& var_of = J->tmp_c;
    var_of.resize(nl);
    int nv = 1;
    for (int li = 0; li < nl; ++li) {
      var_of[li] = eval_variant(J->dev[li]);
      nv = std::max(nv, var_of[li] + 1);
    }
    J->eval_vstart.assign(static_cast<size_t>(nv) + 1, 0);
    for (int s = 0; s < kLists; ++s) {
      int o = 0;
      for (int v = 0; v < (s == kStageEval ? nv : 1); ++v) {
        if (s == kStageEval) J->eval_vstart[v] = o;
        for (int li = 0; li < nl; ++li) {
          if (s == kStageEval && var_of[li] != v) continue;
          off[static_cast<size_t>(li) * kLists + s] = o;
          o += cnt[static_cast<size_t>(li) * kLists + s];
        }
      }
      if (s == kStageEval) J->eval_vstart[nv] = o;
      std::vector<WorkItem>& v = s < kNumStages ? J->items[s] : J->hseg_items;
      v.clear();
      v.resize(o);
    }
    parallel_for(nl, 16, [&](int li) {
      ProbLayout& L = J->lay[li];
      for (int s = 0; s < kLists; ++s) {
        const size_t at = static_cast<size_t>(li) * kLists + s;
        std::vector<WorkItem>& v = s < kNumStages ? J->items[s] : J->hseg_items;
        emit(li, s, v.data() + off[at]);
        if (s < kNumStages) {
          L.item_begin[s] = off[at];
          L.item_end[s] = off[at] + cnt[at];
        } else {
          L.hseg_begin = off[at];
          L.hseg_end = off[at] + cnt[at];
        }
      }
    });
  }

  // wide CRT items, problem by problem
  for (int pass = 0; pass < 3; ++pass) J->wide_items[pass].clear();
  J->wide_mfma = false;
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    const DevProblem& d = J->dev[li];
    ProbLayout& L = J->lay[li];
    for (int pass = 0; pass < 3; ++pass) L.wide_begin[pass] = static_cast<int>(J->wide_items[pass].size());
    if (P.wide) {
      for (int b = 0; b < blocks_of(P.D + 1, kWideTCoeffs); ++b) J->wide_items[0].push_back({li, -1, b, 0});
      // column sums: the blocks of one limb tile read the same columns of
      // the M_i table, so they are dealt onto one XCD (workgroup i of a launch
      // runs on XCD i mod 8; a problem's range starts anywhere, but its items
      // of one tile keep one residue mod 8)
      constexpr int kXcds = 8;
      const bool mfma = d.wide_mfma != 0;
      J->wide_mfma = mfma;
      const int nkt = mfma ? d.wdpad / kWideMfmaKT : blocks_of(P.D + 1, kWideKT);
      const int nht = mfma ? d.wlpad / kWideMfmaTT : blocks_of(P.Lw, kWideHT);
      std::vector<std::vector<WorkItem>> bins(kXcds);
      for (int ht = 0; ht < nht; ++ht)
        for (int kt = 0; kt < nkt; ++kt) bins[ht % kXcds].push_back({li, -1, kt, ht});
      std::vector<size_t> pos(kXcds, 0);
      for (int t = 0; t < nkt * nht; ++t) {
        int x = t % kXcds;
        if (pos[x] >= bins[x].size()) {  // bin x is empty: take from the fullest
          size_t best = 0;
          for (int y = 0; y < kXcds; ++y)
            if (bins[y].size() - pos[y] > best) {
              best = bins[y].size() - pos[y];
              x = y;
            }
        }
        J->wide_items[1].push_back(bins[x][pos[x]++]);
      }
      for (int k = 0; k <= P.D; ++k) J->wide_items[2].push_back({li, -1, k, 0});
    }
    for (int pass = 0; pass < 3; ++pass) L.wide_end[pass] = static_cast<int>(J->wide_items[pass].size());
  }

  // evaluation items: grouped by layout variant as they were written (a
  // problem's items stay together, as the one-pipeline-per-problem schedule needs)
  {
    const std::vector<WorkItem>& ev = J->items[kStageEval];
    const std::vector<int>& vstart = J->eval_vstart;
    const int nv = static_cast<int>(vstart.size()) - 1;
    J->eval_ranges.clear();
    // each variant's launch sized for its own problems (a small register
    // form keeps more waves per CU than the largest problem's LDS would allow)
    std::vector<size_t> vlds(static_cast<size_t>(nv), 0);
    for (int li = 0; li < nl; ++li)
      vlds[J->tmp_c[li]] = std::max(vlds[J->tmp_c[li]], static_cast<size_t>(eval_stage_lds_words(J->dev[li])) * 4);
    for (int v = 0; v < nv; ++v)
      if (vstart[v] < vstart[v + 1])
        J->eval_ranges.push_back({v, static_cast<int>(vstart[v]), static_cast<int>(vstart[v + 1]), vlds[v]});
    // the staged launches take the same items dealt so that all blocks of one
    // (problem, prime) run on the same XCD: workgroup i of a launch goes to
    // XCD i mod 8, so the prime's coefficient tile is fetched into one L2
    // instead of eight.  Per variant range: the g-th (problem, prime) of the
    // range goes to bin g mod 8, and launch position t takes the next item of
    // bin t mod 8 (of the bin with the most items left once that one is empty).
    // The ranges are independent: one host thread each.
    constexpr int kXcds = 8;
    J->eval_staged.resize(ev.size());
    std::vector<int>& bin = J->tmp_a;
    std::vector<int>& order = J->tmp_b;  // items of the range by bin, stable
    bin.resize(ev.size());
    order.resize(ev.size());
    parallel_for(static_cast<int>(J->eval_ranges.size()), 1, [&](int ri) {
      const size_t b0 = static_cast<size_t>(J->eval_ranges[ri].begin), b1 = static_cast<size_t>(J->eval_ranges[ri].end);
      size_t bsize[kXcds] = {}, bstart[kXcds + 1] = {}, pos[kXcds] = {};
      int pairs_seen = -1, last_prob = -1, last_slot = -1;
      for (size_t t = b0; t < b1; ++t) {
        if (ev[t].prob != last_prob || ev[t].slot != last_slot) {
          ++pairs_seen;
          last_prob = ev[t].prob;
          last_slot = ev[t].slot;
        }
        bin[t] = pairs_seen % kXcds;
        ++bsize[bin[t]];
      }
      for (int x = 0; x < kXcds; ++x) bstart[x + 1] = bstart[x] + bsize[x];
      {
        size_t fill[kXcds];
        for (int x = 0; x < kXcds; ++x) fill[x] = bstart[x];
        for (size_t t = b0; t < b1; ++t) order[b0 + fill[bin[t]]++] = static_cast<int>(t);
      }
      for (size_t t = b0; t < b1; ++t) {
        int x = static_cast<int>((t - b0) % kXcds);
        if (pos[x] >= bsize[x]) {  // bin x is empty: take from the fullest
          size_t best = 0;
          for (int y = 0; y < kXcds; ++y)
            if (bsize[y] - pos[y] > best) {
              best = bsize[y] - pos[y];
              x = y;
            }
        }
        J->eval_staged[t] = ev[order[b0 + bstart[x] + pos[x]++]];
      }
    });
  }

  // prime groups for the basis change: every (problem, slot) by global prime
  // index (slots whose points turn out gapped skip their share)
  J->sgroups.clear();
  J->smembers.clear();
  J->sg_items.clear();
  J->sg_lds = 0;
  {
    // (problem, slot) members by global prime index: a stable counting sort
    int gidx = 0;
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      for (int sl = 0; sl < P.np; ++sl) gidx = std::max(gidx, P.pidx[sl] + 1);
    }
    std::vector<int> pstart(static_cast<size_t>(gidx) + 1, 0);
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      for (int sl = 0; sl < P.np; ++sl) ++pstart[P.pidx[sl] + 1];
    }
    for (int gi = 0; gi < gidx; ++gi) pstart[gi + 1] += pstart[gi];
    std::vector<StirMember> by_prime(pstart[gidx]);
    {
      std::vector<int> fill(pstart.begin(), pstart.end() - 1);
      for (int li = 0; li < nl; ++li) {
        const Plan& P = J->plans[J->live[li]];
        for (int sl = 0; sl < P.np; ++sl) by_prime[fill[P.pidx[sl]]++] = StirMember{li, sl};
      }
    }
    int gmax = kStirGroupMax;
    while (gmax > 1 && stir_group_lds_words(gmax, 256) > kLdsWords) --gmax;
    J->smembers.reserve(by_prime.size());
    for (int prime = 0; prime < gidx; ++prime) {
      const StirMember* mem = by_prime.data() + pstart[prime];
      const size_t msize = static_cast<size_t>(pstart[prime + 1] - pstart[prime]);
      for (size_t b = 0; b < msize; b += gmax) {
        StirGroup G{prime, static_cast<int>(J->smembers.size()), static_cast<int>(std::min<size_t>(gmax, msize - b)),
                    0};
        for (int m = 0; m < G.count; ++m) {
          J->smembers.push_back(mem[b + m]);
          G.maxD = std::max(G.maxD, J->dev[mem[b + m].prob].D);
        }
        const int gi = static_cast<int>(J->sgroups.size());
        J->sgroups.push_back(G);
        J->sg_lds = std::max<size_t>(J->sg_lds, static_cast<size_t>(stir_group_lds_words(kStirGroupMax, 256)) * 4);
        for (int jb = 0; jb < blocks_of(G.maxD + 1, 256); ++jb)
          for (int ch = 0; ch * Kc <= G.maxD; ++ch) {
            const int ke = std::min(G.maxD, (ch + 1) * Kc - 1);
            if (ke >= jb * 256) J->sg_items.push_back({gi, -1, jb, ch});
          }
      }
    }
  }

  // matrix-core interpolation: every (problem, slot) by global prime
  // index (a stable counting sort), groups of all members of a prime
  J->mgroups.clear();
  J->mmembers.clear();
  J->dig_items.clear();
  J->mm_items.clear();
  J->mm_lds[0] = J->mm_lds[1] = 0;
  if (mm_req) {
    int gidx = 0;
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      for (int sl = 0; sl < P.np; ++sl) gidx = std::max(gidx, P.pidx[sl] + 1);
    }
    std::vector<int> pstart(static_cast<size_t>(gidx) + 1, 0);
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      for (int sl = 0; sl < P.np; ++sl) ++pstart[P.pidx[sl] + 1];
    }
    for (int gi = 0; gi < gidx; ++gi) pstart[gi + 1] += pstart[gi];
    J->mmembers.resize(pstart[gidx]);
    {
      std::vector<int> fill(pstart.begin(), pstart.end() - 1);
      for (int li = 0; li < nl; ++li) {
        const Plan& P = J->plans[J->live[li]];
        for (int sl = 0; sl < P.np; ++sl) J->mmembers[fill[P.pidx[sl]]++] = StirMember{li, sl};
      }
    }
    for (int prime = 0; prime < gidx; ++prime) {
      const int first = pstart[prime], count = pstart[prime + 1] - first;
      if (count == 0) continue;
      // largest degree bound first: each 16-column tile is bounded by its first column
      std::stable_sort(J->mmembers.begin() + first, J->mmembers.begin() + first + count,
                       [&](const StirMember& a, const StirMember& b) { return J->dev[a.prob].D > J->dev[b.prob].D; });
      StirGroup G{prime, first, count, 0};
      for (int m = first; m < first + count; ++m) G.maxD = std::max(G.maxD, J->dev[J->mmembers[m].prob].D);
      const int gi = static_cast<int>(J->mgroups.size());
      J->mgroups.push_back(G);
      // items: (group, 64 rows, a run of 16-column tiles whose slices add up to
      // about kMmRunSlices); a tile whose largest bound is below the rows has
      // nothing there, and neither have the tiles after it
      const int ntile = blocks_of(count, 16);
      for (int rs = 0; rs < blocks_of(G.maxD + 1, 64); ++rs) {
        const int rs0 = 64 * rs;
        int ct = 0;
        while (ct < ntile) {
          const int tileD0 = J->dev[J->mmembers[first + 16 * ct].prob].D;
          if (tileD0 < rs0) break;
          for (int which = 1; which <= 2; ++which)
            J->mm_lds[which - 1] = std::max(J->mm_lds[which - 1], kMmColBytes + mm_operand_bytes(which, rs0, tileD0));
          int n = 0, cost = 0;
          while (ct + n < ntile && n < kMmTilesMax && cost < kMmRunSlices) {
            const int tD = J->dev[J->mmembers[first + 16 * (ct + n)].prob].D;
            if (tD < rs0) break;
            const int c1 = mm_slices_hi(1, rs0, tD) - mm_slices_lo(1, rs0) + 1;
            const int c2 = mm_slices_hi(2, rs0, tD) - mm_slices_lo(2, rs0) + 1;
            cost += std::max(c1, c2);
            ++n;
          }
          J->mm_items.push_back({gi, rs, ct, n + 32 * tileD0});
          ct += n;
        }
      }
    }
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      const int Dp = static_cast<int>(align_up(static_cast<size_t>(P.D + 1), kCkpt));
      for (int sl = 0; sl < P.np; ++sl)
        for (int b = 0; b < blocks_of(Dp, kDigitsPerBlock); ++b) J->dig_items.push_back({li, sl, b, 0});
    }
  }

  // device layout: [problems | items | inputs | statuses][outputs][intermediates]
  const size_t A = 256;
  size_t o = 0;
  J->probs_off = o;
  o = align_up(o + sizeof(DevProblem) * std::max(nl, 1), A);
  for (int s = 0; s < kNumStages; ++s) {
    J->items_off[s] = o;
    o = align_up(o + sizeof(WorkItem) * J->items[s].size(), A);
  }
  J->evs_off = o;
  o = align_up(o + sizeof(WorkItem) * J->eval_staged.size(), A);
  J->sg_off = o;
  o = align_up(o + sizeof(StirGroup) * J->sgroups.size(), A);
  J->sm_off = o;
  o = align_up(o + sizeof(StirMember) * J->smembers.size(), A);
  J->sgi_off = o;
  o = align_up(o + sizeof(WorkItem) * J->sg_items.size(), A);
  J->hseg_off = o;
  o = align_up(o + sizeof(WorkItem) * J->hseg_items.size(), A);
  J->mg_off = o;
  o = align_up(o + sizeof(StirGroup) * J->mgroups.size(), A);
  J->mm_off = o;
  o = align_up(o + sizeof(StirMember) * J->mmembers.size(), A);
  J->digi_off = o;
  o = align_up(o + sizeof(WorkItem) * J->dig_items.size(), A);
  J->mmi_off = o;
  o = align_up(o + sizeof(WorkItem) * J->mm_items.size(), A);
  for (int pass = 0; pass < 3; ++pass) {
    J->wide_off[pass] = o;
    o = align_up(o + sizeof(WorkItem) * J->wide_items[pass].size(), A);
  }
  J->nclr = 0;
  for (int li = 0; li < nl; ++li)
    J->nclr += (J->dev[li].wide ? 1 : 0) + (J->dev[li].evmf ? 1 : 0) + (J->skip_reduce[li] > 0 ? 1 : 0);
  J->clr_off = o;
  o = align_up(o + sizeof(ClearRange) * J->nclr, A);
  // CRT constants are laid out once per prime list (problems with the same
  // canonical list share them)
  std::map<const CrtConst*, int> crt_owner;
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    const DevProblem& d = J->dev[li];
    ProbLayout& L = J->lay[li];
    L.L_in = d.L_in;
    L.coeff = o; o = align_up(o + static_cast<size_t>(d.ncoef) * d.L_in * 4, 16);
    L.gdeg = o;  o = align_up(o + static_cast<size_t>(d.myp + d.nyp) / kRowGroup * 4, 16);
    L.pidx = o;  o = align_up(o + static_cast<size_t>(P.np) * 4, 16);
    auto own = crt_owner.find(P.crt.get());
    if (own != crt_owner.end()) {
      const ProbLayout& S = J->lay[own->second];
      L.Hm = S.Hm; L.NH = S.NH; L.Mi = S.Mi; L.wdir = S.wdir; L.rinv = S.rinv; L.negM = S.negM;
      L.Mw = S.Mw; L.wMd = S.wMd; L.NHM = S.NHM; L.Tg = S.Tg; L.invM = S.invM; L.Plimb = S.Plimb;
      L.crt_own = false;
      continue;
    }
    crt_owner[P.crt.get()] = li;
    L.crt_own = true;
    L.Hm = o;    o = align_up(o + static_cast<size_t>(P.np) * 4, 16);
    L.NH = o;    o = align_up(o + static_cast<size_t>(P.L_out) * 4, 16);
    L.Mi = o;    o = align_up(o + static_cast<size_t>(P.np) * P.Lw * 4, 16);
    L.wdir = o;  o = align_up(o + static_cast<size_t>(P.np) * 4, 16);
    L.rinv = o;  o = align_up(o + static_cast<size_t>(P.np) * 8, 16);
    L.negM = o;  o = align_up(o + static_cast<size_t>(P.Lw) * 4, 16);
    L.Mw = L.NHM = 0;
    if (P.wide) {
      L.Mw = o;  o = align_up(o + static_cast<size_t>(P.Lw) * 4, 16);
      L.wMd = o; o = align_up(o + static_cast<size_t>(kWideDigits) * d.wlpad * d.wnpad, 16);
      L.NHM = o; o = align_up(o + static_cast<size_t>(P.L_out) * 4, 16);
    }
    if (!P.canonical) {
      L.Tg = o;    o = align_up(o + static_cast<size_t>(P.np) * P.np * 4, 16);
      L.invM = o;  o = align_up(o + static_cast<size_t>(P.np) * 4, 16);
      L.Plimb = o; o = align_up(o + static_cast<size_t>(P.np) * P.L_out * 4, 16);
    }
  }
  // persistent queue: [state | tasks | ready | counters]; an initial image is
  // uploaded with the inputs and copied to the live queue before each launch
  {
    int64_t cap = 0, crt_total = 0, initial = 0;
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      const DevProblem& d = J->dev[li];
      const int64_t ne = blocks_of(P.E + 1, d.evpb), nc = blocks_of(P.D + 1, 64);
      const int64_t ns = blocks_of(P.D + 1, 64) * d.nchunk;
      cap += static_cast<int64_t>(P.np) * (1 + ne + std::max<int64_t>(nc * d.ncchunk + ns + (P.origin != 0), 1));
      const int64_t ncrt = blocks_of(P.D + 1, kCrtPerTask);
      cap += ncrt;
      crt_total += ncrt;
      initial += P.np;
    }
    J->q_capacity = static_cast<int>(std::max<int64_t>(cap, 1));
    J->q_crt_total = static_cast<int>(crt_total);
    J->q_initial = static_cast<int>(initial);
    size_t qo = 0;
    qo = align_up(qo + sizeof(QueueState), A);
    J->q_tasks = qo;
    qo = align_up(qo + sizeof(Task) * J->q_capacity, A);
    J->q_ready = qo;
    qo = align_up(qo + sizeof(int) * J->q_capacity, A);
    J->q_counters = qo;
    qo = align_up(qo + sizeof(ProbCounters) * std::max(nl, 1), A);
    J->queue_bytes = qo;
    o = align_up(o, A);
    J->qinit_off = o;
    o += J->queue_bytes;
  }
  o = align_up(o, A);
  J->status_off = o;
  for (int li = 0; li < nl; ++li) {
    J->lay[li].status = o;
    o += static_cast<size_t>(2 * J->plans[J->live[li]].np + 2) * 4;
  }
  o = align_up(o, A);
  J->status_bytes = o - J->status_off;
  J->up_bytes = o;
  J->down_off = J->status_off;
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    J->lay[li].out = o;
    o = align_up(o + static_cast<size_t>(P.D + 1) * P.L_out * 4, 16);
  }
  o = align_up(o, A);
  J->down_bytes = o - J->down_off;
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    const DevProblem& d = J->dev[li];
    ProbLayout& L = J->lay[li];
    const size_t np = P.np;
    L.resid = o; o = align_up(o + np * d.CS * 4, A);
    L.dig = o;   o = align_up(o + np * d.dfr * 512, A);
    L.zval = o;  o = align_up(o + np * (P.E + 1) * 4, A);
    L.zbad = o;  o = align_up(o + np * (P.E + 1), A);
    L.aconv = o; o = align_up(o + static_cast<size_t>(d.ncchunk) * np * (P.D + 1) * 8, A);
    L.cpart = o; o = align_up(o + static_cast<size_t>(d.nchunk) * np * (P.D + 1) * 8, A);
    L.hseg = o;  o = align_up(o + np * align_up(static_cast<size_t>(P.D + 1), kCkpt) * 4, A);
    L.ydig = L.hdig = 0;
    if (mm_req) {  // digit planes of the matrix-core interpolation
      const size_t planes = np * kDigits * align_up(static_cast<size_t>(P.D + 1), kCkpt);
      L.ydig = o; o = align_up(o + planes, A);
      L.hdig = o; o = align_up(o + planes, A);
    }
    L.wT = L.wq = L.wS = 0;
    if (P.wide) {
      L.wT = o; o = align_up(o + static_cast<size_t>(d.wdpad) * d.wnpad * 4, A);
      L.wq = o; o = align_up(o + static_cast<size_t>(P.D + 1) * 4, A);
      L.wS = o; o = align_up(o + static_cast<size_t>(P.D + 1) * 2 * P.Lw * 8, A);
    }
  }
  J->queue_off = o;
  o = align_up(o + J->queue_bytes, A);
  J->total = o;

  // LDS per stage launch (max over problems)
  for (int s = 0; s < kNumStages; ++s) J->stage_lds[s] = 0;
  for (int li = 0; li < nl; ++li) {
    const DevProblem& d = J->dev[li];
    auto up = [&](int s, size_t words) { J->stage_lds[s] = std::max(J->stage_lds[s], words * 4); };
    up(kStageEval, eval_stage_lds_words(d));
    up(kStageConv, static_cast<size_t>(std::min(d.cchunk, d.D + 1)) + std::min(d.D + 1, d.cchunk + 256));
    up(kStageStir, std::max(basis_lds_words(1, 256, 0), kHsegRows));
    if (J->lay[li].item_end[kStageNewton] > J->lay[li].item_begin[kStageNewton]) up(kStageNewton, newton_lds_words(d, 1024));
    if (!d.wide) up(kStageCrt, crt_lds_words(d, J->crt_ns, crt_block_waves(J->crt_ns)));
    if (d.L_in > 2) up(kStageReduce, reduce_ml_lds_words());
  }
  for (int pass = 0; pass < 3; ++pass) J->wide_lds[pass] = 0;
  for (int li = 0; li < nl; ++li) {
    const DevProblem& d = J->dev[li];
    if (!d.wide) continue;
    J->wide_lds[0] = static_cast<size_t>(wide_t_lds_words()) * 4;
    J->wide_lds[1] = static_cast<size_t>(J->wide_mfma ? wide_mfma_lds_words() : wide_sum_lds_words()) * 4;
    J->wide_lds[2] = std::max(J->wide_lds[2], static_cast<size_t>(wide_fin_lds_words(d)) * 4);
  }
  J->persist_lds = 0;
  for (int li = 0; li < nl; ++li) {
    const DevProblem& d = J->dev[li];
    size_t w = std::max(eval_group_lds_words(d, d.evk), eval_lds_words(d));  // no register form here
    w = std::max<size_t>(w, static_cast<size_t>(std::min(d.cchunk, d.D + 1)) + std::min(d.D + 1, d.cchunk + 64));
    w = std::max<size_t>(w, basis_lds_words(1, 64, d.kchunk));
    if (J->lay[li].item_end[kStageNewton] > J->lay[li].item_begin[kStageNewton])
      w = std::max<size_t>(w, newton_lds_words(d, 64));
    if (!d.wide) w = std::max<size_t>(w, crt_lds_words(d, J->crt_ns, 1));
    J->persist_lds = std::max(J->persist_lds, w * 4);
  }
  for (int s = 0; s < kNumStages; ++s)
    if (J->stage_lds[s] > static_cast<size_t>(kLdsWords) * 4 ||
        (s < 3 && J->wide_lds[s] > static_cast<size_t>(kLdsWords) * 4)) {
      *err = "a stage needs more than 64 KB of LDS";
      return RSL_EINVAL;
    }
  return RSL_OK;
}

void job_bind(Job* J, uint8_t* base, uint8_t* image, bool with_queue) {
  J->base = base;
  J->with_queue = with_queue;
  const int nl = static_cast<int>(J->live.size());
  if (!image) {
    J->blob.assign(J->up_bytes, 0);
    image = J->blob.data();
  } else {
    J->blob.clear();
    // an external image is not zeroed: the queue's ready flags and the
    // statuses must start at zero (every other region is written whole)
    if (with_queue) std::memset(image + J->qinit_off, 0, J->up_bytes - J->qinit_off);
  }
  J->image = image;
  uint8_t* blob = image;
  // each problem writes its own regions (a shared CRT block only by its owner)
  parallel_for(nl, 8, [&](int li) {
    const Plan& P = J->plans[J->live[li]];
    const ProbLayout& L = J->lay[li];
    DevProblem& d = J->dev[li];
    // inputs: f rows 0..my (stride rowf) then g rows 0..ny (stride rowg),
    // sign-extended to L_in limbs
    uint32_t* c = reinterpret_cast<uint32_t*>(blob + L.coeff);
    const int Li = L.L_in;
    auto put = [&](const View& V, int rows, int rowstride, size_t first) {
      for (int j = 0; j < rows; ++j)
        for (int i = 0; i < rowstride; ++i) {
          uint32_t* dst = c + (first + static_cast<size_t>(j) * rowstride + i) * Li;
          if (i <= V.rdeg[j]) {
            const uint32_t* src = &V.c[(static_cast<size_t>(j) * (V.dx + 1) + i) * V.L];
            const uint32_t ext = (src[V.L - 1] >> 31) ? 0xFFFFFFFFu : 0u;
            for (int l = 0; l < Li; ++l) dst[l] = (l < V.L) ? src[l] : ext;
          } else {
            for (int l = 0; l < Li; ++l) dst[l] = 0;
          }
        }
    };
    put(P.f, P.my + 1, P.rowf, 0);
    put(P.g, P.ny + 1, P.rowg, static_cast<size_t>(P.my + 1) * P.rowf);
    int* gd = reinterpret_cast<int*>(blob + L.gdeg);
    const int gf = d.myp / kRowGroup, gg = d.nyp / kRowGroup;
    for (int q = 0; q < gf; ++q) {
      int m = -1;
      for (int j = q * kRowGroup; j < (q + 1) * kRowGroup && j <= P.my; ++j) m = std::max(m, P.f.rdeg[j]);
      gd[q] = m;
    }
    for (int q = 0; q < gg; ++q) {
      int m = -1;
      for (int j = q * kRowGroup; j < (q + 1) * kRowGroup && j <= P.ny; ++j) m = std::max(m, P.g.rdeg[j]);
      gd[gf + q] = m;
    }
    std::memcpy(blob + L.pidx, P.pidx.data(), P.np * 4);
    if (L.crt_own) {
    std::memcpy(blob + L.Hm, P.crt->Hm.data(), P.np * 4);
    std::memcpy(blob + L.NH, P.crt->NH.data(), P.L_out * 4);
    std::memcpy(blob + L.Mi, P.crt->Mi.data(), P.crt->Mi.size() * 4);
    std::memcpy(blob + L.wdir, P.crt->wdir.data(), P.crt->wdir.size() * 4);
    std::memcpy(blob + L.rinv, P.crt->rinv.data(), P.crt->rinv.size() * 4);
    std::memcpy(blob + L.negM, P.crt->negM.data(), P.crt->negM.size() * 4);
    if (P.wide) {
      std::memcpy(blob + L.Mw, P.crt->Mw.data(), P.crt->Mw.size() * 4);
      std::memcpy(blob + L.NHM, P.crt->NHM.data(), P.crt->NHM.size() * 4);
      // 7-bit digit planes of the M_i limbs, [digit][limb][prime], zero padded
      int8_t* md = reinterpret_cast<int8_t*>(blob + L.wMd);
      const size_t plane = static_cast<size_t>(d.wlpad) * d.wnpad;
      for (int i = 0; i < P.np; ++i)
        for (int t = 0; t < P.Lw; ++t) {
          const uint32_t m = P.crt->Mi[static_cast<size_t>(i) * P.Lw + t];
          for (int dd = 0; dd < kWideDigits; ++dd)
            md[dd * plane + static_cast<size_t>(t) * d.wnpad + i] = static_cast<int8_t>((m >> (7 * dd)) & 127u);
        }
    }
    if (!P.canonical) {
      std::memcpy(blob + L.Tg, P.crt->Tg.data(), P.crt->Tg.size() * 4);
      std::memcpy(blob + L.invM, P.crt->invM.data(), P.crt->invM.size() * 4);
      std::memcpy(blob + L.Plimb, P.crt->Plimb.data(), P.crt->Plimb.size() * 4);
    }
    }  // crt_own
    // device pointers
    d.coeff = reinterpret_cast<const uint32_t*>(base + L.coeff);
    d.gdeg = reinterpret_cast<const int*>(base + L.gdeg);
    d.pidx = reinterpret_cast<const int*>(base + L.pidx);
    d.Hm = reinterpret_cast<const uint32_t*>(base + L.Hm);
    d.NH = reinterpret_cast<const uint32_t*>(base + L.NH);
    d.Mi = reinterpret_cast<const uint32_t*>(base + L.Mi);
    d.wdir = reinterpret_cast<const uint32_t*>(base + L.wdir);
    d.rinv = reinterpret_cast<const uint32_t*>(base + L.rinv);
    d.negM = reinterpret_cast<const uint32_t*>(base + L.negM);
    d.Mw = P.wide ? reinterpret_cast<const uint32_t*>(base + L.Mw) : nullptr;
    d.NHM = P.wide ? reinterpret_cast<const uint32_t*>(base + L.NHM) : nullptr;
    d.wT = P.wide ? reinterpret_cast<uint32_t*>(base + L.wT) : nullptr;
    d.wq = P.wide ? reinterpret_cast<uint32_t*>(base + L.wq) : nullptr;
    d.wS = P.wide ? reinterpret_cast<uint64_t*>(base + L.wS) : nullptr;
    d.wMd = (P.wide && d.wide_mfma) ? reinterpret_cast<const int8_t*>(base + L.wMd) : nullptr;
    d.resid = reinterpret_cast<uint32_t*>(base + L.resid);
    d.dig = d.evmf ? reinterpret_cast<uint64_t*>(base + L.dig) : nullptr;
    d.zval = reinterpret_cast<uint32_t*>(base + L.zval);
    d.zbad = base + L.zbad;
    d.aconv = reinterpret_cast<uint64_t*>(base + L.aconv);
    d.cpart = reinterpret_cast<uint64_t*>(base + L.cpart);
    d.hseg = reinterpret_cast<uint32_t*>(base + L.hseg);
    d.ydig = L.ydig ? base + L.ydig : nullptr;
    d.hdig = L.hdig ? base + L.hdig : nullptr;
    d.hstride = static_cast<int>(align_up(static_cast<size_t>(P.D + 1), kCkpt));
    d.out = reinterpret_cast<uint32_t*>(base + L.out);
    d.status = reinterpret_cast<int*>(base + L.status);
  });
  for (int li = 0; li < nl; ++li) {
    const int pa = J->partner[li];
    J->dev[li].presid = (pa >= 0) ? reinterpret_cast<uint32_t*>(base + J->lay[pa].resid) : nullptr;
    J->dev[li].pdig = (pa >= 0 && J->dev[pa].evmf) ? reinterpret_cast<uint64_t*>(base + J->lay[pa].dig) : nullptr;
  }
  // the clear table: the t rows of the wide CRT (their padding stays zero),
  // the digit tiles (only the coefficient positions are written) and the
  // residue tiles a partner fills (its padding)
  {
    ClearRange* cr = reinterpret_cast<ClearRange*>(blob + J->clr_off);
    int c = 0;
    for (int li = 0; li < nl; ++li) {
      const DevProblem& d = J->dev[li];
      if (d.wide) cr[c++] = ClearRange{d.wT, static_cast<uint64_t>(d.wdpad) * d.wnpad};
      if (d.evmf) cr[c++] = ClearRange{reinterpret_cast<uint32_t*>(d.dig), static_cast<uint64_t>(d.np) * d.dfr * 128};
      if (J->skip_reduce[li] > 0)
        cr[c++] = ClearRange{d.resid, static_cast<uint64_t>(J->skip_reduce[li]) * d.CS};
    }
  }
  // initial queue image: one REDUCE task per (problem, prime slot), largest problems first
  // (none when a problem has more primes than the persistent schedule takes)
  if (with_queue && J->max_np <= kMaxSlots) {
    uint8_t* q = blob + J->qinit_off;
    QueueState* qs = reinterpret_cast<QueueState*>(q);
    Task* tasks = reinterpret_cast<Task*>(q + J->q_tasks);
    int* ready = reinterpret_cast<int*>(q + J->q_ready);
    ProbCounters* cnt = reinterpret_cast<ProbCounters*>(q + J->q_counters);
    int t = 0;
    for (int li = 0; li < nl; ++li) {
      const Plan& P = J->plans[J->live[li]];
      const DevProblem& d = J->dev[li];
      const int ne = blocks_of(P.E + 1, d.evpb), nc = blocks_of(P.D + 1, 64);
      cnt[li].slots_left = P.np;
      for (int sl = 0; sl < P.np; ++sl) {
        cnt[li].eval_left[sl] = ne;
        cnt[li].conv_left[sl] = nc * d.ncchunk;
        cnt[li].stir_left[sl] = nc * d.nchunk;
        tasks[t] = Task{(kTaskReduce << 24) | li, sl, 0, 0};
        ready[t] = 1;
        ++t;
      }
    }
    qs->head = 0;
    qs->tail = t;
    qs->done = (J->q_crt_total == 0) ? 1 : 0;
    qs->crt_done = 0;
    qs->err = 0;
  }
  std::memcpy(blob + J->probs_off, J->dev.data(), sizeof(DevProblem) * nl);
  for (int s = 0; s < kNumStages; ++s)
    if (!J->items[s].empty())
      std::memcpy(blob + J->items_off[s], J->items[s].data(), sizeof(WorkItem) * J->items[s].size());
  if (!J->eval_staged.empty())
    std::memcpy(blob + J->evs_off, J->eval_staged.data(), sizeof(WorkItem) * J->eval_staged.size());
  for (int pass = 0; pass < 3; ++pass)
    if (!J->wide_items[pass].empty())
      std::memcpy(blob + J->wide_off[pass], J->wide_items[pass].data(), sizeof(WorkItem) * J->wide_items[pass].size());
  if (!J->hseg_items.empty())
    std::memcpy(blob + J->hseg_off, J->hseg_items.data(), sizeof(WorkItem) * J->hseg_items.size());
  if (!J->mgroups.empty()) {
    std::memcpy(blob + J->mg_off, J->mgroups.data(), sizeof(StirGroup) * J->mgroups.size());
    std::memcpy(blob + J->mm_off, J->mmembers.data(), sizeof(StirMember) * J->mmembers.size());
    std::memcpy(blob + J->digi_off, J->dig_items.data(), sizeof(WorkItem) * J->dig_items.size());
    std::memcpy(blob + J->mmi_off, J->mm_items.data(), sizeof(WorkItem) * J->mm_items.size());
  }
  if (!J->sgroups.empty()) {
    std::memcpy(blob + J->sg_off, J->sgroups.data(), sizeof(StirGroup) * J->sgroups.size());
    std::memcpy(blob + J->sm_off, J->smembers.data(), sizeof(StirMember) * J->smembers.size());
    std::memcpy(blob + J->sgi_off, J->sg_items.data(), sizeof(WorkItem) * J->sg_items.size());
  }
}

// CRT tables: canonical prime lists use the context's global tables.
static void bind_crt_tables(const rsl_ctx* ctx, Job* J) {
  const int nl = static_cast<int>(J->live.size());
  for (int li = 0; li < nl; ++li) {
    const Plan& P = J->plans[J->live[li]];
    const ProbLayout& L = J->lay[li];
    DevProblem& d = J->dev[li];
    if (P.canonical) {
      d.Tg = ctx->d_Tg;
      d.tgs = ctx->garner_np;
      d.invM = ctx->d_invM;
      d.Plimb = ctx->d_Plimb;
      d.LP = ctx->LPg;
    } else {
      d.Tg = reinterpret_cast<const uint32_t*>(J->base + L.Tg);
      d.tgs = P.np;
      d.invM = reinterpret_cast<const uint32_t*>(J->base + L.invM);
      d.Plimb = reinterpret_cast<const uint32_t*>(J->base + L.Plimb);
      d.LP = P.L_out;
    }
  }
  std::memcpy(J->image + J->probs_off, J->dev.data(), sizeof(DevProblem) * nl);
}

int job_upload_copy(rsl_ctx* ctx, Job* J, hipStream_t st, uint8_t* pinned) {
  bind_crt_tables(ctx, J);
  const size_t up = upload_bytes(*J);
  if (up == 0) return RSL_OK;
  if ((J->blob.empty() && J->image) || J->direct_image) {
    pinned = J->image;  // bound straight into pinned staging, or sent from pageable memory
  } else {
    if (!pinned) {
      int rc = ensure_staging(ctx, J->up_bytes, J->down_bytes);
      if (rc) return rc;
      pinned = ctx->h_up;
    }
    std::memcpy(pinned, J->image, up);
  }
  return hip_check(ctx, hipMemcpyAsync(J->base, pinned, up, hipMemcpyHostToDevice, st), "upload");
}

int job_upload(rsl_ctx* ctx, Job* J, hipStream_t st, uint8_t* pinned) {
  int rc = job_upload_copy(ctx, J, st, pinned);
  if (!rc) rc = job_upload_clear(ctx, J, st);
  return rc;
}

int job_upload_clear(rsl_ctx* ctx, Job* J, hipStream_t st) {
  // one launch over the clear table the upload brought (ordered after it)
  return hip_check(ctx, launch_clear_ranges(reinterpret_cast<const ClearRange*>(J->base + J->clr_off), J->nclr, st),
                   "clear ranges");
}

int job_reset(rsl_ctx* ctx, Job* J, hipStream_t st) {
  if (J->status_bytes == 0) return RSL_OK;
  return hip_check(ctx, launch_copy_words(reinterpret_cast<uint32_t*>(J->base + J->status_off), nullptr,
                                          J->status_bytes / 4, st), "status reset");
}

int job_launch(rsl_ctx* ctx, Job* J, int mode, hipStream_t st, bool stage_events) {
  if (J->live.empty()) return RSL_OK;
  const DevTables T = tables_of(ctx);
  const DevProblem* probs = reinterpret_cast<const DevProblem*>(J->base + J->probs_off);
  auto items = [&](int s) { return reinterpret_cast<const WorkItem*>(J->base + J->items_off[s]); };
  auto wide = [&](int pass) { return reinterpret_cast<const WorkItem*>(J->base + J->wide_off[pass]); };
  const WorkItem* hseg_items = reinterpret_cast<const WorkItem*>(J->base + J->hseg_off);
  int rc;
  if (mode == RSL_PLAIN) {
    for (size_t li = 0; li < J->live.size(); ++li) {
      const ProbLayout& L = J->lay[li];
      // the job-wide slot count: CRT kernels exist for 1-4, 6 and 8 slots, and
      // the CRT's LDS size was taken for that count
      const int ns = J->crt_ns;
      for (int s = 0; s < kNumStages; ++s) {
        const int cnt = L.item_end[s] - L.item_begin[s];
        if (s == kStageStir &&
            (rc = hip_check(ctx, launch_hseg(probs, hseg_items + L.hseg_begin, L.hseg_end - L.hseg_begin, T, st),
                            "launch")))
          return rc;
        const hipError_t e = (s == kStageEval)
            ? launch_eval(eval_variant(J->dev[li]), probs, items(s) + L.item_begin[s], cnt,
                          static_cast<size_t>(eval_stage_lds_words(J->dev[li])) * 4, T, st)
            : launch_stage(s, probs, items(s) + L.item_begin[s], cnt, J->stage_lds[s], ns, T, st);
        if ((rc = hip_check(ctx, e, "launch"))) return rc;
      }
      for (int pass = 0; pass < 3; ++pass) {
        const int cnt = L.wide_end[pass] - L.wide_begin[pass];
        const int kp = (pass == 1 && J->wide_mfma) ? 3 : pass;
        if ((rc = hip_check(ctx, launch_crt_wide(kp, probs, wide(pass) + L.wide_begin[pass], cnt, J->wide_lds[pass], T, st),
                            "launch")))
          return rc;
      }
    }
    return RSL_OK;
  }
  if (mode == RSL_BATCHED) {
    if (J->max_np > kMaxSlots)
      return fail(ctx, RSL_EINVAL, "the persistent schedule takes at most 256 primes per problem");
    if (J->any_schur)
      return fail(ctx, RSL_EINVAL, "the persistent schedule does not run the Schur evaluation");
    if (J->persist_lds > static_cast<size_t>(kLdsWords) * 4)
      return fail(ctx, RSL_EINVAL, "persistent launch needs more than 64 KB of LDS per workgroup");
    QueueDesc Q{};
    uint8_t* qb = J->base + J->queue_off;
    Q.state = reinterpret_cast<QueueState*>(qb);
    Q.tasks = reinterpret_cast<Task*>(qb + J->q_tasks);
    Q.ready = reinterpret_cast<int*>(qb + J->q_ready);
    Q.counters = reinterpret_cast<ProbCounters*>(qb + J->q_counters);
    Q.capacity = J->q_capacity;
    Q.crt_total = J->q_crt_total;
    Q.nprob = static_cast<int>(J->live.size());
    Q.wait_ticks = ctx->queue_wait_ticks;
    if (J->persist_grid == 0) {
      // at most two waiting waves per SIMD by default: idle waves only poll
      const int per_cu = std::min(8, persistent_blocks_per_cu(J->crt_ns, J->persist_lds));
      int cus = 256;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) cus = prop.multiProcessorCount;
      J->persist_grid = std::max(1, per_cu * cus * std::max(1, J->tune.grid_mult));
    }
    if ((rc = hip_check(ctx, launch_copy_words(reinterpret_cast<uint32_t*>(qb),
                                               reinterpret_cast<const uint32_t*>(J->base + J->qinit_off),
                                               J->queue_bytes / 4, st),
                        "queue reset")))
      return rc;
    if (stage_events && (rc = hip_check(ctx, hipEventRecord(ctx->ev[0], st), "event"))) return rc;
    if ((rc = hip_check(ctx, launch_persistent(probs, Q, T, J->crt_ns, J->persist_grid, J->persist_lds, st),
                        "persistent launch")))
      return rc;
    if (stage_events)
      for (int s = 1; s <= kNumStages; ++s)
        if ((rc = hip_check(ctx, hipEventRecord(ctx->ev[s], st), "event"))) return rc;
    return RSL_OK;
  }
  for (int s = 0; s < kNumStages; ++s) {
    if (stage_events && (rc = hip_check(ctx, hipEventRecord(ctx->ev[s], st), "event"))) return rc;
    if (s == kStageEval) {
      const WorkItem* evs = reinterpret_cast<const WorkItem*>(J->base + J->evs_off);
      for (const Job::EvalRange& r : J->eval_ranges)
        if ((rc = hip_check(ctx, launch_eval(r.variant, probs, evs + r.begin, r.end - r.begin, r.lds, T, st),
                            "launch")))
          return rc;
      continue;
    }
    if (J->mm_interp && (s == kStageConv || s == kStageStir)) {
      // the interpolation's two products on the matrix cores (the segments'
      // polynomials between them, from the Newton coefficients)
      const StirGroup* mg = reinterpret_cast<const StirGroup*>(J->base + J->mg_off);
      const StirMember* mm = reinterpret_cast<const StirMember*>(J->base + J->mm_off);
      const WorkItem* di = reinterpret_cast<const WorkItem*>(J->base + J->digi_off);
      const WorkItem* mi = reinterpret_cast<const WorkItem*>(J->base + J->mmi_off);
      const int nd = static_cast<int>(J->dig_items.size()), nm = static_cast<int>(J->mm_items.size());
      if (s == kStageStir &&
          (rc = hip_check(ctx, launch_hseg(probs, hseg_items, static_cast<int>(J->hseg_items.size()), T, st),
                          "launch")))
        return rc;
      const int which = s == kStageConv ? 1 : 2;
      if ((rc = hip_check(ctx, launch_interp_mm(which, probs, mg, mm, di, nd, mi, nm, J->mm_lds[which - 1], T, st),
                          "launch")))
        return rc;
      continue;
    }
    if (s == kStageStir &&
        (rc = hip_check(ctx, launch_hseg(probs, hseg_items, static_cast<int>(J->hseg_items.size()), T, st), "launch")))
      return rc;
    if (s == kStageStir && !J->sg_items.empty()) {
      if ((rc = hip_check(ctx, launch_stir_group(probs, reinterpret_cast<const StirGroup*>(J->base + J->sg_off),
                                                 reinterpret_cast<const StirMember*>(J->base + J->sm_off),
                                                 reinterpret_cast<const WorkItem*>(J->base + J->sgi_off),
                                                 static_cast<int>(J->sg_items.size()), J->sg_lds, T, st),
                          "launch")))
        return rc;
      continue;
    }
    // CRT: several items per block once the launch still has a block per CU
    // or more (the degree-24 pair, 146 items, keeps one per block)
    const int crt_per = J->items[kStageCrt].size() >= 1024 ? kCrtItemsPerBlock : 1;
    if ((rc = hip_check(ctx, launch_stage(s, probs, items(s), static_cast<int>(J->items[s].size()),
                                          J->stage_lds[s], J->crt_ns, T, st, crt_per), "launch")))
      return rc;
    if (s == kStageCrt)
      for (int pass = 0; pass < 3; ++pass)
        if ((rc = hip_check(ctx, launch_crt_wide((pass == 1 && J->wide_mfma) ? 3 : pass, probs, wide(pass),
                                                 static_cast<int>(J->wide_items[pass].size()),
                                                 J->wide_lds[pass], T, st), "launch")))
          return rc;
  }
  if (stage_events && (rc = hip_check(ctx, hipEventRecord(ctx->ev[kNumStages], st), "event"))) return rc;
  return RSL_OK;
}

int job_download(rsl_ctx* ctx, Job* J, uint8_t* host, hipStream_t st) {
  if (J->down_bytes == 0) return RSL_OK;
  return hip_check(ctx, hipMemcpyAsync(host, J->base + J->down_off, J->down_bytes, hipMemcpyDeviceToHost, st),
                   "download");
}

int job_decode(rsl_ctx* ctx, const Job& J, const uint8_t* host, rsl_result* out, int* status, rsl_counters* cnt) {
  std::vector<int> li_of(J.n, -1);
  for (size_t li = 0; li < J.live.size(); ++li) li_of[J.live[li]] = static_cast<int>(li);
  // results are independent per problem: decode them on host threads, then
  // gather counters and the first error in problem order
  std::vector<int> rcs(J.n, RSL_OK);
  parallel_for(J.n, 16, [&](int k) {
    int rc = J.pstatus[k];
    const Plan& P = J.plans[k];
    if (!rc) {
      if (P.zero) {
        rc = decode_result(P, nullptr, &out[k]);
      } else {
        const ProbLayout& L = J.lay[li_of[k]];
        const int* st = reinterpret_cast<const int*>(host + (L.status - J.down_off));
        if (st[0] & kErrQueueStall) rc = RSL_EDEVICE;
        else if (st[0] & kErrTooFewGoodPoints) rc = RSL_EPRIMES;
        else rc = decode_result(P, reinterpret_cast<const uint32_t*>(host + (L.out - J.down_off)), &out[k]);
      }
    }
    rcs[k] = rc;
  });
  int first = RSL_OK;
  for (int k = 0; k < J.n; ++k) {
    const int rc = rcs[k];
    const Plan& P = J.plans[k];
    if (!J.pstatus[k]) {
      cnt->problems += 1;
      if (!P.zero) {
        const ProbLayout& L = J.lay[li_of[k]];
        const int* st = reinterpret_cast<const int*>(host + (L.status - J.down_off));
        if (rc == RSL_EDEVICE) ctx->err = "persistent launch: a wave gave up waiting on the task queue";
        else if (rc == RSL_EPRIMES) ctx->err = "fewer than D+1 good points for a prime";
        else if (rc == RSL_ERANGE) ctx->err = "result buffer too small";
        cnt->pairs += static_cast<int64_t>(P.np) * (P.E + 1);
        cnt->bad_pairs += st[P.np + 1];
        cnt->bad_primes += P.bad_primes;
        for (int i = 0; i < P.np; ++i) cnt->slow_primes += st[1 + i];
      }
    }
    if (status) status[k] = rc;
    if (rc && !first) first = rc;
  }
  return first;
}

}  // namespace rsl
