// Launch plans: the instances one term-sweep / reduce launch covers.
//
// Packing (the term -> workgroup schedule).  Each term gets the smallest
// group that runs it well:
//   * one wavefront, for in-place terms of at most kWaveMaxGrid points (a
//     contraction over more fibers than the lanes hold runs in chunks) and
//     for small ping-pong terms;
//   * the eight wavefronts of a workgroup otherwise, with its buffer in LDS
//     when it fits under the per-workgroup cap, else in global scratch.
// A pack's LDS holds the one-mode tables of the levels up to its highest,
// then its terms' buffers, under the cap of two workgroups per compute unit.
// Wave terms are dealt, most expensive first, to the least loaded of enough
// packs (at most kPackTerms terms and the LDS cap each) to give every compute
// unit work; terms taking more than a quarter of the cap instead fill packs
// as densely as the cap allows, so that more of them run at once.  Terms of
// different instances mix freely: every term is computed by the same code
// whatever its pack, so results do not depend on the mix.
//
// Reduce items (one per wavefront): a workgroup's worth per long row, one per
// eight short rows, in each instance's row order, padded to
// whole workgroups; an item's partial sums go to its own slot so that the
// per-instance norm / energy sums run in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sg_internal.h"

namespace sg {

namespace {

struct Cand {
  int32_t inst;
  int32_t term;
  double cost;
  int64_t slice;   // bytes of the term's buffer(s)
  int inplace;     // 1: one buffer, contractions in place
  int wave;        // 1: one wavefront can run it
  int64_t ngrid;
  int maxlev;      // highest level of an active mode
  const int32_t *mbt;  // the term's first M^B entry on the device
};

// Does every in-place contraction of term T fit the registers of a group of
// n lanes?  B->G along modes 1.. and G->B along modes ..na-2 run in place
// (the first and last contractions read or write HBM).
bool inplace_fits(const TermDev &T, int n) {
  const int na = T.na;
  for (int p = 1; p < na; ++p) {           // basis -> grid along mode p
    int64_t s = 1;
    for (int q = 0; q < na; ++q) s *= q < p ? T.nq[q] : T.nb[q];
    const int ni = T.nb[p];
    if (s / ni > (int64_t)inplace_fpt(ni) * n) return false;
  }
  for (int p = 0; p + 1 < na; ++p) {       // grid -> basis along mode p
    int64_t s = 1;
    for (int q = 0; q < na; ++q) s *= q < p ? T.nb[q] : T.nq[q];
    const int ni = T.nq[p];
    if (s / ni > (int64_t)inplace_fpt(ni) * n) return false;
  }
  return true;
}

// The schedule knob in effect for a problem: its own setting, or by default
// (0) a threshold from the problem's size.  A launch over few terms lasts as
// long as its longest term chain, so there terms above 1024 points run on a
// whole workgroup; a launch over many terms is bound by throughput, where a
// wavefront per term (no workgroup barriers, more terms in flight per
// compute unit) wins for terms up to 2048 points and 4096-point terms stay on
// workgroups.  Plans over several problems always hold many terms.
int32_t effective_block_grid(const sg_problem *p, bool multi) {
  if (p->block_grid > 0) return p->block_grid;
  if (!multi && p->h.nterms < 4 * kComputeUnits) return 1025;
  return 4096;
}

// One candidate per term of a pack set.  split: the set applies the split
// operator (no kinetic contractions, so the in-place form applies to the
// standard size maps); elem: bytes of one complex value.
Cand make_cand(int32_t inst, int32_t term, const Compiled &h, bool split, int elem,
               const int32_t *d_mb, int32_t block_grid) {
  const TermDev &T = h.terms[term];
  Cand c{inst, term, h.cost[term], 0, 0, 0, T.ngrid, 0, d_mb ? d_mb + T.off : nullptr};
  for (int p = 0; p < T.na; ++p) c.maxlev = std::max<int>(c.maxlev, T.lev[p]);
  const bool std_maps = h.nbA == 1 && h.nbB == 2 && h.nqA == 2 && h.nqB == 2;
  const int64_t one = (int64_t)T.ngrid * elem;
  if (split && std_maps && T.na == 0) {
    // the scalar case: one product, no grid buffer
    c.inplace = 1;
    c.slice = elem;
    c.wave = 1;
  } else if (split && std_maps && inplace_fits(T, kSweepThreads)) {
    c.inplace = 1;
    c.slice = one + kCoefLdsBytes;
    // a wavefront runs any in-place term up to kWaveMaxGrid points, in chunks
    // of the fibers its registers hold when one pass does not fit
    c.wave = T.ngrid <= kWaveMaxGrid && !(block_grid > 0 && T.ngrid >= block_grid) ? 1 : 0;
  } else {
    c.inplace = 0;
    c.slice = 2 * one;
    c.wave = T.ngrid <= kPingPongWaveMaxGrid ? 1 : 0;
  }
  return c;
}

// dense: as few wave packs as the terms fill (plans over many problems);
// otherwise enough packs to give every compute unit `spread` workgroups (one
// by default: the wavefronts of a sparsely filled pack then have their CU's
// SIMDs to themselves).  costs (nullable) receives the estimated cost of each
// pack appended to out.  tab_bytes: the set's tables in LDS, two_sets: they
// are two sets of tab_bytes / 2 (then a pack keeps room for both whole).
void pack_set(const std::vector<Cand> &cands, int elem, int tab_bytes, bool two_sets,
              std::vector<PackDev> *out, PackSet *set, int64_t *scratch_bytes, bool dense = false,
              std::vector<double> *costs = nullptr, int spread = 1) {
  set->first = (int32_t)out->size();
  set->count = 0;
  set->lds_bytes = 0;
  set->tab_bytes = 0;
  if (cands.empty()) return;
  // two workgroups per compute unit (FP64), four (FP32); a pack's tables come
  // first, the levels up to its highest (pack_lds_base)
  const int cap_total = elem >= 16 ? kLdsPerCU / 2 : kLdsPerCU / 4;
  const int per_cu = kLdsPerCU / cap_total;
  const int tab_a = two_sets ? tab_bytes / 2 : tab_bytes, tab_b = two_sets ? tab_bytes / 2 : 0;
  auto tables = [&](int maxlev) { return pack_lds_base(tab_a, tab_b, elem / 2, maxlev); };
  auto fits = [&](int64_t bytes, int maxlev) { return bytes + tables(maxlev) <= cap_total; };
  std::vector<Cand> big, small;
  for (const Cand &c : cands) (c.wave && fits(c.slice, c.maxlev) ? small : big).push_back(c);
  auto by_cost = [](const Cand &a, const Cand &b) { return a.cost > b.cost; };
  std::stable_sort(big.begin(), big.end(), by_cost);
  std::stable_sort(small.begin(), small.end(), by_cost);
  int lds = 0;
  const int64_t nsmall = (int64_t)small.size();
  int64_t nbins = (nsmall + kPackTerms - 1) / kPackTerms;
  const int64_t want = (int64_t)kComputeUnits * std::min(std::max(spread, 1), per_cu) -
                       (int64_t)big.size();
  if (!dense) nbins = std::max<int64_t>(nbins, std::min<int64_t>(nsmall, want));
  struct Bin {
    double load;
    int64_t id;
  };
  auto worse = [](const Bin &a, const Bin &b) {
    return a.load > b.load || (a.load == b.load && a.id > b.id);
  };
  std::vector<Bin> heap;
  std::vector<PackDev> bins;
  std::vector<int64_t> bin_bytes;
  std::vector<double> bin_load;
  auto new_bin = [&]() {
    PackDev pk;
    std::memset(&pk, 0, sizeof(pk));
    pk.block = kPackWaves;
    bins.push_back(pk);
    bin_bytes.push_back(0);
    bin_load.push_back(0.0);
    heap.push_back({0.0, (int64_t)bins.size() - 1});
    std::push_heap(heap.begin(), heap.end(), worse);
  };
  for (int64_t i = 0; i < nbins; ++i) new_bin();
  // terms taking more than a quarter of a pack's LDS fill packs as densely as
  // LDS allows (first fit), so that more of them run at once on a compute
  // unit; cur is the pack they are filling, held out of the heap meanwhile
  int64_t cur = -1;
  auto release_cur = [&]() {
    if (cur >= 0 && bins[cur].n < kPackTerms) {
      heap.push_back({bin_load[cur], cur});
      std::push_heap(heap.begin(), heap.end(), worse);
    }
    cur = -1;
  };
  for (const Cand &c : small) {
    const bool heavy = 4 * c.slice > cap_total;
    Bin b{0.0, -1};
    if (heavy && cur >= 0 && bins[cur].n < kPackTerms &&
        fits(bin_bytes[cur] + c.slice, std::max<int32_t>(bins[cur].maxlev, c.maxlev)))
      b = {bin_load[cur], cur};
    else
      release_cur();
    // otherwise the least loaded bin with room (bins without room leave the
    // heap for good once full; bins short of LDS are set aside for this term
    // only)
    std::vector<Bin> aside;
    while (b.id < 0 && !heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), worse);
      Bin t = heap.back();
      heap.pop_back();
      if (fits(bin_bytes[t.id] + c.slice, std::max<int32_t>(bins[t.id].maxlev, c.maxlev))) {
        b = t;
        break;
      }
      aside.push_back(t);
    }
    for (const Bin &t : aside) {
      heap.push_back(t);
      std::push_heap(heap.begin(), heap.end(), worse);
    }
    if (b.id < 0) {
      new_bin();
      std::pop_heap(heap.begin(), heap.end(), worse);
      b = heap.back();
      heap.pop_back();
    }
    PackDev &pk = bins[b.id];
    pk.inst[pk.n] = c.inst;
    pk.term[pk.n] = c.term;
    pk.lds_off[pk.n] = (int32_t)bin_bytes[b.id];
    pk.inplace[pk.n] = c.inplace;
    pk.mbt[pk.n] = c.mbt;
    pk.maxlev = std::max<int32_t>(pk.maxlev, c.maxlev);
    bin_bytes[b.id] += c.slice;
    pk.n += 1;
    b.load += c.cost;
    bin_load[b.id] = b.load;
    if (heavy)
      cur = b.id;
    else if (pk.n < kPackTerms) {
      heap.push_back(b);
      std::push_heap(heap.begin(), heap.end(), worse);
    }
  }
  release_cur();
  for (const Cand &c : big) {
    PackDev pk;
    std::memset(&pk, 0, sizeof(pk));
    pk.n = 1;
    for (int w = 0; w < kPackTerms; ++w) {   // only slot 0 is read; all hold the term
      pk.inst[w] = c.inst;
      pk.term[w] = c.term;
      pk.mbt[w] = c.mbt;
    }
    pk.inplace[0] = c.inplace;
    pk.maxlev = c.maxlev;
    if (fits(c.slice, c.maxlev)) {
      pk.block = kPackBlockLds;
      pk.slices = (int32_t)c.slice;
    } else {
      // global scratch holds the two ping-pong buffers
      pk.block = kPackBlockScratch;
      pk.inplace[0] = 0;
      pk.scratch_off = *scratch_bytes;
      *scratch_bytes += (2 * c.ngrid * elem + 255) & ~(int64_t)255;
    }
    pk.lds_base = tables(pk.maxlev);
    lds = std::max<int>(lds, pk.lds_base + pk.slices);
    out->push_back(pk);
    if (costs) costs->push_back(c.cost);
  }
  std::vector<int64_t> order(bins.size());
  for (size_t i = 0; i < bins.size(); ++i) order[i] = (int64_t)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return bin_load[a] > bin_load[b]; });
  for (int64_t i : order) {
    PackDev &pk = bins[i];
    if (pk.n == 0) continue;
    // every wavefront reads its slot's term record before it tests whether
    // the slot is used: unused slots repeat slot 0's term (a valid record)
    for (int w = pk.n; w < kPackTerms; ++w) {
      pk.inst[w] = pk.inst[0];
      pk.term[w] = pk.term[0];
      pk.mbt[w] = pk.mbt[0];
    }
    pk.slices = (int32_t)bin_bytes[i];
    pk.lds_base = tables(pk.maxlev);
    out->push_back(pk);
    if (costs) costs->push_back(bin_load[i]);
    lds = std::max<int>(lds, pk.lds_base + pk.slices);
  }
  set->count = (int32_t)(out->size() - set->first);
  set->tab_bytes = tab_bytes;
  set->lds_bytes = lds;
}

template <typename T>
hipError_t ensure(T **ptr, int64_t *cap, int64_t n, int64_t *bytes_delta) {
  if (n <= *cap && *ptr) return hipSuccess;
  hipFree(*ptr);
  *ptr = nullptr;
  const int64_t m = std::max<int64_t>(n, 1);
  hipError_t e = hipMalloc((void **)ptr, (size_t)m * sizeof(T));
  if (e == hipSuccess) {
    if (bytes_delta) *bytes_delta += (m - *cap) * (int64_t)sizeof(T);
    *cap = m;
  } else {
    *cap = 0;
  }
  return e;
}

}  // namespace

void inst_from_problem(const sg_problem *p, InstDev *d) {
  std::memset(d, 0, sizeof(*d));
  const Compiled &h = p->h;
  d->terms = p->d_terms;
  d->pairs = p->d_pairs;
  d->potc = p->d_potc;
  d->mb = p->d_mb;
  d->inv_ptr = p->d_inv_ptr;
  d->inv_col = p->d_inv_col;
  d->rows = p->d_rows;
  d->h0 = p->d_h0;
  d->tab64 = p->d_tables;
  d->tab32 = p->d_tables32;
  d->tab32r = p->d_tables32r;
  d->tm = p->d_tm;
  d->x0 = p->d_work;
  d->x1 = p->d_work + h.ncs;
  d->acc = p->d_work + 2 * h.ncs;
  d->partials = p->d_partials;
  d->abc = p->d_abc;
  d->nfib = p->h.nfib;
  d->veff = p->d_veff;
  d->voff = p->d_voff;
  d->result = p->d_result;
  d->cheb_a = p->d_cheb_a;
  d->ncs = h.ncs;
  d->nlong = h.n_long_rows;
  d->nitems = (int32_t)h.n_items;
  d->std_maps = (h.nbA == 1 && h.nbB == 2 && h.nqA == 2 && h.nqB == 2) ? 1 : 0;
  d->round32 = 0;
  d->K = 0;
  d->inv_half = 1.0;
  d->phase_re = 1.0;
  d->active = 1;
}

namespace {

// LDS bytes of the standard tables up to level 7 (the largest a cached pack
// set leaves room for).
constexpr int kTabMax64 = ((std_table_base(8) * 8 + 15) / 16) * 16;
constexpr int kTabMax32 = ((std_table_base(8) * 4 + 15) / 16) * 16;

void reduce_items(const sg_problem *p, int32_t inst, std::vector<RedItem> *items) {
  const Compiled &h = p->h;
  auto at = [&](int64_t q, const int32_t *base) { return base ? base + q : nullptr; };
  int32_t local = 0;
  for (int64_t q = 0; q < h.n_long_rows; ++q)
    for (int32_t w = 0; w < kRowWaves; ++w)
      items->push_back({inst, (int32_t)q, local++, (1 << 12) | (w << 24), at(q, p->d_rows),
                        at(q, p->d_inv_ptr)});
  const int64_t nshort = h.ncs - h.n_long_rows;
  for (int64_t q = 0; q < nshort; q += kShortLanes) {
    const int64_t first = h.n_long_rows + q;
    items->push_back({inst, (int32_t)first, local++,
                      (int32_t)std::min<int64_t>(kShortLanes, h.ncs - first),
                      at(first, p->d_rows), at(first, p->d_inv_ptr)});
  }
  // whole workgroups: padding items cover no row
  while (local % kRowWaves) items->push_back({inst, (int32_t)h.ncs, local++, 0, nullptr, nullptr});
}

void build_cache(sg_problem *p) {
  PackCache &c = p->pcache;
  const Compiled &h = p->h;
  if (c.valid && c.thr == h.mixed_max_fp32_coeff && c.grid_kinetic == p->grid_kinetic &&
      c.block_grid == p->block_grid)
    return;
  std::vector<Cand> cg64, cs64, m64, m32;
  c.inst32 = false;
  for (int64_t t = 0; t < h.nterms; ++t) {
    const int32_t bg = effective_block_grid(p, true);
    cg64.push_back(make_cand(0, (int32_t)t, h, false, 16, p->d_mb, bg));
    cs64.push_back(make_cand(0, (int32_t)t, h, true, 16, p->d_mb, bg));
    if (std::abs(h.coeff[t]) <= h.mixed_max_fp32_coeff) {
      m32.push_back(make_cand(0, (int32_t)t, h, true, 8, p->d_mb, bg));
      c.inst32 = true;
    } else {
      m64.push_back(make_cand(0, (int32_t)t, h, true, 16, p->d_mb, bg));
    }
  }
  const std::vector<Cand> *cs[kPackSets] = {&cg64, &cs64, &m64, &m32};
  const int elem[kPackSets] = {16, 16, 16, 8};
  // the mixed path's FP64 terms hold the exact and the FP32-rounded tables
  // only when the instance has FP32 terms; otherwise they pack like the FP64
  // split set (no term pushed out of LDS into global scratch)
  const int tab[kPackSets] = {0, kTabMax64, c.inst32 ? 2 * kTabMax64 : kTabMax64, kTabMax32};
  for (int k = 0; k < kPackSets; ++k) {
    c.packs[k].clear();
    c.cost[k].clear();
    PackSet ps;
    c.scratch[k] = 0;
    pack_set(*cs[k], elem[k], tab[k], k == kSetMixed64 && c.inst32, &c.packs[k], &ps,
             &c.scratch[k], true, &c.cost[k]);
  }
  c.items.clear();
  reduce_items(p, 0, &c.items);
  c.thr = h.mixed_max_fp32_coeff;
  c.grid_kinetic = p->grid_kinetic;
  c.block_grid = p->block_grid;
  c.valid = true;
}

}  // namespace

// Does every pack of each set run its terms in place?  Such a set launches
// the sweep without the ping-pong form.
static void mark_inplace_sets(Plan *pl) {
  for (int k = 0; k < kPackSets; ++k) {
    PackSet &set = pl->sets[k];
    bool all = set.count > 0;
    for (int32_t i = set.first; all && i < set.first + set.count; ++i) {
      const PackDev &pk = pl->packs[i];
      if (pk.block == kPackBlockScratch) all = false;
      const int n = pk.block == kPackWaves ? pk.n : 1;
      for (int w = 0; w < n; ++w) all = all && pk.inplace[w] != 0;
    }
    set.all_inplace = all ? 1 : 0;
  }
}

sg_status plan_build(Plan *pl, const std::vector<sg_problem *> &probs, std::string *err) {
  pl->probs = probs;
  pl->inst.assign(probs.size(), InstDev{});
  pl->packs.clear();
  pl->items.clear();
  pl->scratch_bytes = 0;
  pl->any32 = false;
  pl->fp64_split = false;
  pl->any_tab = false;
  const bool multi = probs.size() > 1;
  std::vector<Cand> cg64, cs64, m64, m32;
  bool split_all = true;
  for (size_t i = 0; i < probs.size(); ++i) {
    sg_problem *p = probs[i];
    const Compiled &h = p->h;
    inst_from_problem(p, &pl->inst[i]);
    split_all = split_all && h.split_exact && !p->grid_kinetic;
    bool inst32 = false;
    if (multi) {
      build_cache(p);
      inst32 = p->pcache.inst32;
      const size_t first = pl->items.size();
      pl->items.insert(pl->items.end(), p->pcache.items.begin(), p->pcache.items.end());
      for (size_t q = first; q < pl->items.size(); ++q) pl->items[q].inst = (int32_t)i;
    } else {
      for (int64_t t = 0; t < h.nterms; ++t) {
        const int32_t bg = effective_block_grid(p, false);
        cg64.push_back(make_cand((int32_t)i, (int32_t)t, h, false, 16, p->d_mb, bg));
        cs64.push_back(make_cand((int32_t)i, (int32_t)t, h, true, 16, p->d_mb, bg));
        if (std::abs(h.coeff[t]) <= h.mixed_max_fp32_coeff) {
          m32.push_back(make_cand((int32_t)i, (int32_t)t, h, true, 8, p->d_mb, bg));
          inst32 = true;
        } else {
          m64.push_back(make_cand((int32_t)i, (int32_t)t, h, true, 16, p->d_mb, bg));
        }
      }
      reduce_items(p, (int32_t)i, &pl->items);
    }
    pl->inst[i].round32 = inst32 ? 1 : 0;
    pl->any32 = pl->any32 || inst32;
    pl->any_tab = pl->any_tab || p->d_veff != nullptr;
  }
  pl->fp64_split = split_all;
  // standard-map tables (identical for every such instance) for LDS
  pl->stab_L = -1;
  pl->any_round32 = false;
  const sg_problem *src = nullptr;
  for (size_t i = 0; i < probs.size(); ++i) {
    if (!pl->inst[i].std_maps) continue;
    pl->any_round32 = pl->any_round32 || pl->inst[i].round32;
    if (probs[i]->h.L > pl->stab_L) {
      pl->stab_L = probs[i]->h.L;
      src = probs[i];
    }
  }
  pl->stab64.clear();
  pl->stab32.clear();
  pl->stab32r.clear();
  if (src) {
    const Compiled &h = src->h;
    for (int l = 0; l <= pl->stab_L; ++l) {
      const LevelDev &ld = h.tdesc.lev[l];
      const int nb = 2 * l + 1, nq = 2 * l + 2;
      if ((int)pl->stab64.size() != std_table_base(l)) {
        *err = "standard table layout mismatch";
        return SG_EINVAL;
      }
      auto take = [&](int off, int n) {
        for (int i = 0; i < n; ++i) {
          pl->stab64.push_back(h.tables[off + i]);
          pl->stab32.push_back(h.tables32[off + i]);
          pl->stab32r.push_back(h.tables32r[off + i]);
        }
      };
      take(ld.bt, nq * nb);
      take(ld.wt, nb * nq);
      take(ld.x, nq);
    }
  }
  const int64_t E = (int64_t)pl->stab64.size();
  const int t64 = (int)((E * 8 + 15) & ~(int64_t)15);
  const int t32 = (int)((E * 4 + 15) & ~(int64_t)15);
  const int tabs[kPackSets] = {0, t64, pl->any_round32 ? 2 * t64 : t64, t32};
  if (!multi) {
    // the set SG_FP64 launches do not use stays empty
    if (split_all) cg64.clear(); else cs64.clear();
    const int sp = probs[0]->packs_per_cu;
    pack_set(cg64, 16, tabs[kSetGrid64], false, &pl->packs, &pl->sets[kSetGrid64],
             &pl->scratch_bytes, false, nullptr, sp);
    pack_set(cs64, 16, tabs[kSetSplit64], false, &pl->packs, &pl->sets[kSetSplit64],
             &pl->scratch_bytes, false, nullptr, sp);
    pack_set(m64, 16, tabs[kSetMixed64], pl->any_round32, &pl->packs, &pl->sets[kSetMixed64],
             &pl->scratch_bytes, false, nullptr, sp);
    pack_set(m32, 8, tabs[kSetMixed32], false, &pl->packs, &pl->sets[kSetMixed32],
             &pl->scratch_bytes, false, nullptr, sp);
    mark_inplace_sets(pl);
    return SG_OK;
  }
  // concatenate the problems' cached packs, most expensive first
  for (int k = 0; k < kPackSets; ++k) {
    PackSet &set = pl->sets[k];
    set.first = (int32_t)pl->packs.size();
    set.count = 0;
    set.tab_bytes = 0;
    set.lds_bytes = 0;
    if ((k == kSetGrid64 && split_all) || (k == kSetSplit64 && !split_all)) continue;
    std::vector<std::pair<double, PackDev>> all;
    for (size_t i = 0; i < probs.size(); ++i) {
      const PackCache &c = probs[i]->pcache;
      const int64_t base = pl->scratch_bytes;
      for (size_t q = 0; q < c.packs[k].size(); ++q) {
        PackDev pk = c.packs[k][q];
        for (int w = 0; w < kPackTerms; ++w) pk.inst[w] = (int32_t)i;   // unused slots too
        if (pk.block == kPackBlockScratch) pk.scratch_off += base;
        all.push_back({c.cost[k][q], pk});
      }
      pl->scratch_bytes += c.scratch[k];
    }
    std::stable_sort(all.begin(), all.end(),
                     [](const std::pair<double, PackDev> &a, const std::pair<double, PackDev> &b) {
                       return a.first > b.first;
                     });
    // the launch's table layout (two sets: the mixed FP64 terms of a plan
    // with FP32-rounded instances), and each pack's buffers after it
    const bool two = k == kSetMixed64 && pl->any_round32;
    const int tab_a = two ? tabs[k] / 2 : tabs[k], tab_b = two ? tabs[k] / 2 : 0;
    for (auto &x : all) {
      x.second.lds_base = pack_lds_base(tab_a, tab_b, k == kSetMixed32 ? 4 : 8, x.second.maxlev);
      set.lds_bytes = std::max(set.lds_bytes, x.second.lds_base + x.second.slices);
      pl->packs.push_back(x.second);
    }
    set.count = (int32_t)all.size();
    if (set.count) set.tab_bytes = tabs[k];
  }
  mark_inplace_sets(pl);
  return SG_OK;
}

sg_status plan_upload(Plan *pl, hipStream_t s) {
  hipError_t e;
  if ((e = ensure(&pl->d_packs, &pl->packs_capacity, (int64_t)pl->packs.size(), nullptr)) != hipSuccess)
    return fail(SG_ENOMEM, "device allocation of packs failed");
  if ((e = ensure(&pl->d_items, &pl->items_capacity, (int64_t)pl->items.size(), nullptr)) != hipSuccess)
    return fail(SG_ENOMEM, "device allocation of reduce items failed");
  if ((e = ensure(&pl->d_scratch, &pl->scratch_capacity, pl->scratch_bytes, nullptr)) != hipSuccess)
    return fail(SG_ENOMEM, "device allocation of sweep scratch failed");

  if (!pl->packs.empty() &&
      (e = hipMemcpyAsync(pl->d_packs, pl->packs.data(), pl->packs.size() * sizeof(PackDev),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "upload packs");
  if (!pl->items.empty() &&
      (e = hipMemcpyAsync(pl->d_items, pl->items.data(), pl->items.size() * sizeof(RedItem),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "upload reduce items");
  const int64_t E = (int64_t)pl->stab64.size();
  if (E > pl->stab_capacity) {
    hipFree(pl->d_stab64);
    hipFree(pl->d_stab32r);
    hipFree(pl->d_stab32);
    pl->d_stab64 = pl->d_stab32r = nullptr;
    pl->d_stab32 = nullptr;
    pl->stab_capacity = 0;
    if (hipMalloc((void **)&pl->d_stab64, E * 8) != hipSuccess ||
        hipMalloc((void **)&pl->d_stab32r, E * 8) != hipSuccess ||
        hipMalloc((void **)&pl->d_stab32, E * 4) != hipSuccess)
      return fail(SG_ENOMEM, "device allocation of the standard tables failed");
    pl->stab_capacity = E;
  }
  if (E > 0 &&
      ((e = hipMemcpyAsync(pl->d_stab64, pl->stab64.data(), E * 8, hipMemcpyHostToDevice, s)) !=
           hipSuccess ||
       (e = hipMemcpyAsync(pl->d_stab32r, pl->stab32r.data(), E * 8, hipMemcpyHostToDevice, s)) !=
           hipSuccess ||
       (e = hipMemcpyAsync(pl->d_stab32, pl->stab32.data(), E * 4, hipMemcpyHostToDevice, s)) !=
           hipSuccess))
    return hip_fail(e, "upload standard tables");
  return plan_upload_inst(pl, s);
}

sg_status plan_upload_inst(Plan *pl, hipStream_t s) {
  hipError_t e;
  if ((e = ensure(&pl->d_inst, &pl->inst_capacity, (int64_t)pl->inst.size(), nullptr)) != hipSuccess)
    return fail(SG_ENOMEM, "device allocation of instance descriptors failed");
  if (!pl->inst.empty() &&
      (e = hipMemcpyAsync(pl->d_inst, pl->inst.data(), pl->inst.size() * sizeof(InstDev),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "upload instance descriptors");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "plan upload");
  return SG_OK;
}

void plan_free(Plan *pl) {
  if (!pl) return;
  hipFree(pl->d_inst);
  hipFree(pl->d_packs);
  hipFree(pl->d_items);
  hipFree(pl->d_scratch);
  hipFree(pl->d_stab64);
  hipFree(pl->d_stab32r);
  hipFree(pl->d_stab32);
  pl->d_stab64 = pl->d_stab32r = nullptr;
  pl->d_stab32 = nullptr;
  pl->stab_capacity = 0;
  pl->d_inst = nullptr;
  pl->d_packs = nullptr;
  pl->d_items = nullptr;
  pl->d_scratch = nullptr;
  pl->inst_capacity = pl->packs_capacity = pl->items_capacity = pl->scratch_capacity = 0;
}

}  // namespace sg
