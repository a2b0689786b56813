// Host-only check of the plan builder (no GPU): the device addresses a plan
// hands the sweep and reduce kernels.  Every wavefront of a wave pack reads
// its slot's instance, term and M^B pointer before it tests whether the slot
// is used, so every slot of every pack must name a real term of its own
// problem; every reduce item's row and bound pointers must stay inside its
// problem's arrays; every compact-basis row must be finished by exactly one
// item.  Problems get fake, disjoint device addresses; nothing is
// dereferenced.  Built and run by the host test suite.
#include <cstdio>
#include <cstdint>
#include <algorithm>
#include "sg_internal.h"
using namespace sg;

// the plan builder's device-side neighbours, not exercised here
namespace sg {
hipError_t launch_sweep(const Plan *, const LaunchCtl &, hipStream_t) { return hipSuccess; }
hipError_t launch_reduce(const Plan *, const LaunchCtl &, hipStream_t) { return hipSuccess; }
hipError_t launch_finalize(const Plan *, hipStream_t) { return hipSuccess; }
hipError_t launch_dot(const sg_problem *, const double2 *, const double2 *, hipStream_t) { return hipSuccess; }
hipError_t launch_axpby(int64_t, double2 *, const double2 *, double, double, double, hipStream_t) { return hipSuccess; }
}
namespace sg {
sg_status fail(sg_status s, const std::string &) { return s; }
sg_status hip_fail(hipError_t, const char *) { return SG_EDEVICE; }
}

int main() {
  int bad = 0;
  std::vector<sg_problem *> all;
  for (auto [D, L] : std::vector<std::pair<int,int>>{{2,4},{6,6},{12,6},{7,7},{3,3},{1,7},{5,7}}) {
    std::vector<double> om(D, 1.0), c(D * D, 0.01), k(D * D, 0.005);
    sg_problem_desc d{D, L, 1, 2, 2, 2, om.data(), c.data(), k.data()};
    sg_problem *p = new sg_problem();
    std::string err;
    if (compile_problem(&d, &p->h, &err) != SG_OK) { printf("compile fail\n"); return 1; }
    // fake device arrays, disjoint per problem
    static uintptr_t next = 0x100000000ull;
    auto fake = [&](size_t bytes) { uintptr_t a = next; next += (bytes + 4096) & ~(uintptr_t)255; return a; };
    p->d_terms = (TermDev *)fake(p->h.nterms * sizeof(TermDev));
    p->d_mb = (int32_t *)fake(p->h.MB.size() * 4);
    p->d_rows = (int32_t *)fake(p->h.ncs * 4);
    p->d_inv_ptr = (int32_t *)fake((p->h.ncs + 1) * 4);
    all.push_back(p);
  }
  auto in = [](const void *x, const void *base, size_t n, size_t sz) {
    return (uintptr_t)x >= (uintptr_t)base && (uintptr_t)x + sz <= (uintptr_t)base + n * sz;
  };
  auto check = [&](const Plan &pl, const std::vector<sg_problem *> &probs) {
    // every pack's tables (levels up to its highest) and term buffers fit
    // the launch's LDS, and that stays within two workgroups per compute unit
    for (int k = 0; k < kPackSets; ++k) {
      const PackSet &set = pl.sets[k];
      const bool two = k == kSetMixed64 && pl.any_round32;
      const int ta = two ? set.tab_bytes / 2 : set.tab_bytes, tb = two ? set.tab_bytes / 2 : 0;
      const int er = k == kSetMixed32 ? 4 : 8;
      if (set.count && set.lds_bytes > kLdsPerCU / (k == kSetMixed32 ? 4 : 2)) {
        printf("set %d lds %d\n", k, set.lds_bytes); bad++;
      }
      for (int q = set.first; q < set.first + set.count; ++q) {
        const PackDev &pk = pl.packs[q];
        if (pk.lds_base != pack_lds_base(ta, tb, er, pk.maxlev) || pk.lds_base + pk.slices > set.lds_bytes) {
          printf("pack %d lds\n", q); bad++;
        }
        if (pk.block == kPackWaves)
          for (int w = 0; w < pk.n; ++w) {
            const sg_problem *p = probs[pk.inst[w]];
            const TermDev &T = p->h.terms[pk.term[w]];
            int ml = 0;
            for (int m = 0; m < T.na; ++m) ml = std::max<int>(ml, T.lev[m]);
            if (ml > pk.maxlev || pk.lds_off[w] < 0 || pk.lds_off[w] > pk.slices) {
              printf("pack %d slot %d maxlev/offset\n", q, w); bad++;
            }
          }
      }
    }
    for (const PackDev &pk : pl.packs) {
      const int slots = pk.block == kPackWaves ? kPackTerms : 1;
      for (int w = 0; w < slots; ++w) {
        if (pk.inst[w] < 0 || pk.inst[w] >= (int)probs.size()) { printf("inst slot %d\n", w); bad++; continue; }
        const sg_problem *p = probs[pk.inst[w]];
        if (pk.term[w] < 0 || pk.term[w] >= p->h.nterms) { printf("term slot %d n %d\n", w, pk.n); bad++; continue; }
        if (pk.mbt[w] != p->d_mb + p->h.terms[pk.term[w]].off) { printf("mbt slot %d\n", w); bad++; }
      }
    }
    for (const RedItem &it : pl.items) {
      const sg_problem *p = probs[it.inst];
      const int nch = (it.chunk >> 12) & 0xfff;
      if (nch) {
        if (!in(it.rows, p->d_rows, p->h.ncs, 4) || !in(it.ptr + 1, p->d_inv_ptr, p->h.ncs + 1, 4) ||
            it.rows != p->d_rows + it.first || it.first >= p->h.n_long_rows) { printf("long item\n"); bad++; }
      } else {
        for (int r = 0; r < it.chunk; ++r)
          if (!in(it.rows + r, p->d_rows, p->h.ncs, 4) || !in(it.ptr + r + 1, p->d_inv_ptr, p->h.ncs + 1, 4) ||
              it.first < p->h.n_long_rows) { printf("short item\n"); bad++; }
        if (it.chunk < 0 || it.chunk > kShortLanes) { printf("short count\n"); bad++; }
      }
    }
    // a long row is one workgroup: kRowWaves consecutive items from a
    // workgroup boundary, waves 0..kRowWaves-1
    for (size_t q = 0; q < pl.items.size(); ++q) {
      const RedItem &it = pl.items[q];
      const int nch = (it.chunk >> 12) & 0xfff;
      if (nch && (nch != 1 || (int)(q % kRowWaves) != (it.chunk >> 24))) { printf("long row item\n"); bad++; }
    }
    // every row is covered exactly once by short items or chunk 0 wave 0 of long rows
    for (size_t i = 0; i < probs.size(); ++i) {
      std::vector<int> cov(probs[i]->h.ncs, 0);
      for (const RedItem &it : pl.items) {
        if (it.inst != (int)i) continue;
        const int nch = (it.chunk >> 12) & 0xfff;
        if (nch) { if ((it.chunk & 0xfff) == 0 && (it.chunk >> 24) == 0) cov[it.first]++; }
        else for (int r = 0; r < it.chunk; ++r) cov[it.first + r]++;
      }
      for (int64_t r = 0; r < probs[i]->h.ncs; ++r) if (cov[r] != 1) { printf("row %ld covered %d\n", (long)r, cov[r]); bad++; break; }
    }
  };
  std::string err;
  for (sg_problem *p : all)
    for (int bg : {0, 256, 1024})
      for (int sp : {1, 2, 4}) {
        p->block_grid = bg; p->packs_per_cu = sp; p->pcache.valid = false;
        Plan pl; plan_build(&pl, {p}, &err); check(pl, {p});
      }
  for (sg_problem *p : all) { p->block_grid = 0; p->packs_per_cu = 1; p->pcache.valid = false; }
  Plan pm; plan_build(&pm, all, &err); check(pm, all);
  std::vector<sg_problem *> two = {all[1], all[1], all[0]};
  Plan p2; plan_build(&p2, two, &err); check(p2, two);
  printf("packs/items pointer check: %d bad\n", bad);
  return bad ? 1 : 0;
}
