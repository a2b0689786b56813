// Host term compiler: turns a problem description into the Smolyak term set,
// combination coefficients, compact basis, mapping table M^B, its inverse, the
// one-mode tables and the per-term operator coefficients the kernels read.
//
// Sec. 2: terms l (l_i >= 0) with L-D+1 <= |l| <= L, weight
// D_l = (-1)^(L-|l|) C(D-1, L-|l|), per-mode sizes N_l = A + B l.
// Sec. 3 / Table 2: compact basis = union of the term bases without
// duplicates; M^B maps (term, position) to the compact index.  Orderings:
// terms with l_1 fastest, positions with mode 1 fastest, compact basis
// lexicographic with mode 1 slowest.
//
// Closed form used for the compact basis: index n of one mode first appears
// at level g(n) = min{l : nb(l) > n}; a tuple n is in some term's basis iff
// sum_i g(n_i) <= L (raise any level of g(n) to land inside R(l)).
//
// Modes with a single basis function (nb(l_i) = 1, level 0 in the standard
// maps) are integrated out exactly per term: along such a mode Alg. 1 takes
// b_0(Q_u) psi to the grid, multiplies by the operator and projects back with
// wt_u b_0(Q_u), which only needs the rule's moments
// m_p = sum_u wt_u b_0(Q_u)^2 Q_u^p (p = 1, 2) and the kinetic element
// t = sum_u wt_u b_0(Q_u) b_0''(Q_u).  The polynomial family then gives an
// effective potential over the active modes only:
//   V_eff = c0 + sum_p (alpha_p Q_p^2 + beta_p Q_p)
//           + sum_{p<q active} (c Q_p^2 Q_q^2 + k Q_p^2 Q_q),
// identical (up to rounding) to the literal per-term sweep over all modes.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "sg_internal.h"

namespace sg {

namespace {

inline int size_map(int A, int B, int l) { return A + B * l; }

}  // namespace

sg_status count_sizes(int D, int L, int nbA, int nbB, int64_t out[3]) {
  if (D < 1 || D > 4096 || L < 0 || L > 64 || nbA < 1 || nbB < 1) return SG_EINVAL;
  // Polynomials in the level variable, truncated at degree L; entries are
  // counts, accumulated in long double with an overflow guard.
  const long double lim = 9.0e18L;
  std::vector<long double> P(L + 1), G(L + 1), C(L + 1, 1.0L);
  for (int l = 0; l <= L; ++l) {
    P[l] = size_map(nbA, nbB, l);
    G[l] = size_map(nbA, nbB, l) - (l > 0 ? size_map(nbA, nbB, l - 1) : 0);
  }
  auto power = [&](const std::vector<long double> &poly) {
    std::vector<long double> res(L + 1, 0.0L), nxt(L + 1);
    res[0] = 1.0L;
    for (int e = 0; e < D; ++e) {
      std::fill(nxt.begin(), nxt.end(), 0.0L);
      for (int a = 0; a <= L; ++a) {
        if (res[a] == 0.0L) continue;
        for (int b = 0; a + b <= L; ++b) nxt[a + b] += res[a] * poly[b];
      }
      res.swap(nxt);
    }
    return res;
  };
  int lo = std::max(0, L - D + 1);
  auto PD = power(P), GD = power(G), CD = power(C);
  long double ns = 0, ncs = 0, nst = 0;
  for (int m = lo; m <= L; ++m) { ns += PD[m]; nst += CD[m]; }
  for (int m = 0; m <= L; ++m) ncs += GD[m];
  if (ns > lim || ncs > lim || nst > lim) return SG_EINVAL;
  out[0] = (int64_t)std::llround((double)nst);
  out[1] = (int64_t)std::llround((double)ns);
  out[2] = (int64_t)std::llround((double)ncs);
  // exact integer recount when the doubles could round (large values)
  if (ns > 1e15L || ncs > 1e15L) {
    // same recursion in unsigned 128-bit integers
    using u128 = unsigned __int128;
    auto ipower = [&](const std::vector<long double> &poly) {
      std::vector<u128> res(L + 1, 0), nxt(L + 1);
      res[0] = 1;
      for (int e = 0; e < D; ++e) {
        std::fill(nxt.begin(), nxt.end(), (u128)0);
        for (int a = 0; a <= L; ++a)
          for (int b = 0; a + b <= L; ++b) nxt[a + b] += res[a] * (u128)(uint64_t)poly[b];
        res.swap(nxt);
      }
      return res;
    };
    auto iP = ipower(P), iG = ipower(G), iC = ipower(C);
    u128 a = 0, b = 0, c = 0;
    for (int m = lo; m <= L; ++m) { a += iP[m]; c += iC[m]; }
    for (int m = 0; m <= L; ++m) b += iG[m];
    out[0] = (int64_t)c;
    out[1] = (int64_t)a;
    out[2] = (int64_t)b;
  }
  return SG_OK;
}

sg_status compile_problem(const sg_problem_desc *desc, Compiled *out, std::string *err) {
  Compiled &h = *out;
  if (!desc) { *err = "desc is NULL"; return SG_EINVAL; }
  const int D = desc->D, L = desc->L;
  if (D < 1 || D > 64) { *err = "D must be in 1..64"; return SG_EINVAL; }
  if (L < 0 || L >= kMaxLevels) { *err = "L must be in 0..15"; return SG_EINVAL; }
  if (desc->nb_A < 1 || desc->nb_B < 1 || desc->nq_A < 1 || desc->nq_B < 1) {
    *err = "size maps need A >= 1 and B >= 1"; return SG_EINVAL;
  }
  if (!desc->omega || !desc->c) { *err = "omega and c are required"; return SG_EINVAL; }
  h.D = D; h.L = L;
  h.nbA = desc->nb_A; h.nbB = desc->nb_B; h.nqA = desc->nq_A; h.nqB = desc->nq_B;
  for (int l = 0; l <= L; ++l) {
    int nb = size_map(h.nbA, h.nbB, l), nq = size_map(h.nqA, h.nqB, l);
    if (nq < nb) { *err = "nq(l) must be >= nb(l)"; return SG_EINVAL; }
    if (nq > kMaxN || nb > kMaxN) { *err = "nb(L), nq(L) must be <= 16"; return SG_EINVAL; }
  }
  h.omega.assign(desc->omega, desc->omega + D);
  h.c.assign(desc->c, desc->c + size_t(D) * D);
  h.k.assign(size_t(D) * D, 0.0);
  if (desc->k) h.k.assign(desc->k, desc->k + size_t(D) * D);
  for (int i = 0; i < D; ++i) {
    if (!(h.omega[i] > 0.0) || !std::isfinite(h.omega[i])) { *err = "omega must be finite and > 0"; return SG_EINVAL; }
    for (int j = 0; j < D; ++j) {
      if (j <= i) { h.c[size_t(i) * D + j] = 0.0; h.k[size_t(i) * D + j] = 0.0; }
      if (!std::isfinite(h.c[size_t(i) * D + j]) || !std::isfinite(h.k[size_t(i) * D + j])) {
        *err = "c and k must be finite"; return SG_EINVAL;
      }
    }
  }
  int64_t sizes[3];
  if (count_sizes(D, L, h.nbA, h.nbB, sizes) != SG_OK) { *err = "problem too large"; return SG_EINVAL; }
  if (sizes[1] > (int64_t)2000000000 || sizes[0] > (int64_t)50000000) {
    *err = "N_s or N_st beyond int32 layout limits"; return SG_EINVAL;
  }

  // lowest level of each one-mode index
  h.nmax = size_map(h.nbA, h.nbB, L) - 1;
  h.g.assign(h.nmax + 1, 0);
  for (int n = 0; n <= h.nmax; ++n) {
    int l = 0;
    while (size_map(h.nbA, h.nbB, l) <= n) ++l;
    h.g[n] = l;
  }

  // ---- term set, canonical order (l_1 fastest) ---------------------------
  h.nterms = sizes[0];
  h.lev.resize(size_t(h.nterms) * D);
  h.coeff.resize(h.nterms);
  {
    const int lo = L - D + 1;
    std::vector<int> l(D, 0);
    int64_t t = 0;
    // iterate with an odometer in which mode 1 (index 0) moves fastest,
    // restricted to |l| <= L
    int sum = 0;
    while (true) {
      if (sum >= lo) {
        for (int i = 0; i < D; ++i) h.lev[size_t(t) * D + i] = (uint8_t)l[i];
        int s = L - sum;  // 0 <= s <= D-1 here
        double bin = 1.0;
        for (int j = 1; j <= s; ++j) bin = bin * (D - 1 - s + j) / j;
        h.coeff[t] = (int32_t)std::llround(bin) * ((s % 2) ? -1 : 1);
        ++t;
      }
      int i = 0;
      while (i < D) {
        if (sum < L) { ++l[i]; ++sum; break; }
        sum -= l[i]; l[i] = 0; ++i;
      }
      if (i == D) break;
    }
    if (t != h.nterms) { *err = "internal: term count mismatch"; return SG_EINVAL; }
  }

  // ---- compact basis ranking tables --------------------------------------
  const int NX = h.nmax + 1;
  // cnt[d][b]: tuples over d modes with sum g <= b
  std::vector<int64_t> cnt(size_t(D + 1) * (L + 1), 0);
  for (int b = 0; b <= L; ++b) cnt[b] = 1;
  for (int d = 1; d <= D; ++d)
    for (int b = 0; b <= L; ++b) {
      int64_t s = 0;
      for (int x = 0; x < NX; ++x)
        if (h.g[x] <= b) s += cnt[size_t(d - 1) * (L + 1) + b - h.g[x]];
      cnt[size_t(d) * (L + 1) + b] = s;
    }
  h.ncs = cnt[size_t(D) * (L + 1) + L];
  if (h.ncs != sizes[2]) { *err = "internal: compact count mismatch"; return SG_EINVAL; }
  // pre[(d*(L+1)+b)*(NX+1)+x] = sum_{v<x, g(v)<=b} cnt[d][b-g(v)]
  std::vector<int64_t> pre(size_t(D + 1) * (L + 1) * (NX + 1), 0);
  for (int d = 0; d <= D; ++d)
    for (int b = 0; b <= L; ++b) {
      int64_t acc = 0;
      int64_t *row = &pre[(size_t(d) * (L + 1) + b) * (NX + 1)];
      for (int x = 0; x < NX; ++x) {
        row[x] = acc;
        if (h.g[x] <= b) acc += cnt[size_t(d) * (L + 1) + b - h.g[x]];
      }
      row[NX] = acc;
    }
  auto rank = [&](const uint8_t *n) -> int64_t {
    int64_t r = 0;
    int b = L;
    for (int i = 0; i < D; ++i) {
      r += pre[(size_t(D - 1 - i) * (L + 1) + b) * (NX + 1) + n[i]];
      b -= h.g[n[i]];
    }
    return r;
  };

  // compact basis enumeration (lexicographic, mode 1 slowest)
  h.compact.resize(size_t(h.ncs) * D);
  {
    std::vector<uint8_t> n(D, 0);
    int64_t idx = 0;
    // depth-first over modes, mode 1 outermost: lexicographic, mode 1 slowest
    std::function<void(int, int)> rec = [&](int i, int budget) {
      if (i == D) {
        std::memcpy(&h.compact[size_t(idx) * D], n.data(), D);
        ++idx;
        return;
      }
      for (int x = 0; x <= h.nmax; ++x) {
        if (h.g[x] > budget) continue;
        n[i] = (uint8_t)x;
        rec(i + 1, budget - h.g[x]);
      }
    };
    rec(0, L);
    if (idx != h.ncs) { *err = "internal: compact enumeration mismatch"; return SG_EINVAL; }
  }

  // ---- mapping table M^B and term offsets -------------------------------
  h.off.resize(h.nterms + 1);
  h.off[0] = 0;
  for (int64_t t = 0; t < h.nterms; ++t) {
    int64_t sz = 1;
    for (int i = 0; i < D; ++i) sz *= size_map(h.nbA, h.nbB, h.lev[size_t(t) * D + i]);
    h.off[t + 1] = h.off[t] + sz;
  }
  if (h.off[h.nterms] != sizes[1]) { *err = "internal: N_s mismatch"; return SG_EINVAL; }
  // M^B in Table 2's position order (mode 1 fastest), and the device copy
  // with positions in lexicographic order (mode D fastest, as the compact
  // basis): consecutive compact indices then sit at consecutive positions of
  // every term holding them, so the term sweep writes each term contiguously
  // and the reduce's reads of neighbouring rows share cache lines.
  h.MB.resize(h.off[h.nterms]);
  h.mbd.resize(h.off[h.nterms]);
  {
    std::vector<uint8_t> n(D);
    std::vector<int> nb(D);
    for (int64_t t = 0; t < h.nterms; ++t) {
      for (int i = 0; i < D; ++i) { nb[i] = size_map(h.nbA, h.nbB, h.lev[size_t(t) * D + i]); n[i] = 0; }
      for (int64_t s = h.off[t]; s < h.off[t + 1]; ++s) {
        h.MB[s] = (int32_t)rank(n.data());
        for (int i = 0; i < D; ++i) {  // mode 1 fastest
          if (++n[i] < nb[i]) break;
          n[i] = 0;
        }
      }
      for (int i = 0; i < D; ++i) n[i] = 0;
      for (int64_t s = h.off[t]; s < h.off[t + 1]; ++s) {
        h.mbd[s] = (int32_t)rank(n.data());
        for (int i = D - 1; i >= 0; --i) {  // mode D fastest
          if (++n[i] < nb[i]) break;
          n[i] = 0;
        }
      }
    }
  }

  // ---- inverse of the device mapping (CSR over compact indices) ----------
  h.inv_ptr.assign(h.ncs + 1, 0);
  for (int32_t cs : h.mbd) h.inv_ptr[cs + 1]++;
  for (int64_t i = 0; i < h.ncs; ++i) h.inv_ptr[i + 1] += h.inv_ptr[i];
  h.inv_col.resize(h.mbd.size());
  {
    std::vector<int32_t> fill(h.inv_ptr.begin(), h.inv_ptr.end() - 1);
    for (size_t s = 0; s < h.mbd.size(); ++s) h.inv_col[fill[h.mbd[s]]++] = (int32_t)s;
  }

  // ---- exact diagonal harmonic part on the compact basis ----------------
  h.h0.resize(h.ncs);
  for (int64_t i = 0; i < h.ncs; ++i) {
    double e = 0.0;
    for (int j = 0; j < D; ++j) e += h.omega[j] * (h.compact[size_t(i) * D + j] + 0.5);
    h.h0[i] = e;
  }

  // ---- one-mode tables per level ----------------------------------------
  std::vector<double> m1(L + 1, 0.0), m2(L + 1, 0.0), t0(L + 1, 0.0);
  h.tables.clear();
  for (int l = 0; l <= L; ++l) {
    int nb = size_map(h.nbA, h.nbB, l), nq = size_map(h.nqA, h.nqB, l);
    std::vector<double> x, wt;
    gauss_hermite_nodes(nq, &x, &wt);
    std::vector<double> b(size_t(nq) * nb), d2(size_t(nq) * nb), tmp(nb);
    for (int u = 0; u < nq; ++u) {
      hermite_function_values(nb, x[u], tmp.data());
      for (int k = 0; k < nb; ++k) {
        b[size_t(u) * nb + k] = tmp[k];
        d2[size_t(u) * nb + k] = (x[u] * x[u] - (2.0 * k + 1.0)) * tmp[k];
      }
    }
    LevelDev &ld = h.tdesc.lev[l];
    ld.nb = nb; ld.nq = nq;
    ld.bt = (int32_t)h.tables.size();
    h.tables.insert(h.tables.end(), b.begin(), b.end());
    ld.wt = (int32_t)h.tables.size();
    for (int k = 0; k < nb; ++k)
      for (int u = 0; u < nq; ++u) h.tables.push_back(wt[u] * b[size_t(u) * nb + k]);
    ld.kg = (int32_t)h.tables.size();
    for (int u = 0; u < nq; ++u)
      for (int v = 0; v < nq; ++v) {
        double s = 0.0;
        for (int k = 0; k < nb; ++k) s += d2[size_t(u) * nb + k] * wt[v] * b[size_t(v) * nb + k];
        h.tables.push_back(s);
      }
    ld.x = (int32_t)h.tables.size();
    h.tables.insert(h.tables.end(), x.begin(), x.end());
    // single-function moments (used when nb == 1)
    for (int u = 0; u < nq; ++u) {
      double w0 = wt[u] * b[size_t(u) * nb] * b[size_t(u) * nb];
      m1[l] += w0 * x[u];
      m2[l] += w0 * x[u] * x[u];
      t0[l] += wt[u] * b[size_t(u) * nb] * d2[size_t(u) * nb];
    }
  }
  // pad the table array to a multiple of 2 doubles
  if (h.tables.size() % 2) h.tables.push_back(0.0);

  // ---- per-term operator coefficients -------------------------------------
  h.terms.resize(h.nterms);
  h.pairs.assign((size_t)h.nterms * kPairStride, 0.0);
  h.potc.assign((size_t)h.nterms * 2 * kCoefStride, 0.0);
  h.grid_literal = h.grid_active = h.max_basis = h.max_grid = 0;
  h.flops_fp64 = h.flops_mixed = 0.0;
  h.nfib = 0;
  std::vector<double> cost(h.nterms);
  for (int64_t t = 0; t < h.nterms; ++t) {
    TermDev &T = h.terms[t];
    std::memset(&T, 0, sizeof(T));
    const uint8_t *lv = &h.lev[size_t(t) * D];
    std::vector<int> act, zero;
    int64_t glit = 1;
    // active modes in decreasing mode id: the first is the fastest index of
    // the device position order
    for (int i = D - 1; i >= 0; --i) {
      glit *= size_map(h.nqA, h.nqB, lv[i]);
      if (size_map(h.nbA, h.nbB, lv[i]) > 1) act.push_back(i); else zero.push_back(i);
    }
    std::reverse(zero.begin(), zero.end());   // the level-0 sums below take zero ascending
    if ((int)act.size() > kMaxActive) { *err = "a term has more than 8 active modes"; return SG_EINVAL; }
    T.off = (int32_t)h.off[t];
    T.na = (int32_t)act.size();
    T.coeff = h.coeff[t];
    int64_t nbas = 1, ngr = 1;
    for (size_t p = 0; p < act.size(); ++p) {
      const int l = lv[act[p]];
      T.lev[p] = l;
      T.mode[p] = act[p];
      T.nb[p] = size_map(h.nbA, h.nbB, l);
      T.nq[p] = size_map(h.nqA, h.nqB, l);
      T.bt[p] = h.tdesc.lev[l].bt;
      T.wt[p] = h.tdesc.lev[l].wt;
      T.kg[p] = h.tdesc.lev[l].kg;
      T.xo[p] = h.tdesc.lev[l].x;
      T.rcp_nq[p] = 1.0f / (float)T.nq[p];
      nbas *= T.nb[p];
      ngr *= T.nq[p];
    }
    for (size_t p = act.size(); p < (size_t)kMaxActive; ++p) {
      T.nb[p] = T.nq[p] = 1;
      T.rcp_nq[p] = 1.0f;
    }
    if (!act.empty()) {
      T.foff = (int32_t)h.nfib;
      h.nfib += ngr / T.nq[0];
    }
    auto r32 = [](double v) { return (double)(float)v; };
    double *pr = &h.pairs[(size_t)t * kPairStride];
    double *prr = pr + 2 * kMaxPairs;
    for (size_t q = 0; q < act.size(); ++q)
      for (size_t r = q + 1; r < act.size(); ++r) {
        // act[q] > act[r]: c is symmetric; k_ij Q_i^2 Q_j (i < j) is the
        // coefficient of x_r^2 x_q here
        const int pi = pair_index((int)q, (int)r);
        pr[2 * pi] = h.c[(size_t)act[r] * D + act[q]];
        pr[2 * pi + 1] = h.k[(size_t)act[r] * D + act[q]];
        prr[2 * pi] = r32(pr[2 * pi]);
        prr[2 * pi + 1] = r32(pr[2 * pi + 1]);
      }
    T.nbasis = (int32_t)nbas;
    T.ngrid = (int32_t)ngr;
    auto C = [&](int i, int j) { return h.c[size_t(std::min(i, j)) * D + std::max(i, j)]; };
    auto K = [&](int i, int j) { return h.k[size_t(i) * D + j]; };  // i < j
    double c0s = 0.0, c0h = 0.0;
    for (size_t a = 0; a < zero.size(); ++a) {
      int z = zero[a], lz = lv[z];
      c0h += 0.5 * h.omega[z] * m2[lz] - 0.5 * h.omega[z] * t0[lz];
      for (size_t b2 = a + 1; b2 < zero.size(); ++b2) {
        int z2 = zero[b2], lz2 = lv[z2];
        c0s += C(z, z2) * m2[lz] * m2[lz2] + K(z, z2) * m2[lz] * m1[lz2];
      }
    }
    T.c0[kPotFull] = c0s + c0h;
    T.c0[kPotSplit] = c0s;
    T.c0[kPotSplitRounded] = r32(c0s);
    for (size_t p = 0; p < act.size(); ++p) {
      int m = act[p];
      double al = 0.0, be = 0.0;
      for (int z : zero) {
        int lz = lv[z];
        al += C(m, z) * m2[lz];
        if (m < z) al += K(m, z) * m1[lz];
        else be += K(z, m) * m2[lz];
      }
      T.alpha[kPotFull][p] = al + 0.5 * h.omega[m];
      T.alpha[kPotSplit][p] = al;
      T.alpha[kPotSplitRounded][p] = r32(al);
      T.beta[0][p] = be;
      T.beta[1][p] = r32(be);
      T.kin[p] = -0.5 * h.omega[m];
    }
    // split coefficient blocks (exact, then rounded to FP32)
    for (int v = 0; v < 2; ++v) {
      double *cb = &h.potc[((size_t)t * 2 + v) * kCoefStride];
      const int pot = v == 0 ? kPotSplit : kPotSplitRounded;
      const double *pv = pr + (v == 0 ? 0 : 2 * kMaxPairs);
      const int na = (int)act.size();
      cb[0] = T.c0[pot];
      if (na > 0) {
        cb[1] = T.alpha[pot][0];
        cb[2] = T.beta[v][0];
      }
      for (int q = 1; q < na; ++q) {
        cb[2 + q] = T.alpha[pot][q];
        cb[9 + q] = T.beta[v][q];
        cb[16 + q] = pv[2 * pair_index(0, q)];
        cb[23 + q] = pv[2 * pair_index(0, q) + 1];
        for (int r = q + 1; r < na; ++r) {
          cb[coef_pair(q, r)] = pv[2 * pair_index(q, r)];
          cb[coef_pair(q, r) + 1] = pv[2 * pair_index(q, r) + 1];
        }
      }
    }
    // sizes and algorithmic flops (4 per complex x real multiply-add)
    h.grid_literal += glit;
    h.grid_active += ngr;
    h.max_basis = std::max<int64_t>(h.max_basis, nbas);
    h.max_grid = std::max<int64_t>(h.max_grid, ngr);
    double f_bg = 0.0, f_kin = 0.0;
    {
      double sz = (double)nbas;
      for (size_t p = 0; p < act.size(); ++p) {
        int nb = size_map(h.nbA, h.nbB, lv[act[p]]), nq = size_map(h.nqA, h.nqB, lv[act[p]]);
        sz = sz / nb * nq;
        f_bg += 4.0 * sz * nb;       // basis -> grid along mode p
        f_kin += 4.0 * (double)ngr * nq;
      }
    }
    // grid -> basis mirrors basis -> grid (same multiply-add count)
    double f_common = 2.0 * f_bg + 2.0 * (double)ngr + 2.0 * (double)nbas;
    h.flops_fp64 += f_common + f_kin + 2.0 * (double)ngr;
    h.flops_mixed += f_common;
    cost[t] = f_common + f_kin + 64.0;
  }
  // reduce: one complex add per term-major entry (+ the diagonal in mixed)
  h.flops_fp64 += 2.0 * (double)h.MB.size();
  h.flops_mixed += 2.0 * (double)h.MB.size() + 4.0 * (double)h.ncs;
  // algorithmic bytes: psi in and out, M^B + inverse map, term-major results
  // written and read, term descriptors
  h.bytes_apply = 32.0 * (double)h.ncs + 8.0 * (double)h.MB.size() + 4.0 * (double)h.ncs +
                  32.0 * (double)h.MB.size() + (double)sizeof(TermDev) * (double)h.nterms;

  h.split_exact = true;
  for (int l = 0; l <= L; ++l)
    if (size_map(h.nqA, h.nqB, l) <= size_map(h.nbA, h.nbB, l)) h.split_exact = false;
  h.cost = cost;
  h.tables32.assign(h.tables.begin(), h.tables.end());
  h.tables32r.assign(h.tables32.begin(), h.tables32.end());
  if (h.max_grid > 65536) {
    *err = "a term grid exceeds 65536 points";
    return SG_EINVAL;
  }
  if (h.nfib > INT32_MAX) {
    *err = "too many grid fibers for 32-bit offsets";
    return SG_EINVAL;
  }

  // reduce rows: long rows (a wavefront each) first, then short rows
  h.rows.clear();
  h.rows.reserve(h.ncs);
  for (int64_t r = 0; r < h.ncs; ++r)
    if (h.inv_ptr[r + 1] - h.inv_ptr[r] > kLongRow) h.rows.push_back((int32_t)r);
  h.n_long_rows = (int64_t)h.rows.size();
  for (int64_t r = 0; r < h.ncs; ++r)
    if (h.inv_ptr[r + 1] - h.inv_ptr[r] <= kLongRow) h.rows.push_back((int32_t)r);
  // reduce items: kRowWaves per long row, then one per kShortLanes
  // short rows, padded to whole workgroups
  h.n_items = (h.ncs - h.n_long_rows + kShortLanes - 1) / kShortLanes;
  h.n_items = (h.n_items + kRowWaves - 1) / kRowWaves * kRowWaves;
  for (int64_t q = 0; q < h.n_long_rows; ++q) {
    const int64_t len = h.inv_ptr[h.rows[q] + 1] - h.inv_ptr[h.rows[q]];
    if (len > (int64_t)INT32_MAX / 2) {
      *err = "a compact row has too many term contributions";
      return SG_EINVAL;
    }
    h.n_items += kRowWaves;
  }
  // the inverse CSR in that row order: the reduce loads a row's id and its
  // bounds at the same index, in parallel
  h.red_ptr.assign(h.ncs + 1, 0);
  h.red_col.clear();
  h.red_col.reserve(h.inv_col.size());
  for (int64_t i = 0; i < h.ncs; ++i) {
    const int32_t r = h.rows[i];
    h.red_col.insert(h.red_col.end(), h.inv_col.begin() + h.inv_ptr[r],
                     h.inv_col.begin() + h.inv_ptr[r + 1]);
    h.red_ptr[i + 1] = (int32_t)h.red_col.size();
  }
  return SG_OK;
}

bool group_terms(const Compiled &h, std::vector<int32_t> *order, std::vector<TermGroup> *groups) {
  const int64_t nt = h.nterms;
  std::vector<int32_t> shape_of(nt, -1);
  for (int64_t t = 0; t < nt; ++t) {
    const TermDev &T = h.terms[t];
    int maxlev = 0;
    for (int q = 0; q < T.na; ++q) maxlev = std::max(maxlev, (int)T.lev[q]);
    for (int k = kGroupShapes - 1; k >= 0; --k)
      if (T.ngrid <= kGroupShape[k].max_grid && maxlev <= kGroupShape[k].max_level) {
        shape_of[t] = k;
        break;
      }
    if (shape_of[t] < 0) return false;
  }
  order->resize(nt);
  std::iota(order->begin(), order->end(), 0);
  std::stable_sort(order->begin(), order->end(), [&](int32_t a, int32_t b) {
    if (shape_of[a] != shape_of[b]) return shape_of[a] < shape_of[b];
    return h.terms[a].ngrid > h.terms[b].ngrid;
  });
  groups->clear();
  for (int64_t i = 0; i < nt;) {
    TermGroup G;
    G.first = (int32_t)i;
    G.shape = shape_of[(*order)[i]];
    G.max_grid = h.terms[(*order)[i]].ngrid;
    while (i < nt && shape_of[(*order)[i]] == G.shape) ++i;
    G.count = (int32_t)(i - G.first);
    groups->push_back(G);
  }
  return true;
}

}  // namespace sg
