// Internal definitions shared by the host term compiler, the drivers and the
// HIP kernels of the Smolyak library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sg.h"

namespace sg {

// Largest number of active modes (l_i > 0) in one term and largest one-mode
// grid the kernels handle.
constexpr int kMaxActive = 8;
constexpr int kMaxN = 16;

// Per-term operator description, one per Smolyak term, in canonical (Table 2)
// term order.  Level-0 modes are integrated out exactly (see term compiler),
// so a term only carries its active modes.
// Everything a kernel needs about a term sits at constant offsets here (and in
// the term's pair-coefficient block), so a workgroup issues independent
// scalar loads instead of chains of dependent ones.
constexpr int kMaxPairs = kMaxActive * (kMaxActive - 1) / 2;
__host__ __device__ constexpr int pair_index(int q, int r) {  // q < r < kMaxActive
  return q * (2 * kMaxActive - q - 1) / 2 + (r - q - 1);
}

// The first kTermHdrDwords dwords (the header) are what the in-place sweep
// reads; a wavefront loads them with one vector load and reads fields from
// lanes.
struct alignas(16) TermDev {
  int32_t off;       // start of the term in the term-major layout (N_s)
  int32_t nbasis;    // prod over active modes of nb
  int32_t ngrid;     // prod over active modes of nq
  int32_t na;        // number of active modes
  int32_t lev[kMaxActive];  // levels of the active modes, decreasing mode id
  int32_t nb[kMaxActive];   // per active mode: basis size
  int32_t nq[kMaxActive];   //   grid size
  float rcp_nq[kMaxActive]; //   1/nq for fast index division
  double coeff;             // D_l
  int32_t foff;             // first mode-0 fiber of the term in the per-fiber arrays
  // ---- end of header ----
  int32_t mode[kMaxActive]; // mode ids of the active modes
  int32_t bt[kMaxActive];   // offsets of each level's tables in the table array
  int32_t wt[kMaxActive];
  int32_t kg[kMaxActive];
  int32_t xo[kMaxActive];
  // Effective-potential coefficients in three variants (kPot*): the FP64
  // path; the mixed path (no separable harmonic part); the mixed path's
  // values rounded to FP32 (held in FP64), for instances whose FP64 terms
  // must apply the same rounded operator as their FP32 terms.
  double c0[3];                    // constant part
  double alpha[3][kMaxActive];     // coefficient of Q_p^2
  double beta[2][kMaxActive];      // coefficient of Q_p: exact, rounded
  double kin[kMaxActive];          // -1/2 omega_p (kinetic prefactor)
};
constexpr int kPotFull = 0, kPotSplit = 1, kPotSplitRounded = 2;
constexpr int kTermHdrDwords = 39;
static_assert(offsetof(TermDev, coeff) == 4 * (kTermHdrDwords - 3), "term header layout");
static_assert(offsetof(TermDev, foff) == 4 * (kTermHdrDwords - 1), "term header layout");
static_assert(offsetof(TermDev, lev) == 16 && offsetof(TermDev, nb) == 48 &&
                  offsetof(TermDev, nq) == 80 && offsetof(TermDev, rcp_nq) == 112,
              "term header layout");
// Per-term coefficient block of the split coupling potential (exact and
// FP32-rounded variants), which an in-place term copies into LDS next to its
// grid buffer:  [0] c0, [1] alpha_0, [2] beta_0, [2+q] alpha_q, [9+q] beta_q,
// [16+q] c_0q, [23+q] k_0q (q = 1..7), [31 + 2 (pair_index(q,r) - 7)] c_qr,
// k_qr (1 <= q < r <= 7).
constexpr int kCoefUsed = 73;
constexpr int kCoefStride = 80;          // doubles per variant
constexpr int kCoefLdsBytes = 640;       // LDS reserved per in-place term
__host__ __device__ constexpr int coef_pair(int q, int r) { return 31 + 2 * (q * (2 * 8 - q - 1) / 2 + (r - q - 1) - 7); }
// Pair coefficients per term: [2 variants: exact, FP32-rounded][kMaxPairs][c, k].
constexpr int kPairStride = 4 * kMaxPairs;

// Offsets of the one-mode tables of a level inside the packed table array.
struct LevelDev {
  int32_t nb, nq;
  int32_t bt;   // b(Q_u)            [nq][nb]   basis -> grid
  int32_t wt;   // wt_u b(Q_u)^T     [nb][nq]   grid -> basis
  int32_t kg;   // d2b (wt b)^T      [nq][nq]   second derivative on the grid
  int32_t x;    // nodes             [nq]
};

constexpr int kMaxLevels = 16;

struct DeviceTables {
  LevelDev lev[kMaxLevels];
};

// Per-instance view read by the kernels.  A launch covers one or more
// problem instances ("plan"); packs and reduce items name their instance.
struct InstDev {
  const TermDev *terms;
  const double *pairs;
  const double *potc;       // [nterms][2][kCoefStride] split coefficient blocks
  const int32_t *mb;
  const int32_t *inv_ptr;   // [N_cs+1] indexed by reduce item row, not compact index
  const int32_t *inv_col;   // [N_s] term-major entries of rows[0], rows[1], ...
  const int32_t *rows;      // long rows first, then short rows
  const double *h0;
  const double *tab64;      // one-mode tables, exact
  const float *tab32;       // the same in FP32
  const double *tab32r;     // FP32-rounded, held in FP64
  // Per mode-0 fiber of every term with active modes (fiber f of term t at
  // t.foff + f): the split coupling potential along the fiber is
  // A + x0 (C + B x0).  [2 variants: exact, FP32-rounded][A, B, C][nfib]
  const double *abc;
  int64_t nfib;
  double2 *tm;              // term-major results
  double2 *x0, *x1;         // apply: x0 -> x1.  Chebyshev: phi buffers, x0 = psi
  double2 *acc;             // Chebyshev running sum
  double *partials;         // [2 * nitems] norm / energy partial sums
  double *result;           // [2] finalised sums
  const double *cheb_a;     // [K] series coefficients (2 - delta_k0) J_k(R)
  int64_t ncs;
  int64_t nlong;            // long rows
  int32_t nitems;           // reduce work items of this instance
  int32_t std_maps;         // nb = 1 + 2l, nq = 2 + 2l
  int32_t round32;          // mixed path: FP64 terms read the FP32-rounded tables
  int32_t K;                // Chebyshev terms (applies per step = K-1)
  double ebar, inv_half, phase_re, phase_im;
  int32_t active;           // 0: the launch skips this instance
  int32_t pad;
  int64_t vec_off;          // added to the launch's vector overrides (x0o, x1o) for this
                            // instance: the electronic states of a two-state problem
                            // are instances over consecutive halves of one vector
  const double *veff;       // tabulated coupling potential, or null (polynomial couplings)
  const int64_t *voff;      //   term t's V_eff from veff + voff[t]
};

// Term-sweep packing.  A workgroup (kSweepThreads threads, eight wavefronts)
// runs one pack: up to kPackTerms terms, one per wavefront, or one term on
// all eight wavefronts, its buffers in LDS or (too large for LDS) in a global
// scratch region.  A term runs "in place" (one grid buffer: each contraction
// holds all its input fibers in registers before writing) or "ping-pong"
// (two buffers).  The host picks, per term, the smallest group whose
// registers hold every in-place contraction (inplace_fpt below), and packs
// wave terms under an LDS cap so that two workgroups share a compute unit.
constexpr int kSweepThreads = 512;
constexpr int kPackTerms = 8;
constexpr int kLdsPerCU = 160 * 1024;
constexpr int kComputeUnits = 256;   // MI355X; used to size the packing only
constexpr int kPingPongWaveMaxGrid = 512;
// Largest in-place term a single wavefront runs (its contractions in chunks
// of inplace_fpt(NI) fibers per lane when the fibers exceed the lanes).
constexpr int kWaveMaxGrid = 4096;
// Fibers of NI values one thread holds in an in-place contraction.
__host__ __device__ constexpr int inplace_fpt(int ni) { return ni <= 18 ? 18 / ni : 1; }
enum PackKind : int32_t { kPackWaves = 0, kPackBlockLds = 1, kPackBlockScratch = 2 };
struct PackDev {
  int32_t n;                    // terms in the pack
  int32_t block;                // PackKind
  int32_t inst[kPackTerms];
  int32_t term[kPackTerms];
  int32_t lds_off[kPackTerms];  // byte offset of each wavefront's LDS slice
  int32_t inplace[kPackTerms];  // 1: in place (one buffer), 0: ping-pong
  int32_t maxlev;               // highest level of an active mode of the pack's terms
  int32_t slices;               // LDS bytes of the pack's term buffers (after its tables)
  int32_t lds_base;             // byte offset of those buffers in LDS (pack_lds_base)
  int32_t pad;
  int64_t scratch_off;          // kPackBlockScratch: byte offset in the plan's scratch
  const int32_t *mbt[kPackTerms];  // each term's first M^B entry (device), for its gather
};
struct PackSet {
  int32_t first = 0;            // index of the first pack
  int32_t count = 0;
  int32_t lds_bytes = 0;        // dynamic LDS of the launch (tables + largest pack)
  int32_t tab_bytes = 0;        // LDS at offset 0 holding the standard-map tables
  int32_t all_inplace = 0;      // every term of the set runs in place (or is scalar)
};
// The one-mode tables of the standard size maps (nb = 2l+1, nq = 2l+2) are
// the same for every instance; a launch copies them into LDS once per
// workgroup.  Compact layout per level l: b (nq x nb), wt b^T (nb x nq),
// nodes (nq), at element offset std_table_base(l).
__host__ __device__ constexpr int std_table_base(int l) {
  return 8 * ((l - 1) * l * (2 * l - 1) / 6) + 7 * l * (l - 1) + 6 * l;
}
// Where a pack's term buffers start in LDS.  The tables come first, laid out
// by level.  With one table set (tab_b = 0) a pack holds the levels up to its
// highest only, so its buffers start right after those; with two sets (the
// exact and the FP32-rounded FP64 tables) after both whole sets.  elem_r:
// bytes of one table entry.  The planner stores it in each pack.
__host__ __device__ constexpr int pack_lds_base(int tab_a, int tab_b, int elem_r, int maxlev) {
  return tab_b > 0 ? tab_a + tab_b
                   : (((elem_r * std_table_base(maxlev + 1) < tab_a ? elem_r * std_table_base(maxlev + 1)
                                                                     : tab_a) + 15) & ~15);
}
// Pack sets: FP64 with the kinetic matrices on the grid (all terms); FP64
// with the separable part split off (all terms); the mixed path's FP64 terms;
// its FP32 terms.
constexpr int kPackSets = 4;
enum PackSetId { kSetGrid64 = 0, kSetSplit64 = 1, kSetMixed64 = 2, kSetMixed32 = 3 };
// Rows of the inverse mapping longer than this are reduced by a whole
// wavefront, shorter ones by a group of 8 lanes.
constexpr int kLongRow = 64;
// A long row is summed by one workgroup of kRowWaves wavefronts: wavefront w
// takes the w-th of kRowWaves consecutive runs of the row's entries (runs of
// at least kRowRun entries), and the run sums are added in wavefront order
// through LDS.  Long rows come first in the reduce order, so the longest
// (the ground function takes one contribution from every term) start first.
constexpr int kRowWaves = 4;
constexpr int kRowRun = 256;
constexpr int kShortLanes = 8;
// One reduce work item = one wavefront: a long row, or 8 short rows.
struct RedItem {
  int32_t inst;
  int32_t first;    // index into the instance's row list
  int32_t local;    // item index inside the instance (partial-sum slot)
  int32_t chunk;    // long rows: 1 << 12 | (wavefront << 24);
                    // short rows: how many of the item's rows exist (0 for padding)
  const int32_t *rows;  // the instance's row list and row bounds at `first`
  const int32_t *ptr;   // (device), so that they load without the instance record
};

// Host-side term compiler output.
struct Compiled {
  int D = 0, L = 0, nbA = 1, nbB = 1, nqA = 1, nqB = 1;
  std::vector<double> omega, c, k;   // c, k dense D*D, only i<j used
  int nmax = 0;                      // largest one-mode basis index
  std::vector<int> g;                // lowest level holding index n
  // terms, canonical order
  int64_t nterms = 0;
  std::vector<uint8_t> lev;          // [nterms*D]
  std::vector<int32_t> coeff;        // [nterms]
  std::vector<int64_t> off;          // [nterms+1] canonical term-major offsets
  // compact basis
  int64_t ncs = 0;
  std::vector<uint8_t> compact;      // [ncs*D]
  std::vector<int32_t> MB;           // [N_s]
  std::vector<int32_t> inv_ptr;      // [ncs+1] inverse CSR row pointers
  std::vector<int32_t> inv_col;      // [N_s] term-major positions, ascending
  std::vector<int32_t> red_ptr;      // [ncs+1] the inverse CSR with its rows in `rows` order
  std::vector<int32_t> red_col;      // [N_s]   (what the reduce kernel reads)
  std::vector<int32_t> mbd;          // [N_s] M^B, positions lexicographic (device order)
  std::vector<double> h0;            // [ncs] sum_i omega_i (n_i + 1/2)
  // tables
  std::vector<double> tables;
  DeviceTables tdesc;
  std::vector<TermDev> terms;        // [nterms]
  std::vector<double> pairs;         // [nterms][kMaxPairs][2]: c_pq, k_pq of active pairs
  std::vector<double> potc;          // [nterms][2][kCoefStride]: split coefficient blocks
  int64_t nfib = 0;                  // mode-0 fibers over all terms with active modes
  std::vector<float> tables32;       // the same tables in FP32 (mixed path)
  std::vector<double> tables32r;     // FP32-rounded tables held in FP64 (mixed-path
                                     // FP64 terms: same operator as the FP32 terms)
  std::vector<double> cost;          // estimated work per term
  int32_t mixed_max_fp32_coeff = 16; // mixed path: |D_l| at most this -> FP32
  // nq(l) > nb(l) at every level used: every term's rule then integrates the
  // separable harmonic part exactly, so it can be split off as the diagonal.
  bool split_exact = false;
  std::vector<int32_t> rows;         // compact rows, long rows first
  int64_t n_long_rows = 0;
  int64_t n_items = 0;               // reduce work items
  // sizes
  int64_t grid_literal = 0, grid_active = 0, max_basis = 0, max_grid = 0;
  double flops_fp64 = 0, flops_mixed = 0, bytes_apply = 0;
};

// Term compiler (sg_terms.cpp)
sg_status compile_problem(const sg_problem_desc *desc, Compiled *out,
                          std::string *err);
sg_status count_sizes(int D, int L, int nbA, int nbB, int64_t out[3]);

// One-mode tables (sg_tables.cpp)
void gauss_hermite_nodes(int n, std::vector<double> *x, std::vector<double> *wt);
// Eigenvalues (ascending) and, if evecs != nullptr, column eigenvectors of a
// small dense symmetric matrix (cyclic Jacobi rotations).
void jacobi_eigen(std::vector<double> a, int n, std::vector<double> *evals,
                  std::vector<double> *evecs);
void hermite_function_values(int nb, double x, double *b);

// Bessel J_0..J_{n-1}(x) by backward recurrence (sg_cheb.cpp)
void bessel_j_sequence(double x, int n, double *out);
int chebyshev_terms(double R, double tol);

struct Plan;

}  // namespace sg

namespace sg {
// A problem's own term packs and reduce items, kept so that plans over many
// problems (batches, the server) concatenate them instead of packing every
// term again.  Built for a fixed mixed threshold and operator form.
struct PackCache {
  bool valid = false;
  int32_t thr = -1, grid_kinetic = -1, block_grid = -1;
  std::vector<PackDev> packs[kPackSets];   // inst = 0
  std::vector<double> cost[kPackSets];
  int64_t scratch[kPackSets] = {0, 0, 0, 0};    // scratch bytes of each set
  std::vector<RedItem> items;              // inst = 0
  bool inst32 = false;
};
}  // namespace sg

// Device-resident state of a built problem.
struct sg_problem {
  sg::Compiled h;
  int device = 0;
  bool host_only = false;          // built without device tables
  // device tables
  sg::TermDev *d_terms = nullptr;
  float *d_tables32 = nullptr;
  double *d_tables32r = nullptr;
  int32_t *d_mb = nullptr;
  int32_t *d_inv_ptr = nullptr;
  int32_t *d_inv_col = nullptr;
  int32_t *d_rows = nullptr;
  double *d_tables = nullptr;
  double *d_pairs = nullptr;       // [nterms][kPairStride]
  double *d_potc = nullptr;        // [nterms][2][kCoefStride]
  double *d_abc = nullptr;         // [2][3][nfib] per-fiber potential coefficients
  double *d_h0 = nullptr;
  // work buffers
  double2 *d_tm = nullptr;         // term-major results [N_s]
  double2 *d_work = nullptr;       // 4 * N_cs: Chebyshev phi, ACC, spares
  double *d_partials = nullptr;    // [2 * n_items] reduction partials
  double *d_cheb_a = nullptr;      // [kMaxChebTerms] series coefficients
  int grid_kinetic = 0;            // 1: SG_FP64 applies the kinetic matrices on the grid
  int32_t block_grid = 0;          // > 0: terms of at least this many grid points run on a
                                   // whole workgroup even when a wavefront could hold them
  int32_t packs_per_cu = 1;        // workgroups per compute unit that wave terms spread over
  sg::PackCache pcache;            // packs for multi-problem plans
  double *d_result = nullptr;      // 8 doubles
  double *h_result = nullptr;      // pinned host mirror of d_result
  int64_t device_bytes = 0;
  sg::Plan *plan = nullptr;        // launch plan of this problem alone
  // tabulated coupling potential (sg_set_potential), or none: V_eff of every
  // term on its active grid (mode 0 fastest), term t's from d_voff[t]
  double *d_veff = nullptr;
  int64_t *d_voff = nullptr;
  // optional per-kernel timing with HIP events (sg_set_timing)
  struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs (start, stop)
    std::vector<int> kind;        // 0 sweep, 1 reduce, per pair
    int used = 0;                 // pairs recorded and not yet read
    double ms[2] = {0.0, 0.0};
    int64_t n[2] = {0, 0};
    hipStream_t stream = nullptr;
  } timing;
};

namespace sg {

constexpr int kMaxChebTerms = 4096;

// A launch plan: the instances one sweep/reduce launch covers, their packs
// and reduce items, resident on the device.
struct Plan {
  std::vector<sg_problem *> probs;
  std::vector<InstDev> inst;       // host mirror
  std::vector<PackDev> packs;
  PackSet sets[kPackSets];
  std::vector<RedItem> items;
  InstDev *d_inst = nullptr;
  PackDev *d_packs = nullptr;
  RedItem *d_items = nullptr;
  char *d_scratch = nullptr;
  int64_t scratch_bytes = 0;
  int64_t packs_capacity = 0, items_capacity = 0, inst_capacity = 0, scratch_capacity = 0;
  bool any32 = false;              // some term of some instance runs in FP32
  bool fp64_split = false;         // SG_FP64 launches use the split form
  bool any_round32 = false;        // some instance's FP64 terms use rounded tables
  bool any_tab = false;            // some instance has a tabulated potential
  // standard-map tables for levels 0..stab_L (stab_L < 0: no standard-map instance)
  int stab_L = -1;
  std::vector<double> stab64, stab32r;
  std::vector<float> stab32;
  double *d_stab64 = nullptr, *d_stab32r = nullptr;
  float *d_stab32 = nullptr;
  int64_t stab_capacity = 0;
};

// Plans (sg_plan.cpp)
sg_status plan_build(Plan *pl, const std::vector<sg_problem *> &probs, std::string *err);
sg_status plan_upload(Plan *pl, hipStream_t s);   // packs, items, scratch, descriptors
sg_status plan_upload_inst(Plan *pl, hipStream_t s);  // descriptors only
void plan_free(Plan *pl);
// Fills the static part of an instance descriptor from a problem.
void inst_from_problem(const sg_problem *p, InstDev *d);

// Kernel launchers.  `k` is the Chebyshev term being produced (1..K-1);
// apply mode ignores it.  x0o / x1o, when non-null, replace the x0 / x1
// buffers of a single-instance plan.
enum class Mode : int { Apply = 0, Cheb = 1 };
struct LaunchCtl {
  Mode mode = Mode::Apply;
  sg_precision prec = SG_FP64;
  int k = 1;
  int want_partials = 0;
  double2 *x0o = nullptr;
  double2 *x1o = nullptr;
  // Optional timing events attached to the dispatches themselves (start of
  // the first kernel of the launch, end of the last one).
  hipEvent_t ev0 = nullptr;
  hipEvent_t ev1 = nullptr;
};
// Does a launch of this precision apply the split operator (separable
// harmonic part as the exact FP64 diagonal in the reduce)?
inline bool split_form(const Plan *pl, sg_precision prec) {
  return prec == SG_MIXED || pl->fp64_split;
}
hipError_t launch_sweep(const Plan *pl, const LaunchCtl &c, hipStream_t s);
// Fills abc ([2][3][nfib]) from the term records, coefficient blocks and
// one-mode tables of one problem (device pointers).
hipError_t launch_fiber_coeffs(const TermDev *terms, int64_t nterms, const double *potc,
                               const double *tab64, const double *tab32r, double *abc,
                               int64_t nfib, hipStream_t s);
hipError_t launch_reduce(const Plan *pl, const LaunchCtl &c, hipStream_t s);
hipError_t launch_finalize(const Plan *pl, hipStream_t s);  // per-instance partials
hipError_t launch_dot(const sg_problem *p, const double2 *a, const double2 *b,
                      hipStream_t s);  // result in d_result[0..1] (re, im)
hipError_t launch_axpby(int64_t n, double2 *y, const double2 *x, double a_re,
                        double a_im, double b, hipStream_t s);  // y = a x + b y

// Vector kernels of the eigensolver (sg_blas.hip).  out[2j..2j+1] =
// sum_i conj(V_j[i]) w[i] with V_j = V + j*ld; partials holds
// 2 * dot_partials_per_vector() doubles per j.
int dot_partials_per_vector();
hipError_t launch_multi_dot(const double2 *V, int64_t ld, int m, const double2 *w, int64_t n,
                            double *partials, double *out, hipStream_t s);
hipError_t launch_multi_axpy(double2 *x, double beta, const double2 *V, int64_t ld, int m,
                             const double *c, int64_t n, hipStream_t s);  // x = beta x + V c
hipError_t launch_precondition(double2 *t, const double2 *r, const double *d, double theta,
                               int64_t n, hipStream_t s);
hipError_t launch_zero(double2 *y, int64_t n, hipStream_t s);
// Lanczos steps on the device (sg_blas.hip).  project: coef = -conj(V_j)^T w
// for j < m (m <= 64; partials as launch_multi_dot) and alpha (+)= the real
// part of the last.  norm: beta = sqrt(nrm2[0]) with scale = 1/beta, or both
// 0 when beta < thr * beta0[0] (beta0 null: when beta is 0).  multi_axpy_norm:
// x += sum_j c_j V_j, with npart (lanczos_norm_partials() doubles) holding
// block sums of |x|^2 for norm_partials, which then acts as norm.
// scale_copy: dst = scale[0] * src.
hipError_t launch_lanczos_project(const double2 *V, int64_t ld, int m, const double2 *w,
                                  int64_t n, double *partials, double *coef, double *alpha,
                                  bool accumulate, hipStream_t s);
int lanczos_norm_partials();
hipError_t launch_multi_axpy_norm(double2 *x, const double2 *V, int64_t ld, int m,
                                  const double *c, int64_t n, double *npart, hipStream_t s);
hipError_t launch_lanczos_norm_partials(const double *npart, int64_t n, double *beta,
                                        const double *beta0, double thr, double *scale,
                                        hipStream_t s);
hipError_t launch_lanczos_norm(const double *nrm2, double *beta, const double *beta0, double thr,
                               double *scale, hipStream_t s);
hipError_t launch_scale_copy(double2 *dst, const double2 *src, const double *scale, int64_t n,
                             hipStream_t s);
// Propagator vector updates (sg_blas.hip), complex coefficients:
// comb3: y = c0 x0 + c1 x1 (+ c2 x2 if x2), y may alias an x;
// scale_accumulate: t = c x, acc += t.
hipError_t launch_comb3(int64_t n, double2 *y, const double2 *x0, double2 c0, const double2 *x1,
                        double2 c1, const double2 *x2, double2 c2, hipStream_t s);
hipError_t launch_scale_accumulate(int64_t n, double2 *t, const double2 *x, double2 c,
                                   double2 *acc, hipStream_t s);
hipError_t launch_embed(const double2 *x, const int32_t *map, int64_t nx, double2 *y, int64_t ny,
                        hipStream_t s);

// Launch with optional event timing (sg_api.cpp); the drivers use these.
hipError_t run_sweep(sg_problem *timing_owner, const Plan *pl, const LaunchCtl &c,
                     hipStream_t s);
hipError_t run_reduce(sg_problem *timing_owner, const Plan *pl, const LaunchCtl &c,
                      hipStream_t s);
sg_status fail(sg_status st, const std::string &msg);
sg_status hip_fail(hipError_t e, const char *what);

// Device upload of a compiled problem (takes ownership; frees on failure),
// its device-memory estimate, and release.
sg_status upload_problem(sg_problem *p, sg_problem **out);
int64_t estimate_device_bytes(const Compiled &h);
void release_problem(sg_problem *p);

// Chebyshev series for one instance: K and coefficients for R = dE dt / 2.
int chebyshev_series(double R, std::vector<double> *a);

// Two-state (vibronic) term sweep (sg_vibronic.hip).  Coefficient block per
// term: kVibSurf doubles per state (constant, Q_p^2, Q_p, pair Q_p^2 Q_q^2
// coefficients of the active modes) and the interstate Q_p coefficients.
constexpr int kVibSurf = 17 + kMaxPairs;   // 45
constexpr int kVibCoef = 104;              // 2 kVibSurf + kMaxActive, padded
static_assert(2 * kVibSurf + kMaxActive <= kVibCoef, "vibronic coefficient block");
// Launch shapes of the term sweeps that run one term per workgroup (the
// two-state operator): threads per term, the largest
// term grid and the highest active level a shape's kernel takes.  With the
// standard maps and L <= 6 every term fits one of them (grids above 1024
// points have levels <= 2, above 256 levels <= 3).  Every shape is one
// dispatch, and a dispatch of small terms lasts about one term's chain of
// dependent steps, so the small terms share one shape.
struct GroupShape {
  int vt, max_grid, max_level;
};
constexpr int kGroupShapes = 3;
constexpr GroupShape kGroupShape[kGroupShapes] = {{512, 4096, 2}, {256, 1024, 3}, {64, 256, 6}};
struct TermGroup {
  int32_t first = 0, count = 0;   // range of the term order launched together
  int32_t max_grid = 0;           // largest grid of the group (sizes its LDS)
  int32_t shape = 0;              // index into kGroupShape
};
// Orders the terms of a compiled problem for such sweeps: each term goes to
// the smallest shape that takes its grid and highest level, groups in shape
// order, largest grids first within a group.  False if a term fits no shape.
bool group_terms(const Compiled &h, std::vector<int32_t> *order, std::vector<TermGroup> *groups);
struct VibLaunch {
  const TermDev *terms = nullptr;
  const int32_t *mb = nullptr;
  const double *tab = nullptr;    // standard-map tables, levels 0..L
  const double *coef = nullptr;   // [nterms][kVibCoef]
  const int32_t *order = nullptr; // device: terms, largest grid first
  std::vector<TermGroup> groups;
  int64_t ncs = 0, ns = 0;
  int tab_elems = 0;
};
// vin: [2 N_cs] state-major; tm: [2 N_s].  ev0 / ev1 (nullable) attach to the
// first / last dispatch.
hipError_t launch_vib_sweep(const VibLaunch &v, const double2 *vin, double2 *tm, hipStream_t s,
                            hipEvent_t ev0, hipEvent_t ev1);
// the same, timed as a sweep by owner's events when its timing is on
hipError_t run_vib_sweep(sg_problem *owner, const VibLaunch &v, const double2 *vin, double2 *tm,
                         hipStream_t s);

// Rebuilds and re-uploads a problem's own launch plan after one of its
// settings changed (the device is synchronised first).
sg_status problem_replan(sg_problem *p);

// Work buffers of one sg_propagate call (sg_step.cpp): allocated for the call
// (owned), or carved out of a region the caller provides (not owned).
struct PropBuffers {
  double2 *v = nullptr;        // vectors, n each
  double *partials = nullptr;  // multi-dot partial sums
  double *coef = nullptr;      // multi-axpy coefficients (re, im)
  double *lz = nullptr;        // Lanczos scalars on the device
  double *npart = nullptr;     // block sums of |w|^2
  bool owned = true;
  ~PropBuffers();
};
// Argument checks and work sizes (m: Krylov dimension used; nvec: work
// vectors besides the check vector).
sg_status propagate_check(sg_problem *p, void *psi, double dt, int32_t nsteps, int32_t method,
                          int32_t order, sg_precision prec, int32_t check_every, int *m,
                          int *nvec);
// Byte offsets (256-byte aligned) of v, partials, coef, lz, npart in one
// region; returns the region's size.
int64_t propagate_layout(int64_t n, int32_t method, int32_t order, int m, int nvec,
                         int64_t off[5]);
// The propagation on prepared buffers; zero_kernel clears the work vectors
// with a fill kernel instead of hipMemsetAsync.
sg_status propagate_run(sg_problem *p, void *psi, double dt, int32_t nsteps, int32_t method,
                        int32_t order, int m, int nvec, double tol, sg_precision prec,
                        int32_t check_every, sg_prop_stats *stats, double *norm_trace,
                        double *energy_trace, void *stream, PropBuffers &B, bool zero_kernel);
}  // namespace sg
