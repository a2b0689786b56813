// Internal definitions shared by the host term compiler, the drivers and the
// HIP kernels of the Smolyak library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

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

struct alignas(16) TermDev {
  int32_t off;       // start of the term in the term-major layout (N_s)
  int32_t nbasis;    // prod over active modes of nb
  int32_t ngrid;     // prod over active modes of nq
  int32_t na;        // number of active modes
  int8_t lev[kMaxActive];   // levels of the active modes, increasing mode id
  int8_t mode[kMaxActive];  // their mode ids
  int32_t nb[kMaxActive];   // per active mode: basis size
  int32_t nq[kMaxActive];   //   grid size
  int32_t bt[kMaxActive];   //   offsets of its level's tables in the table array
  int32_t wt[kMaxActive];
  int32_t kg[kMaxActive];
  int32_t xo[kMaxActive];
  float rcp_nq[kMaxActive]; //   1/nq for fast index division
  double coeff;             // D_l
  double c0_full;           // constant part of the effective potential, FP64 path
  double c0_split;          // ... without the harmonic part (mixed path)
  double alpha_full[kMaxActive];   // coefficient of Q_p^2, FP64 path
  double alpha_split[kMaxActive];  // ... without 1/2 omega_p (mixed path)
  double beta[kMaxActive];         // coefficient of Q_p
  double kin[kMaxActive];          // -1/2 omega_p (kinetic prefactor)
};

// Offsets of the one-mode tables of a level inside the packed table array.
struct LevelDev {
  int32_t nb, nq;
  int32_t bt;   // b(Q_u)            [nq][nb]   basis -> grid
  int32_t wt;   // wt_u b(Q_u)^T     [nb][nq]   grid -> basis
  int32_t kg;   // d2b (wt b)^T      [nq][nq]   second derivative on the grid
  int32_t x;    // nodes             [nq]
};

constexpr int kMaxLevels = 16;

// Term-sweep packing.  A workgroup (512 threads) runs one pack: one term with
// more than kWaveMaxGrid grid points on all its wavefronts, or up to
// kPackTerms smaller terms, one per wavefront.
constexpr int kPackTerms = 8;
constexpr int kWaveMaxGrid = 512;
constexpr int kLdsPerCU = 160 * 1024;
constexpr int kComputeUnits = 256;   // MI355X; used to size the packing only
struct PackDev {
  int32_t n;                  // terms in the pack
  int32_t block;              // 1: term[0] runs on the whole workgroup
  int32_t term[kPackTerms];
  int32_t lds_off[kPackTerms];  // byte offset of each wavefront's LDS slice
};
struct PackSet {
  int32_t first = 0;          // index of the first pack
  int32_t count = 0;
  int32_t lds_bytes = 0;      // dynamic LDS of the launch
};
// Pack sets: FP64 path (all terms), mixed path FP64 terms, mixed path FP32 terms.
constexpr int kPackSets = 3;
// Rows of the inverse mapping longer than this are reduced by a whole
// wavefront, shorter ones by a group of 8 lanes.
constexpr int kLongRow = 64;

struct DeviceTables {
  LevelDev lev[kMaxLevels];
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
  std::vector<double> h0;            // [ncs] sum_i omega_i (n_i + 1/2)
  // tables
  std::vector<double> tables;
  DeviceTables tdesc;
  std::vector<TermDev> terms;        // [nterms]
  std::vector<double> pairs;         // [nterms][kMaxPairs][2]: c_pq, k_pq of active pairs
  std::vector<float> tables32;       // the same tables in FP32 (mixed path)
  std::vector<double> tables32r;     // FP32-rounded tables held in FP64 (mixed-path
                                     // FP64 terms: same operator as the FP32 terms)
  std::vector<double> cost;          // estimated work per term
  std::vector<PackDev> packs;        // all pack sets, concatenated
  PackSet sets[kPackSets];
  int32_t mixed_max_fp32_coeff = 16; // mixed path: |D_l| at most this -> FP32
  std::vector<int32_t> rows;         // compact rows, long rows first
  int64_t n_long_rows = 0;
  // sizes
  int64_t grid_literal = 0, grid_active = 0, max_basis = 0, max_grid = 0;
  double flops_fp64 = 0, flops_mixed = 0, bytes_apply = 0;
};

// Term compiler (sg_terms.cpp)
sg_status compile_problem(const sg_problem_desc *desc, Compiled *out,
                          std::string *err);
sg_status count_sizes(int D, int L, int nbA, int nbB, int64_t out[3]);
// (Re)builds the three pack sets from the term records and the mixed-path
// coefficient threshold.
sg_status build_pack_sets(Compiled *h, std::string *err);

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

}  // namespace sg

// Device-resident state of a built problem.
struct sg_problem {
  sg::Compiled h;
  int device = 0;
  bool host_only = false;          // built without device tables
  // device tables
  sg::TermDev *d_terms = nullptr;
  sg::PackDev *d_packs = nullptr;
  int64_t d_packs_capacity = 0;
  float *d_tables32 = nullptr;
  double *d_tables32r = nullptr;
  int32_t *d_mb = nullptr;
  int32_t *d_inv_ptr = nullptr;
  int32_t *d_inv_col = nullptr;
  int32_t *d_rows = nullptr;
  double *d_tables = nullptr;
  sg::LevelDev *d_lvt = nullptr;   // [kMaxLevels]
  double *d_pairs = nullptr;       // [nterms][kMaxPairs][2]
  double *d_h0 = nullptr;
  double *d_c = nullptr;           // [D*D]
  double *d_k = nullptr;           // [D*D]
  // work buffers
  double2 *d_tm = nullptr;         // term-major results [N_s]
  double2 *d_work = nullptr;       // 3 * N_cs: Chebyshev P, ACC, spare
  double *d_partials = nullptr;    // reduction partials
  double *d_result = nullptr;      // 4 doubles
  double *h_result = nullptr;      // pinned host mirror of d_result
  int64_t device_bytes = 0;
  int n_partials = 0;
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
// Kernel launchers (sg_kernels.hip)
enum class Epi : int { Apply = 0, Cheb = 1 };

struct ChebArgs {
  const double2 *psi_in;   // the vector H was applied to (phi_k)
  double2 *prev;           // phi_{k-1} on input, phi_{k+1} on output
  double2 *acc;            // running sum
  double2 *final_out;      // ChebLast: exp(-i Ebar dt) * acc
  double ebar, inv_half;   // Ebar and 2 / dE
  double a_k;              // coefficient of the produced phi
  double a_0;              // ChebFirst: coefficient of phi_0
  double phase_re, phase_im;
  int split;               // add the exact FP64 diagonal part
  int want_partials;       // first: norm/energy partials
  int first;               // produce phi_1 from phi_0
  int last;                // write exp(-i Ebar dt) * acc instead of phi, acc
};

hipError_t launch_sweep(const sg_problem *p, const double2 *psi, sg_precision prec,
                        hipStream_t s);
hipError_t launch_reduce(const sg_problem *p, Epi epi, const double2 *psi_in,
                         double2 *out, const ChebArgs *ca, hipStream_t s);
hipError_t launch_finalize_partials(const sg_problem *p, hipStream_t s);
hipError_t launch_init_vector(const sg_problem *p, const double *coef_dev,
                              double2 *psi, hipStream_t s);
hipError_t launch_dot(const sg_problem *p, const double2 *a, const double2 *b,
                      hipStream_t s);  // result in d_result[0..1] (re, im)
hipError_t launch_axpby(int64_t n, double2 *y, const double2 *x, double a_re,
                        double a_im, double b, hipStream_t s);  // y = a x + b y
int64_t reduce_blocks(const sg_problem *p);

// Launch with optional event timing (sg_api.cpp); the drivers use these.
hipError_t run_sweep(sg_problem *p, const double2 *psi, sg_precision prec, hipStream_t s);
hipError_t run_reduce(sg_problem *p, Epi epi, const double2 *psi_in, double2 *out,
                      const ChebArgs *ca, hipStream_t s);
sg_status fail(sg_status st, const std::string &msg);
sg_status hip_fail(hipError_t e, const char *what);
}  // namespace sg
