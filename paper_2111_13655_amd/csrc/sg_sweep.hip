// Term sweep of the Smolyak operator action (Alg. 1, Sec. 3) for gfx950.
//
// One launch covers every term.  A workgroup of 512 threads runs a "pack":
// either one large term processed by all eight wavefronts, or up to eight
// small terms processed one per wavefront with wave-level synchronisation.
// The host packs terms by LDS need and estimated cost (longest first), so a
// single dispatch fills the chip without charging small terms the LDS of the
// largest one.  For one term:
//   1. gather through M^B fused with the basis -> grid contraction of the
//      first active mode (each thread loads whole fibers straight from HBM);
//   2. basis -> grid along the remaining active modes (eq_transfer_b_to_g),
//      ping-ponging between two LDS buffers;
//   3. the operator on the grid: the effective potential (closed form, per
//      fiber) fused with the kinetic second-derivative matrix of the first
//      mode, then the kinetic matrices of the other modes accumulated (the
//      mixed path carries no harmonic part and no kinetic term here: that part
//      is diagonal and is added exactly in the reduce);
//   4. grid -> basis (eq_transfer_g_to_b); the last mode's contraction writes
//      D_l times the result, in FP64, straight to the term-major buffer.
// Every contraction gives one thread a whole fiber along the contracted mode:
// the fiber sits in registers and the one-mode matrix is wave-uniform, so its
// entries arrive through scalar loads.  Per-term data sit at constant offsets
// of the term record, so a wave issues independent scalar loads.
// The arithmetic type R is double (FP64 path, and the high-|D_l| terms of the
// mixed path) or float (the other terms of the mixed path).
#include <hip/hip_ext.h>

#include "sg_internal.h"

namespace sg {

namespace {

constexpr int kThreads = kSweepThreads;

// Address-space-qualified pointers.  Grid buffers live in LDS (or, for terms
// too large for LDS, in global scratch); HBM data are global; per-term
// records, coefficient blocks and one-mode matrices are wave-uniform and are
// read through the constant address space, i.e. with scalar loads.
template <typename T> using lds_p = __attribute__((address_space(3))) T *;
template <typename T> using glb_p = __attribute__((address_space(1))) T *;
template <typename T> using cptr = const __attribute__((address_space(4))) T *;

// Plain complex values (trivially copyable across address spaces; the
// layout of double2 / float2).
struct alignas(16) Z64 { double x, y; };
struct alignas(8) Z32 { float x, y; };
// What one term's computation reads and writes.
struct TermCtx {
  glb_p<const int32_t> mb;
  glb_p<const int32_t> mbt;  // the term's first M^B entry (from the pack)
  glb_p<const Z64> psi;      // the vector H is applied to
  glb_p<Z64> tm;             // term-major contributions
  const void *tab;           // one-mode tables in the arithmetic type
  cptr<double> pc;           // the term's pair coefficients (variant chosen)
  int std_maps;              // nb = 1 + 2l, nq = 2 + 2l
  int split;                 // operator without the separable harmonic part
  int pot;                   // kPotFull / kPotSplit / kPotSplitRounded
  int lt_off;                // byte offset of this term's tables in LDS
  glb_p<const double> pcoef; // the term's split coefficient block (variant chosen)
  glb_p<const double> abc;   // per-fiber A, B, C (variant chosen; FP64 terms)
  const void *gtab;          // the standard-map tables in HBM (variant chosen)
  int64_t nfib;              // stride between the A, B and C arrays
  glb_p<const double> vt;    // tabulated potential: the term's V_eff (null: polynomial)
};

struct SweepArgs {
  cptr<InstDev> inst;
  cptr<PackDev> packs;
  char *scratch;
  double2 *x0o, *x1o;    // single-instance buffer overrides (nullable)
  int mode;              // 0 apply, 1 Chebyshev
  int k;                 // Chebyshev term being produced
  int split;             // split operator (no kinetic or harmonic part on the grids)
  int mixed;             // SG_MIXED launch (instances with FP32 terms use rounded tables)
  const void *stab;      // standard-map tables (launch precision) copied to LDS at 0
  const void *stab_r;    // FP32-rounded FP64 tables, copied after them (or null)
  int tab_a, tab_b;      // their LDS bytes (multiples of 16)
};

// Element access through address-space-qualified pointers (member-wise: the
// implicit copy of a struct binds a generic reference).
template <typename C, typename P>
__device__ __forceinline__ C ldc(P p) {
  C v;
  v.x = p->x;
  v.y = p->y;
  return v;
}
template <typename P, typename C>
__device__ __forceinline__ void stc(P p, const C &v) {
  p->x = v.x;
  p->y = v.y;
}

// Where a term's outputs go: entry i of the term lands at tm[i].
struct Out {
  glb_p<Z64> tm;
};

template <typename R> struct Cx;
template <> struct Cx<double> {
  typedef Z64 T;
  static __device__ __forceinline__ Z64 make(double a, double b) { return Z64{a, b}; }
};
template <> struct Cx<float> {
  typedef Z32 T;
  static __device__ __forceinline__ Z32 make(float a, float b) { return Z32{a, b}; }
};

// Threads of one term: a single wavefront, or the whole workgroup.
struct WaveGroup {
  static constexpr int N = 64;
  static __device__ __forceinline__ int tid() { return threadIdx.x & 63; }
  static __device__ __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};
struct BlockGroup {
  static constexpr int N = kThreads;
  static __device__ __forceinline__ int tid() { return threadIdx.x; }
  static __device__ __forceinline__ void sync() { __syncthreads(); }
};

// floor(f / d) for 0 <= f, d < 2^20 via a float reciprocal (exact in this
// range: f + 0.5 is at least 0.5 away from any multiple of d).
__device__ __forceinline__ int fdiv(int f, float rcp) {
  return __float2int_rz(((float)f + 0.5f) * rcp);
}
// a * b for 0 <= a, b < 2^24 (full-rate 24-bit multiply)
__device__ __forceinline__ int mul24(int a, int b) {
  return (int)__umul24((unsigned)a, (unsigned)b);
}

// A wave-uniform pointer re-derived inside a divergent loop.  readfirstlane
// is convergent, so it and the scalar loads through the pointer stay in the
// loop body; hoisting every matrix entry or coefficient out of the fiber loop
// would exhaust the scalar registers and spill.
template <typename T>
__device__ __forceinline__ cptr<T> in_loop_uniform(const T *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (cptr<T>)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ cptr<T> in_loop_uniform(cptr<T> p) {
  return in_loop_uniform((const T *)p);
}

// Compile-time size when N_ > 0, run-time size n otherwise (loops are then
// unrolled to kMaxN with guards so that fibers stay in registers).
#define SG_CN(N_) ((N_) > 0 ? (N_) : kMaxN)
#define SG_IN(N_, k, n) ((N_) > 0 || (k) < (n))

// ---------------------------------------------------------------------------
// One-mode contraction over fibers.  Layout: out[lo + stride*(u + NO*hi)]
// (+)= scale * sum_k M[u*NI + k] in[lo + stride*(k + NI*hi)].
// P is the buffer pointer type (LDS or global scratch).
// ---------------------------------------------------------------------------
template <typename G, typename R, typename P, int NI_, int NO_, bool ACC>
__device__ __forceinline__ void contract(P in, P out, const R *M, R scale, int ni, int no,
                                         int stride, int nouter) {
  typedef typename Cx<R>::T C;
  const int NI = NI_ > 0 ? NI_ : ni;
  const int NO = NO_ > 0 ? NO_ : no;
  const int F = stride * nouter;
  const float rcp = 1.0f / (float)stride;
  for (int f = G::tid(); f < F; f += G::N) {
    const int hi = fdiv(f, rcp);
    const int lo = f - hi * stride;
    P src = in + lo + hi * (stride * NI);
    P dst = out + lo + hi * (stride * NO);
    const cptr<R> Mw = in_loop_uniform(M);
    C x[SG_CN(NI_)];
#pragma unroll
    for (int k = 0; k < SG_CN(NI_); ++k) x[k] = SG_IN(NI_, k, NI) ? ldc<C>(src + k * stride) : Cx<R>::make(0, 0);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      R re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < SG_CN(NI_); ++k) {
        if (SG_IN(NI_, k, NI)) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[k].x, re);
          im = fma(m, x[k].y, im);
        }
      }
      if (ACC) {
        C o = ldc<C>(dst + u * stride);
        o.x = fma(scale, re, o.x);
        o.y = fma(scale, im, o.y);
        stc(dst + u * stride, o);
      } else {
        stc(dst + u * stride, Cx<R>::make(re, im));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-size contractions (standard size maps), processed in rounds: in one
// round a thread takes FPT fibers (f = f0 + tid + j*N), issues all their
// loads together, then forms each output row for all FPT fibers from one
// row of the one-mode matrix.  Outputs are the same FMA chains, in the same
// order, as one fiber at a time.
// ---------------------------------------------------------------------------
template <int NI>
struct Fpt {
  static constexpr int value = NI <= 4 ? 4 : NI == 5 ? 3 : NI <= 8 ? 2 : 1;
};

template <typename G, typename R, typename P, int NI, int NO, bool ACC>
__device__ __forceinline__ void contract_fixed(P in, P out, const R *M, R scale, int stride,
                                               int nouter) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = Fpt<NI>::value;
  const int F = stride * nouter;
  const float rcp = 1.0f / (float)stride;
  const int sNI = stride * NI, sNO = stride * NO;
  for (int f0 = 0; f0 < F; f0 += FPT * G::N) {
    int ib[FPT], ob[FPT];
    bool ok[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      int f = f0 + G::tid() + j * G::N;
      ok[j] = f < F;
      f = ok[j] ? f : 0;
      const int hi = fdiv(f, rcp);
      const int lo = f - hi * stride;
      ib[j] = lo + hi * sNI;
      ob[j] = lo + hi * sNO;
    }
    C x[FPT][NI];
#pragma unroll
    for (int j = 0; j < FPT; ++j)
#pragma unroll
      for (int k = 0; k < NI; ++k) x[j][k] = ldc<C>(in + ib[j] + k * stride);
    const cptr<R> Mw = in_loop_uniform(M);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        R re = 0, im = 0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[j][k].x, re);
          im = fma(m, x[j][k].y, im);
        }
        if (ok[j]) {
          P d = out + ob[j] + u * stride;
          if (ACC) {
            C o = ldc<C>(d);
            o.x = fma(scale, re, o.x);
            o.y = fma(scale, im, o.y);
            stc(d, o);
          } else {
            stc(d, Cx<R>::make(re, im));
          }
        }
      }
    }
  }
}

template <typename G, typename R, typename P, int NI, int NO>
__device__ __forceinline__ void gather_fixed(const TermCtx &a, int off, int nfib, const R *M,
                                             P out) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = Fpt<NI>::value;
  for (int f0 = 0; f0 < nfib; f0 += FPT * G::N) {
    int idx[FPT][NI];
    bool ok[FPT];
    int fb[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + G::tid() + j * G::N;
      ok[j] = f < nfib;
      fb[j] = ok[j] ? f : 0;
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j)
#pragma unroll
      for (int k = 0; k < NI; ++k) idx[j][k] = a.mb[off + fb[j] * NI + k];
    C x[FPT][NI];
#pragma unroll
    for (int j = 0; j < FPT; ++j)
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const Z64 v = ldc<Z64>(a.psi + idx[j][k]);
        x[j][k] = Cx<R>::make((R)v.x, (R)v.y);
      }
    const cptr<R> Mw = in_loop_uniform(M);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        R re = 0, im = 0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[j][k].x, re);
          im = fma(m, x[j][k].y, im);
        }
        if (ok[j]) stc(out + fb[j] * NO + u, Cx<R>::make(re, im));
      }
    }
  }
}

template <typename G, typename R, typename P, int NI, int NO>
__device__ __forceinline__ void g2b_fixed(P in, Out o, const R *M, double cf,
                                          int stride) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = Fpt<NI>::value;
  for (int f0 = 0; f0 < stride; f0 += FPT * G::N) {
    bool ok[FPT];
    int lo[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + G::tid() + j * G::N;
      ok[j] = f < stride;
      lo[j] = ok[j] ? f : 0;
    }
    C x[FPT][NI];
#pragma unroll
    for (int j = 0; j < FPT; ++j)
#pragma unroll
      for (int k = 0; k < NI; ++k) x[j][k] = ldc<C>(in + lo[j] + k * stride);
    const cptr<R> Mw = in_loop_uniform(M);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        R re = 0, im = 0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[j][k].x, re);
          im = fma(m, x[j][k].y, im);
        }
        if (ok[j]) stc(o.tm + lo[j] + u * stride, Z64{cf * (double)re, cf * (double)im});
      }
    }
  }
}

// kind 0: basis -> grid (NI = nb, NO = nq); 1: kinetic on the grid
// (NI = NO = nq); 2: grid -> basis (NI = nq, NO = nb)
template <typename G, typename R, typename P, bool ACC>
__device__ __forceinline__ void contract_level(int kind, int level, int std_maps, int nb, int nq,
                                               P in, P out, const R *M, R scale, int stride,
                                               int nouter) {
  if (std_maps) {
#define SG_CASE(L_, NB_, NQ_)                                                                       \
  case L_:                                                                                          \
    if (kind == 0) contract_fixed<G, R, P, NB_, NQ_, ACC>(in, out, M, scale, stride, nouter);      \
    else if (kind == 1) contract_fixed<G, R, P, NQ_, NQ_, ACC>(in, out, M, scale, stride, nouter); \
    else contract_fixed<G, R, P, NQ_, NB_, ACC>(in, out, M, scale, stride, nouter);                \
    return;
    switch (level) {
      SG_CASE(1, 3, 4)
      SG_CASE(2, 5, 6)
      SG_CASE(3, 7, 8)
      SG_CASE(4, 9, 10)
      SG_CASE(5, 11, 12)
      SG_CASE(6, 13, 14)
      SG_CASE(7, 15, 16)
      default: break;
    }
#undef SG_CASE
  }
  const int NI = kind == 0 ? nb : nq;
  const int NO = kind == 2 ? nb : nq;
  contract<G, R, P, 0, 0, ACC>(in, out, M, scale, NI, NO, stride, nouter);
}

// ---------------------------------------------------------------------------
// Step 1 fused with the first basis -> grid contraction: fibers along mode 0
// are contiguous runs of the term-major layout, so each thread gathers its
// fiber through M^B and writes the nq transformed values to the buffer.
// ---------------------------------------------------------------------------
template <typename G, typename R, typename P, int NI_, int NO_>
__device__ __forceinline__ void gather_b2g_impl(const TermCtx &a, int off, int nfib, int ni,
                                                int no, const R *M, P out) {
  typedef typename Cx<R>::T C;
  const int NI = NI_ > 0 ? NI_ : ni;
  const int NO = NO_ > 0 ? NO_ : no;
  for (int f = G::tid(); f < nfib; f += G::N) {
    glb_p<const int32_t> mb = a.mb + off + f * NI;
    const cptr<R> Mw = in_loop_uniform(M);
    C x[SG_CN(NI_)];
#pragma unroll
    for (int k = 0; k < SG_CN(NI_); ++k) {
      if (SG_IN(NI_, k, NI)) {
        const Z64 v = ldc<Z64>(a.psi + mb[k]);
        x[k] = Cx<R>::make((R)v.x, (R)v.y);
      } else {
        x[k] = Cx<R>::make(0, 0);
      }
    }
    P dst = out + f * NO;
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      R re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < SG_CN(NI_); ++k) {
        if (SG_IN(NI_, k, NI)) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[k].x, re);
          im = fma(m, x[k].y, im);
        }
      }
      stc(dst + u, Cx<R>::make(re, im));
    }
  }
}

template <typename G, typename R, typename P>
__device__ __forceinline__ void gather_b2g(const TermCtx &a, int level, int nb, int nq, int off,
                                           int nfib, const R *M, P out) {
  if (a.std_maps) {
    switch (level) {
      case 1: gather_fixed<G, R, P, 3, 4>(a, off, nfib, M, out); return;
      case 2: gather_fixed<G, R, P, 5, 6>(a, off, nfib, M, out); return;
      case 3: gather_fixed<G, R, P, 7, 8>(a, off, nfib, M, out); return;
      case 4: gather_fixed<G, R, P, 9, 10>(a, off, nfib, M, out); return;
      case 5: gather_fixed<G, R, P, 11, 12>(a, off, nfib, M, out); return;
      case 6: gather_fixed<G, R, P, 13, 14>(a, off, nfib, M, out); return;
      case 7: gather_fixed<G, R, P, 15, 16>(a, off, nfib, M, out); return;
      default: break;
    }
  }
  gather_b2g_impl<G, R, P, 0, 0>(a, off, nfib, nb, nq, M, out);
}

// ---------------------------------------------------------------------------
// Step 4's last contraction: grid -> basis along the slowest active mode
// (nouter = 1), written as D_l * result in FP64 to the term-major buffer.
// ---------------------------------------------------------------------------
template <typename G, typename R, typename P, int NI_, int NO_>
__device__ __forceinline__ void g2b_store_impl(P in, Out o, const R *M, double cf,
                                               int ni, int no, int stride) {
  typedef typename Cx<R>::T C;
  const int NI = NI_ > 0 ? NI_ : ni;
  const int NO = NO_ > 0 ? NO_ : no;
  for (int lo = G::tid(); lo < stride; lo += G::N) {
    const cptr<R> Mw = in_loop_uniform(M);
    C x[SG_CN(NI_)];
#pragma unroll
    for (int k = 0; k < SG_CN(NI_); ++k)
      x[k] = SG_IN(NI_, k, NI) ? ldc<C>(in + lo + k * stride) : Cx<R>::make(0, 0);
#pragma unroll 1
    for (int u = 0; u < NO; ++u) {
      R re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < SG_CN(NI_); ++k) {
        if (SG_IN(NI_, k, NI)) {
          const R m = Mw[u * NI + k];
          re = fma(m, x[k].x, re);
          im = fma(m, x[k].y, im);
        }
      }
      stc(o.tm + lo + u * stride, Z64{cf * (double)re, cf * (double)im});
    }
  }
}

template <typename G, typename R, typename P>
__device__ __forceinline__ void g2b_store(int std_maps, int level, int nb, int nq, P in,
                                          Out o, const R *M, double cf, int stride) {
  if (std_maps) {
    switch (level) {
      case 1: g2b_fixed<G, R, P, 4, 3>(in, o, M, cf, stride); return;
      case 2: g2b_fixed<G, R, P, 6, 5>(in, o, M, cf, stride); return;
      case 3: g2b_fixed<G, R, P, 8, 7>(in, o, M, cf, stride); return;
      case 4: g2b_fixed<G, R, P, 10, 9>(in, o, M, cf, stride); return;
      case 5: g2b_fixed<G, R, P, 12, 11>(in, o, M, cf, stride); return;
      case 6: g2b_fixed<G, R, P, 14, 13>(in, o, M, cf, stride); return;
      case 7: g2b_fixed<G, R, P, 16, 15>(in, o, M, cf, stride); return;
      default: break;
    }
  }
  g2b_store_impl<G, R, P, 0, 0>(in, o, M, cf, nq, nb, stride);
}

// ---------------------------------------------------------------------------
// Step 3, first part: dst = V_eff * src (+ kin_0 K_0 x_0 src on the FP64
// path) over fibers along mode 0.  Along one fiber only Q_0 varies, so the
// potential is A + B Q_0^2 + C Q_0 with A, B, C computed once per fiber from
// V_eff = c0 + sum_p (alpha_p Q_p^2 + beta_p Q_p)
//       + sum_{p<q} (c_pq Q_p^2 Q_q^2 + k_pq Q_p^2 Q_q).
// The coefficients are read with scalar loads from the term record and the
// term's pair block, in the variant the context selects.
// ---------------------------------------------------------------------------
template <typename G, typename R, typename P, int NQ_, bool KIN>
__device__ __forceinline__ void potential_impl(const TermCtx &a, cptr<TermDev> T, P src, P dst,
                                               int nfib) {
  typedef typename Cx<R>::T C;
  const R *tab = (const R *)a.tab;
  const glb_p<const R> tg = (glb_p<const R>)tab;   // per-lane node reads
  const int na = T->na;
  const int NQ = NQ_ > 0 ? NQ_ : T->nq[0];
  const R *x0 = tab + T->xo[0];
  const R *K0 = tab + T->kg[0];
  const R kin0 = (R)T->kin[0];
  const int pot = a.pot;
  const int bv = pot == kPotSplitRounded ? 1 : 0;
  const R c0 = (R)T->c0[pot];
  const R al0 = (R)T->alpha[pot][0];
  const R be0 = (R)T->beta[bv][0];
  for (int f = G::tid(); f < nfib; f += G::N) {
    R xq[kMaxActive];
    int rem = f;
#pragma unroll
    for (int q = 1; q < kMaxActive; ++q) {
      xq[q] = 0;
      if (q < na) {
        const int hi = fdiv(rem, T->rcp_nq[q]);
        const int u = rem - hi * T->nq[q];
        rem = hi;
        xq[q] = tg[T->xo[q] + u];
      }
    }
    const cptr<double> al = in_loop_uniform(&T->alpha[pot][0]);
    const cptr<double> be = in_loop_uniform(&T->beta[bv][0]);
    const cptr<double> pc = in_loop_uniform(a.pc);
    R A = c0, B = al0, Cc = be0;
#pragma unroll
    for (int q = 1; q < kMaxActive; ++q) {
      if (q < na) {
        const R x2 = xq[q] * xq[q];
        A = fma((R)al[q], x2, A);
        A = fma((R)be[q], xq[q], A);
        B = fma((R)pc[2 * pair_index(0, q)], x2, B);
        Cc = fma((R)pc[2 * pair_index(0, q) + 1], x2, Cc);
#pragma unroll
        for (int r = q + 1; r < kMaxActive; ++r) {
          if (r < na) {
            const R y2 = xq[r] * xq[r];
            A = fma((R)pc[2 * pair_index(q, r)] * x2, y2, A);
            A = fma((R)pc[2 * pair_index(q, r) + 1] * y2, xq[q], A);
          }
        }
      }
    }
    P s = src + f * NQ;
    P d = dst + f * NQ;
    const cptr<R> Kw = in_loop_uniform(K0);
    const cptr<R> xw = in_loop_uniform(x0);
    C x[SG_CN(NQ_)];
    if (KIN) {
#pragma unroll
      for (int u = 0; u < SG_CN(NQ_); ++u) x[u] = SG_IN(NQ_, u, NQ) ? ldc<C>(s + u) : Cx<R>::make(0, 0);
    }
#pragma unroll 1
    for (int u = 0; u < NQ; ++u) {
      const R xv = xw[u];
      const R V = fma(fma(B, xv, Cc), xv, A);
      const C xu = ldc<C>(s + u);
      R re = V * xu.x, im = V * xu.y;
      if (KIN) {
        R kr = 0, ki = 0;
#pragma unroll
        for (int k = 0; k < SG_CN(NQ_); ++k) {
          if (SG_IN(NQ_, k, NQ)) {
            const R m = Kw[u * NQ + k];
            kr = fma(m, x[k].x, kr);
            ki = fma(m, x[k].y, ki);
          }
        }
        re = fma(kin0, kr, re);
        im = fma(kin0, ki, im);
      }
      stc(d + u, Cx<R>::make(re, im));
    }
  }
}

// Fixed-size potential step (standard maps), in rounds of FPT fibers: each
// coefficient read with a scalar load updates all FPT fibers of the round.
template <typename G, typename R, typename P, int NQ, bool KIN>
__device__ __forceinline__ void potential_fixed(const TermCtx &a, cptr<TermDev> T, P src, P dst,
                                                int nfib) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = NQ <= 8 ? 2 : 1;
  const R *tab = (const R *)a.tab;
  const glb_p<const R> tg = (glb_p<const R>)tab;   // per-lane node reads
  const int na = T->na;
  const R *x0 = tab + T->xo[0];
  const R *K0 = tab + T->kg[0];
  const R kin0 = (R)T->kin[0];
  const int pot = a.pot;
  const int bv = pot == kPotSplitRounded ? 1 : 0;
  const R c0 = (R)T->c0[pot];
  const R al0 = (R)T->alpha[pot][0];
  const R be0 = (R)T->beta[bv][0];
  for (int f0 = 0; f0 < nfib; f0 += FPT * G::N) {
    bool ok[FPT];
    int fb[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + G::tid() + j * G::N;
      ok[j] = f < nfib;
      fb[j] = ok[j] ? f : 0;
    }
    // the fibers (held only for the fused kinetic contraction)
    C x[FPT][KIN ? NQ : 1];
    if (KIN) {
#pragma unroll
      for (int j = 0; j < FPT; ++j)
#pragma unroll
        for (int u = 0; u < NQ; ++u) x[j][u] = ldc<C>(src + fb[j] * NQ + u);
    }
    R xq[FPT][kMaxActive];
    int rem[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) rem[j] = fb[j];
#pragma unroll
    for (int q = 1; q < kMaxActive; ++q) {
      if (q < na) {
        const float rq = T->rcp_nq[q];
        const int nq = T->nq[q];
        const int xo = T->xo[q];
#pragma unroll
        for (int j = 0; j < FPT; ++j) {
          const int hi = fdiv(rem[j], rq);
          const int uq = rem[j] - hi * nq;
          rem[j] = hi;
          xq[j][q] = tg[xo + uq];
        }
      } else {
#pragma unroll
        for (int j = 0; j < FPT; ++j) xq[j][q] = 0;
      }
    }
    const cptr<double> al = in_loop_uniform(&T->alpha[pot][0]);
    const cptr<double> be = in_loop_uniform(&T->beta[bv][0]);
    const cptr<double> pc = in_loop_uniform(a.pc);
    R A[FPT], B[FPT], Cl[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      A[j] = c0;
      B[j] = al0;
      Cl[j] = be0;
    }
#pragma unroll
    for (int q = 1; q < kMaxActive; ++q) {
      if (q < na) {
        const R alq = (R)al[q], beq = (R)be[q];
        const R c0q = (R)pc[2 * pair_index(0, q)], k0q = (R)pc[2 * pair_index(0, q) + 1];
#pragma unroll
        for (int j = 0; j < FPT; ++j) {
          const R x2 = xq[j][q] * xq[j][q];
          A[j] = fma(alq, x2, A[j]);
          A[j] = fma(beq, xq[j][q], A[j]);
          B[j] = fma(c0q, x2, B[j]);
          Cl[j] = fma(k0q, x2, Cl[j]);
        }
#pragma unroll
        for (int r = q + 1; r < kMaxActive; ++r) {
          if (r < na) {
            const R cqr = (R)pc[2 * pair_index(q, r)], kqr = (R)pc[2 * pair_index(q, r) + 1];
#pragma unroll
            for (int j = 0; j < FPT; ++j) {
              const R x2 = xq[j][q] * xq[j][q];
              const R y2 = xq[j][r] * xq[j][r];
              A[j] = fma(cqr * x2, y2, A[j]);
              A[j] = fma(kqr * y2, xq[j][q], A[j]);
            }
          }
        }
      }
    }
    const cptr<R> Kw = in_loop_uniform(K0);
    const cptr<R> xw = in_loop_uniform(x0);
#pragma unroll 1
    for (int u = 0; u < NQ; ++u) {
      const R xv = xw[u];
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        const R V = fma(fma(B[j], xv, Cl[j]), xv, A[j]);
        const C xu = ldc<C>(src + fb[j] * NQ + u);
        R re = V * xu.x, im = V * xu.y;
        if (KIN) {
          R kr = 0, ki = 0;
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            const R m = Kw[u * NQ + k];
            kr = fma(m, x[j][k].x, kr);
            ki = fma(m, x[j][k].y, ki);
          }
          re = fma(kin0, kr, re);
          im = fma(kin0, ki, im);
        }
        if (ok[j]) stc(dst + fb[j] * NQ + u, Cx<R>::make(re, im));
      }
    }
  }
}

template <typename G, typename R, typename P>
__device__ __forceinline__ void potential(const TermCtx &a, cptr<TermDev> T, int level0, P src,
                                          P dst, int nfib) {
  const bool kin = a.split == 0;
  if (a.std_maps) {
#define SG_PCASE(L_, NQ_)                                                     \
  case L_:                                                                    \
    if (kin) potential_fixed<G, R, P, NQ_, true>(a, T, src, dst, nfib);       \
    else potential_fixed<G, R, P, NQ_, false>(a, T, src, dst, nfib);          \
    return;
    switch (level0) {
      SG_PCASE(1, 4)
      SG_PCASE(2, 6)
      SG_PCASE(3, 8)
      SG_PCASE(4, 10)
      SG_PCASE(5, 12)
      SG_PCASE(6, 14)
      SG_PCASE(7, 16)
      default: break;
    }
#undef SG_PCASE
  }
  if (kin) potential_impl<G, R, P, 0, true>(a, T, src, dst, nfib);
  else potential_impl<G, R, P, 0, false>(a, T, src, dst, nfib);
}

// The whole of Alg. 1 for one term, by the threads of G, with two buffers of
// `buf` complex values each starting at `base`.
template <typename G, typename R, typename P>
__device__ __forceinline__ void run_term(const TermCtx &a, cptr<TermDev> T, P base, int buf) {
  const R *tab = (const R *)a.tab;
  const int na = T->na;
  const int nbasis = T->nbasis;
  const int ngrid = T->ngrid;
  const int off = T->off;
  const double cf = T->coeff;
  if (na == 0) {  // every mode at a one-function level: a scalar term
    if (G::tid() == 0) {
      const double c0 = a.vt ? a.vt[0] : T->c0[a.split ? kPotSplit : kPotFull];
      const Z64 x = ldc<Z64>(a.psi + a.mb[off]);
      stc(a.tm + off, Z64{cf * c0 * x.x, cf * c0 * x.y});
    }
    return;
  }
  P src = base, dst = base + buf;

  // steps 1-2: gather + basis -> grid along mode 0, then the other modes
  {
    const int nb0 = T->nb[0], nq0 = T->nq[0];
    gather_b2g<G, R, P>(a, T->lev[0], nb0, nq0, off, nbasis / nb0, tab + T->bt[0], src);
    G::sync();
    int stride = nq0;
    int nouter = nbasis / nb0;
    for (int p = 1; p < na; ++p) {
      const int nb = T->nb[p], nq = T->nq[p];
      nouter /= nb;
      contract_level<G, R, P, false>(0, T->lev[p], a.std_maps, nb, nq, src, dst, tab + T->bt[p],
                                     (R)1, stride, nouter);
      G::sync();
      P tmp = src; src = dst; dst = tmp;
      stride *= nq;
    }
  }
  // step 3: potential (+ mode-0 kinetic), then the other modes' kinetic
  {
    const int nq0 = T->nq[0];
    potential<G, R, P>(a, T, T->lev[0], src, dst, ngrid / nq0);
    G::sync();
    if (!a.split) {
      int stride = nq0;
      int nouter = ngrid / nq0;
      for (int p = 1; p < na; ++p) {
        const int nb = T->nb[p], nq = T->nq[p];
        nouter /= nq;
        contract_level<G, R, P, true>(1, T->lev[p], a.std_maps, nb, nq, src, dst, tab + T->kg[p],
                                      (R)T->kin[p], stride, nouter);
        G::sync();
        stride *= nq;
      }
    }
    P tmp = src; src = dst; dst = tmp;
  }
  // step 4: grid -> basis; the last mode writes D_l * result to HBM
  {
    int stride = 1;
    int nouter = ngrid;
    for (int p = 0; p < na - 1; ++p) {
      const int nb = T->nb[p], nq = T->nq[p];
      nouter /= nq;
      contract_level<G, R, P, false>(2, T->lev[p], a.std_maps, nb, nq, src, dst, tab + T->wt[p],
                                     (R)1, stride, nouter);
      G::sync();
      P tmp = src; src = dst; dst = tmp;
      stride *= nb;
    }
    const int p = na - 1;
    g2b_store<G, R, P>(a.std_maps, T->lev[p], T->nb[p], T->nq[p], src, Out{a.tm + off},
                       tab + T->wt[p], cf, stride);
  }
}

// ---------------------------------------------------------------------------
// In-place form (split operator, standard size maps): one buffer per term,
// one-mode tables read from the workgroup's LDS copy.  A contraction first
// loads every input fiber of the group into registers (the host guarantees
// at most inplace_fpt(NI) fibers per thread), syncs the group, then writes
// the outputs over the inputs.  Matrix rows are read one row ahead.  Outputs
// are the same FMA chains, in the same order, as in the ping-pong form.
// ---------------------------------------------------------------------------
// The term record's header held across a wavefront: lane i has dword i.
// Fields are read with v_readlane (no memory access after the one load).
struct TermHdr {
  uint32_t v;
  __device__ __forceinline__ int i32(int idx) const {
    return (int)__builtin_amdgcn_readlane((int)v, idx);
  }
  __device__ __forceinline__ int off() const { return i32(0); }
  __device__ __forceinline__ int nbasis() const { return i32(1); }
  __device__ __forceinline__ int ngrid() const { return i32(2); }
  __device__ __forceinline__ int na() const { return i32(3); }
  __device__ __forceinline__ int lev(int p) const { return i32(4 + p); }
  __device__ __forceinline__ int nb(int p) const { return i32(12 + p); }
  __device__ __forceinline__ int nq(int p) const { return i32(20 + p); }
  __device__ __forceinline__ float rcp_nq(int p) const { return __int_as_float(i32(28 + p)); }
  __device__ __forceinline__ double coeff() const {
    return __hiloint2double(i32(37), i32(36));
  }
  __device__ __forceinline__ int foff() const { return i32(38); }
};
__device__ __forceinline__ TermHdr load_hdr(cptr<TermDev> T) {
  const int lane = threadIdx.x & 63;
  const glb_p<const uint32_t> w = (glb_p<const uint32_t>)(const TermDev *)T;
  return TermHdr{w[lane < kTermHdrDwords ? lane : 0]};
}

template <typename R, int NI>
__device__ __forceinline__ void ld_row(lds_p<const R> M, int u, R (&r)[NI]) {
#pragma unroll
  for (int k = 0; k < NI; ++k) r[k] = M[u * NI + k];
}

// LDS bank skew for fibers stored contiguously, one fiber per lane (the
// mode-0 fibers at grid size, whose length n is even): lane t visits entry
// (i + fiber_skew) mod n at step i, so that the lanes of one 128-byte LDS pass
// (8 lanes of 16-byte or 16 lanes of 8-byte values) hit distinct banks, also
// when a pass spans twice as many lanes.  Zero for odd n.
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
constexpr int igcd(int a, int b) { return b == 0 ? a : igcd(b, a % b); }
template <int N, int ELEM>
__device__ __forceinline__ int fiber_skew() {
  if constexpr (N % 2 != 0) {
    return 0;
  } else {
    constexpr int P = 128 / ELEM;
    constexpr int S = ilog2(P / igcd(N, P));
    const int t = (int)threadIdx.x;
    return ((t & (P - 1)) >> S) ^ ((t / P) & 1);
  }
}
__device__ __forceinline__ int wrap_add(int i, int s, int n) {
  const int v = i + s;
  return v >= n ? v - n : v;
}
// row u of M with its columns rotated by cs: r[k] = M[u*NI + (k + cs) mod NI]
template <typename R, int NI>
__device__ __forceinline__ void ld_row_rot(lds_p<const R> M, int u, int cs, R (&r)[NI]) {
#pragma unroll
  for (int k = 0; k < NI; ++k) r[k] = M[u * NI + wrap_add(k, cs, NI)];
}
// Rows are prefetched one ahead for short rows only (long rows would cost
// more registers than the latency they hide).
template <int NI> struct RowAhead { static constexpr bool value = NI <= 8; };

// The rows of a one-mode matrix (NO rows of NI entries, row-major in LDS) as
// a contraction walks its outputs.  Level-1 matrices (at most 4 rows) are held
// whole: every row load is issued before the first output and the row loop
// is unrolled.  Longer matrices are read one row ahead in a rolled loop.
// SKEW: per-lane rotations (rs of the rows, cs of the columns): step u reads
// row (u + rs) mod NO with column k holding entry (k + cs) mod NI.
template <typename R, int NI, int NO, bool SKEW = false>
struct Rows {
  static constexpr bool kAll = NO <= 4;
  R all[kAll ? NO : 1][NI];
  R cur[NI], nxt[NI];
  lds_p<const R> M;
  int rs = 0, cs = 0;
  __device__ __forceinline__ explicit Rows(lds_p<const R> m) : M(m) {}
  __device__ __forceinline__ Rows(lds_p<const R> m, int row_skew, int col_skew)
      : M(m), rs(row_skew), cs(col_skew) {}
  __device__ __forceinline__ void ld(int u, R (&r)[NI]) const {
    if constexpr (SKEW) ld_row_rot<R, NI>(M, wrap_add(u, rs, NO), cs, r);
    else ld_row<R, NI>(M, u, r);
  }
  // issue the first loads (before the group sync that precedes the outputs)
  __device__ __forceinline__ void prime() {
    if constexpr (kAll) {
#pragma unroll
      for (int u = 0; u < NO; ++u) ld(u, all[u]);
    } else {
      ld(0, cur);
    }
  }
  // body(u, j, row) for every output row u and fiber slot j < nj: all rows of
  // one fiber before the next when the rows are held whole (one guard per
  // fiber), one row for all fibers at a time otherwise.
  template <int FPT, typename Body>
  __device__ __forceinline__ void for_outputs(int nj, Body &&body) {
    if constexpr (kAll) {
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        if (j >= nj) break;
#pragma unroll
        for (int u = 0; u < NO; ++u) body(u, j, all[u]);
      }
    } else {
      run([&](int u, const R (&row)[NI]) {
#pragma unroll
        for (int j = 0; j < FPT; ++j) {
          if (j >= nj) break;
          body(u, j, row);
        }
      });
    }
  }
  // body(u, row) for u = 0..NO-1 in order
  template <typename Body>
  __device__ __forceinline__ void run(Body &&body) {
    if constexpr (kAll) {
#pragma unroll
      for (int u = 0; u < NO; ++u) body(u, all[u]);
    } else if constexpr (NO <= 8) {
      // levels 2 and 3: two rows per iteration, loaded together, so that one
      // LDS wait serves two rows
#pragma unroll 1
      for (int u = 0; u < NO; u += 2) {
        R ra[NI], rb[NI];
        ld(u, ra);
        if (u + 1 < NO) ld(u + 1, rb);
        body(u, ra);
        if (u + 1 < NO) body(u + 1, rb);
      }
    } else {
#pragma unroll 1
      for (int u = 0; u < NO; ++u) {
        if (!RowAhead<NI>::value) ld(u, cur);
        else if (u + 1 < NO) ld(u + 1, nxt);
        body(u, cur);
        if (RowAhead<NI>::value) {
#pragma unroll
          for (int k = 0; k < NI; ++k) cur[k] = nxt[k];
        }
      }
    }
  }
};

// Chunks of an in-place contraction over more fibers than the group holds
// at once (FPT fibers per thread): each chunk loads all its input fibers,
// syncs the group, then writes its outputs.  A compacting contraction (fewer
// outputs than inputs per fiber) visits its chunks in increasing fiber order
// and an expanding one in decreasing order; then a chunk's outputs never
// land on inputs of a chunk not yet read.  (Fiber f = lo + stride hi reads
// in[lo + stride (k + NI hi)] and writes out[lo + stride (u + NO hi)];
// positions of two fibers coincide only for the same lo, where NO < NI puts
// every output of hi below the inputs of any later hi' > hi, and NO > NI puts
// them above the inputs of any earlier hi' < hi.)  A chunk's results do not
// depend on the chunking: every output is the same FMA chain.
__device__ __forceinline__ int chunk_index(int cc, int nch, bool compacting) {
  return compacting ? cc : nch - 1 - cc;
}

// One chunk of an in-place contraction: fibers base + tid + j N (j < FPT).
template <typename G, typename R, int NI, int NO>
__device__ __forceinline__ void contract_ip_chunk(lds_p<typename Cx<R>::T> buf,
                                                  lds_p<const R> M, int stride, int F,
                                                  int base) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = inplace_fpt(NI);
  const float rcp = 1.0f / (float)stride;
  const int sNI = stride * NI, sNO = stride * NO;
  // fiber slots this chunk needs (wave-uniform)
  const int nj = min(FPT, (F - base + G::N - 1) / G::N);
  int ob[FPT];
  bool ok[FPT];
  C x[FPT][NI];
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    if (j >= nj) break;
    int f = base + G::tid() + j * G::N;
    ok[j] = f < F;
    f = ok[j] ? f : 0;
    const int hi = fdiv(f, rcp);
    const int lo = f - mul24(hi, stride);
    const int ib = lo + mul24(hi, sNI);
    ob[j] = lo + mul24(hi, sNO);
#pragma unroll
    for (int k = 0; k < NI; ++k) x[j][k] = ldc<C>(buf + ib + k * stride);
  }
  Rows<R, NI, NO> rows(M);
  rows.prime();
  G::sync();
  rows.template for_outputs<FPT>(nj, [&](int u, int j, const R (&row)[NI]) {
    R re = 0, im = 0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      re = fma(row[k], x[j][k].x, re);
      im = fma(row[k], x[j][k].y, im);
    }
    if (ok[j]) stc(buf + ob[j] + u * stride, Cx<R>::make(re, im));
  });
}

template <typename G, typename R, int NI, int NO>
__device__ __forceinline__ void contract_ip(lds_p<typename Cx<R>::T> buf, lds_p<const R> M,
                                            int stride, int nouter) {
  constexpr int CH = inplace_fpt(NI) * G::N;
  const int F = stride * nouter;
  const int nch = (F + CH - 1) / CH;
  if (nch <= 1) {
    contract_ip_chunk<G, R, NI, NO>(buf, M, stride, F, 0);
    return;
  }
  for (int cc = 0; cc < nch; ++cc) {
    // the previous chunk's stores before this chunk's loads (disjoint, but
    // the group's accesses of one chunk must not move across another's sync)
    if (cc > 0) G::sync();
    contract_ip_chunk<G, R, NI, NO>(buf, M, stride, F, chunk_index(cc, nch, NO < NI) * CH);
  }
}

// Two consecutive in-place contractions along level-1 modes p and p+1 (the
// same one-mode matrix M, NO x NI, for both) in one step: a thread takes a
// whole NI x NI input slab (one per thread: the caller checks that the slabs
// fit), keeps the intermediate in registers and writes the NO x NO outputs.
// Layout: in[lo + stride*(k1 + NI*(k2 + NI*hi))] ->
// out[lo + stride*(u1 + NO*(u2 + NO*hi))].  M is read with scalar loads.
template <typename G, typename R, int NI, int NO>
__device__ __forceinline__ void contract2_ip(lds_p<typename Cx<R>::T> buf, cptr<R> Ms, int stride,
                                             int nouter) {
  typedef typename Cx<R>::T C;
  const int F = stride * nouter;
  const float rcp = 1.0f / (float)stride;
  int f = G::tid();
  const bool ok = f < F;
  f = ok ? f : 0;
  const int hi = fdiv(f, rcp);
  const int lo = f - mul24(hi, stride);
  const int ib = lo + mul24(hi, stride * NI * NI);
  const int ob = lo + mul24(hi, stride * NO * NO);
  C x[NI][NI];
#pragma unroll
  for (int k2 = 0; k2 < NI; ++k2)
#pragma unroll
    for (int k1 = 0; k1 < NI; ++k1) x[k2][k1] = ldc<C>(buf + ib + stride * (k1 + NI * k2));
  R m[NO][NI];
#pragma unroll
  for (int u = 0; u < NO; ++u)
#pragma unroll
    for (int k = 0; k < NI; ++k) m[u][k] = Ms[u * NI + k];
  G::sync();
  if (!ok) return;
#pragma unroll
  for (int u1 = 0; u1 < NO; ++u1) {
    // t[k2] = sum_k1 M[u1][k1] x[k2][k1]: mode p done for output u1
    C t[NI];
#pragma unroll
    for (int k2 = 0; k2 < NI; ++k2) {
      R re = 0, im = 0;
#pragma unroll
      for (int k1 = 0; k1 < NI; ++k1) {
        re = fma(m[u1][k1], x[k2][k1].x, re);
        im = fma(m[u1][k1], x[k2][k1].y, im);
      }
      t[k2] = Cx<R>::make(re, im);
    }
#pragma unroll
    for (int u2 = 0; u2 < NO; ++u2) {
      R re = 0, im = 0;
#pragma unroll
      for (int k2 = 0; k2 < NI; ++k2) {
        re = fma(m[u2][k2], t[k2].x, re);
        im = fma(m[u2][k2], t[k2].y, im);
      }
      stc(buf + ob + stride * (u1 + NO * u2), Cx<R>::make(re, im));
    }
  }
}

template <typename G, typename R, int NI, int NO>
__device__ __forceinline__ void gather_ip(const TermCtx &a, int off, int nfib, lds_p<const R> M,
                                          lds_p<typename Cx<R>::T> out) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = Fpt<NI>::value;
  for (int f0 = 0; f0 < nfib; f0 += FPT * G::N) {
    const int nj = min(FPT, (nfib - f0 + G::N - 1) / G::N);
    int idx[FPT][NI];
    bool ok[FPT];
    int fb[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + G::tid() + j * G::N;
      ok[j] = f < nfib;
      fb[j] = ok[j] ? f : 0;
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (j >= nj) break;
#pragma unroll
      for (int k = 0; k < NI; ++k) idx[j][k] = a.mbt[fb[j] * NI + k];
    }
    C x[FPT][NI];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (j >= nj) break;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const Z64 v = ldc<Z64>(a.psi + idx[j][k]);
        x[j][k] = Cx<R>::make((R)v.x, (R)v.y);
      }
    }
    // the outputs of one fiber are contiguous: rows visited in a per-lane
    // rotated order keep the stores free of LDS bank conflicts
    const int sk = fiber_skew<NO, (int)sizeof(C)>();
    Rows<R, NI, NO, true> rows(M, sk, 0);
    rows.prime();
    rows.template for_outputs<FPT>(nj, [&](int u, int j, const R (&row)[NI]) {
      R re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        re = fma(row[k], x[j][k].x, re);
        im = fma(row[k], x[j][k].y, im);
      }
      if (ok[j]) stc(out + fb[j] * NO + wrap_add(u, sk, NO), Cx<R>::make(re, im));
    });
  }
}

template <typename G, typename R, int NI, int NO>
__device__ __forceinline__ void g2b_ip(lds_p<typename Cx<R>::T> in, Out o, lds_p<const R> M,
                                       double cf, int stride) {
  typedef typename Cx<R>::T C;
  constexpr int FPT = Fpt<NI>::value;
  for (int f0 = 0; f0 < stride; f0 += FPT * G::N) {
    const int nj = min(FPT, (stride - f0 + G::N - 1) / G::N);
    bool ok[FPT];
    int lo[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = f0 + G::tid() + j * G::N;
      ok[j] = f < stride;
      lo[j] = ok[j] ? f : 0;
    }
    C x[FPT][NI];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (j >= nj) break;
#pragma unroll
      for (int k = 0; k < NI; ++k) x[j][k] = ldc<C>(in + lo[j] + k * stride);
    }
    Rows<R, NI, NO> rows(M);
    rows.prime();
    rows.template for_outputs<FPT>(nj, [&](int u, int j, const R (&row)[NI]) {
      R re = 0, im = 0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        re = fma(row[k], x[j][k].x, re);
        im = fma(row[k], x[j][k].y, im);
      }
      if (ok[j]) stc(o.tm + lo[j] + u * stride, Z64{cf * (double)re, cf * (double)im});
    });
  }
}

// The first grid -> basis contraction (along mode 0, whose fibers are
// contiguous) with the split coupling potential applied to the fibers as they
// are loaded.  Along a mode-0 fiber the potential is A + x0 (C + B x0), where
// A, B, C depend on the fiber's coordinates in the other active modes (nodes
// from the LDS tables, coefficients from the term's LDS block).  STORE: mode 0
// is the only active mode and the outputs, times D_l, go to HBM; otherwise
// they overwrite the fibers in place (at most inplace_fpt(NQ) fibers per
// thread).
// The A, B, C of the mode-0 fibers a thread takes in the first grid -> basis
// contraction (fiber tid + j N), read from the per-problem arrays; FP64
// terms issue these loads before the group sync that ends basis -> grid.
template <typename R, int FPT>
struct FiberABC {
  R A[FPT], B[FPT], C[FPT];
  bool have = false;
};
template <typename G, typename R, int NQ>
__device__ __forceinline__ FiberABC<R, inplace_fpt(NQ)> load_abc(const TermCtx &a,
                                                                 const TermHdr &T, int nfib,
                                                                 int base = 0) {
  constexpr int FPT = inplace_fpt(NQ);
  FiberABC<R, FPT> r;
  if (a.vt) return r;   // a tabulated potential reads V_eff instead
  if constexpr (sizeof(R) == sizeof(double)) {
    const int nj = min(FPT, (nfib - base + G::N - 1) / G::N);
    const glb_p<const double> A = a.abc + T.foff();
    const glb_p<const double> B = A + a.nfib, Cc = B + a.nfib;
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      if (j >= nj) break;
      const int f = base + G::tid() + j * G::N;
      const int fi = f < nfib ? f : 0;
      r.A[j] = A[fi];
      r.B[j] = B[fi];
      r.C[j] = Cc[fi];
    }
    r.have = true;
  }
  return r;
}

template <typename G, typename R, int NQ, int NB, bool STORE, int FPT>
__device__ __forceinline__ void pot_g2b0_chunk(const TermHdr &T, lds_p<typename Cx<R>::T> buf,
                                               lds_p<const R> lt, lds_p<const R> cf, int nfib,
                                               Out o, double dl, const FiberABC<R, FPT> &pre,
                                               int base, glb_p<const double> vt) {
  typedef typename Cx<R>::T C;
  const int na = T.na();
  const int l0 = T.lev(0);
  const int nj = min(FPT, (nfib - base + G::N - 1) / G::N);
  bool ok[FPT];
  int fb[FPT], rem[FPT];
  R A[FPT], B[FPT], Cl[FPT];
  R xq[FPT][kMaxActive];
  if (vt) {   // tabulated potential: V_eff is read per point below
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = base + G::tid() + j * G::N;
      ok[j] = f < nfib && j < nj;
      fb[j] = ok[j] ? f : 0;
      A[j] = B[j] = Cl[j] = (R)0;
    }
  } else if (pre.have) {
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = base + G::tid() + j * G::N;
      ok[j] = f < nfib && j < nj;
      fb[j] = ok[j] ? f : 0;
      A[j] = pre.A[j];
      B[j] = pre.B[j];
      Cl[j] = pre.C[j];
    }
  } else {
    const R c0 = cf[0], al0 = cf[1], be0 = cf[2];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int f = base + G::tid() + j * G::N;
      ok[j] = f < nfib && j < nj;
      fb[j] = ok[j] ? f : 0;
      rem[j] = fb[j];
      A[j] = c0;
      B[j] = al0;
      Cl[j] = be0;
    }
    // the fibers' coordinates along modes 1.. and their A, B, C; each
    // coefficient is read once for all of the thread's fibers
#pragma unroll
    for (int q = 1; q < kMaxActive; ++q) {
      if (q >= na) break;
      const float rq = T.rcp_nq(q);
      const int nq = T.nq(q);
      const int lq = T.lev(q);
      const lds_p<const R> xn = lt + std_table_base(lq) + 2 * (2 * lq + 1) * (2 * lq + 2);
      const R alq = cf[2 + q], beq = cf[9 + q], c0q = cf[16 + q], k0q = cf[23 + q];
#pragma unroll
      for (int j = 0; j < FPT; ++j) {
        if (j >= nj) break;
        const int hi = fdiv(rem[j], rq);
        const int uq = rem[j] - hi * nq;
        rem[j] = hi;
        xq[j][q] = xn[uq];
        const R x2 = xq[j][q] * xq[j][q];
        A[j] = fma(alq, x2, A[j]);
        A[j] = fma(beq, xq[j][q], A[j]);
        B[j] = fma(c0q, x2, B[j]);
        Cl[j] = fma(k0q, x2, Cl[j]);
      }
#pragma unroll
      for (int r = 1; r < q; ++r) {   // pair (r, q), r < q
        const R cqr = cf[coef_pair(r, q)], kqr = cf[coef_pair(r, q) + 1];
#pragma unroll
        for (int j = 0; j < FPT; ++j) {
          if (j >= nj) break;
          const R x2 = xq[j][q] * xq[j][q];
          A[j] = fma(cqr * (xq[j][r] * xq[j][r]), x2, A[j]);
          A[j] = fma(kqr * x2, xq[j][r], A[j]);
        }
      }
    }
  }
  // fiber entries in a per-lane rotated order (free of LDS bank conflicts):
  // slot k holds entry (k + sk) mod NQ, with its node and matrix column
  const int sk = fiber_skew<NQ, (int)sizeof(C)>();
  const lds_p<const R> x0 = lt + std_table_base(l0) + 2 * NB * NQ;
  C x[FPT][NQ];
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    if (j >= nj) break;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int kk = wrap_add(k, sk, NQ);
      const C v = ldc<C>(buf + fb[j] * NQ + kk);
      const R xv = x0[kk];
      const R V = vt ? (R)vt[fb[j] * NQ + kk] : fma(fma(B[j], xv, Cl[j]), xv, A[j]);
      x[j][k] = Cx<R>::make(V * v.x, V * v.y);
    }
  }
  Rows<R, NQ, NB, true> rows(lt + std_table_base(l0) + NB * NQ, 0, sk);
  rows.prime();
  if (!STORE) G::sync();
  rows.template for_outputs<FPT>(nj, [&](int v, int j, const R (&row)[NQ]) {
    R re = 0, im = 0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      re = fma(row[k], x[j][k].x, re);
      im = fma(row[k], x[j][k].y, im);
    }
    if (ok[j]) {
      if (STORE) stc(o.tm + fb[j] * NB + v, Z64{dl * (double)re, dl * (double)im});
      else stc(buf + fb[j] * NB + v, Cx<R>::make(re, im));
    }
  });
}

// A compacting contraction: chunks in increasing fiber order (see
// chunk_index).  The first chunk (inplace_fpt(NQ) fibers per thread) takes
// the prefetched A, B, C (FP64 terms); the rest, when the fibers exceed one
// pass, run in chunks of one fiber per thread that load theirs (any partition
// into increasing contiguous ranges is safe; small chunks keep the
// registers of the first pass free).
template <typename G, typename R, int NQ, int NB, bool STORE>
__device__ __forceinline__ void pot_g2b0_ip(const TermCtx &a, const TermHdr &T,
                                            lds_p<typename Cx<R>::T> buf, lds_p<const R> lt,
                                            lds_p<const R> cf, int nfib, Out o, double dl,
                                            const FiberABC<R, inplace_fpt(NQ)> &pre0) {
  constexpr int FPT = inplace_fpt(NQ);
  pot_g2b0_chunk<G, R, NQ, NB, STORE, FPT>(T, buf, lt, cf, nfib, o, dl, pre0, 0, a.vt);
  for (int base = FPT * G::N; base < nfib; base += G::N) {
    if (!STORE) G::sync();
    FiberABC<R, 1> pre;
    if constexpr (sizeof(R) == sizeof(double)) {
      if (pre0.have) {
        const int f = base + G::tid();
        const glb_p<const double> A = a.abc + T.foff() + (f < nfib ? f : 0);
        pre.A[0] = A[0];
        pre.B[0] = A[a.nfib];
        pre.C[0] = A[2 * a.nfib];
        pre.have = true;
      }
    }
    pot_g2b0_chunk<G, R, NQ, NB, STORE, 1>(T, buf, lt, cf, nfib, o, dl, pre, base, a.vt);
  }
}

// Level dispatch of the in-place steps (standard maps: nb = 2l+1, nq = 2l+2).
#define SG_LEVELS(X) X(1, 3, 4) X(2, 5, 6) X(3, 7, 8) X(4, 9, 10) X(5, 11, 12) X(6, 13, 14) X(7, 15, 16)

template <typename G, typename R>
__device__ __forceinline__ void contract_ip_level(int kind, int level,
                                                  lds_p<typename Cx<R>::T> buf,
                                                  lds_p<const R> lt, int stride, int nouter) {
  const lds_p<const R> base = lt + std_table_base(level);
#define SG_IPCASE(L_, NB_, NQ_)                                                          \
  case L_:                                                                              \
    if (kind == 0) contract_ip<G, R, NB_, NQ_>(buf, base, stride, nouter);               \
    else contract_ip<G, R, NQ_, NB_>(buf, base + NB_ * NQ_, stride, nouter);             \
    return;
  switch (level) { SG_LEVELS(SG_IPCASE) default: break; }
#undef SG_IPCASE
}

// Alg. 1 for one term of the split operator in place: gather + basis -> grid,
// then grid -> basis with the coupling potential applied to the fibers of the
// first contraction, D_l * result to HBM.
template <typename G, typename R>
__device__ __forceinline__ void run_term_inplace(const TermCtx &a, const TermHdr &T,
                                                 lds_p<typename Cx<R>::T> buf,
                                                 lds_p<const R> lt) {
  const int na = T.na();
  const int nbasis = T.nbasis();
  const int ngrid = T.ngrid();
  const int off = T.off();
  const double cf = T.coeff();
  // the coefficient block, into LDS after the grid buffer (published by the
  // sync after the gather)
  const lds_p<R> coef = (lds_p<R>)(buf + ngrid);
  if (sizeof(R) != sizeof(double) || na == 1)   // FP64 terms read A, B, C from HBM
    for (int i = G::tid(); i < kCoefUsed; i += G::N) coef[i] = (R)a.pcoef[i];
  const int l0 = T.lev(0);
  {
    const int nb0 = T.nb(0), nq0 = T.nq(0);
    const lds_p<const R> M0 = lt + std_table_base(l0);
#define SG_GCASE(L_, NB_, NQ_)                                                   \
  case L_: gather_ip<G, R, NB_, NQ_>(a, off, nbasis / NB_, M0, buf); break;
    switch (l0) { SG_LEVELS(SG_GCASE) default: break; }
#undef SG_GCASE
    G::sync();
    int stride = nq0;
    int nouter = nbasis / nb0;
    for (int p = 1; p < na;) {
      // two level-1 modes in one step when every slab has a thread
      if (p + 1 < na && T.lev(p) == 1 && T.lev(p + 1) == 1 && stride * (nouter / 9) <= G::N) {
        nouter /= 9;
        contract2_ip<G, R, 3, 4>(buf, (cptr<R>)a.gtab + std_table_base(1), stride, nouter);
        stride *= 16;
        p += 2;
      } else {
        nouter /= T.nb(p);
        contract_ip_level<G, R>(0, T.lev(p), buf, lt, stride, nouter);
        stride *= T.nq(p);
        p += 1;
      }
      if (p < na) G::sync();   // the last sync follows the A, B, C loads
    }
  }
  const int nfib = ngrid / T.nq(0);
  if (na == 1) {
#define SG_P1CASE(L_, NB_, NQ_)                                                  \
  case L_:                                                                      \
    pot_g2b0_ip<G, R, NQ_, NB_, true>(a, T, buf, lt, coef, nfib, Out{a.tm + off}, cf,  \
                                      FiberABC<R, inplace_fpt(NQ_)>{});               \
    break;
    switch (l0) { SG_LEVELS(SG_P1CASE) default: break; }
#undef SG_P1CASE
    return;
  }
#define SG_PCASE(L_, NB_, NQ_)                                                   \
  case L_: {                                                                    \
    const auto pre = load_abc<G, R, NQ_>(a, T, nfib);                           \
    G::sync();                                                                  \
    pot_g2b0_ip<G, R, NQ_, NB_, false>(a, T, buf, lt, coef, nfib, Out{a.tm + off}, cf, pre); \
    break;                                                                      \
  }
  switch (l0) { SG_LEVELS(SG_PCASE) default: G::sync(); break; }
#undef SG_PCASE
  G::sync();
  {
    int stride = T.nb(0);
    int nouter = nfib;
    for (int p = 1; p < na - 1;) {
      if (p + 1 < na - 1 && T.lev(p) == 1 && T.lev(p + 1) == 1 &&
          stride * (nouter / 16) <= G::N) {
        nouter /= 16;
        contract2_ip<G, R, 4, 3>(buf, (cptr<R>)a.gtab + std_table_base(1) + 12, stride, nouter);
        stride *= 9;
        p += 2;
      } else {
        nouter /= T.nq(p);
        contract_ip_level<G, R>(2, T.lev(p), buf, lt, stride, nouter);
        stride *= T.nb(p);
        p += 1;
      }
      G::sync();
    }
    const int p = na - 1;
    const int lp = T.lev(p);
    const lds_p<const R> Mw = lt + std_table_base(lp) + (2 * lp + 1) * (2 * lp + 2);
#define SG_SCASE(L_, NB_, NQ_)                                                   \
  case L_: g2b_ip<G, R, NQ_, NB_>(buf, Out{a.tm + off}, Mw, cf, stride); break;
    switch (lp) { SG_LEVELS(SG_SCASE) default: break; }
#undef SG_SCASE
  }
}

// One term: the scalar case, then the in-place or the ping-pong form (IP: the
// launch holds in-place terms only, and the ping-pong form is not compiled in).
template <typename G, typename R, typename P, bool IP>
__device__ __forceinline__ void run_any(const TermCtx &a, cptr<TermDev> T, const TermHdr &hdr,
                                        P base, int inplace, char *lds_raw) {
  if (T->na == 0) {
    if (G::tid() == 0) {
      const double c0 = a.vt ? a.vt[0] : T->c0[a.split ? kPotSplit : kPotFull];
      const Z64 x = ldc<Z64>(a.psi + a.mb[T->off]);
      stc(a.tm + T->off, Z64{T->coeff * c0 * x.x, T->coeff * c0 * x.y});
    }
    return;
  }
  if (IP || inplace)
    run_term_inplace<G, R>(a, hdr, (lds_p<typename Cx<R>::T>)base,
                           (lds_p<const R>)(lds_raw + a.lt_off));
  else if constexpr (!IP) run_term<G, R, P>(a, T, base, T->ngrid);
}

// Is instance I part of this launch, and which vector does H act on?
__device__ __forceinline__ bool live(const SweepArgs &a, cptr<InstDev> I) {
  return I->active && (a.mode == 0 || a.k <= I->K - 1);
}
__device__ __forceinline__ const double2 *input_of(const SweepArgs &a, cptr<InstDev> I) {
  double2 *x0 = a.x0o ? a.x0o + I->vec_off : I->x0;
  double2 *x1 = a.x1o ? a.x1o + I->vec_off : I->x1;
  if (a.mode == 0) return x0;
  return ((a.k - 1) & 1) ? x1 : x0;   // phi_{k-1}
}

template <typename R, bool TAB>
__device__ __forceinline__ TermCtx make_ctx(const SweepArgs &a, cptr<InstDev> I, int t) {
  TermCtx c;
  c.mb = (glb_p<const int32_t>)I->mb;
  c.psi = (glb_p<const Z64>)input_of(a, I);
  c.tm = (glb_p<Z64>)I->tm;
  c.std_maps = I->std_maps;
  c.split = a.split;
  const bool r32 = a.mixed && I->round32;
  c.pot = a.split ? (r32 ? kPotSplitRounded : kPotSplit) : kPotFull;
  c.pc = (cptr<double>)(I->pairs + (size_t)t * kPairStride + (r32 ? 2 * kMaxPairs : 0));
  if (sizeof(R) == sizeof(float)) c.tab = I->tab32;
  else c.tab = r32 ? (const void *)I->tab32r : (const void *)I->tab64;
  c.lt_off = (sizeof(R) == sizeof(double) && r32) ? a.tab_a : 0;
  c.gtab = (sizeof(R) == sizeof(double) && r32) ? a.stab_r : a.stab;
  c.pcoef = (glb_p<const double>)(I->potc + ((size_t)t * 2 + (r32 ? 1 : 0)) * kCoefStride);
  c.abc = (glb_p<const double>)(I->abc + (r32 ? 3 * I->nfib : 0));
  c.nfib = I->nfib;
  c.vt = nullptr;
  if constexpr (TAB)
    if (I->veff) c.vt = (glb_p<const double>)(I->veff + I->voff[t]);
  return c;
}

// IP: every term of the launch runs in place.  TAB: the instance's coupling
// potential is tabulated (V_eff per term, read along the fibers).  Two
// workgroups per compute unit: at most 128 VGPRs per lane.
template <typename R, bool IP, bool TAB>
__global__ __launch_bounds__(kThreads, 4) void sweep_kernel(SweepArgs a) {
  extern __shared__ char lds_raw[];
  typedef typename Cx<R>::T C;
  // this wavefront's term (slot 0 of a one-term pack; unused slots of a wave
  // pack repeat slot 0's term) and its record header, loaded before the
  // table copy so that their latency overlaps it
  const cptr<PackDev> P = a.packs + blockIdx.x;
  const int kind = P->block;
  const int w = kind == kPackWaves ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const bool has_term = kind != kPackWaves || w < P->n;
  const cptr<InstDev> I = a.inst + P->inst[w];
  const int t = P->term[w];
  const cptr<TermDev> T = (cptr<TermDev>)(I->terms + t);
  const TermHdr hdr = load_hdr(T);
  TermCtx c = make_ctx<R, TAB>(a, I, t);
  c.mbt = (glb_p<const int32_t>)P->mbt[w];
  // the standard-map tables into LDS (every wavefront takes part): the
  // exact set at 0, the FP32-rounded FP64 set (if any) at tab_a, levels up to
  // the pack's highest only; the pack's term buffers follow (at lds_base)
  {
    const lds_p<Z64> dst = (lds_p<Z64>)lds_raw;
    const glb_p<const Z64> sa = (glb_p<const Z64>)a.stab;
    const glb_p<const Z64> sb = (glb_p<const Z64>)a.stab_r;
    const int pre = min(a.tab_a, (int)sizeof(R) * std_table_base(P->maxlev + 1));
    const int na16 = (pre + 15) >> 4, nb16 = a.tab_b > 0 ? na16 : 0, off_b = a.tab_a >> 4;
    for (int i = threadIdx.x; i < na16 + nb16; i += kThreads)
      stc(dst + (i < na16 ? i : off_b + (i - na16)),
          i < na16 ? ldc<Z64>(sa + i) : ldc<Z64>(sb + (i - na16)));
    if (na16 + nb16 > 0) __syncthreads();
  }
  if (!has_term || !live(a, I)) return;
  char *const pack_lds = lds_raw + __builtin_amdgcn_readfirstlane(P->lds_base);
  if (kind != kPackWaves) {
    if constexpr (IP) {
      run_any<BlockGroup, R, lds_p<C>, true>(c, T, hdr, (lds_p<C>)pack_lds, 1, lds_raw);
    } else {
      if (kind == kPackBlockLds)
        run_any<BlockGroup, R, lds_p<C>, false>(c, T, hdr, (lds_p<C>)pack_lds, P->inplace[0],
                                                lds_raw);
      else
        run_any<BlockGroup, R, glb_p<C>, false>(c, T, hdr,
                                                (glb_p<C>)(a.scratch + P->scratch_off), 0,
                                                lds_raw);
    }
    return;
  }
  run_any<WaveGroup, R, lds_p<C>, IP>(c, T, hdr, (lds_p<C>)(pack_lds + P->lds_off[w]),
                                      P->inplace[w], lds_raw);
}
template <typename R, bool IP, bool TAB>
hipError_t launch_packs_as(const SweepArgs &a, int npacks, int lds, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<R, IP, TAB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (ev0 || ev1)
    hipExtLaunchKernelGGL((sweep_kernel<R, IP, TAB>), dim3((unsigned)npacks), dim3(kThreads), lds, s,
                          ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL((sweep_kernel<R, IP, TAB>), dim3((unsigned)npacks), dim3(kThreads), lds, s,
                       a);
  return hipGetLastError();
}

// tab: some instance of the plan has a tabulated potential (FP64; its terms
// run in place, the others as they would)
template <typename R>
hipError_t launch_packs(const SweepArgs &a, const PackSet &ps, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1, bool tab = false) {
  if constexpr (sizeof(R) == sizeof(double))
    if (tab) {
      if (ps.all_inplace) return launch_packs_as<R, true, true>(a, ps.count, ps.lds_bytes, s, ev0, ev1);
      return launch_packs_as<R, false, true>(a, ps.count, ps.lds_bytes, s, ev0, ev1);
    }
  if (ps.all_inplace) return launch_packs_as<R, true, false>(a, ps.count, ps.lds_bytes, s, ev0, ev1);
  return launch_packs_as<R, false, false>(a, ps.count, ps.lds_bytes, s, ev0, ev1);
}

}  // namespace

// The per-fiber A, B, C of the split coupling potential along the mode-0
// fibers of every term, for both coefficient variants (exact, and the
// FP32-rounded coefficients and nodes): the sums the in-kernel form takes,
// once per problem.  Nodes come from the problem's one-mode tables.
__global__ __launch_bounds__(256) void fiber_coeff_kernel(const TermDev *terms,
                                                          const double *potc,
                                                          const double *tab64,
                                                          const double *tab32r, double *abc,
                                                          int64_t nfib) {
  const int64_t t = blockIdx.x;
  const TermDev &T = terms[t];
  const int na = T.na;
  if (na == 0) return;
  const int nf = T.ngrid / T.nq[0];
  for (int v = 0; v < 2; ++v) {
    const double *cf = potc + ((size_t)t * 2 + v) * kCoefStride;
    const double *tab = v ? tab32r : tab64;
    double *A = abc + (size_t)v * 3 * nfib + T.foff;
    double *B = A + nfib, *Cc = B + nfib;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      double xq[kMaxActive] = {};
      int rem = f;
      double va = cf[0], vb = cf[1], vc = cf[2];
      for (int q = 1; q < na; ++q) {
        const int hi = rem / T.nq[q];
        const int uq = rem - hi * T.nq[q];
        rem = hi;
        xq[q] = tab[T.xo[q] + uq];
        const double x2 = xq[q] * xq[q];
        va = fma(cf[2 + q], x2, va);
        va = fma(cf[9 + q], xq[q], va);
        vb = fma(cf[16 + q], x2, vb);
        vc = fma(cf[23 + q], x2, vc);
        for (int r = 1; r < q; ++r) {
          const double cqr = cf[coef_pair(r, q)], kqr = cf[coef_pair(r, q) + 1];
          va = fma(cqr * (xq[r] * xq[r]), x2, va);
          va = fma(kqr * x2, xq[r], va);
        }
      }
      A[f] = va;
      B[f] = vb;
      Cc[f] = vc;
    }
  }
}

hipError_t launch_fiber_coeffs(const TermDev *terms, int64_t nterms, const double *potc,
                               const double *tab64, const double *tab32r, double *abc,
                               int64_t nfib, hipStream_t s) {
  if (nterms <= 0 || nfib <= 0) return hipSuccess;
  hipLaunchKernelGGL(fiber_coeff_kernel, dim3((unsigned)nterms), dim3(256), 0, s, terms, potc,
                     tab64, tab32r, abc, nfib);
  return hipGetLastError();
}

hipError_t launch_sweep(const Plan *pl, const LaunchCtl &c, hipStream_t s) {
  SweepArgs a;
  a.inst = (cptr<InstDev>)pl->d_inst;
  a.scratch = pl->d_scratch;
  a.x0o = c.x0o;
  a.x1o = c.x1o;
  a.mode = c.mode == Mode::Cheb ? 1 : 0;
  a.k = c.k;
  a.split = split_form(pl, c.prec) ? 1 : 0;
  a.mixed = c.prec == SG_MIXED ? 1 : 0;
  a.stab = a.stab_r = nullptr;
  a.tab_a = a.tab_b = 0;
  hipError_t e = hipSuccess;
  if (c.prec == SG_FP64) {
    const PackSet &ps = pl->sets[pl->fp64_split ? kSetSplit64 : kSetGrid64];
    if (ps.count == 0) return hipSuccess;
    a.packs = (cptr<PackDev>)(pl->d_packs + ps.first);
    a.stab = pl->d_stab64;
    a.tab_a = ps.tab_bytes;
    return launch_packs<double>(a, ps, s, c.ev0, c.ev1, pl->any_tab);
  }
  if (pl->any_tab) return hipErrorInvalidValue;   // tabulated potentials run in FP64
  // mixed: terms with large |D_l| in FP64, the rest in FP32.  The FP64 terms
  // of an instance that also has FP32 terms read the FP32-rounded tables, so
  // that all its terms apply the same one-mode operators and the Smolyak
  // combination cancels their rounding as it does when all run in FP32.
  const PackSet &p64 = pl->sets[kSetMixed64], &p32 = pl->sets[kSetMixed32];
  if (p64.count > 0) {
    a.packs = (cptr<PackDev>)(pl->d_packs + p64.first);
    a.stab = pl->d_stab64;
    a.stab_r = pl->d_stab32r;
    a.tab_a = pl->any_round32 ? p64.tab_bytes / 2 : p64.tab_bytes;
    a.tab_b = pl->any_round32 ? p64.tab_bytes / 2 : 0;
    e = launch_packs<double>(a, p64, s, c.ev0,
                             p32.count > 0 ? nullptr : c.ev1);
    if (e != hipSuccess) return e;
  }
  if (p32.count > 0) {
    a.packs = (cptr<PackDev>)(pl->d_packs + p32.first);
    a.stab = pl->d_stab32;
    a.stab_r = nullptr;
    a.tab_a = p32.tab_bytes;
    a.tab_b = 0;
    e = launch_packs<float>(a, p32, s, p64.count > 0 ? nullptr : c.ev0,
                            c.ev1);
  }
  return e;
}

}  // namespace sg
