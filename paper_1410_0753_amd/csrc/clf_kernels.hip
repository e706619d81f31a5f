// HIP kernels of the split-step shallow-water library (gfx950).
//
// The hot path is one fused "march" kernel per time step.  A wavefront owns
// a tile: a strip of 64 consecutive columns (58 output columns plus a
// 3-column halo on each side) and a segment of rows.  It walks along the
// segment one row at a time (alternate segment rows in opposite directions,
// so that neighbouring segments read their shared halo rows together):
//   * the x-sweep of the row (eq2A) runs across the 64 lanes; the neighbour
//     values of steps (b), (d) and (e) come from the adjacent lanes, and each
//     of the three neighbour stages costs one lane of validity on each side,
//     hence the 3-column halo;
//   * the post-x row enters a per-lane y-sweep pipeline (eq2B) held in
//     registers: stage A = step (a), B = step (b), C = steps (c)+(d),
//     D = step (e).  Each stage needs its neighbours one row up and down, so
//     the row leaving the pipeline lags the row entering it by 3 and a
//     segment re-reads 3 rows above and below it.
// The eqQ value of an interface is the same bits for the two nodes it
// separates when both are wet, so each sweep evaluates it once, on the node
// above or left of it, and hands it on: across lanes in the x-sweep, in a
// register down the y pipeline.  Selecting its operands first (the real
// neighbour, or the node's own mirror ghost) covers the wall cases with the
// same single evaluation.
// Every node of the state is read once and written once per step (plus the
// depth and the maxwave read-modify-write); rows are read with fully
// coalesced loads along x.  There is no LDS and no barrier.
//
// FP64 arithmetic follows the literal form of the paper's formulas in the
// operation order fixed by the formulation note (eqQ, solver2/solver1,
// stateu/stateh), compiled without FMA contraction, so that results are
// reproducible bit for bit by any implementation of the same note.
// The FP32 path stores the surface eta instead of h and advances
// perturbations (algebraically identical form, exact at rest).

#include "clf_internal.h"

#include <math.h>

#include <type_traits>

namespace clf {
namespace {

constexpr double kG = 9.81;

// ---------------------------------------------------------------------------
// Cross-lane exchange: value held by lane-1 / lane+1 of the wavefront, by
// DPP whole-wave shifts (wave_shr:1 / wave_shl:1).  Lanes without a source
// (lane 0, lane 63) read 0 (bound_ctrl); they lie in the halo and a zero
// flag word makes their neighbour look missing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_prev_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int lane_next_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);
}

template <class T>
__device__ __forceinline__ T from_prev(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "4-byte multiple");
  union U { T v; int i[sizeof(T) / 4]; };
  U a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) b.i[k] = lane_prev_i(a.i[k]);
  return b.v;
}

template <class T>
__device__ __forceinline__ T from_next(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "4-byte multiple");
  union U { T v; int i[sizeof(T) / 4]; };
  U a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) b.i[k] = lane_next_i(a.i[k]);
  return b.v;
}

// Loads through the global address space (the field pointers come from a
// descriptor in memory, so the compiler cannot infer it).
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
// Load of read-only data at a wavefront-uniform address (row metrics):
// through the constant address space the compiler may use a scalar load,
// which is counted apart from the vector loads, so waiting for it does not
// also wait for the rows prefetched before it.
template <class T>
__device__ __forceinline__ T cload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}
template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// An array element through a 32-bit byte offset from the array's base: the
// access takes the uniform base in scalar registers and the offset in one
// vector register, shared by all fields of a node (field arrays up to 4 GiB;
// larger ones take the 64-bit variant of the step kernel).
template <class T>
__device__ __forceinline__ T gload_at(const T* base, unsigned boff) {
  return *(const __attribute__((address_space(1))) T*)((const char*)base + boff);
}
template <class T>
__device__ __forceinline__ void gstore_at(T* base, unsigned boff, T v) {
  *(__attribute__((address_space(1))) T*)((char*)base + boff) = v;
}

// Wet after (a) and before (b).  A node flooded in (b) carries F_FLD, so a
// post-(b) view answers this as its post-(a) state did: (b) changes no other
// node, and a flooded node was dry before it.
__device__ __forceinline__ bool wet_before_b(int f) {
  return (f & (F_EX | F_WET | F_FLD)) == (F_EX | F_WET);
}

// ---------------------------------------------------------------------------
// FP64 node stages (literal form).
// ---------------------------------------------------------------------------
#ifndef CLF_PREFETCH64
#define CLF_PREFETCH64 2
#endif
#ifndef CLF_PREFETCH32
#define CLF_PREFETCH32 2
#endif
// Rows of the 2-D march are prefetched into registers P::kPrefetch rows
// ahead of use, or (G_LDSROWS, FP32 variants for grids that stream from
// HBM) staged in LDS through direct global-to-LDS loads kLdsAhead rows
// ahead, with the maxwave of their output rows.  Staging gains where the
// rows come from HBM; on a grid that the last-level cache holds, and in the
// FP64 kernel, whose vector ALU is the busier unit, its extra instructions
// cost more than it saves.
constexpr int kLdsSlots = 4;               // LDS row slots per wavefront (a power of 2)
constexpr int kLdsAhead = kLdsSlots - 1;   // rows in flight ahead of the one in use

// Wait until at most N vector memory operations of this wavefront are
// outstanding.  Vector memory operations complete in issue order, so this
// waits for every operation issued before the last N.  The memory clobber
// keeps the compiler from moving LDS reads above the wait.
template <int N>
__device__ __forceinline__ void wait_vmem() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// A wavefront-uniform pointer passed through readfirstlane: the compiler can
// then not fold per-lane terms into it, and forms it with scalar
// instructions.
__device__ __forceinline__ const char* uniform_ptr(const char* p) {
  const unsigned long long a = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return (const char*)(((unsigned long long)hi << 32) | lo);
}

// One direct global-to-LDS load of a dword per lane: lane l's dword lands at
// lds + 4 l (bytes).
__device__ __forceinline__ void dma_dword(const char* g, void* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                   (__attribute__((address_space(3))) void*)lds, 4, 0, 0);
}

// This lane's values of a row staged in LDS: four fields `stride` bytes apart
// from byte address a, and the maxwave pair from am.  The reads are written
// out here, with their wait in the same block, because the compiler would
// otherwise wait for every direct-to-LDS load still in flight before any LDS
// read; the order against those loads is kept by wait_vmem before this.
template <class R>
__device__ __forceinline__ void lds_row(unsigned a, unsigned am, R& h, R& d, R& u, R& v, R& e,
                                        R& s2);
template <>
__device__ __forceinline__ void lds_row<double>(unsigned a, unsigned am, double& h, double& d,
                                                double& u, double& v, double& e, double& s2) {
  asm volatile(
      "ds_read_b64 %0, %6\n\t"
      "ds_read_b64 %1, %6 offset:512\n\t"
      "ds_read_b64 %2, %6 offset:1024\n\t"
      "ds_read_b64 %3, %6 offset:1536\n\t"
      "ds_read_b64 %4, %7\n\t"
      "ds_read_b64 %5, %7 offset:512\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h), "=&v"(d), "=&v"(u), "=&v"(v), "=&v"(e), "=&v"(s2)
      : "v"(a), "v"(am)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_row<float>(unsigned a, unsigned am, float& h, float& d,
                                               float& u, float& v, float& e, float& s2) {
  asm volatile(
      "ds_read_b32 %0, %6\n\t"
      "ds_read_b32 %1, %6 offset:256\n\t"
      "ds_read_b32 %2, %6 offset:512\n\t"
      "ds_read_b32 %3, %6 offset:768\n\t"
      "ds_read_b32 %4, %7\n\t"
      "ds_read_b32 %5, %7 offset:256\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h), "=&v"(d), "=&v"(u), "=&v"(v), "=&v"(e), "=&v"(s2)
      : "v"(a), "v"(am)
      : "memory");
}

template <class T>
__device__ __forceinline__ unsigned lds_addr(T* p) {
  return (unsigned)(uintptr_t)(__attribute__((address_space(3))) T*)p;
}

struct P64 {
  typedef double R;
  // march rows between a row's load and its use (latency cover)
  static constexpr int kPrefetch = CLF_PREFETCH64;
  // post-(a) view of a node along the sweep line: w normal, t tangential
  struct A { double H, w, t, D; int f; int pad; };
  // post-(b) view: c = sqrt(g H) on wet nodes
  struct B { double H, w, t, D, c; int f; int src; };
  // what the neighbours need from a post-(b) node
  struct Bx { double w, t, D, c; int f; int pad; };
  // post-(d) view
  struct C { double H, w, t; };
  struct Cx { double H, w; };

  struct Par {
    double dt, hdt, dt2, hmin, gn2, inv16g, dwall;
    int flags;
  };

  // (a) marks the wet nodes. A node in the grid at or below the threshold is
  // dry; its values are not emptied here, because nothing that reaches a
  // result reads them: its neighbours take its mirror ghost in (c)+(d), (b)
  // reads wet neighbours and the dry node's own depth only, (b) overwrites
  // a flooded node, and (d) replaces its own update by the dry state. (The
  // oracle empties it, as step (a) is written; the results are the same
  // bits.)
  static __device__ __forceinline__ void stage_a(A& a, const Par& p) {
    const bool ex = (a.f & F_EX) != 0;
    const bool wet = a.H > p.hmin;
    a.f |= (ex && wet) ? F_WET : 0;
  }

  static __device__ __forceinline__ B stage_b(const A& l, const A& c, const A& r, const Par& p) {
    B b;
    b.H = c.H; b.w = c.w; b.t = c.t; b.D = c.D; b.f = c.f; b.src = 0;
    const bool blocked = (p.flags & G_WALLMODE) && (c.D < p.dwall);
    if ((c.f & F_EX) && !(c.f & (F_WET | F_FIX)) && !blocked) {
      bool qL = false, qR = false;
      double fL = 0.0, fR = 0.0;
      if (wet_before_b(l.f)) {
        fL = (l.H - l.D) + c.D;
        qL = fL > p.hmin;
      }
      if (wet_before_b(r.f)) {
        fR = (r.H - r.D) + c.D;
        qR = fR > p.hmin;
      }
      int s = 0;
      if (qL && qR) s = (fL > fR) ? -1 : ((fR > fL) ? 1 : 2);
      else if (qL) s = -1;
      else if (qR) s = 1;
      if (s != 0) {
        b.src = s;
        b.f |= F_WET | F_FLD;
        b.H = p.hmin;
        if (s == 2) {
          b.w = 0.5 * (l.w + r.w);
          b.t = 0.5 * (l.t + r.t);
        } else if (s == -1) {
          b.w = l.w; b.t = l.t;
        } else {
          b.w = r.w; b.t = r.t;
        }
      }
    }
    return b;
  }

  // post-(b) view of a node when no lane of the wavefront can flood
  static __device__ __forceinline__ B stage_b_copy(const A& c) {
    B b;
    b.H = c.H; b.w = c.w; b.t = c.t; b.D = c.D; b.f = c.f; b.src = 0; b.c = 0.0;
    return b;
  }

  // a dry node next to a wet one (flags of the neighbours after (a))
  static __device__ __forceinline__ bool flood_candidate(int f, int fl, int fr) {
    return (f & F_EX) && !(f & (F_WET | F_FIX)) && (wet_before_b(fl) || wet_before_b(fr));
  }
  // a post-(b) node as the neighbour of a node in (b): the fields that
  // neighbour reads are those of its post-(a) state (wet_before_b)
  static __device__ __forceinline__ A pre_b(const B& b) {
    A a;
    a.H = b.H; a.w = b.w; a.t = b.t; a.D = b.D; a.f = b.f; a.pad = 0;
    return a;
  }

  // c = sqrt(g h) on every node: dry nodes hold h = 0 (so c = 0), and c of
  // a node outside the grid is never used (it is no real neighbour)
  // c = sqrt(g H).  Wet nodes hold H >= h_min and dry ones H = 0, so where
  // g h_min >= 2^-767 the argument the sweep uses is 0 or at least that
  // large, and the square root skips the rescaling of smaller arguments.
  // Both forms round correctly there and agree bit for bit; grids with a
  // smaller h_min (G_TINYH) run the general kernel, which keeps the full form.
  static __device__ __forceinline__ void set_c(B& b, const Par& p) {
    const double x = kG * b.H;
    b.c = (p.flags & G_TINYH) ? sqrt(x) : sqrt_large(x);
  }
  // Square root of 0 or of x >= 2^-767: an estimate of 1/sqrt(x), one
  // coupled Newton step on sqrt(x) and 1/(2 sqrt(x)), then two corrections
  // of sqrt(x) by its residual x - s^2 (Goldschmidt's iteration with a
  // final correction, as in Markstein's correctly rounded square root).
  // 0 and +inf are returned unchanged.
  static __device__ __forceinline__ double sqrt_large(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    // class mask: -0 (bit 5), +0 (bit 6), +inf (bit 9)
    return __builtin_amdgcn_class(x, 0x260) ? x : g;
  }

  static __device__ __forceinline__ Bx bx(const B& b) {
    Bx x;
    x.w = b.w; x.t = b.t; x.D = b.D; x.c = b.c; x.f = b.f; x.pad = 0;
    return x;
  }

  static __device__ __forceinline__ double qhat(double la, double xa, double Da, double lb,
                                                double xb, double Db, double inv) {
    double s = lb + la;
    double h = 0.5 * s;
    double dx = xb - xa;
    double m = h * dx;
    double dd = Db - Da;
    double gd = kG * dd;
    double num = m - gd;
    return num * inv;
  }

  static __device__ __forceinline__ double qhat_t(double la, double xa, double lb, double xb,
                                                  double inv) {
    double s = lb + la;
    double h = 0.5 * s;
    double dx = xb - xa;
    double m = h * dx;
    return m * inv;
  }

  static __device__ __forceinline__ double advance(const Par& p, double xi, double lam, double QL,
                                                   double QR, double Qc, double iS) {
    double a3;
    if (p.flags & G_SOLVER1) {
      double a2 = p.dt * Qc;
      a3 = xi - a2;
    } else {
      double a1 = QL + QR;
      double a2 = p.hdt * a1;
      a3 = xi - a2;
    }
    double b1 = QR - QL;
    double b2 = lam * p.dt2;
    double b3 = b2 * b1;
    double b4 = b3 * iS;
    return a3 + b4;
  }

  // eqQ across the interface a|b for the P, M and T families.  Between two
  // real wet nodes the value is the same bits whichever node evaluates it
  // (the sums are taken b + a in both), so a sweep computes it once per
  // interface and hands it to the node on the other side.
  struct Fx { double P, M, T; };
  static __device__ __forceinline__ Fx flux(double wa, double ca, double Da, double ta,
                                            double wb, double cb, double Db, double tb,
                                            double inv) {
    Fx f;
    f.P = qhat(wa + ca, wa + 2.0 * ca, Da, wb + cb, wb + 2.0 * cb, Db, inv);
    f.M = qhat(wa - ca, wa - 2.0 * ca, Da, wb - cb, wb - 2.0 * cb, Db, inv);
    f.T = qhat_t(wa, ta, wb, tb, inv);
    return f;
  }
  // The value an interface a|b must have for whichever of its two nodes is
  // real (inside the grid and wet after (b)): with both real it is eqQ over
  // a and b; with one real, eqQ between that node and its own mirror ghost
  // (h, -w, t, d).  Selecting the operands first gives all three cases from
  // one evaluation; with neither real the value is never used.
  static __device__ __forceinline__ Fx interface(const B& a, bool areal, const Bx& b, bool breal,
                                                 double inv) {
    const double aw = areal ? a.w : -b.w, ac = areal ? a.c : b.c;
    const double bw = breal ? b.w : -a.w, bc = breal ? b.c : a.c;
    // a ghost copies the node's own d and t, so across a ghost both
    // differences are exactly zero: select the differences, not the operands
    const bool both = areal && breal;
    const double dD = both ? b.D - a.D : 0.0, dt = both ? b.t - a.t : 0.0;
    Fx f;
    f.P = qhat_d(aw + ac, aw + 2.0 * ac, bw + bc, bw + 2.0 * bc, dD, inv);
    f.M = qhat_d(aw - ac, aw - 2.0 * ac, bw - bc, bw - 2.0 * bc, dD, inv);
    const double s = bw + aw;
    const double h = 0.5 * s;
    f.T = (h * dt) * inv;
    return f;
  }
  // qhat with the depth difference given
  static __device__ __forceinline__ double qhat_d(double la, double xa, double lb, double xb,
                                                  double dd, double inv) {
    double s = lb + la;
    double h = 0.5 * s;
    double dx = xb - xa;
    double m = h * dx;
    double gd = kG * dd;
    double num = m - gd;
    return num * inv;
  }

  // (d) from the values of the interfaces on each side of the node
  static __device__ __forceinline__ C stage_cd_shared(const B& c, const Fx& FL, const Fx& FR,
                                                      double iS, double tanR, const Par& p) {
    return finish(c, FL.P, FR.P, FL.M, FR.M, FL.T, FR.T, 0.0, 0.0, 0.0, iS, tanR, p);
  }

  // (d) with every neighbour evaluated in place (needed by solver1, whose
  // centred term spans both neighbours)
  // Ghost beyond an open (radiating) edge: it carries the node's outgoing
  // Riemann invariant and the still-water incoming one (p0 = 2 sqrt(g d) from
  // the left, q0 = -2 sqrt(g d) from the right); w = (p + q)/2 and
  // c = max((p - q)/4, 0).
  static __device__ __forceinline__ void open_ghost(double w, double c, double D, bool right,
                                                    double& wg, double& cg) {
    const double c0 = sqrt(kG * (D > 0.0 ? D : 0.0));
    const double pp = right ? w + 2.0 * c : 2.0 * c0;
    const double qq = right ? -2.0 * c0 : w - 2.0 * c;
    wg = 0.5 * (pp + qq);
    const double cc = 0.25 * (pp - qq);
    cg = cc < 0.0 ? 0.0 : cc;
  }

  static __device__ __forceinline__ C stage_cd(const Bx& l, const B& c, const Bx& r, double iL,
                                               double iR, double iS, double tanR, const Par& p) {
    const bool lreal = (l.f & (F_EX | F_WET)) == (F_EX | F_WET);
    const bool rreal = (r.f & (F_EX | F_WET)) == (F_EX | F_WET);
    const double Cw = c.w, Ct = c.t, CD = c.D, Cc = c.c;
    // mirror ghost (h_k, -w_k, t_k, d_k) where the neighbour is dry or missing
    double Lw = lreal ? l.w : -Cw, Lc = lreal ? l.c : Cc;
    double Rw = rreal ? r.w : -Cw, Rc = rreal ? r.c : Cc;
    const double Lt = lreal ? l.t : Ct, LD = lreal ? l.D : CD;
    const double Rt = rreal ? r.t : Ct, RD = rreal ? r.D : CD;
    if (p.flags & G_OPEN_ANY) {
      if (!lreal && (l.f & F_OPEN)) open_ghost(Cw, Cc, CD, false, Lw, Lc);
      if (!rreal && (r.f & F_OPEN)) open_ghost(Cw, Cc, CD, true, Rw, Rc);
    }
    const Fx QL = flux(Lw, Lc, LD, Lt, Cw, Cc, CD, Ct, iL);
    const Fx QR = flux(Cw, Cc, CD, Ct, Rw, Rc, RD, Rt, iR);
    double QPc = 0.0, QMc = 0.0, QTc = 0.0;
    if (p.flags & G_SOLVER1) {
      const Fx Qc = flux(Lw, Lc, LD, Lt, Rw, Rc, RD, Rt, iS);
      QPc = Qc.P; QMc = Qc.M; QTc = Qc.T;
    }
    return finish(c, QL.P, QR.P, QL.M, QR.M, QL.T, QR.T, QPc, QMc, QTc, iS, tanR, p);
  }

  static __device__ __forceinline__ C finish(const B& c, double QPL, double QPR, double QML,
                                             double QMR, double QTL, double QTR, double QPc,
                                             double QMc, double QTc, double iS, double tanR,
                                             const Par& p) {
    // Every lane computes the update; dry and held nodes select their value
    // at the end (a wet node's result is the same bits either way).
    const double Cw = c.w, Ct = c.t, Cc = c.c;
    const double xPC = Cw + 2.0 * Cc, lPC = Cw + Cc, xMC = Cw - 2.0 * Cc, lMC = Cw - Cc;
    double Pn = advance(p, xPC, lPC, QPL, QPR, QPc, iS);
    double Mn = advance(p, xMC, lMC, QML, QMR, QMc, iS);
    double Tn = advance(p, Ct, Cw, QTL, QTR, QTc, iS);
    if (tanR != 0.0) {
      double s1 = p.dt * Cc;
      double s2 = s1 * Cw;
      double s3 = s2 * tanR;
      Pn = Pn + s3;
      Mn = Mn - s3;
    }
    // Manning friction: fr = dt g n^2 |U| / h^(4/3) with h^(-1/3) from a
    // single-precision seed (hardware log2 / exp2) and one Newton step
    // r <- r (4 - h r^3) / 3 (relative error about 1e-13), and |U| from the
    // square root without argument rescaling (speeds below 1e-115 m/s count
    // as 0): no libm cbrt and no division. The friction term agrees with the
    // direct form to about 1e-13 of itself; the rest of the update is the
    // oracle's operation order.
    double fr = 0.0;
    if (p.flags & G_FRICTION) {
      const double s2 = Cw * Cw + Ct * Ct;
      const double sp = s2 < 0x1p-767 ? 0.0 : sqrt_large(s2);
      const double h = c.H;
      double r = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)h) * (-1.0f / 3.0f));
      r = r * ((4.0 - h * ((r * r) * r)) * (1.0 / 3.0));
      const double r2 = r * r;
      fr = ((p.dt * p.gn2) * sp) * (r2 * r2);
      if (!(p.flags & G_FRIC_SEMI)) {
        // the -alpha dt term of solver2 / solver1 on p and q (old level),
        // alpha dt = fr w with fr capped at 1: friction does not reverse the flow
        const double a = (fr < 1.0 ? fr : 1.0) * Cw;
        Pn = Pn - a;
        Mn = Mn - a;
      }
    }
    double ws = Pn + Mn;
    double wv = 0.5 * ws;
    double dd = Pn - Mn;
    dd = (dd < 0.0) ? 0.0 : dd;
    double Hv = (dd * dd) * p.inv16g;
    // option: semi-implicit friction on the normal velocity
    if ((p.flags & G_FRICTION) && (p.flags & G_FRIC_SEMI)) wv = wv / (1.0 + fr);
    const bool wet = (c.f & F_WET) != 0;
    C o;
    o.H = wet ? Hv : 0.0;
    o.w = wet ? wv : 0.0;
    o.t = wet ? Tn : 0.0;
    if ((p.flags & (G_FIX_W | G_FIX_E | G_FIX_S | G_FIX_N)) && (c.f & F_FIX)) {
      o.H = c.H; o.w = c.w; o.t = c.t;
    }
    return o;
  }

  static __device__ __forceinline__ Cx cx(const C& c) {
    Cx x;
    x.H = c.H; x.w = c.w;
    return x;
  }

  static __device__ __forceinline__ void stage_e(C& o, const Cx& l, const Cx& r, int src,
                                                 double /*D*/) {
    // source on the left (src -1), right (+1), tie (2) or none (0)
    const double m = (r.H < l.H) ? r.H : l.H;
    const double sh = (src == -1) ? l.H : r.H;
    const double cap = 0.5 * ((src == 2) ? m : sh);
    o.H = (src != 0 && o.H > cap) ? cap : o.H;
    const double sw = (src == -1) ? l.w : r.w;
    const bool capw = (src == -1) ? (o.w > sw) : ((src == 1) && (o.w < sw));
    o.w = capw ? sw : o.w;
  }

  static __device__ __forceinline__ bool wet_out(const C& o, double /*D*/, const Par& p) {
    return o.H > p.hmin;
  }
  static __device__ __forceinline__ double eta_out(const C& o, double D) { return o.H - D; }
};

// ---------------------------------------------------------------------------
// FP32 node stages.  The stored state is the surface eta (field "H" of the
// views holds eta), so that a node at rest over 4000 m keeps its surface to
// the last bit.  The update is the algebraically identical perturbation form
// of eqQ and solver2:
//   Q_P = [ (l_a + l_b)/2 (w_b - w_a) + g (eta_b - eta_a)
//           + g (h_b - h_a) (w_a + w_b)/(c_a + c_b) ] / dx,   Q_M: minus sign,
//   p' - p = -dt/2 (QL + QR) + lambda dt^2 (QR - QL)/(dx_l + dx_r),
//   u' = u + (dp + dq)/2,  h' = h + d (8c + d)/16g with d = dp - dq,
// which is zero to the bit for a lake at rest.  Products that feed a sum
// are fused (one rounding instead of two; the FP64 stages keep the written
// order with separate roundings, which the oracle shares).  A fused
// multiply-add of negated operands is the negated result, so mirror-image
// nodes still get mirror-image bits.
// ---------------------------------------------------------------------------
struct P32 {
  typedef float R;
  static constexpr int kPrefetch = CLF_PREFETCH32;
  static constexpr float kGf = 9.81f;
  struct A { float H, w, t, D; int f; int pad; };          // H = eta
  struct B { float H, w, t, D, c, h; int f; int src; };   // h = total height
  struct Bx { float w, t, D, c, H; int f; };
  struct C { float H, w, t, h; };                         // eta', u', v', h'
  struct Cx { float h, w; };

  struct Par {
    float dt, hdt, dt2, hmin, gn2, inv16g, dwall;
    int flags;
  };

  // (a): as in the FP64 stages, dry nodes are only marked
  static __device__ __forceinline__ void stage_a(A& a, const Par& p) {
    const bool ex = (a.f & F_EX) != 0;
    const bool wet = a.D + a.H > p.hmin;
    a.f |= (ex && wet) ? F_WET : 0;
  }

  static __device__ __forceinline__ B stage_b(const A& l, const A& c, const A& r, const Par& p) {
    B b;
    b.H = c.H; b.w = c.w; b.t = c.t; b.D = c.D; b.f = c.f; b.src = 0;
    b.h = c.D + c.H;
    const bool blocked = (p.flags & G_WALLMODE) && (c.D < p.dwall);
    if ((c.f & F_EX) && !(c.f & (F_WET | F_FIX)) && !blocked) {
      bool qL = false, qR = false;
      float fL = 0.f, fR = 0.f;
      if (wet_before_b(l.f)) {
        fL = l.H + c.D;
        qL = fL > p.hmin;
      }
      if (wet_before_b(r.f)) {
        fR = r.H + c.D;
        qR = fR > p.hmin;
      }
      int s = 0;
      if (qL && qR) s = (fL > fR) ? -1 : ((fR > fL) ? 1 : 2);
      else if (qL) s = -1;
      else if (qR) s = 1;
      if (s != 0) {
        b.src = s;
        b.f |= F_WET | F_FLD;
        b.h = p.hmin;
        b.H = p.hmin - c.D;
        if (s == 2) {
          b.w = 0.5f * (l.w + r.w);
          b.t = 0.5f * (l.t + r.t);
        } else if (s == -1) {
          b.w = l.w; b.t = l.t;
        } else {
          b.w = r.w; b.t = r.t;
        }
      }
    }
    return b;
  }

  static __device__ __forceinline__ B stage_b_copy(const A& c) {
    B b;
    b.H = c.H; b.w = c.w; b.t = c.t; b.D = c.D; b.f = c.f; b.src = 0; b.c = 0.f;
    b.h = c.D + c.H;
    return b;
  }

  static __device__ __forceinline__ bool flood_candidate(int f, int fl, int fr) {
    return (f & F_EX) && !(f & (F_WET | F_FIX)) && (wet_before_b(fl) || wet_before_b(fr));
  }
  static __device__ __forceinline__ A pre_b(const B& b) {
    A a;
    a.H = b.H; a.w = b.w; a.t = b.t; a.D = b.D; a.f = b.f; a.pad = 0;
    return a;
  }

  static __device__ __forceinline__ void set_c(B& b, const Par&) {
    b.c = __builtin_amdgcn_sqrtf(kGf * b.h);
  }

  static __device__ __forceinline__ Bx bx(const B& b) {
    Bx x;
    x.w = b.w; x.t = b.t; x.D = b.D; x.c = b.c; x.H = b.H; x.f = b.f;
    return x;
  }

  // perturbation-form Q of the P (sg = +1) or M (sg = -1) family across the
  // interface a|b
  static __device__ __forceinline__ float qpm(float sg, float wa, float ca, float ea, float Da,
                                              float wb, float cb, float eb, float Db, float inv) {
    const float sw = wb + wa, dw = wb - wa, sc = cb + ca;
    const float de = eb - ea;
    const float dh = (Db - Da) + de;
    const float lam2 = sw + sg * sc;
    const float cross = kGf * dh * (sw * __builtin_amdgcn_rcpf(sc));
    return __builtin_fmaf(0.5f * lam2, dw, __builtin_fmaf(kGf, de, sg * cross)) * inv;
  }

  static __device__ __forceinline__ float qt(float wa, float ta, float wb, float tb, float inv) {
    return (0.5f * (wb + wa) * (tb - ta)) * inv;
  }

  // dt2iS = dt^2 / (Delta_l + Delta_r), formed once per node for the three
  // families
  static __device__ __forceinline__ float incr(const Par& p, float lam, float QL, float QR, float Qc,
                                               float dt2iS) {
    const float first = (p.flags & G_SOLVER1) ? -(p.dt * Qc) : -(p.hdt * (QL + QR));
    return __builtin_fmaf(lam * (QR - QL), dt2iS, first);
  }

  // the interface values of the three families (shared between the two
  // nodes of a real wet interface, as in the FP64 stages)
  struct Fx { float P, M, T; };
  static __device__ __forceinline__ Fx flux(float wa, float ca, float ea, float Da, float ta,
                                            float wb, float cb, float eb, float Db, float tb,
                                            float inv) {
    Fx f;
    f.P = qpm(1.f, wa, ca, ea, Da, wb, cb, eb, Db, inv);
    f.M = qpm(-1.f, wa, ca, ea, Da, wb, cb, eb, Db, inv);
    f.T = qt(wa, ta, wb, tb, inv);
    return f;
  }
  static __device__ __forceinline__ Fx interface(const B& a, bool areal, const Bx& b, bool breal,
                                                 float inv) {
    const float aw = areal ? a.w : -b.w, ac = areal ? a.c : b.c;
    const float bw = breal ? b.w : -a.w, bc = breal ? b.c : a.c;
    // across a ghost the surface, depth and tangential differences are zero
    const bool both = areal && breal;
    const float de = both ? b.H - a.H : 0.f, dD = both ? b.D - a.D : 0.f,
                dt = both ? b.t - a.t : 0.f;
    Fx f;
    f.P = qpm_d(1.f, aw, ac, bw, bc, de, dD, inv);
    f.M = qpm_d(-1.f, aw, ac, bw, bc, de, dD, inv);
    f.T = (0.5f * (bw + aw) * dt) * inv;
    return f;
  }
  // qpm with the surface and depth differences given
  static __device__ __forceinline__ float qpm_d(float sg, float wa, float ca, float wb, float cb,
                                                float de, float dD, float inv) {
    const float sw = wb + wa, dw = wb - wa, sc = cb + ca;
    const float dh = dD + de;
    const float lam2 = sw + sg * sc;
    const float cross = kGf * dh * (sw * __builtin_amdgcn_rcpf(sc));
    return __builtin_fmaf(0.5f * lam2, dw, __builtin_fmaf(kGf, de, sg * cross)) * inv;
  }

  static __device__ __forceinline__ C stage_cd_shared(const B& c, const Fx& FL, const Fx& FR,
                                                      float iS, float tanR, const Par& p) {
    return finish(c, FL.P, FR.P, FL.M, FR.M, FL.T, FR.T, 0.f, 0.f, 0.f, iS, tanR, p);
  }

  // Ghost beyond an open edge (as in the FP64 stages).  Its surface differs
  // from the node's by the height difference (c_g^2 - c^2)/g, formed as a
  // product of differences so that it is exactly zero at rest.
  static __device__ __forceinline__ void open_ghost(float w, float c, float e, float D, bool right,
                                                    float& wg, float& cg, float& eg) {
    const float c0 = __builtin_amdgcn_sqrtf(kGf * (D > 0.f ? D : 0.f));
    const float pp = right ? w + 2.f * c : 2.f * c0;
    const float qq = right ? -2.f * c0 : w - 2.f * c;
    wg = 0.5f * (pp + qq);
    const float cc = 0.25f * (pp - qq);
    cg = cc < 0.f ? 0.f : cc;
    eg = e + ((cg - c) * (cg + c)) * (1.f / kGf);
  }

  static __device__ __forceinline__ C stage_cd(const Bx& l, const B& c, const Bx& r, float iL,
                                               float iR, float iS, float tanR, const Par& p) {
    const bool lreal = (l.f & (F_EX | F_WET)) == (F_EX | F_WET);
    const bool rreal = (r.f & (F_EX | F_WET)) == (F_EX | F_WET);
    const float Cw = c.w, Ct = c.t, CD = c.D, Cc = c.c, Ce = c.H;
    // mirror ghost where the neighbour is dry or missing
    float Lw = lreal ? l.w : -Cw, Lc = lreal ? l.c : Cc, Le = lreal ? l.H : Ce;
    float Rw = rreal ? r.w : -Cw, Rc = rreal ? r.c : Cc, Re = rreal ? r.H : Ce;
    const float Lt = lreal ? l.t : Ct, LD = lreal ? l.D : CD;
    const float Rt = rreal ? r.t : Ct, RD = rreal ? r.D : CD;
    if (p.flags & G_OPEN_ANY) {
      if (!lreal && (l.f & F_OPEN)) open_ghost(Cw, Cc, Ce, CD, false, Lw, Lc, Le);
      if (!rreal && (r.f & F_OPEN)) open_ghost(Cw, Cc, Ce, CD, true, Rw, Rc, Re);
    }
    const Fx QL = flux(Lw, Lc, Le, LD, Lt, Cw, Cc, Ce, CD, Ct, iL);
    const Fx QR = flux(Cw, Cc, Ce, CD, Ct, Rw, Rc, Re, RD, Rt, iR);
    float QPc = 0.f, QMc = 0.f, QTc = 0.f;
    if (p.flags & G_SOLVER1) {
      const Fx Qc = flux(Lw, Lc, Le, LD, Lt, Rw, Rc, Re, RD, Rt, iS);
      QPc = Qc.P; QMc = Qc.M; QTc = Qc.T;
    }
    return finish(c, QL.P, QR.P, QL.M, QR.M, QL.T, QR.T, QPc, QMc, QTc, iS, tanR, p);
  }

  static __device__ __forceinline__ C finish(const B& c, float QPL, float QPR, float QML,
                                             float QMR, float QTL, float QTR, float QPc,
                                             float QMc, float QTc, float iS, float tanR,
                                             const Par& p) {
    const float Cw = c.w, Ct = c.t, CD = c.D, Cc = c.c, Ce = c.H;
    const float dt2iS = p.dt2 * iS;
    float dP = incr(p, Cw + Cc, QPL, QPR, QPc, dt2iS);
    float dM = incr(p, Cw - Cc, QML, QMR, QMc, dt2iS);
    const float dT = incr(p, Cw, QTL, QTR, QTc, dt2iS);
    if (tanR != 0.f) {
      const float s3 = ((p.dt * Cc) * Cw) * tanR;
      dP = dP + s3;
      dM = dM - s3;
    }
    float wv = __builtin_fmaf(0.5f, dP + dM, Cw);
    const float dd = dP - dM;
    const float dh = (dd * __builtin_fmaf(8.f, Cc, dd)) * p.inv16g;
    const bool drained = __builtin_fmaf(4.f, Cc, dd) < 0.f;
    if (p.flags & G_FRICTION) {
      // fr = dt g n^2 |U| h^(-4/3) through the hardware log2 / exp2.  The
      // -alpha dt term on p and q moves u by -alpha dt and leaves p - q
      // (hence h) unchanged, so it is applied to u directly.
      const float sp = __builtin_amdgcn_sqrtf(__builtin_fmaf(Cw, Cw, Ct * Ct));
      const float hm43 = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(c.h) * (-4.0f / 3.0f));
      const float fr = ((p.dt * p.gn2) * sp) * hm43;
      if (p.flags & G_FRIC_SEMI)
        wv = wv * __builtin_amdgcn_rcpf(1.f + fr);
      else
        wv = __builtin_fmaf(-(fr < 1.f ? fr : 1.f), Cw, wv);
    }
    const bool wet = (c.f & F_WET) != 0;
    // a drained or dry node holds no water (one select per field: the two
    // conditions are combined as lane masks)
    const bool holds = wet && !drained;
    C o;
    o.H = holds ? Ce + dh : -CD;
    o.w = wet ? wv : 0.f;
    o.t = wet ? Ct + dT : 0.f;
    o.h = holds ? c.h + dh : 0.f;
    if ((p.flags & (G_FIX_W | G_FIX_E | G_FIX_S | G_FIX_N)) && (c.f & F_FIX)) {
      o.H = c.H; o.w = c.w; o.t = c.t; o.h = c.h;
    }
    return o;
  }

  static __device__ __forceinline__ Cx cx(const C& c) {
    Cx x;
    x.h = c.h; x.w = c.w;
    return x;
  }

  static __device__ __forceinline__ void stage_e(C& o, const Cx& l, const Cx& r, int src,
                                                 float D) {
    const float m = (r.h < l.h) ? r.h : l.h;
    const float sh = (src == -1) ? l.h : r.h;
    const float cap = 0.5f * ((src == 2) ? m : sh);
    const bool caph = src != 0 && o.h > cap;
    o.h = caph ? cap : o.h;
    o.H = caph ? cap - D : o.H;
    const float sw = (src == -1) ? l.w : r.w;
    const bool capw = (src == -1) ? (o.w > sw) : ((src == 1) && (o.w < sw));
    o.w = capw ? sw : o.w;
  }

  static __device__ __forceinline__ bool wet_out(const C& o, float D, const Par& p) {
    return D + o.H > p.hmin;
  }
  static __device__ __forceinline__ float eta_out(const C& o, float /*D*/) { return o.H; }
};

// ---------------------------------------------------------------------------
// The march kernel.
// ---------------------------------------------------------------------------
template <class P>
struct Ctx {
  typedef typename P::R R;
  const R* H;
  const R* U;
  const R* V;
  R* Ho;
  R* Uo;
  R* Vo;
  const R* D;
  R* emax;
  R* smax2;
  const R* yib;
  const R* yisb;
  const R* tanR;
  int nx, ny, gflags;
  typename P::Par par;
};

__device__ __forceinline__ int ring_flag(int gflags, int xc, int r, int nx, int ny) {
  return ((gflags & G_FIX_W) && xc == 0) || ((gflags & G_FIX_E) && xc == nx - 1) ||
                 ((gflags & G_FIX_S) && r == 0) || ((gflags & G_FIX_N) && r == ny - 1)
             ? F_FIX
             : 0;
}

// a node outside the grid beyond an open edge (its ghost is the open one)
__device__ __forceinline__ int open_flag(int gflags, int xc, int r, int nx, int ny) {
  return ((gflags & G_OPEN_W) && xc < 0) || ((gflags & G_OPEN_E) && xc >= nx) ||
                 ((gflags & G_OPEN_S) && r < 0) || ((gflags & G_OPEN_N) && r >= ny)
             ? F_OPEN
             : 0;
}

// a neighbour that takes part in (d) with its own values: inside the grid
// and wet after (b); any other neighbour is replaced by the mirror ghost
__device__ __forceinline__ bool is_real(int f) { return (f & (F_EX | F_WET)) == (F_EX | F_WET); }

// x-sweep of one row across the wavefront.  In: this lane's node along x
// (w = u, t = v), unflagged wet state.  Out: post-sweep (H, u, v), valid on
// lanes 3..60.  The flooding exchange of step (b) and the limiter exchange
// of step (e) run only when some lane of the wavefront needs them.
template <class P>
__device__ __forceinline__ typename P::C xsweep_row(typename P::A a, typename P::R iL,
                                                    typename P::R iR, typename P::R iS,
                                                    const typename P::Par& par) {
  typedef typename P::A A;
  typedef typename P::B B;
  typedef typename P::C C;
  P::stage_a(a, par);
  const int fl = lane_prev_i(a.f), fr = lane_next_i(a.f);
  B b;
  if (__ballot(P::flood_candidate(a.f, fl, fr)) != 0) {
    A al = from_prev(a);
    A ar = from_next(a);
    b = P::stage_b(al, a, ar, par);
  } else {
    b = P::stage_b_copy(a);
  }
  P::set_c(b, par);
  typename P::Bx bx = P::bx(b);
  typename P::Bx br = from_next(bx);
  C c;
  if (par.flags & (G_SOLVER1 | G_OPEN_ANY)) {
    typename P::Bx bl = from_prev(bx);
    c = P::stage_cd(bl, b, br, iL, iR, iS, (typename P::R)0, par);
  } else {
    // each lane evaluates the interface to its right and passes it on
    const typename P::Fx FR = P::interface(b, is_real(b.f), br, is_real(br.f), iR);
    const typename P::Fx FL = from_prev(FR);
    c = P::stage_cd_shared(b, FL, FR, iS, (typename P::R)0, par);
  }
  if (__ballot(b.src != 0) != 0) {
    typename P::Cx cc = P::cx(c);
    typename P::Cx cl = from_prev(cc);
    typename P::Cx cr = from_next(cc);
    P::stage_e(c, cl, cr, b.src, b.D);
  }
  return c;
}

// Per-lane y pipeline: rotating register windows of the stages.  Row r is
// pushed in phase K = (r - first) mod 3; slot indices are compile-time so the
// windows rotate by renaming, not by moves.  After the push of row r:
//   a[(K+2)%3], a[K] = post-(a) rows r-1, r (a[(K+1)%3] is not read)
//   b[(K+1)%3], b[(K+2)%3], b[K] = post-(b) rows r-3, r-2, r-1
//   c[(K+1)%3], c[(K+2)%3], c[K] = post-(d) rows r-4, r-3, r-2
//   F[K] = interface values between rows r-2 and r-1
template <class P>
struct YPipe {
  typename P::A a[3];
  typename P::B b[3];
  typename P::C c[3];
  typename P::Fx F[3];

  __device__ __forceinline__ void reset() {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = typename P::A{};
      b[k] = typename P::B{};
      c[k] = typename P::C{};
      F[k] = typename P::Fx{};
    }
  }
};

// Push row r (y view: w = v, t = u) in phase K of a march in direction D
// (+1: rows in increasing index, -1: decreasing); returns the final state of
// row r - 3D in `out` and its post-(b) view (flags, depth, flood source) in
// `ob`.  The segment writes rows y0..ylast.  SH: interfaces are evaluated
// once and carried to the next push (else each node evaluates both of its
// own).  "Lower" and "upper" below are row indices; a node's stages see its
// lower neighbour as left and its upper neighbour as right in either
// direction, so every node computes the same bits.
template <class P, int K, bool SH, int D>
__device__ __forceinline__ void ypipe_push(YPipe<P>& y, const typename P::A& a_in, int r,
                                           int y0, int ylast, const Ctx<P>& cx,
                                           typename P::C& out, typename P::B& ob) {
  typedef typename P::R R;
  constexpr int K1 = (K + 1) % 3, K2 = (K + 2) % 3;
  // window slots by row: a[K] = r, a[K2] = r - D (likewise b one row behind
  // a, c two rows behind)
  y.a[K] = a_in;
  P::stage_a(y.a[K], cx.par);
  // (b) on row r - D (centre a[K2]).  Its neighbour behind, row r - 2D, is
  // read from that row's post-(b) view b[K2] (wet_before_b), so the post-(a)
  // row dies once (b) has read it.  The flooding logic runs only when some
  // lane of the wavefront has a dry node next to a wet one.
  const typename P::A ab = P::pre_b(y.b[K2]);
  const typename P::A& al = D > 0 ? ab : y.a[K];
  const typename P::A& au = D > 0 ? y.a[K] : ab;
  if (__ballot(P::flood_candidate(y.a[K2].f, al.f, au.f)) != 0)
    y.b[K] = P::stage_b(al, y.a[K2], au, cx.par);
  else
    y.b[K] = P::stage_b_copy(y.a[K2]);
  P::set_c(y.b[K], cx.par);
  // (c)+(d) on row rc = r - 2D (centre b[K2]; b[K] = row r - D, b[K1] = row r - 3D)
  constexpr int BL = D > 0 ? K1 : K, BU = D > 0 ? K : K1;
  const int rc = r - 2 * D;
  R iL = 1, iR = 1, iS = 1, tr = 0;
  if (rc >= 0 && rc < cx.ny) {
    iS = cload(cx.yisb + rc);
    if (cx.par.flags & G_SPHSRC) tr = cload(cx.tanR + rc);
  }
  // the interface between rows k and k + 1 has spacing index k + 1; the edge
  // interfaces of rows 0 and ny - 1 are evaluated from rows -1 and ny
  if (rc >= 0 && rc <= cx.ny) iL = cload(cx.yib + rc);
  if (rc >= -1 && rc < cx.ny) iR = cload(cx.yib + rc + 1);
  // Rows y0 - 1 and ylast + 1 lie outside the segment. Their (c)+(d) values
  // feed only (e) of the adjacent end row, which reads them only when some
  // node of that row was flooded in (b) (the ballot before stage_e), so
  // their update is skipped otherwise. That end row's post-(b) view is b[K]
  // when the march reaches the edge it starts from, and b[K1] at the edge it
  // ends on (the push that also finishes the end row). FP64 only: the
  // issue-bound FP32 kernel loses more to the extra branches than it saves.
  constexpr bool kEdgeSkip = std::is_same<P, P64>::value;
  const bool start_edge = kEdgeSkip && (D > 0 ? rc == y0 - 1 : rc == ylast + 1);
  const bool end_edge = kEdgeSkip && (D > 0 ? rc == ylast + 1 : rc == y0 - 1);
  bool edge_need = true;
  if (start_edge) edge_need = __ballot(y.b[K].src != 0) != 0;
  if (end_edge) edge_need = __ballot(y.b[K1].src != 0) != 0;
  if (!SH || (cx.par.flags & G_SOLVER1)) {
    // rows beyond y0 - 1 and ylast + 1 feed nothing written
    if ((!kEdgeSkip || (rc >= y0 - 1 && rc <= ylast + 1)) && edge_need)
      y.c[K] = P::stage_cd(P::bx(y.b[BL]), y.b[K2], P::bx(y.b[BU]), iL, iR, iS, tr, cx.par);
  } else if (D > 0) {
    // the interface above row rc was evaluated by the previous push (as the
    // one below row rc - 1); evaluate the one below and keep it for the next.
    // Rows above y0 - 1 only feed rows above the segment, so their update is
    // skipped (a uniform branch), and of row y0 - 2 only the interface below
    // it is kept. Row y0 - 1 always keeps its interface below (row y0 reads
    // it); row ylast + 1 is the last row of the march.
    if (rc >= y0 - 2 && (edge_need || !end_edge)) {
      const typename P::Fx FR =
          P::interface(y.b[K2], is_real(y.b[K2].f), P::bx(y.b[BU]), is_real(y.b[BU].f), iR);
      if (rc >= y0 - 1 && edge_need)
        y.c[K] = P::stage_cd_shared(y.b[K2], y.F[K2], FR, iS, tr, cx.par);
      y.F[K] = FR;
    }
  } else {
    // mirrored: the interface below row rc came from the previous push;
    // evaluate the one above (rows below ylast + 1 feed nothing written)
    if (rc <= ylast + 2 && (edge_need || !end_edge)) {
      const typename P::Fx FL =
          P::interface(y.b[BL], is_real(y.b[BL].f), P::bx(y.b[K2]), is_real(y.b[K2].f), iL);
      if (rc <= ylast + 1 && edge_need)
        y.c[K] = P::stage_cd_shared(y.b[K2], FL, y.F[K2], iS, tr, cx.par);
      y.F[K] = FL;
    }
  }
  // (e) on row r - 3D (c[K2]; c[K] = row r - 2D, c[K1] = row r - 4D)
  constexpr int CL = D > 0 ? K1 : K, CU = D > 0 ? K : K1;
  out = y.c[K2];
  ob = y.b[K1];
  if (__ballot(ob.src != 0) != 0)
    P::stage_e(out, P::cx(y.c[CL]), P::cx(y.c[CU]), ob.src, ob.D);
}

// FL: the grid flags this instantiation honours (others are compiled out).
constexpr int FL_FAST = G_SPHSRC;
// runup workloads: the common case plus bottom friction (the explicit
// -alpha dt form), and the same with the semi-implicit option
constexpr int FL_FRIC = G_SPHSRC | G_FRICTION;
constexpr int FL_FRIC_SEMI = FL_FRIC | G_FRIC_SEMI;
// grids driven by boundary forcing (a forcing ring), without and with
// friction. These sets also take wall mode, which changes only step (b) in
// the ballot-guarded flooding branch (in the common set the extra code
// alone cost 0.5-0.8%).
constexpr int FL_RING = FL_FAST | G_WALLMODE | G_FIX_W | G_FIX_E | G_FIX_S | G_FIX_N;
constexpr int FL_RING_FRIC = FL_RING | G_FRICTION | G_FRIC_SEMI;
constexpr int FL_ALL = G_FIX_W | G_FIX_E | G_FIX_S | G_FIX_N | G_WALLMODE | G_SOLVER1 |
                       G_SPHSRC | G_FRICTION | G_FRIC_SEMI | G_TINYH | G_OPEN_ANY;
// grids whose field arrays exceed 4 GiB: the same three flag sets with
// 64-bit addresses
constexpr int FL_FAST_WIDE = FL_FAST | G_WIDE;
constexpr int FL_FAST_LDS = FL_FAST | G_LDSROWS;
constexpr int FL_FRIC_LDS = FL_FRIC | G_LDSROWS;
constexpr int FL_FRIC_WIDE = FL_FRIC | G_WIDE;
constexpr int FL_WIDE = FL_ALL | G_WIDE;

// Lower bound on resident waves per SIMD handed to the register allocator:
// it holds the common FP64 kernel within the three-wave limit of 168 VGPRs.
template <class P, int ORDER, int FL>
constexpr int kStepWaves() {
  return std::is_same<P, P64>::value && FL == FL_FAST && ORDER == ORD_XY ? 3 : 2;
}

template <class P, int ORDER, int FL>
__global__ void __launch_bounds__(WAVE * WAVES_PER_BLOCK)
__attribute__((amdgpu_waves_per_eu(kStepWaves<P, ORDER, FL>())))
step_kernel(const GridDesc* __restrict__ grids, const Tile* __restrict__ tiles, int ntiles,
            StepState* st, int parity, int do_max, int rec_slot) {
  typedef typename P::R R;
  typedef typename P::A A;
  typedef typename P::C C;
  // Each interface is evaluated once and handed to the node on its other
  // side, except in the y pipeline of the FP64 variants with the
  // semi-implicit friction option and of the general variants (both forms
  // give the same bits). In the first, the carried interface values would
  // raise register use past the three resident waves per SIMD (the explicit
  // friction variant fits: 163 VGPRs). In the second, solver1 takes the
  // per-node form at run time, and with both forms in one kernel the FP32
  // pipeline windows were left in scratch memory (four times slower).
  constexpr bool kShY =
      !(std::is_same<P, P64>::value && (FL & G_FRICTION) != 0 && (FL & G_FRIC_SEMI) != 0) &&
      (FL & G_SOLVER1) == 0;
  const int lane = threadIdx.x & (WAVE - 1);
  // the wave index is uniform across the wavefront: say so, so that the
  // tile, the row counter and the row metrics live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  // LDS ring of the 2-D march (G_LDSROWS): per wavefront and slot, a row
  // of h, d, u, v and the maxwave pair of an output row
  constexpr bool kLds = ORDER != ORD_X && (FL & G_LDSROWS) != 0;
  // In FP32 the row slots are padded (7 field rows for 4): 36 KB per
  // workgroup hold residency at 4 workgroups, 16 waves, per CU. Without the
  // padding the kernel fits 5 (96 VGPRs), and the 8000x6000 step was 2%
  // slower at every segment length (more row streams in flight at once).
  constexpr int kLdsFieldRows = kLds && std::is_same<P, P32>::value ? 7 : 4;
  __shared__ R lrow[kLds ? kLdsSlots : 1][WAVES_PER_BLOCK][kLdsFieldRows][WAVE];
  __shared__ R lmw[kLds ? kLdsSlots : 1][WAVES_PER_BLOCK][2][WAVE];
  // grid-stride over the tile list: one tile per wavefront when the grid
  // covers the list, a persistent loop when it is launched smaller
  const int stride = gridDim.x * WAVES_PER_BLOCK;
  int bad = 0;
  for (int tid = blockIdx.x * WAVES_PER_BLOCK + wave; tid < ntiles; tid += stride) {
    Tile tl = tiles[tid];
    tl.grid = __builtin_amdgcn_readfirstlane(tl.grid);
    const bool rev = (tl.grid & kTileReverse) != 0;
    tl.grid &= ~kTileReverse;
    tl.x0 = __builtin_amdgcn_readfirstlane(tl.x0);
    tl.y0 = __builtin_amdgcn_readfirstlane(tl.y0);
    tl.rows = __builtin_amdgcn_readfirstlane(tl.rows);
    tl.g0 = __builtin_amdgcn_readfirstlane(tl.g0);
    tl.gn = __builtin_amdgcn_readfirstlane(tl.gn);
    if (tl.rows <= 0) continue;   // padding slot of the XCD-aware order
    const GridDesc& g = grids[tl.grid];
    Ctx<P> cx;
    cx.H = (const R*)g.H[parity];
    cx.U = (const R*)g.U[parity];
    cx.V = (const R*)g.V[parity];
    cx.Ho = (R*)g.H[parity ^ 1];
    cx.Uo = (R*)g.U[parity ^ 1];
    cx.Vo = (R*)g.V[parity ^ 1];
    cx.D = (const R*)g.D;
    cx.emax = (R*)g.emax;
    cx.smax2 = (R*)g.smax2;
    cx.yib = (const R*)g.yib;
    cx.yisb = (const R*)g.yisb;
    cx.tanR = (const R*)g.tanR;
    cx.nx = g.nx;
    cx.ny = g.ny;
    cx.gflags = g.flags & FL;
    cx.par.dt = (R)g.dt;
    cx.par.hdt = (R)g.hdt;
    cx.par.dt2 = (R)g.dt2;
    cx.par.hmin = (R)g.hmin;
    cx.par.gn2 = (R)g.gn2;
    cx.par.inv16g = (R)g.inv16g;
    cx.par.dwall = (R)g.dwall;
    cx.par.flags = g.flags & FL;
    const R* xfac = (const R*)g.xfac;
    constexpr bool kRing = (FL & (G_FIX_W | G_FIX_E | G_FIX_S | G_FIX_N)) != 0;
    constexpr bool kOpen = (FL & G_OPEN_ANY) != 0;

    const int nx = cx.nx, ny = cx.ny;
    const int xc = tl.x0 - HALO + lane;
    const bool col_in = xc >= 0 && xc < nx;
    const bool out_lane = lane >= HALO && lane < WAVE - HALO && col_in;
    // per-lane x metrics (constant along the march)
    R xiL = 1, xiR = 1, xiS = 1;
    if (col_in) {
      xiL = gload((const R*)g.xib + xc);
      xiS = gload((const R*)g.xisb + xc);
    }
    // the lane left of the grid evaluates the edge interface of column 0
    if (xc >= -1 && xc < nx) xiR = gload((const R*)g.xib + xc + 1);
    // Loads use clamped, always in-bounds indices; nodes outside the grid
    // only lose their existence flag (no divergent branches, no zero fill).
    const int xcl = xc < 0 ? 0 : (xc >= nx ? nx - 1 : xc);
    // node offsets: bytes in 32 bits, or elements (below 2^32) with 64-bit
    // address arithmetic for field arrays above 4 GiB
    constexpr bool kWide = (FL & G_WIDE) != 0;
    auto node = [&](int r, int x) -> unsigned {
      const unsigned k = (unsigned)r * (unsigned)nx + (unsigned)x;
      return kWide ? k : k * (unsigned)sizeof(R);
    };
    auto ld = [&](const R* base, unsigned o) { return kWide ? gload(base + o) : gload_at(base, o); };
    auto put = [&](R* base, unsigned o, R v) {
      if (kWide) gstore(base + o, v); else gstore_at(base, o, v);
    };
    auto load_row = [&](int r, A& a) {
      const int rc = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
      const unsigned b = node(rc, xcl);
      a.H = ld(cx.H, b);
      a.D = ld(cx.D, b);
      a.w = ld(cx.U, b);   // x view: w = u, t = v
      a.t = ld(cx.V, b);
      a.f = (col_in && r >= 0 && r < ny) ? F_EX : 0;
      if (kRing) a.f |= ring_flag(cx.gflags, xc, r, nx, ny);
      if (kOpen) a.f |= open_flag(cx.gflags, xc, r, nx, ny);
    };
    // maxwave values of an output row, read one march row ahead of use
    struct MW { R e, s2; };
    // A row that is not one of the tile's output rows (the halo rows at the
    // start of the march, the rows past its end) reads the maxwave of the
    // first output row instead, which the tile reads anyway: the load is
    // still issued (every path of the march issues the same loads, which
    // keeps the compiler's waits as tight as before) but costs no new lines.
    const int yout0 = tl.y0, yout1 = tl.y0 + tl.rows - 1;
    auto load_mw = [&](int r, MW& m) {
      m.e = 0; m.s2 = 0;
      if (do_max) {
        const int rc = (r < yout0 || r > yout1) ? yout0 : r;
        const unsigned b = node(rc, xcl);
        m.e = ld(cx.emax, b);
        m.s2 = ld(cx.smax2, b);
      }
    };
    auto store = [&](int r, const C& o, R D, const MW& m) {
      // o in x view: H, w = u, t = v
      if (!out_lane || r < 0 || r >= ny) return;
      const unsigned b = node(r, xc);
      put(cx.Ho, b, o.H);
      put(cx.Uo, b, o.w);
      put(cx.Vo, b, o.t);
      // one test: a NaN or an infinity in any term makes the sum non-finite
      if (!isfinite((o.H + o.w) + o.t)) bad = 1;
      if (do_max && P::wet_out(o, D, cx.par)) {
        R e = P::eta_out(o, D);
        if (e > m.e) put(cx.emax, b, e);
        R s2 = o.w * o.w + o.t * o.t;
        if (s2 > m.s2) put(cx.smax2, b, s2);
      }
      // gauge records of this tile's nodes on record steps (eta, u, v on
      // wet nodes, zeros on dry ones), written by the lane holding the node
      if (rec_slot >= 0 && tl.gn > 0) {
        for (int k = tl.g0; k < tl.g0 + tl.gn; ++k) {
          if (cload(g.gtab + 3 * k) != r) continue;
          if (cload(g.gtab + 3 * k + 1) != xc) continue;
          const int gi = cload(g.gtab + 3 * k + 2);
          const bool w = P::wet_out(o, D, cx.par);
          double* rec = g.grec + ((size_t)rec_slot * (size_t)g.ngauge + (size_t)gi) * 3;
          gstore(rec, w ? (double)P::eta_out(o, D) : 0.0);
          gstore(rec + 1, w ? (double)o.w : 0.0);
          gstore(rec + 2, w ? (double)o.t : 0.0);
        }
      }
    };

    if (ORDER == ORD_X) {
      A nxt;
      MW mnxt;
      load_row(tl.y0, nxt);
      load_mw(tl.y0, mnxt);
      for (int r = tl.y0; r < tl.y0 + tl.rows; ++r) {
        A a = nxt;
        MW m = mnxt;
        // past the last row: the row in use again (its lines are loaded)
        load_row(r < yout1 ? r + 1 : r, nxt);
        load_mw(r + 1, mnxt);
        R f = cload(xfac + r);
        C o = xsweep_row<P>(a, f * xiL, f * xiR, f * xiS, cx.par);
        store(r, o, a.D, m);
      }
    } else {
      // Alternate segment rows march in opposite directions, so that two
      // vertically adjacent segments read the rows around their common edge
      // at the same phase of their marches (both at the start or both at
      // the end), when one XCD's L2 can serve the second read.
      // Rows staged in LDS: each lane loads dwords of the 64-column window
      // (FP64: two loads of 64 dwords per field row, FP32: one), at byte
      // offsets within the row that depend only on the column, so they are
      // computed once per tile; the row itself enters through the scalar
      // base address.
      constexpr int kDw = sizeof(R) / 4;   // dwords per value
      unsigned dma_off[kDw];
#pragma unroll
      for (int h = 0; h < kDw; ++h) {
        const int d = h * WAVE + lane;     // dword of the window this lane loads
        int col = tl.x0 - HALO + d / kDw;
        col = col < 0 ? 0 : (col >= nx ? nx - 1 : col);
        dma_off[h] = (unsigned)col * (unsigned)sizeof(R) + (unsigned)(d % kDw) * 4u;
      }
      auto dma_row = [&](const R* base, int r, R* lds) {
        const int rc = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
        // The row's address, formed by scalar instructions (its byte offset
        // is below 4 GiB: the staged form is not used with 64-bit
        // addresses); otherwise the compiler folds the row offset into a
        // per-lane 64-bit multiply-add for every load, and keeps a 64-bit
        // base-plus-lane-offset pair per load alive across the march.
        const unsigned rowoff = (unsigned)rc * (unsigned)nx * (unsigned)sizeof(R);
        const char* g = uniform_ptr((const char*)base + rowoff);
#pragma unroll
        for (int h = 0; h < kDw; ++h) dma_dword(g + dma_off[h], lds + h * (WAVE / kDw));
      };
      // vector memory operations one march row issues: the row's four fields,
      // and the maxwave pair of an output row
      constexpr int kVmRow = 4 * kDw, kVmMw = 2 * kDw;
      auto march = [&](auto dir) {
        constexpr int D = decltype(dir)::value;
        YPipe<P> yp;
        yp.reset();
        A pf[3];
        MW pm[3];
        const int ylast = tl.y0 + tl.rows - 1;
        const int r_first = D > 0 ? tl.y0 - HALO : ylast + HALO;
        const int npush = tl.rows + 2 * HALO;
        // rows are loaded PF = P::kPrefetch march rows ahead of use (1 or 2:
        // the three slots hold the row in use and up to two in flight)
        constexpr int PF = P::kPrefetch;
        // LDS ring: march row i sits in slot i % kLdsSlots, with the maxwave
        // of its output row r - 3D; rows i + 1 .. i + kLdsAhead are in flight
        auto issue_dir = [&](int i) {
          const int r = r_first + D * i;
          const int slot = i & (kLdsSlots - 1);
          dma_row(cx.H, r, &lrow[slot][wave][0][0]);
          dma_row(cx.D, r, &lrow[slot][wave][1][0]);
          dma_row(cx.U, r, &lrow[slot][wave][2][0]);
          dma_row(cx.V, r, &lrow[slot][wave][3][0]);
          // the maxwave pair of output rows only (march rows 2 HALO on)
          if (do_max && i >= 2 * HALO) {
            dma_row(cx.emax, r - D * HALO, &lmw[slot][wave][0][0]);
            dma_row(cx.smax2, r - D * HALO, &lmw[slot][wave][1][0]);
          }
        };
        if (kLds) {
          // Every load issued before the march (the tile's column metrics)
          // has landed, in a wait the compiler sees: the waits inside the
          // march are its own, and without this one the compiler would wait
          // for all loads in flight before the first use of those values
          // in each row.  (simm16: vmcnt 0, expcnt and lgkmcnt not waited)
          __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
          for (int j = 0; j < kLdsAhead; ++j) issue_dir(j);
        } else {
          load_row(r_first, pf[0]);
          if (PF == 2) load_row(r_first + D, pf[1]);
          load_mw(r_first - D * HALO, pm[0]);
        }
        // one march row in phase K: consume row r and the maxwave of the
        // output row r - 3D; prefetch the rows ahead
        auto body = [&](auto phase, int r, int i) {
          constexpr int K = decltype(phase)::value;
          A a;
          MW m;
          if (kLds) {
            // Row i and its maxwave pair were issued kLdsAhead rows ago; the
            // kLdsAhead - 1 rows issued since may still be in flight. From
            // step 2 HALO + kLdsAhead on, each of the kLdsAhead steps since
            // that issue has also stored its output row (h, u, v: one store
            // each, issued after the step's loads), so those stores may be
            // in flight as well, and every row since carries its maxwave
            // pair. Before that, the count leaves out the stores and the
            // maxwave pairs (march rows below 2 HALO load none), and at the
            // end of the march it counts only the rows issued (none past the
            // last): a count below the operations issued after row i still
            // waits for row i. (The conditional maxwave and gauge stores
            // only add to the operations issued after row i.)
            constexpr int kRowOps = kVmRow + kVmMw, kRowOps0 = kVmRow;
            constexpr int kStores = kLdsAhead * 3;
            static_assert(kLdsAhead == 3, "the end-of-march waits below assume 3 rows ahead");
            const int after = npush - 1 - i;
            if (after <= 0) {
              wait_vmem<0>();
            } else if (after == 1) {
              wait_vmem<kRowOps0>();
            } else if (i >= 2 * HALO + kLdsAhead) {
              if (do_max)
                wait_vmem<(kLdsAhead - 1) * kRowOps + kStores>();
              else
                wait_vmem<(kLdsAhead - 1) * kRowOps0 + kStores>();
            } else {
              wait_vmem<(kLdsAhead - 1) * kRowOps0>();
            }
            const int slot = i & (kLdsSlots - 1);
            // x view: w = u, t = v
            lds_row<R>(lds_addr(&lrow[slot][wave][0][lane]), lds_addr(&lmw[slot][wave][0][lane]),
                       a.H, a.D, a.w, a.t, m.e, m.s2);
            a.f = (col_in && r >= 0 && r < ny) ? F_EX : 0;
            if (kRing) a.f |= ring_flag(cx.gflags, xc, r, nx, ny);
            if (kOpen) a.f |= open_flag(cx.gflags, xc, r, nx, ny);
            if (!do_max) {
              m.e = 0;
              m.s2 = 0;
            }
            if (i + kLdsAhead < npush) issue_dir(i + kLdsAhead);
          } else {
            a = pf[K];
            m = pm[K];
            // past the end of the march: the last march row again (its
            // lines are loaded by then; the slot is never read)
            load_row(i + PF < npush ? r + D * PF : r_first + D * (npush - 1), pf[(K + PF) % 3]);
            load_mw(r + D * (1 - HALO), pm[(K + 1) % 3]);
          }
          const int ro = r - D * HALO;
          const bool writes = D > 0 ? ro >= tl.y0 : ro <= ylast;
          if (ORDER == ORD_YX) {
            A ay = a;
            ay.w = a.t;
            ay.t = a.w;
            C oy;
            typename P::B ob;
            ypipe_push<P, K, kShY, D>(yp, ay, r, tl.y0, ylast, cx, oy, ob);
            if (writes && ro < ny) {
              A ax;
              ax.H = oy.H; ax.w = oy.t; ax.t = oy.w;
              ax.f = ob.f & (F_EX | F_FIX | F_OPEN);
              ax.D = ob.D;
              R f = cload(xfac + ro);
              C o = xsweep_row<P>(ax, f * xiL, f * xiR, f * xiS, cx.par);
              store(ro, o, ax.D, m);
            }
          } else {
            if (ORDER == ORD_XY && r >= 0 && r < ny) {
              R f = cload(xfac + r);
              C o = xsweep_row<P>(a, f * xiL, f * xiR, f * xiS, cx.par);
              a.H = o.H; a.w = o.w; a.t = o.t;
              a.f &= (F_EX | F_FIX);
            }
            A ay = a;   // y view: w = v, t = u
            ay.w = a.t;
            ay.t = a.w;
            C oy;
            typename P::B ob;
            ypipe_push<P, K, kShY, D>(yp, ay, r, tl.y0, ylast, cx, oy, ob);
            if (writes) {
              C o;
              o.H = oy.H; o.w = oy.t; o.t = oy.w;   // back to x view
              store(ro, o, ob.D, m);
            }
          }
        };
        // whole triples in the loop, so that its back edge sees the slots in
        // one rotation (no register copies); the last 0-2 rows after it
        int i = 0;
        for (; i + 3 <= npush; i += 3) {
          body(std::integral_constant<int, 0>(), r_first + D * i, i);
          body(std::integral_constant<int, 1>(), r_first + D * (i + 1), i + 1);
          body(std::integral_constant<int, 2>(), r_first + D * (i + 2), i + 2);
        }
        if (i < npush) body(std::integral_constant<int, 0>(), r_first + D * i, i);
        if (i + 1 < npush) body(std::integral_constant<int, 1>(), r_first + D * (i + 1), i + 1);
        // the loads of the last row have landed (its wait was for all
        // operations), so the LDS ring is free for the next tile
      };
      if (rev)
        march(std::integral_constant<int, -1>());
      else
        march(std::integral_constant<int, 1>());
    }
  }
  if (bad) st->bad = 1;
}

// ---------------------------------------------------------------------------
// Small kernels: state set-up and read-out, maxwave, sampling, forcing.
// ---------------------------------------------------------------------------
template <class R>
__global__ void init_state_kernel(GridDesc g, const double* eta, const double* u, const double* v,
                                  int deform, long long N, int parity) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  R* H = (R*)g.H[parity];
  R* U = (R*)g.U[parity];
  R* V = (R*)g.V[parity];
  R* D = (R*)g.D;
  const bool fp32 = sizeof(R) == 4;
  double d = (double)D[k];
  double e = eta ? eta[k] : 0.0;
  double h;
  if (deform) {
    h = d > 0.0 ? d : 0.0;
    d = d - e;
    D[k] = (R)d;
  } else {
    h = d + e;
    if (h < 0.0) h = 0.0;
  }
  double uu = u ? u[k] : 0.0, vv = v ? v[k] : 0.0;
  const bool blocked = (g.flags & G_WALLMODE) && (d < g.dwall);
  if (!(h > g.hmin) || blocked) {
    h = 0.0; uu = 0.0; vv = 0.0;
  }
  if (fp32) {
    // FP32 state: surface eta = h - d (dry: -d so that h = 0 exactly)
    float df = (float)D[k];
    H[k] = (R)(h > 0.0 ? (float)(h - d) : -df);
  } else {
    H[k] = (R)h;
  }
  U[k] = (R)uu;
  V[k] = (R)vv;
}

template <class R>
__global__ void set_raw_kernel(GridDesc g, const double* h, const double* u, const double* v,
                               long long N, int parity) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  R* H = (R*)g.H[parity];
  const R* D = (const R*)g.D;
  if (sizeof(R) == 4) {
    H[k] = (R)(h[k] > 0.0 ? (float)(h[k] - (double)D[k]) : -(float)D[k]);
  } else {
    H[k] = (R)h[k];
  }
  ((R*)g.U[parity])[k] = (R)u[k];
  ((R*)g.V[parity])[k] = (R)v[k];
}

template <class R>
__global__ void get_raw_kernel(GridDesc g, double* h, double* u, double* v, long long N,
                               int parity) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const R* H = (const R*)g.H[parity];
  const R* D = (const R*)g.D;
  if (h) {
    if (sizeof(R) == 4) {
      float hh = (float)D[k] + (float)H[k];
      h[k] = hh > 0.f ? (double)hh : 0.0;
    } else {
      h[k] = (double)H[k];
    }
  }
  if (u) u[k] = (double)((const R*)g.U[parity])[k];
  if (v) v[k] = (double)((const R*)g.V[parity])[k];
}

template <class R>
__device__ __forceinline__ bool node_wet(const GridDesc& g, R Hs, R D, R& eta) {
  if (sizeof(R) == 4) {
    R h = D + Hs;
    eta = Hs;
    return h > (R)g.hmin;
  }
  eta = Hs - D;
  return Hs > (R)g.hmin;
}

template <class R>
__global__ void get_state_kernel(GridDesc g, double* eta, double* u, double* v, uint8_t* wet,
                                 long long N, int parity) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const R* H = (const R*)g.H[parity];
  const R* D = (const R*)g.D;
  R e;
  const bool w = node_wet<R>(g, H[k], D[k], e);
  if (eta) eta[k] = w ? (double)e : 0.0;
  if (u) u[k] = w ? (double)((const R*)g.U[parity])[k] : 0.0;
  if (v) v[k] = w ? (double)((const R*)g.V[parity])[k] : 0.0;
  if (wet) wet[k] = w ? 1 : 0;
}

template <class R>
__global__ void read_maxwave_kernel(GridDesc g, double* emax, double* smax, long long N) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  if (emax) emax[k] = (double)((const R*)g.emax)[k];
  if (smax) smax[k] = sqrt((double)((const R*)g.smax2)[k]);
}

template <class R>
__global__ void clear_maxwave_kernel(GridDesc g, long long N) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  ((R*)g.emax)[k] = (R)0;
  ((R*)g.smax2)[k] = (R)0;
}

template <class R>
__global__ void get_depth_kernel(GridDesc g, double* d, long long N) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  d[k] = (double)((const R*)g.D)[k];
}

// Gauge and enclosed-grid records at the level n reached by the last step.
template <class R>
__global__ void sample_kernel(const GridDesc* grids, const SampleDesc* sd, long long n,
                              int parity, int do_gauges) {
  const SampleDesc s = *sd;
  const GridDesc& g = grids[s.grid];
  const R* H = (const R*)g.H[parity];
  const R* U = (const R*)g.U[parity];
  const R* V = (const R*)g.V[parity];
  const R* D = (const R*)g.D;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (do_gauges && s.ngauge > 0 && n % s.gout == 0 && n >= s.g_first && i < s.ngauge) {
    const long long slot = (n - s.g_first) / s.gout;
    if (slot < s.gcap) {
      const long long k = s.gidx[i];
      R e;
      const bool w = node_wet<R>(g, H[k], D[k], e);
      double* o = s.grec + ((size_t)slot * s.ngauge + i) * 3;
      o[0] = w ? (double)e : 0.0;
      o[1] = w ? (double)U[k] : 0.0;
      o[2] = w ? (double)V[k] : 0.0;
    }
  }
  if (s.npts > 0 && n % s.bndout == 0 && n >= s.s_first && i < s.npts) {
    const long long slot = (n - s.s_first) / s.bndout;
    if (slot < s.scap) {
      double ws = 0.0, au = 0.0, av = 0.0, ae = 0.0;
      for (int c = 0; c < 4; ++c) {
        const long long k = s.sidx[(size_t)4 * i + c];
        const double wt = s.swt[(size_t)4 * i + c];
        R e;
        if (!node_wet<R>(g, H[k], D[k], e)) continue;
        ws = ws + wt;
        au = au + wt * (double)U[k];
        av = av + wt * (double)V[k];
        ae = ae + wt * (double)e;
      }
      double* o = s.srec + (size_t)slot * s.rec_len;
      const int off = s.sout[i];   // index of u inside the record; v at +np, eta at +2np
      const int np = s.sout[s.npts + i];
      if (ws > 0.0) {
        o[off] = au / ws;
        o[off + np] = av / ws;
        o[off + 2 * np] = ae / ws;
      } else {
        o[off] = 0.0;
        o[off + np] = 0.0;
        o[off + 2 * np] = 0.0;
      }
    }
  }
}

// Forcing ring at t = n dt (start of the step).
__device__ __forceinline__ double interp_series(const double* tt, int nt, const double* vals,
                                                int np, int q, int pt, double t) {
  const int stride = 3 * np;
  if (t <= tt[0]) return vals[(size_t)q * np + pt];
  if (t >= tt[nt - 1]) return vals[(size_t)(nt - 1) * stride + (size_t)q * np + pt];
  int lo = 0, hi = nt - 1;  // tt[lo] <= t < tt[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tt[mid] <= t) lo = mid;
    else hi = mid;
  }
  double a = (t - tt[lo]) / (tt[lo + 1] - tt[lo]);
  double v0 = vals[(size_t)lo * stride + (size_t)q * np + pt];
  double v1 = vals[(size_t)(lo + 1) * stride + (size_t)q * np + pt];
  return v0 + a * (v1 - v0);
}

template <class R>
__global__ void forcing_kernel(const GridDesc* grids, const ForceDesc* fd, long long n,
                               int parity) {
  const ForceDesc f = *fd;
  const GridDesc& g = grids[f.grid];
  const double t = (double)n * g.dt;
  R* H = (R*)g.H[parity];
  R* U = (R*)g.U[parity];
  R* V = (R*)g.V[parity];
  const R* D = (const R*)g.D;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // sides in order W, E, S, N: a later side overwrites a shared corner, so
  // the four sides run one after the other inside this thread's column of
  // work; corners are written by S/N threads after W/E threads of the same
  // index.  To keep the order deterministic, W/E corner points are skipped
  // when S/N are forced.
  for (int s = 0; s < 4; ++s) {
    if (f.nt[s] <= 0 || i >= f.np[s]) continue;
    int x, y;
    if (s == 0) { x = 0; y = i; }
    else if (s == 1) { x = g.nx - 1; y = i; }
    else if (s == 2) { x = i; y = 0; }
    else { x = i; y = g.ny - 1; }
    if (s < 2 && ((y == 0 && f.nt[2] > 0) || (y == g.ny - 1 && f.nt[3] > 0))) continue;
    const long long k = (long long)y * g.nx + x;
    double uu = interp_series(f.t[s], f.nt[s], f.vals[s], f.np[s], 0, i, t);
    double vv = interp_series(f.t[s], f.nt[s], f.vals[s], f.np[s], 1, i, t);
    double ee = interp_series(f.t[s], f.nt[s], f.vals[s], f.np[s], 2, i, t);
    double d = (double)D[k];
    double h = d + ee;
    if (h < 0.0) h = 0.0;
    if (h > g.hmin) {
      if (sizeof(R) == 4) H[k] = (R)((float)ee);
      else H[k] = (R)h;
      U[k] = (R)uu;
      V[k] = (R)vv;
    } else {
      H[k] = sizeof(R) == 4 ? (R)(-(float)D[k]) : (R)0;
      U[k] = (R)0;
      V[k] = (R)0;
    }
  }
}

// Halo rows of a y-band decomposition (one exchange per blockIdx.y): after a
// step, the HALO rows beyond an inner band edge take the values of the band
// that owns them.  Rows are contiguous, so each copy is HALO * nx elements
// of each field.
template <class R>
__global__ void band_exchange_kernel(const GridDesc* grids, const BandXchg* xt, int nx,
                                     int parity) {
  const BandXchg x = xt[blockIdx.y];
  const long long n = (long long)HALO * nx;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const GridDesc& gs = grids[x.src];
  const GridDesc& gd = grids[x.dst];
  const long long so = (long long)x.src_row * nx + k;
  const long long dof = (long long)x.dst_row * nx + k;
  ((R*)gd.H[parity])[dof] = ((const R*)gs.H[parity])[so];
  ((R*)gd.U[parity])[dof] = ((const R*)gs.U[parity])[so];
  ((R*)gd.V[parity])[dof] = ((const R*)gs.V[parity])[so];
}

inline int nblk(long long N, int bs) { return (int)((N + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <class P, int FL>
static void launch_order(int order, dim3 grid, dim3 block, hipStream_t s, const GridDesc* grids,
                         const Tile* tiles, int ntiles, StepState* st, int parity,
                         int do_max, int rec_slot) {
  switch (order) {
    case ORD_XY:
      hipLaunchKernelGGL((step_kernel<P, ORD_XY, FL>), grid, block, 0, s, grids, tiles, ntiles,
                         st, parity, do_max, rec_slot);
      break;
    case ORD_YX:
      hipLaunchKernelGGL((step_kernel<P, ORD_YX, FL>), grid, block, 0, s, grids, tiles, ntiles,
                         st, parity, do_max, rec_slot);
      break;
    case ORD_X:
      hipLaunchKernelGGL((step_kernel<P, ORD_X, FL>), grid, block, 0, s, grids, tiles, ntiles,
                         st, parity, do_max, rec_slot);
      break;
    default:
      hipLaunchKernelGGL((step_kernel<P, ORD_Y, FL>), grid, block, 0, s, grids, tiles, ntiles,
                         st, parity, do_max, rec_slot);
      break;
  }
}

hipError_t launch_step(int fp32, int order, int gflags, const GridDesc* grids, const Tile* tiles,
                       int ntiles, StepState* st, int parity, int do_max, int nblocks,
                       hipStream_t s, int rec_slot) {
  dim3 grid(nblocks), block(WAVE * WAVES_PER_BLOCK);
  const int base = gflags & ~(G_WIDE | G_LDSROWS);
  const bool fast = (base & ~FL_FAST) == 0;
  const bool fric = (base & ~FL_FRIC) == 0;
  const bool fric_semi = (base & ~FL_FRIC_SEMI) == 0;
  const bool ring = (base & ~FL_RING) == 0;
  const bool ring_fric = (base & ~FL_RING_FRIC) == 0;
  if (gflags & G_WIDE) {
    if (fp32) {
      if (fast)
        launch_order<P32, FL_FAST_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                        do_max, rec_slot);
      else if (fric)
        launch_order<P32, FL_FRIC_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                        do_max, rec_slot);
      else
        launch_order<P32, FL_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                   do_max, rec_slot);
    } else {
      if (fast)
        launch_order<P64, FL_FAST_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                        do_max, rec_slot);
      else if (fric)
        launch_order<P64, FL_FRIC_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                        do_max, rec_slot);
      else
        launch_order<P64, FL_WIDE>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                   do_max, rec_slot);
    }
  } else if (fp32) {
    const bool lds = (gflags & G_LDSROWS) != 0;
    if (fast && lds)
      launch_order<P32, FL_FAST_LDS>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                     do_max, rec_slot);
    else if (fric && lds)
      launch_order<P32, FL_FRIC_LDS>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                     do_max, rec_slot);
    else if (fast)
      launch_order<P32, FL_FAST>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (fric)
      launch_order<P32, FL_FRIC>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (fric_semi)
      launch_order<P32, FL_FRIC_SEMI>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                      do_max, rec_slot);
    else if (ring)
      launch_order<P32, FL_RING>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (ring_fric)
      launch_order<P32, FL_RING_FRIC>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                    do_max, rec_slot);
    else
      launch_order<P32, FL_ALL>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                do_max, rec_slot);
  } else {
    if (fast)
      launch_order<P64, FL_FAST>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (fric)
      launch_order<P64, FL_FRIC>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (fric_semi)
      launch_order<P64, FL_FRIC_SEMI>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                      do_max, rec_slot);
    else if (ring)
      launch_order<P64, FL_RING>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                 do_max, rec_slot);
    else if (ring_fric)
      launch_order<P64, FL_RING_FRIC>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                    do_max, rec_slot);
    else
      launch_order<P64, FL_ALL>(order, grid, block, s, grids, tiles, ntiles, st, parity,
                                do_max, rec_slot);
  }
  return hipGetLastError();
}

template <class P, int FL>
static hipError_t occupancy_of(int order, int* n) {
  const int bs = WAVE * WAVES_PER_BLOCK;
  switch (order) {
    case ORD_XY:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, reinterpret_cast<const void*>(&step_kernel<P, ORD_XY, FL>), bs, 0);
    case ORD_YX:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, reinterpret_cast<const void*>(&step_kernel<P, ORD_YX, FL>), bs, 0);
    case ORD_X:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, reinterpret_cast<const void*>(&step_kernel<P, ORD_X, FL>), bs, 0);
    default:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          n, reinterpret_cast<const void*>(&step_kernel<P, ORD_Y, FL>), bs, 0);
  }
}

hipError_t step_blocks_per_cu(int fp32, int order, int gflags, int* n) {
  *n = 0;
  const int base = gflags & ~(G_WIDE | G_LDSROWS);
  const bool fast = (base & ~FL_FAST) == 0;
  const bool fric = (base & ~FL_FRIC) == 0;
  const bool fric_semi = (base & ~FL_FRIC_SEMI) == 0;
  const bool ring = (base & ~FL_RING) == 0;
  const bool ring_fric = (base & ~FL_RING_FRIC) == 0;
  if (gflags & G_WIDE) {
    if (fp32)
      return fast ? occupancy_of<P32, FL_FAST_WIDE>(order, n)
                  : (fric ? occupancy_of<P32, FL_FRIC_WIDE>(order, n)
                          : occupancy_of<P32, FL_WIDE>(order, n));
    return fast ? occupancy_of<P64, FL_FAST_WIDE>(order, n)
                : (fric ? occupancy_of<P64, FL_FRIC_WIDE>(order, n)
                        : occupancy_of<P64, FL_WIDE>(order, n));
  }
  if (fp32 && (gflags & G_LDSROWS) && (fast || fric))
    return fast ? occupancy_of<P32, FL_FAST_LDS>(order, n) : occupancy_of<P32, FL_FRIC_LDS>(order, n);
  if (fp32)
    return fast ? occupancy_of<P32, FL_FAST>(order, n)
                : fric      ? occupancy_of<P32, FL_FRIC>(order, n)
                : fric_semi ? occupancy_of<P32, FL_FRIC_SEMI>(order, n)
                : ring      ? occupancy_of<P32, FL_RING>(order, n)
                : ring_fric ? occupancy_of<P32, FL_RING_FRIC>(order, n)
                            : occupancy_of<P32, FL_ALL>(order, n);
  return fast ? occupancy_of<P64, FL_FAST>(order, n)
              : fric      ? occupancy_of<P64, FL_FRIC>(order, n)
              : fric_semi ? occupancy_of<P64, FL_FRIC_SEMI>(order, n)
              : ring      ? occupancy_of<P64, FL_RING>(order, n)
              : ring_fric ? occupancy_of<P64, FL_RING_FRIC>(order, n)
                          : occupancy_of<P64, FL_ALL>(order, n);
}

#define CLF_SMALL_LAUNCH(KERNEL, N, ...)                                           \
  do {                                                                             \
    const int bs = 256;                                                            \
    if (fp32)                                                                      \
      hipLaunchKernelGGL(KERNEL<float>, dim3(nblk(N, bs)), dim3(bs), 0, s, __VA_ARGS__); \
    else                                                                           \
      hipLaunchKernelGGL(KERNEL<double>, dim3(nblk(N, bs)), dim3(bs), 0, s, __VA_ARGS__); \
    return hipGetLastError();                                                      \
  } while (0)

hipError_t launch_init_state(int fp32, const GridDesc* gh, const GridDesc*, const double* eta,
                             const double* u, const double* v, int deform, long long N, int parity,
                             hipStream_t s) {
  CLF_SMALL_LAUNCH(init_state_kernel, N, *gh, eta, u, v, deform, N, parity);
}

hipError_t launch_set_raw(int fp32, const GridDesc* gh, const GridDesc*, const double* h,
                          const double* u, const double* v, long long N, int parity,
                          hipStream_t s) {
  CLF_SMALL_LAUNCH(set_raw_kernel, N, *gh, h, u, v, N, parity);
}

hipError_t launch_get_raw(int fp32, const GridDesc* gh, const GridDesc*, double* h, double* u,
                          double* v, long long N, int parity, hipStream_t s) {
  CLF_SMALL_LAUNCH(get_raw_kernel, N, *gh, h, u, v, N, parity);
}

hipError_t launch_get_state(int fp32, const GridDesc* gh, const GridDesc*, double* eta, double* u,
                            double* v, uint8_t* wet, long long N, int parity, hipStream_t s) {
  CLF_SMALL_LAUNCH(get_state_kernel, N, *gh, eta, u, v, wet, N, parity);
}

hipError_t launch_read_maxwave(int fp32, const GridDesc* gh, const GridDesc*, double* emax,
                               double* smax, long long N, hipStream_t s) {
  CLF_SMALL_LAUNCH(read_maxwave_kernel, N, *gh, emax, smax, N);
}

hipError_t launch_get_depth(int fp32, const GridDesc* gh, const GridDesc*, double* d, long long N,
                            hipStream_t s) {
  CLF_SMALL_LAUNCH(get_depth_kernel, N, *gh, d, N);
}

hipError_t launch_clear_maxwave(int fp32, const GridDesc* gh, long long N, hipStream_t s) {
  CLF_SMALL_LAUNCH(clear_maxwave_kernel, N, *gh, N);
}

hipError_t launch_sample(int fp32, const GridDesc* gd, const SampleDesc* sd, int nthreads,
                         long long n, int parity, int do_gauges, hipStream_t s) {
  CLF_SMALL_LAUNCH(sample_kernel, (long long)nthreads, gd, sd, n, parity, do_gauges);
}

hipError_t launch_forcing(int fp32, const GridDesc* gd, const ForceDesc* fd, int nthreads,
                          long long n, int parity, hipStream_t s) {
  CLF_SMALL_LAUNCH(forcing_kernel, (long long)nthreads, gd, fd, n, parity);
}

hipError_t launch_band_exchange(int fp32, const GridDesc* grids, const BandXchg* xt, int nxchg,
                                int nx, int parity, hipStream_t s) {
  if (nxchg <= 0) return hipSuccess;
  const int bs = 256;
  dim3 grid(nblk((long long)HALO * nx, bs), nxchg);
  if (fp32)
    hipLaunchKernelGGL(band_exchange_kernel<float>, grid, dim3(bs), 0, s, grids, xt, nx, parity);
  else
    hipLaunchKernelGGL(band_exchange_kernel<double>, grid, dim3(bs), 0, s, grids, xt, nx, parity);
  return hipGetLastError();
}

}  // namespace clf
