// HIP kernels of the split-step shallow-water library (gfx950).
//
// The hot path is one fused "march" kernel per time step.  A wavefront owns
// a tile: a strip of 64 consecutive columns (58 output columns plus a
// 3-column halo on each side) and a segment of rows.  It walks down the
// segment one row at a time:
//   * the x-sweep of the row (eq2A) runs across the 64 lanes; the neighbour
//     values of steps (b), (d) and (e) come from the adjacent lanes, and each
//     of the three neighbour stages costs one lane of validity on each side,
//     hence the 3-column halo;
//   * the post-x row enters a per-lane y-sweep pipeline (eq2B) held in
//     registers: stage A = step (a), B = step (b), C = steps (c)+(d),
//     D = step (e).  Each stage needs its neighbours one row up and down, so
//     the row leaving the pipeline lags the row entering it by 3 and a
//     segment re-reads 3 rows above and below it.
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

namespace clf {
namespace {

constexpr double kG = 9.81;

// ---------------------------------------------------------------------------
// Cross-lane exchange: value held by lane-1 / lane+1 of the wavefront.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T from_prev(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "4-byte multiple");
  union U { T v; int i[sizeof(T) / 4]; };
  U a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) b.i[k] = __shfl_up(a.i[k], 1, WAVE);
  return b.v;
}

template <class T>
__device__ __forceinline__ T from_next(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "4-byte multiple");
  union U { T v; int i[sizeof(T) / 4]; };
  U a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) b.i[k] = __shfl_down(a.i[k], 1, WAVE);
  return b.v;
}

// ---------------------------------------------------------------------------
// FP64 node stages (literal form).
// ---------------------------------------------------------------------------
struct P64 {
  typedef double R;
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

  static __device__ __forceinline__ void stage_a(A& a, const Par& p) {
    if (a.f & F_EX) {
      if (a.H > p.hmin) {
        a.f |= F_WET;
      } else {
        a.H = 0.0; a.w = 0.0; a.t = 0.0;
      }
    }
  }

  static __device__ __forceinline__ B stage_b(const A& l, const A& c, const A& r, const Par& p) {
    B b;
    b.H = c.H; b.w = c.w; b.t = c.t; b.D = c.D; b.f = c.f; b.src = 0;
    const bool blocked = (p.flags & G_WALLMODE) && (c.D < p.dwall);
    if ((c.f & F_EX) && !(c.f & (F_WET | F_FIX)) && !blocked) {
      bool qL = false, qR = false;
      double fL = 0.0, fR = 0.0;
      if ((l.f & (F_EX | F_WET)) == (F_EX | F_WET)) {
        fL = (l.H - l.D) + c.D;
        qL = fL > p.hmin;
      }
      if ((r.f & (F_EX | F_WET)) == (F_EX | F_WET)) {
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
    b.c = (b.f & F_WET) ? sqrt(kG * b.H) : 0.0;
    return b;
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

  static __device__ __forceinline__ C stage_cd(const Bx& l, const B& c, const Bx& r, double iL,
                                               double iR, double iS, double tanR, const Par& p) {
    C o;
    if (c.f & F_FIX) {
      o.H = c.H; o.w = c.w; o.t = c.t;
      return o;
    }
    if (!(c.f & F_WET)) {
      o.H = 0.0; o.w = 0.0; o.t = 0.0;
      return o;
    }
    double Lw, Lt, LD, Lc, Rw, Rt, RD, Rc;
    if ((l.f & (F_EX | F_WET)) == (F_EX | F_WET)) {
      Lw = l.w; Lt = l.t; LD = l.D; Lc = l.c;
    } else {
      Lw = -c.w; Lt = c.t; LD = c.D; Lc = c.c;   // mirror ghost
    }
    if ((r.f & (F_EX | F_WET)) == (F_EX | F_WET)) {
      Rw = r.w; Rt = r.t; RD = r.D; Rc = r.c;
    } else {
      Rw = -c.w; Rt = c.t; RD = c.D; Rc = c.c;
    }
    const double Cw = c.w, Ct = c.t, CD = c.D, Cc = c.c;
    double xPL = Lw + 2.0 * Lc, xPC = Cw + 2.0 * Cc, xPR = Rw + 2.0 * Rc;
    double lPL = Lw + Lc, lPC = Cw + Cc, lPR = Rw + Rc;
    double xML = Lw - 2.0 * Lc, xMC = Cw - 2.0 * Cc, xMR = Rw - 2.0 * Rc;
    double lML = Lw - Lc, lMC = Cw - Cc, lMR = Rw - Rc;
    double QPL = qhat(lPL, xPL, LD, lPC, xPC, CD, iL);
    double QPR = qhat(lPC, xPC, CD, lPR, xPR, RD, iR);
    double QML = qhat(lML, xML, LD, lMC, xMC, CD, iL);
    double QMR = qhat(lMC, xMC, CD, lMR, xMR, RD, iR);
    double QTL = qhat_t(Lw, Lt, Cw, Ct, iL);
    double QTR = qhat_t(Cw, Ct, Rw, Rt, iR);
    double QPc = 0.0, QMc = 0.0, QTc = 0.0;
    if (p.flags & G_SOLVER1) {
      QPc = qhat(lPL, xPL, LD, lPR, xPR, RD, iS);
      QMc = qhat(lML, xML, LD, lMR, xMR, RD, iS);
      QTc = qhat_t(Lw, Lt, Rw, Rt, iS);
    }
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
    double ws = Pn + Mn;
    double wv = 0.5 * ws;
    double dd = Pn - Mn;
    if (dd < 0.0) dd = 0.0;
    double Hv = (dd * dd) * p.inv16g;
    if (p.flags & G_FRICTION) {
      double sp = sqrt(Cw * Cw + Ct * Ct);
      double den = c.H * cbrt(c.H);
      double fr = ((p.dt * p.gn2) * sp) / den;
      wv = wv / (1.0 + fr);
    }
    o.H = Hv; o.w = wv; o.t = Tn;
    return o;
  }

  static __device__ __forceinline__ Cx cx(const C& c) {
    Cx x;
    x.H = c.H; x.w = c.w;
    return x;
  }

  static __device__ __forceinline__ void stage_e(C& o, const Cx& l, const Cx& r, int src) {
    if (src == 0) return;
    if (src == 2) {
      double a = l.H, b = r.H;
      double m = (b < a) ? b : a;
      double cap = 0.5 * m;
      if (o.H > cap) o.H = cap;
      return;
    }
    const Cx& s = (src == -1) ? l : r;
    double cap = 0.5 * s.H;
    if (o.H > cap) o.H = cap;
    if (src == -1) {
      if (o.w > s.w) o.w = s.w;
    } else {
      if (o.w < s.w) o.w = s.w;
    }
  }

  static __device__ __forceinline__ bool wet_out(const C& o, double /*D*/, const Par& p) {
    return o.H > p.hmin;
  }
  static __device__ __forceinline__ double eta_out(const C& o, double D) { return o.H - D; }
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
  const R* xib;
  const R* xisb;
  const R* xfac;
  const R* yib;
  const R* yisb;
  const R* tanR;
  int nx, ny, gflags;
  typename P::Par par;
};

template <class P>
__device__ __forceinline__ int ring_flag(int gflags, int xc, int r, int nx, int ny) {
  return ((gflags & G_FIX_W) && xc == 0) || ((gflags & G_FIX_E) && xc == nx - 1) ||
                 ((gflags & G_FIX_S) && r == 0) || ((gflags & G_FIX_N) && r == ny - 1)
             ? F_FIX
             : 0;
}

// x-sweep of one row across the wavefront.  In: post-(a) node of this lane
// along x (w = u, t = v).  Out: post-sweep (H, u, v) (valid on lanes 3..60).
template <class P>
__device__ __forceinline__ typename P::C xsweep_row(typename P::A a, typename P::R iL,
                                                    typename P::R iR, typename P::R iS,
                                                    const typename P::Par& par) {
  typedef typename P::A A;
  typedef typename P::B B;
  typedef typename P::C C;
  P::stage_a(a, par);
  A al = from_prev(a);
  A ar = from_next(a);
  B b = P::stage_b(al, a, ar, par);
  typename P::Bx bx = P::bx(b);
  typename P::Bx bl = from_prev(bx);
  typename P::Bx br = from_next(bx);
  C c = P::stage_cd(bl, b, br, iL, iR, iS, (typename P::R)0, par);
  typename P::Cx cc = P::cx(c);
  typename P::Cx cl = from_prev(cc);
  typename P::Cx cr = from_next(cc);
  if (b.f & F_EX) P::stage_e(c, cl, cr, b.src);
  return c;
}

// Per-lane y pipeline: register windows of the stages.
template <class P>
struct YPipe {
  typename P::A a0, a1, a2;   // rows r-2, r-1, r  (post-(a))
  typename P::B b0, b1, b2;   // rows r-3, r-2, r-1 (post-(b))
  typename P::C c0, c1, c2;   // rows r-4, r-3, r-2 (post-(d))

  __device__ __forceinline__ void reset() {
    a0.f = a1.f = a2.f = 0;
    b0.f = b1.f = b2.f = 0;
    b0.src = b1.src = b2.src = 0;
    a0.H = a1.H = a2.H = 0; a0.w = a1.w = a2.w = 0; a0.t = a1.t = a2.t = 0;
    a0.D = a1.D = a2.D = 0;
    b0.H = b1.H = b2.H = 0; b0.w = b1.w = b2.w = 0; b0.t = b1.t = b2.t = 0;
    b0.D = b1.D = b2.D = 0; b0.c = b1.c = b2.c = 0;
    c0.H = c1.H = c2.H = 0; c0.w = c1.w = c2.w = 0; c0.t = c1.t = c2.t = 0;
  }
};

// Push row r (y view: w = v, t = u) into the pipeline; returns the final
// state of row r-3 in `out` and its post-(b) view (flags, depth, flood
// source) in `ob`.
template <class P>
__device__ __forceinline__ void ypipe_push(YPipe<P>& y, typename P::A a, int r,
                                           const Ctx<P>& cx, typename P::C& out,
                                           typename P::B& ob) {
  typedef typename P::R R;
  P::stage_a(a, cx.par);
  y.a0 = y.a1; y.a1 = y.a2; y.a2 = a;
  // (b) on row r-1
  typename P::B bn = P::stage_b(y.a0, y.a1, y.a2, cx.par);
  y.b0 = y.b1; y.b1 = y.b2; y.b2 = bn;
  // (c)+(d) on row r-2 (the centre of the b window)
  const int rc = r - 2;
  R iL = 1, iR = 1, iS = 1, tr = 0;
  if (rc >= 0 && rc < cx.ny) {
    iL = cx.yib[rc];
    iR = cx.yib[rc + 1];
    iS = cx.yisb[rc];
    if (cx.gflags & G_SPHSRC) tr = cx.tanR[rc];
  }
  typename P::C cn = P::stage_cd(P::bx(y.b0), y.b1, P::bx(y.b2), iL, iR, iS, tr, cx.par);
  y.c0 = y.c1; y.c1 = y.c2; y.c2 = cn;
  // (e) on row r-3: centre of the c window; its (b) view is now b0
  out = y.c1;
  ob = y.b0;
  if (ob.f & F_EX) P::stage_e(out, P::cx(y.c0), P::cx(y.c2), ob.src);
}

template <class P, int ORDER>
__global__ void __launch_bounds__(WAVE * WAVES_PER_BLOCK)
step_kernel(const GridDesc* __restrict__ grids, const Tile* __restrict__ tiles, int ntiles,
            StepState* st, int parity, int count_step) {
  typedef typename P::R R;
  typedef typename P::A A;
  typedef typename P::C C;
  const int lane = threadIdx.x & (WAVE - 1);
  const int wave = threadIdx.x / WAVE;
  const int tid = blockIdx.x * WAVES_PER_BLOCK + wave;
  const long long n0 = st->n;
  if (tid < ntiles) {
    const Tile tl = tiles[tid];
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
    cx.xib = (const R*)g.xib;
    cx.xisb = (const R*)g.xisb;
    cx.xfac = (const R*)g.xfac;
    cx.yib = (const R*)g.yib;
    cx.yisb = (const R*)g.yisb;
    cx.tanR = (const R*)g.tanR;
    cx.nx = g.nx;
    cx.ny = g.ny;
    cx.gflags = g.flags;
    cx.par.dt = (R)g.dt;
    cx.par.hdt = (R)g.hdt;
    cx.par.dt2 = (R)g.dt2;
    cx.par.hmin = (R)g.hmin;
    cx.par.gn2 = (R)g.gn2;
    cx.par.inv16g = (R)g.inv16g;
    cx.par.dwall = (R)g.dwall;
    cx.par.flags = g.flags;
    const bool do_max = count_step && ((n0 + 1) % g.maxout == 0);

    const int nx = cx.nx, ny = cx.ny;
    const int xc = tl.x0 - HALO + lane;
    const bool col_in = xc >= 0 && xc < nx;
    const bool out_lane = lane >= HALO && lane < WAVE - HALO && col_in;
    // per-lane x metrics (constant along the march)
    R xiL = 1, xiR = 1, xiS = 1;
    if (col_in) {
      xiL = cx.xib[xc];
      xiR = cx.xib[xc + 1];
      xiS = cx.xisb[xc];
    }
    int bad = 0;

    auto load_row = [&](int r, A& a) {
      a.f = 0;
      a.H = 0; a.w = 0; a.t = 0; a.D = 0;
      if (r >= 0 && r < ny && col_in) {
        const long long k = (long long)r * nx + xc;
        a.H = cx.H[k];
        a.D = cx.D[k];
        a.w = cx.U[k];   // x view: w = u, t = v
        a.t = cx.V[k];
        a.f = F_EX | ring_flag<P>(cx.gflags, xc, r, nx, ny);
      }
    };
    auto store = [&](int r, const C& o, R D) {
      // o in x view: H, w = u, t = v
      if (!out_lane || r < 0 || r >= ny) return;
      const long long k = (long long)r * nx + xc;
      cx.Ho[k] = o.H;
      cx.Uo[k] = o.w;
      cx.Vo[k] = o.t;
      if (!(isfinite(o.H) && isfinite(o.w) && isfinite(o.t))) bad = 1;
      if (do_max && P::wet_out(o, D, cx.par)) {
        R e = P::eta_out(o, D);
        if (e > cx.emax[k]) cx.emax[k] = e;
        R s2 = o.w * o.w + o.t * o.t;
        if (s2 > cx.smax2[k]) cx.smax2[k] = s2;
      }
    };

    if (ORDER == ORD_X) {
      for (int r = tl.y0; r < tl.y0 + tl.rows; ++r) {
        A a;
        load_row(r, a);
        R f = cx.xfac[r];
        C o = xsweep_row<P>(a, f * xiL, f * xiR, f * xiS, cx.par);
        store(r, o, a.D);
      }
    } else if (ORDER == ORD_Y || ORDER == ORD_XY) {
      YPipe<P> yp;
      yp.reset();
      for (int r = tl.y0 - HALO; r < tl.y0 + tl.rows + HALO; ++r) {
        A a;
        load_row(r, a);
        if (ORDER == ORD_XY && r >= 0 && r < ny) {
          R f = cx.xfac[r];
          C o = xsweep_row<P>(a, f * xiL, f * xiR, f * xiS, cx.par);
          a.H = o.H; a.w = o.w; a.t = o.t;
          a.f &= (F_EX | F_FIX);
        }
        // y view: w = v, t = u
        A ay = a;
        ay.w = a.t;
        ay.t = a.w;
        C oy;
        typename P::B ob;
        ypipe_push<P>(yp, ay, r, cx, oy, ob);
        const int ro = r - HALO;
        if (ro >= tl.y0) {
          C o;
          o.H = oy.H; o.w = oy.t; o.t = oy.w;   // back to x view
          store(ro, o, ob.D);
        }
      }
    } else {  // ORD_YX: y pipeline on the loaded rows, then the x-sweep of its output row
      YPipe<P> yp;
      yp.reset();
      for (int r = tl.y0 - HALO; r < tl.y0 + tl.rows + HALO; ++r) {
        A a;
        load_row(r, a);
        A ay = a;
        ay.w = a.t;
        ay.t = a.w;
        C oy;
        typename P::B ob;
        ypipe_push<P>(yp, ay, r, cx, oy, ob);
        const int ro = r - HALO;
        if (ro >= tl.y0 && ro < ny) {
          A ax;
          ax.H = oy.H; ax.w = oy.t; ax.t = oy.w;
          ax.f = ob.f & (F_EX | F_FIX);
          ax.D = ob.D;
          R f = cx.xfac[ro];
          C o = xsweep_row<P>(ax, f * xiL, f * xiR, f * xiS, cx.par);
          store(ro, o, ax.D);
        }
      }
    }
    if (bad) st->bad = 1;
  }
  // step counter: the last wave to finish advances n (every wave has read
  // n0 before it arrives here)
  if (count_step && lane == 0) {
    __threadfence();
    const unsigned total = gridDim.x * WAVES_PER_BLOCK;
    unsigned prev = atomicAdd(&st->done, 1u);
    if (prev == total - 1) {
      st->done = 0;
      st->n = n0 + 1;
      __threadfence();
    }
  }
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
__global__ void sample_kernel(const GridDesc* grids, const SampleDesc* sd, StepState* st,
                              int parity) {
  const long long n = st->n;
  const SampleDesc s = *sd;
  const GridDesc& g = grids[s.grid];
  const R* H = (const R*)g.H[parity];
  const R* U = (const R*)g.U[parity];
  const R* V = (const R*)g.V[parity];
  const R* D = (const R*)g.D;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (s.ngauge > 0 && n % s.gout == 0 && n >= st->g_first && i < s.ngauge) {
    const long long slot = (n - st->g_first) / s.gout;
    if (slot < s.gcap) {
      const int k = s.gidx[i];
      R e;
      const bool w = node_wet<R>(g, H[k], D[k], e);
      double* o = s.grec + ((size_t)slot * s.ngauge + i) * 3;
      o[0] = w ? (double)e : 0.0;
      o[1] = w ? (double)U[k] : 0.0;
      o[2] = w ? (double)V[k] : 0.0;
    }
  }
  if (s.npts > 0 && n % s.bndout == 0 && n >= st->s_first && i < s.npts) {
    const long long slot = (n - st->s_first) / s.bndout;
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
__global__ void forcing_kernel(const GridDesc* grids, const ForceDesc* fd, StepState* st,
                               int parity) {
  const ForceDesc f = *fd;
  const GridDesc& g = grids[f.grid];
  const double t = (double)st->n * g.dt;
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

inline int nblk(long long N, int bs) { return (int)((N + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_step(int fp32, int order, const GridDesc* grids, const Tile* tiles, int ntiles,
                       StepState* st, int parity, int count_step, int nblocks, hipStream_t s) {
  dim3 grid(nblocks), block(WAVE * WAVES_PER_BLOCK);
  (void)fp32;
  switch (order) {
    case ORD_XY:
      hipLaunchKernelGGL((step_kernel<P64, ORD_XY>), grid, block, 0, s, grids, tiles, ntiles, st,
                         parity, count_step);
      break;
    case ORD_YX:
      hipLaunchKernelGGL((step_kernel<P64, ORD_YX>), grid, block, 0, s, grids, tiles, ntiles, st,
                         parity, count_step);
      break;
    case ORD_X:
      hipLaunchKernelGGL((step_kernel<P64, ORD_X>), grid, block, 0, s, grids, tiles, ntiles, st,
                         parity, count_step);
      break;
    default:
      hipLaunchKernelGGL((step_kernel<P64, ORD_Y>), grid, block, 0, s, grids, tiles, ntiles, st,
                         parity, count_step);
      break;
  }
  return hipGetLastError();
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
                         StepState* st, int parity, hipStream_t s) {
  CLF_SMALL_LAUNCH(sample_kernel, (long long)nthreads, gd, sd, st, parity);
}

hipError_t launch_forcing(int fp32, const GridDesc* gd, const ForceDesc* fd, int nthreads,
                          StepState* st, int parity, hipStream_t s) {
  CLF_SMALL_LAUNCH(forcing_kernel, (long long)nthreads, gd, fd, st, parity);
}

}  // namespace clf
