// Adjoint (reverse mode) of the FP64 split step, for gradients of a gauge
// misfit with respect to the initial state.
//
// One sweep maps the pre-sweep state of a line to the post-sweep state;
// with the branch decisions of steps (a), (b), (e) and the clipping of
// stateh frozen at the forward values, node k's output depends on the inputs
// at k-3..k+3 (radius 1 where the neighbourhood is wet and nothing floods).
// The adjoint of a sweep is the transposed Jacobian-vector product
//     lambda_in[j] = sum_{k=j-3..j+3} (d out_k / d in_j)^T lambda_out[k]
// (deterministic, no atomics).  In the wet interior only k = j-1..j+1
// contribute, each through the radius-1 update (c)+(d): every output node
// forms its own product once in hand-written reverse mode and the three
// contributions are gathered (lane shuffles along x, a register march down
// the columns along y).  Near the shoreline each 3x3 block d out_k / d in_j
// (fields h, w, t) comes from evaluating node k's update (a)-(e) once in a
// forward-mode dual number carrying the three directions of in_j.  Both
// restate the step of the paper (eqQ, solver2/solver1, stateu/stateh,
// inundation (a)-(e)) for one node from a window of the pre-sweep state, in
// the forward kernel's operation order, so that the branch decisions are
// the forward ones.

#include "clf_internal.h"

#include <math.h>

namespace clf {
namespace {

constexpr double kG = 9.81;

// ---------------------------------------------------------------------------
// Dual number with three derivative directions.
// ---------------------------------------------------------------------------
struct D3 {
  double v, d0, d1, d2;
};

__device__ __forceinline__ D3 dc(double v) { return D3{v, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ D3 operator+(const D3& a, const D3& b) {
  return D3{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2};
}
__device__ __forceinline__ D3 operator-(const D3& a, const D3& b) {
  return D3{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2};
}
__device__ __forceinline__ D3 operator-(const D3& a) { return D3{-a.v, -a.d0, -a.d1, -a.d2}; }
__device__ __forceinline__ D3 operator*(const D3& a, const D3& b) {
  return D3{a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1,
            a.d2 * b.v + a.v * b.d2};
}
__device__ __forceinline__ D3 operator*(double s, const D3& a) {
  return D3{s * a.v, s * a.d0, s * a.d1, s * a.d2};
}
__device__ __forceinline__ D3 operator*(const D3& a, double s) {
  return D3{a.v * s, a.d0 * s, a.d1 * s, a.d2 * s};
}
__device__ __forceinline__ D3 operator/(const D3& a, const D3& b) {
  const double q = a.v / b.v;
  const double ib = 1.0 / b.v;
  return D3{q, (a.d0 - q * b.d0) * ib, (a.d1 - q * b.d1) * ib, (a.d2 - q * b.d2) * ib};
}
__device__ __forceinline__ D3 dsqrt(const D3& a) {
  const double s = sqrt(a.v);
  const double k = s > 0.0 ? 0.5 / s : 0.0;
  return D3{s, a.d0 * k, a.d1 * k, a.d2 * k};
}
__device__ __forceinline__ D3 dcbrt(const D3& a) {
  const double s = cbrt(a.v);
  const double k = s != 0.0 ? 1.0 / (3.0 * s * s) : 0.0;
  return D3{s, a.d0 * k, a.d1 * k, a.d2 * k};
}

struct AdjPar {
  double dt, hdt, dt2, hmin, gn2, inv16g, dwall;
  int flags;
};

// Node of a line after step (a)/(b): value and flags.
struct Nd {
  D3 H, w, t;
  double D;
  int ex;   // exists
  int wet;  // wet after (a) / after (b)
  int src;  // flood source after (b): -1, +1, 2 (tie), 0
};

__device__ __forceinline__ double qv(const D3& x) { return x.v; }

__device__ __forceinline__ D3 qhat(const D3& la, const D3& xa, double Da, const D3& lb,
                                   const D3& xb, double Db, double inv) {
  D3 s = lb + la;
  D3 h = 0.5 * s;
  D3 dx = xb - xa;
  D3 m = h * dx;
  double gd = kG * (Db - Da);
  return (m - dc(gd)) * inv;
}

__device__ __forceinline__ D3 qhat_t(const D3& la, const D3& xa, const D3& lb, const D3& xb,
                                     double inv) {
  D3 s = lb + la;
  D3 h = 0.5 * s;
  D3 dx = xb - xa;
  return (h * dx) * inv;
}

__device__ __forceinline__ D3 advance(const AdjPar& p, const D3& xi, const D3& lam, const D3& QL,
                                      const D3& QR, const D3& Qc, double iS) {
  D3 a3;
  if (p.flags & G_SOLVER1) {
    a3 = xi - p.dt * Qc;
  } else {
    a3 = xi - p.hdt * (QL + QR);
  }
  D3 b3 = (lam * p.dt2) * (QR - QL);
  return a3 + b3 * iS;
}

// Steps (c)+(d) for node C with neighbours L, R (post-(b) views).
__device__ void update_node(const Nd& L, const Nd& C, const Nd& R, double iL, double iR, double iS,
                            double tanR, const AdjPar& p, D3& Ho, D3& wo, D3& to) {
  if (!C.wet) {
    Ho = dc(0.0); wo = dc(0.0); to = dc(0.0);
    return;
  }
  const bool lr = L.ex && L.wet, rr = R.ex && R.wet;
  const D3 Lw = lr ? L.w : -C.w, Lt = lr ? L.t : C.t;
  const double LD = lr ? L.D : C.D;
  const D3 Rw = rr ? R.w : -C.w, Rt = rr ? R.t : C.t;
  const double RD = rr ? R.D : C.D;
  const D3 cC = dsqrt(kG * C.H);
  const D3 cL = lr ? dsqrt(kG * L.H) : cC;
  const D3 cR = rr ? dsqrt(kG * R.H) : cC;
  const D3 xPL = Lw + 2.0 * cL, xPC = C.w + 2.0 * cC, xPR = Rw + 2.0 * cR;
  const D3 lPL = Lw + cL, lPC = C.w + cC, lPR = Rw + cR;
  const D3 xML = Lw - 2.0 * cL, xMC = C.w - 2.0 * cC, xMR = Rw - 2.0 * cR;
  const D3 lML = Lw - cL, lMC = C.w - cC, lMR = Rw - cR;
  const D3 QPL = qhat(lPL, xPL, LD, lPC, xPC, C.D, iL);
  const D3 QPR = qhat(lPC, xPC, C.D, lPR, xPR, RD, iR);
  const D3 QML = qhat(lML, xML, LD, lMC, xMC, C.D, iL);
  const D3 QMR = qhat(lMC, xMC, C.D, lMR, xMR, RD, iR);
  const D3 QTL = qhat_t(Lw, Lt, C.w, C.t, iL);
  const D3 QTR = qhat_t(C.w, C.t, Rw, Rt, iR);
  D3 QPc = dc(0.0), QMc = dc(0.0), QTc = dc(0.0);
  if (p.flags & G_SOLVER1) {
    QPc = qhat(lPL, xPL, LD, lPR, xPR, RD, iS);
    QMc = qhat(lML, xML, LD, lMR, xMR, RD, iS);
    QTc = qhat_t(Lw, Lt, Rw, Rt, iS);
  }
  D3 Pn = advance(p, xPC, lPC, QPL, QPR, QPc, iS);
  D3 Mn = advance(p, xMC, lMC, QML, QMR, QMc, iS);
  D3 Tn = advance(p, C.t, C.w, QTL, QTR, QTc, iS);
  if (tanR != 0.0) {
    D3 s3 = ((p.dt * cC) * C.w) * tanR;
    Pn = Pn + s3;
    Mn = Mn - s3;
  }
  D3 fr = dc(0.0);
  if (p.flags & G_FRICTION) {
    D3 sp = dsqrt(C.w * C.w + C.t * C.t);
    D3 den = C.H * dcbrt(C.H);
    fr = ((p.dt * p.gn2) * sp) / den;
    if (!(p.flags & G_FRIC_SEMI)) {
      // -alpha dt on p and q (solver2), alpha at the old level, alpha dt =
      // fr w with fr capped at 1 (friction does not reverse the flow)
      const D3 a = (fr.v < 1.0 ? fr : dc(1.0)) * C.w;
      Pn = Pn - a;
      Mn = Mn - a;
    }
  }
  D3 wv = 0.5 * (Pn + Mn);
  D3 dd = Pn - Mn;
  if (dd.v < 0.0) dd = dc(0.0);
  D3 Hv = (dd * dd) * p.inv16g;
  if ((p.flags & G_FRICTION) && (p.flags & G_FRIC_SEMI)) wv = wv / (dc(1.0) + fr);
  Ho = Hv; wo = wv; to = Tn;
}

// Step (b) for node C (post-(a) views in, post-(b) view out).
__device__ Nd flood_node(const Nd& L, const Nd& C, const Nd& R, const AdjPar& p) {
  Nd b = C;
  b.src = 0;
  const bool blocked = (p.flags & G_WALLMODE) && (C.D < p.dwall);
  if (!C.ex || C.wet || blocked) return b;
  bool qL = false, qR = false;
  double fL = 0.0, fR = 0.0;
  if (L.ex && L.wet) {
    fL = (L.H.v - L.D) + C.D;
    qL = fL > p.hmin;
  }
  if (R.ex && R.wet) {
    fR = (R.H.v - R.D) + C.D;
    qR = fR > p.hmin;
  }
  int s = 0;
  if (qL && qR) s = (fL > fR) ? -1 : ((fR > fL) ? 1 : 2);
  else if (qL) s = -1;
  else if (qR) s = 1;
  if (s == 0) return b;
  b.src = s;
  b.wet = 1;
  b.H = dc(p.hmin);
  if (s == 2) {
    b.w = 0.5 * (L.w + R.w);
    b.t = 0.5 * (L.t + R.t);
  } else if (s == -1) {
    b.w = L.w; b.t = L.t;
  } else {
    b.w = R.w; b.t = R.t;
  }
  return b;
}

// ---------------------------------------------------------------------------
// Reverse mode of the (c)+(d) update of one wet node k whose line neighbours
// are wet or outside the grid (a missing neighbour is the mirror ghost of k).
// Given the adjoint (gH, gW, gT) of node k's output (h, w, t), returns the
// adjoints of the inputs (h, w, t) of nodes k-1, k, k+1: one evaluation per
// output node, against three dual-number evaluations in the gather form.
// The forward part repeats the kernel's operation order, so the clip of
// stateh takes the forward decision.
// ---------------------------------------------------------------------------
struct NodeIn {
  double H, w, t, D;
};
struct Vjp3 {
  double LH, Lw, Lt, CH, Cw, Ct, RH, Rw, Rt;
};

__device__ __forceinline__ void qhat_rev(double la, double xa, double lb, double xb, double inv,
                                         double g, double& gla, double& gxa, double& glb,
                                         double& gxb) {
  // Q = (0.5 (lb + la) (xb - xa) - g (Db - Da)) inv
  const double gs = g * inv;
  const double a = 0.5 * (xb - xa) * gs;
  const double b = 0.5 * (lb + la) * gs;
  gla += a; glb += a;
  gxb += b; gxa -= b;
}

__device__ __forceinline__ Vjp3 vjp_local(const NodeIn& nl, const NodeIn& nc, const NodeIn& nr,
                                          bool lex, bool rex, double iL, double iR, double iS,
                                          double tanR, const AdjPar& p, double gH, double gW,
                                          double gT) {
  // ---- forward (same order as the step kernel) ----
  const double Cw = nc.w, Ct = nc.t, CD = nc.D;
  const double Cc = sqrt(kG * nc.H);
  const double Lw = lex ? nl.w : -Cw, Lt = lex ? nl.t : Ct, LD = lex ? nl.D : CD;
  const double Lc = lex ? sqrt(kG * nl.H) : Cc;
  const double Rw = rex ? nr.w : -Cw, Rt = rex ? nr.t : Ct, RD = rex ? nr.D : CD;
  const double Rc = rex ? sqrt(kG * nr.H) : Cc;
  const double xPL = Lw + 2.0 * Lc, xPC = Cw + 2.0 * Cc, xPR = Rw + 2.0 * Rc;
  const double lPL = Lw + Lc, lPC = Cw + Cc, lPR = Rw + Rc;
  const double xML = Lw - 2.0 * Lc, xMC = Cw - 2.0 * Cc, xMR = Rw - 2.0 * Rc;
  const double lML = Lw - Lc, lMC = Cw - Cc, lMR = Rw - Rc;
  auto qh = [](double la, double xa, double Da, double lb, double xb, double Db, double inv) {
    double s = lb + la;
    double h = 0.5 * s;
    double dx = xb - xa;
    double m = h * dx;
    double gd = kG * (Db - Da);
    return (m - gd) * inv;
  };
  auto qt = [](double la, double xa, double lb, double xb, double inv) {
    double s = lb + la;
    double h = 0.5 * s;
    double dx = xb - xa;
    return (h * dx) * inv;
  };
  const bool s1 = (p.flags & G_SOLVER1) != 0;
  const double QPL = qh(lPL, xPL, LD, lPC, xPC, CD, iL), QPR = qh(lPC, xPC, CD, lPR, xPR, RD, iR);
  const double QML = qh(lML, xML, LD, lMC, xMC, CD, iL), QMR = qh(lMC, xMC, CD, lMR, xMR, RD, iR);
  const double QTL = qt(Lw, Lt, Cw, Ct, iL), QTR = qt(Cw, Ct, Rw, Rt, iR);
  auto adv = [&](double xi, double lam, double QL, double QR, double Qc) {
    double a3 = s1 ? xi - p.dt * Qc : xi - p.hdt * (QL + QR);
    double b3 = (lam * p.dt2) * (QR - QL);
    return a3 + b3 * iS;
  };
  double QPc = 0.0, QMc = 0.0, QTc = 0.0;
  if (s1) {
    QPc = qh(lPL, xPL, LD, lPR, xPR, RD, iS);
    QMc = qh(lML, xML, LD, lMR, xMR, RD, iS);
    QTc = qt(Lw, Lt, Rw, Rt, iS);
  }
  double Pn = adv(xPC, lPC, QPL, QPR, QPc);
  double Mn = adv(xMC, lMC, QML, QMR, QMc);
  if (tanR != 0.0) {
    const double s3 = ((p.dt * Cc) * Cw) * tanR;
    Pn = Pn + s3;
    Mn = Mn - s3;
  }
  const bool fric = (p.flags & G_FRICTION) != 0;
  const bool semi = fric && (p.flags & G_FRIC_SEMI) != 0;
  double sp = 0.0, cb = 0.0, den = 1.0, fr = 0.0;
  if (fric) {
    sp = sqrt(Cw * Cw + Ct * Ct);
    cb = cbrt(nc.H);
    den = nc.H * cb;
    fr = ((p.dt * p.gn2) * sp) / den;
    if (!semi) {
      // -alpha dt on p and q (solver2), alpha dt = fr w, fr capped at 1
      const double fe = fr < 1.0 ? fr : 1.0;
      Pn = Pn - fe * Cw;
      Mn = Mn - fe * Cw;
    }
  }
  const double dd = Pn - Mn;
  const bool clipped = dd < 0.0;

  // ---- reverse ----
  double gCw = 0.0, gCt = 0.0, gCc = 0.0, gCH = 0.0;
  double gLw = 0.0, gLt = 0.0, gLc = 0.0;
  double gRw = 0.0, gRt = 0.0, gRc = 0.0;
  double gwv = gW;
  double gfr = 0.0;
  if (semi) {
    const double wv0 = 0.5 * (Pn + Mn);
    const double q = 1.0 + fr;
    gwv = gW / q;
    gfr = -gW * (wv0 / q) / q;
  }
  const double gdd = clipped ? 0.0 : gH * (2.0 * dd * p.inv16g);
  double gPn = 0.5 * gwv + gdd;
  double gMn = 0.5 * gwv - gdd;
  if (fric && !semi) {
    // a = fe w subtracted from both: da = -(gPn + gMn); the cap fe = 1 has
    // no derivative with respect to fr
    const double ga = -(gPn + gMn);
    gCw += ga * (fr < 1.0 ? fr : 1.0);
    if (fr < 1.0) gfr += ga * Cw;
  }
  if (fric) {
    const double gsp = gfr * (p.dt * p.gn2) / den;
    const double gden = -gfr * fr / den;
    if (sp > 0.0) {
      gCw += gsp * Cw / sp;
      gCt += gsp * Ct / sp;
    }
    gCH += gden * (cb + nc.H * (1.0 / (3.0 * cb * cb)));
  }
  if (tanR != 0.0) {
    const double gs3 = gPn - gMn;
    gCc += gs3 * (p.dt * Cw * tanR);
    gCw += gs3 * (p.dt * Cc * tanR);
  }
  // advance: out = xi - hdt (QL + QR) [or - dt Qc] + (lam dt2 (QR - QL)) iS
  double gxPL = 0, gxPC = 0, gxPR = 0, glPL = 0, glPC = 0, glPR = 0;
  double gxML = 0, gxMC = 0, gxMR = 0, glML = 0, glMC = 0, glMR = 0;
  auto adv_rev = [&](double g, double lam, double QL, double QR, double& gxi, double& glam,
                     double& gQL, double& gQR, double& gQc) {
    gxi += g;
    if (s1) gQc = -p.dt * g;
    else { gQL = -p.hdt * g; gQR = -p.hdt * g; }
    const double k = g * p.dt2 * iS;
    gQR += k * lam;
    gQL -= k * lam;
    glam += k * (QR - QL);
  };
  double gQPL = 0, gQPR = 0, gQPc = 0, gQML = 0, gQMR = 0, gQMc = 0, gQTL = 0, gQTR = 0, gQTc = 0;
  adv_rev(gPn, lPC, QPL, QPR, gxPC, glPC, gQPL, gQPR, gQPc);
  adv_rev(gMn, lMC, QML, QMR, gxMC, glMC, gQML, gQMR, gQMc);
  adv_rev(gT, Cw, QTL, QTR, gCt, gCw, gQTL, gQTR, gQTc);
  qhat_rev(lPL, xPL, lPC, xPC, iL, gQPL, glPL, gxPL, glPC, gxPC);
  qhat_rev(lPC, xPC, lPR, xPR, iR, gQPR, glPC, gxPC, glPR, gxPR);
  qhat_rev(lML, xML, lMC, xMC, iL, gQML, glML, gxML, glMC, gxMC);
  qhat_rev(lMC, xMC, lMR, xMR, iR, gQMR, glMC, gxMC, glMR, gxMR);
  qhat_rev(Lw, Lt, Cw, Ct, iL, gQTL, gLw, gLt, gCw, gCt);
  qhat_rev(Cw, Ct, Rw, Rt, iR, gQTR, gCw, gCt, gRw, gRt);
  if (s1) {
    qhat_rev(lPL, xPL, lPR, xPR, iS, gQPc, glPL, gxPL, glPR, gxPR);
    qhat_rev(lML, xML, lMR, xMR, iS, gQMc, glML, gxML, glMR, gxMR);
    qhat_rev(Lw, Lt, Rw, Rt, iS, gQTc, gLw, gLt, gRw, gRt);
  }
  // xP = w + 2c, lP = w + c, xM = w - 2c, lM = w - c
  gLw += gxPL + glPL + gxML + glML;
  gLc += 2.0 * gxPL + glPL - 2.0 * gxML - glML;
  gCw += gxPC + glPC + gxMC + glMC;
  gCc += 2.0 * gxPC + glPC - 2.0 * gxMC - glMC;
  gRw += gxPR + glPR + gxMR + glMR;
  gRc += 2.0 * gxPR + glPR - 2.0 * gxMR - glMR;
  Vjp3 o{};
  // ghosts fold into the node itself: (h, -w, t) of k
  if (lex) {
    o.LH = gLc * (0.5 * kG / Lc);
    o.Lw = gLw;
    o.Lt = gLt;
  } else {
    gCw -= gLw;
    gCt += gLt;
    gCc += gLc;
  }
  if (rex) {
    o.RH = gRc * (0.5 * kG / Rc);
    o.Rw = gRw;
    o.Rt = gRt;
  } else {
    gCw -= gRw;
    gCt += gRt;
    gCc += gRc;
  }
  o.CH = gCH + gCc * (0.5 * kG / Cc);
  o.Cw = gCw;
  o.Ct = gCt;
  return o;
}

// Line accessor for one sweep: node index along the line -> memory index,
// existence, inverse spacings and source factor.
struct Line {
  const double* H;
  const double* W;   // normal velocity field of this sweep
  const double* T;   // tangential velocity field
  const double* D;
  long long base;    // memory index of node 0 of the line
  long long step;    // memory stride along the line
  int n;             // nodes on the line
  const double* ib;  // [n+1]
  const double* isb; // [n]
  double fac;        // row factor on the inverse spacings (x-sweep), 1 in y
  const double* tan; // per node tan(lat)/R or null
};

__device__ __forceinline__ Nd load_pre(const Line& ln, int k, double hmin) {
  Nd a;
  a.src = 0;
  if (k < 0 || k >= ln.n) {
    a.ex = 0; a.wet = 0; a.D = 0.0;
    a.H = dc(0.0); a.w = dc(0.0); a.t = dc(0.0);
    return a;
  }
  const long long m = ln.base + (long long)k * ln.step;
  a.ex = 1;
  a.D = ln.D[m];
  a.H = dc(ln.H[m]);
  a.w = dc(ln.W[m]);
  a.t = dc(ln.T[m]);
  // step (a)
  a.wet = a.H.v > hmin;
  if (!a.wet) {
    a.H = dc(0.0); a.w = dc(0.0); a.t = dc(0.0);
  }
  return a;
}

__device__ __forceinline__ void seed(Nd& a) {
  // directions of this input node: h, w, t (only while it carries them:
  // a dry node's values were replaced by constants in step (a))
  if (a.ex && a.wet) {
    a.H.d0 = 1.0;
    a.w.d1 = 1.0;
    a.t.d2 = 1.0;
  }
}

__device__ __forceinline__ double ibk(const Line& ln, int k) { return ln.fac * ln.ib[k]; }

// d(out_k)/d(in_j) for output node k of the line and input node j, general
// radius-3 form: the window k-3..k+3 of the pre-sweep state is re-evaluated
// through steps (a)-(e) with in_j seeded.
__device__ void block_general(const Line& ln, int k, int j, const AdjPar& p, D3& Ho, D3& wo,
                              D3& to) {
  Nd a[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    a[i] = load_pre(ln, k - 3 + i, p.hmin);
    if (k - 3 + i == j) seed(a[i]);
  }
  Nd b[7];
#pragma unroll
  for (int i = 1; i < 6; ++i) b[i] = flood_node(a[i - 1], a[i], a[i + 1], p);
  D3 Hn[7], wn[7], tn[7];
  for (int i = 2; i < 5; ++i) {
    const int kk = k - 3 + i;
    if (kk < 0 || kk >= ln.n) {
      Hn[i] = dc(0.0); wn[i] = dc(0.0); tn[i] = dc(0.0);
      continue;
    }
    const double tr = ln.tan ? ln.tan[kk] : 0.0;
    update_node(b[i - 1], b[i], b[i + 1], ibk(ln, kk), ibk(ln, kk + 1), ln.fac * ln.isb[kk], tr, p,
                Hn[i], wn[i], tn[i]);
  }
  Ho = Hn[3]; wo = wn[3]; to = tn[3];
  const int s = b[3].src;
  if (s == 0) return;
  if (s == 2) {
    const D3 m = (Hn[4].v < Hn[2].v) ? Hn[4] : Hn[2];
    const D3 cap = 0.5 * m;
    if (Ho.v > cap.v) Ho = cap;
    return;
  }
  const int q = 3 + s;
  const D3 cap = 0.5 * Hn[q];
  if (Ho.v > cap.v) Ho = cap;
  if (s == -1) {
    if (wo.v > wn[q].v) wo = wn[q];
  } else {
    if (wo.v < wn[q].v) wo = wn[q];
  }
}

// Radius-1 form where nodes k-1..k+1 are wet or missing (nothing floods):
// steps (c)+(d) of node k only.
__device__ void block_local(const Line& ln, int k, int j, const AdjPar& p, D3& Ho, D3& wo,
                            D3& to) {
  Nd L = load_pre(ln, k - 1, p.hmin), C = load_pre(ln, k, p.hmin), R = load_pre(ln, k + 1, p.hmin);
  if (j == k - 1) seed(L);
  if (j == k) seed(C);
  if (j == k + 1) seed(R);
  const double tr = ln.tan ? ln.tan[k] : 0.0;
  update_node(L, C, R, ibk(ln, k), ibk(ln, k + 1), ln.fac * ln.isb[k], tr, p, Ho, wo, to);
}

__device__ __forceinline__ bool wet_or_missing(const Line& ln, int k, double hmin) {
  if (k < 0 || k >= ln.n) return true;
  return ln.H[ln.base + (long long)k * ln.step] > hmin;
}

// Adjoint of one sweep for input node j of the line.
__device__ void adjoint_node(const Line& ln, int j, const AdjPar& p, const double* lH,
                             const double* lW, const double* lT, double& aH, double& aW,
                             double& aT) {
  aH = 0.0; aW = 0.0; aT = 0.0;
  for (int k = j - 3; k <= j + 3; ++k) {
    if (k < 0 || k >= ln.n) continue;
    const bool local = wet_or_missing(ln, k - 1, p.hmin) && wet_or_missing(ln, k, p.hmin) &&
                       wet_or_missing(ln, k + 1, p.hmin);
    if (local && (k < j - 1 || k > j + 1)) continue;
    D3 Ho, wo, to;
    if (local) block_local(ln, k, j, p, Ho, wo, to);
    else block_general(ln, k, j, p, Ho, wo, to);
    const long long m = ln.base + (long long)k * ln.step;
    const double gH = lH[m], gW = lW[m], gT = lT[m];
    aH += Ho.d0 * gH + wo.d0 * gW + to.d0 * gT;
    aW += Ho.d1 * gH + wo.d1 * gW + to.d1 * gT;
    aT += Ho.d2 * gH + wo.d2 * gW + to.d2 * gT;
  }
}

// True when nodes j-4..j+4 of the line are all wet or missing: then every
// output k = j-3..j+3 has a radius-1 block and only k = j-1..j+1 touch in_j.
__device__ __forceinline__ bool window_local(const Line& ln, int j, double hmin) {
  bool ok = true;
#pragma unroll
  for (int d = -4; d <= 4; ++d) ok &= wet_or_missing(ln, j + d, hmin);
  return ok;
}

// axis 0: lines are rows (w = u, t = v); axis 1: columns (w = v, t = u).
// pre: state before the sweep; lam_*: adjoint of the state after it;
// out_*: adjoint of the state before it.  Node (i, jrow) sits at position
// i (axis 0) or jrow (axis 1) of its line.
constexpr int kAdjBlock = 128;

struct SweepArgs {
  const double *preH, *preU, *preV;
  const double *lamH, *lamU, *lamV;
  double *outH, *outU, *outV;
  unsigned char* flags;  // one per wavefront of the interior launch
};

__device__ __forceinline__ AdjPar adj_par(const GridDesc& g) {
  AdjPar p;
  p.dt = g.dt; p.hdt = g.hdt; p.dt2 = g.dt2; p.hmin = g.hmin; p.gn2 = g.gn2;
  p.inv16g = g.inv16g; p.dwall = g.dwall; p.flags = g.flags;
  return p;
}

template <int AXIS>
__device__ __forceinline__ Line make_line(const GridDesc& g, const SweepArgs& a, int i, int jrow) {
  Line ln;
  ln.H = a.preH;
  ln.D = (const double*)g.D;
  if (AXIS == 0) {
    ln.W = a.preU; ln.T = a.preV;
    ln.base = (long long)jrow * g.nx;
    ln.step = 1;
    ln.n = g.nx;
    ln.ib = (const double*)g.xib;
    ln.isb = (const double*)g.xisb;
    ln.fac = ((const double*)g.xfac)[jrow];
    ln.tan = nullptr;
  } else {
    ln.W = a.preV; ln.T = a.preU;
    ln.base = i;
    ln.step = g.nx;
    ln.n = g.ny;
    ln.ib = (const double*)g.yib;
    ln.isb = (const double*)g.yisb;
    ln.fac = 1.0;
    ln.tan = (g.flags & G_SPHSRC) ? (const double*)g.tanR : nullptr;
  }
  return ln;
}

template <int AXIS>
__device__ __forceinline__ void sweep_node(const GridDesc& g, const SweepArgs& a, const Line& ln,
                                           const AdjPar& p, int i, int jrow) {
  const long long me = (long long)jrow * g.nx + i;
  const int j = AXIS == 0 ? i : jrow;
  // the adjoint's normal / tangential fields follow the sweep axis
  const double* lW = AXIS == 0 ? a.lamU : a.lamV;
  const double* lT = AXIS == 0 ? a.lamV : a.lamU;
  double aH, aW, aT;
  adjoint_node(ln, j, p, a.lamH, lW, lT, aH, aW, aT);
  a.outH[me] = aH;
  if (AXIS == 0) { a.outU[me] = aW; a.outV[me] = aT; }
  else { a.outV[me] = aW; a.outU[me] = aT; }
}

// Flag of the shoreline launch for node (i, row): one per 64 columns of a row
// (the wavefronts of a 128-wide workgroup over the row).
__device__ __forceinline__ int flag_index(int i, int row, int nx) {
  const int gx = (nx + kAdjBlock - 1) / kAdjBlock;
  return row * gx * (kAdjBlock / 64) + i / 64;
}

constexpr int kAdjStrip = 62;  // output nodes per wavefront of the x reverse sweep

// Reverse of the x-sweep for the wet interior.  A wavefront covers nodes
// k = 62 b - 1 + lane of one row; each lane forms the reverse-mode product of
// its own node's update, and the three contributions to input node j come
// from lanes j-1, j, j+1 by lane shuffles.  Lanes 1..62 write input nodes
// whose window j-4..j+4 is wet or outside the grid; the others set the
// shoreline flag.
__global__ __launch_bounds__(64) void adjoint_local_x_kernel(GridDesc g, SweepArgs a) {
  const int lane = threadIdx.x;
  const int row = blockIdx.y;
  const int nx = g.nx;
  const int k = blockIdx.x * kAdjStrip - 1 + lane;
  const AdjPar p = adj_par(g);
  const long long base = (long long)row * nx;
  const double* H = a.preH;
  const double* D = (const double*)g.D;
  auto at = [&](int q) { return base + (q < 0 ? 0 : (q >= nx ? nx - 1 : q)); };
  auto load = [&](int q) {
    const long long m = at(q);
    return NodeIn{H[m], a.preU[m], a.preV[m], D[m]};
  };
  const bool kex = k >= 0 && k < nx, lex = k - 1 >= 0, rex = k + 1 < nx;
  const NodeIn nc = load(k), nl = load(k - 1), nr = load(k + 1);
  const bool ok = kex && nc.H > p.hmin && (!lex || nl.H > p.hmin) && (!rex || nr.H > p.hmin);
  Vjp3 v{};
  if (ok) {
    const double fac = ((const double*)g.xfac)[row];
    const double* ib = (const double*)g.xib;
    const long long m = base + k;
    v = vjp_local(nl, nc, nr, lex, rex, fac * ib[k], fac * ib[k + 1],
                  fac * ((const double*)g.xisb)[k], 0.0, p, a.lamH[m], a.lamU[m], a.lamV[m]);
  }
  // contributions of the left neighbour's update (its R part) and of the
  // right neighbour's (its L part)
  const double fLH = __shfl_up(v.RH, 1), fLw = __shfl_up(v.Rw, 1), fLt = __shfl_up(v.Rt, 1);
  const double fRH = __shfl_down(v.LH, 1), fRw = __shfl_down(v.Lw, 1),
               fRt = __shfl_down(v.Lt, 1);
  if (lane < 1 || lane > kAdjStrip || !kex) return;
  bool local = true;
#pragma unroll
  for (int d = -4; d <= 4; ++d) {
    const int q = k + d;
    local &= (q < 0 || q >= nx || H[at(q)] > p.hmin);
  }
  if (!local) {
    a.flags[flag_index(k, row, nx)] = 1;
    return;
  }
  const long long m = base + k;
  a.outH[m] = (fLH + v.CH) + fRH;
  a.outU[m] = (fLw + v.Cw) + fRw;
  a.outV[m] = (fLt + v.Ct) + fRt;
}

// Reverse of the y-sweep for the wet interior.  A wavefront covers 64
// columns and marches down a band of rows; at row r each lane forms the
// reverse-mode product of node r's update and writes input node r-1 from
// the products of rows r-2, r-1 and r held in registers.
__global__ __launch_bounds__(64) void adjoint_local_y_kernel(GridDesc g, SweepArgs a, int seg) {
  const int lane = threadIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int i = blockIdx.x * 64 + lane;
  const bool col = i < nx;
  const int ic = col ? i : nx - 1;
  const int y0 = blockIdx.y * seg;
  const int y1 = y0 + seg < ny ? y0 + seg : ny;
  const AdjPar p = adj_par(g);
  const double* H = a.preH;
  const double* D = (const double*)g.D;
  const double* yib = (const double*)g.yib;
  const double* yisb = (const double*)g.yisb;
  const double* tanR = (g.flags & G_SPHSRC) ? (const double*)g.tanR : nullptr;
  auto at = [&](int r) { return (long long)(r < 0 ? 0 : (r >= ny ? ny - 1 : r)) * nx + ic; };
  // y view: w = v, t = u
  auto load = [&](int r) {
    const long long m = at(r);
    return NodeIn{H[m], a.preV[m], a.preU[m], D[m]};
  };
  auto wom = [&](int r) { return (r < 0 || r >= ny || H[at(r)] > p.hmin) ? 1u : 0u; };
  // bit b of wb: row r+3-b is wet or outside the grid (b = 0..8 at row r)
  unsigned wb = 0;
  for (int rr = y0 - 6; rr <= y0 + 1; ++rr) wb = (wb << 1) | wom(rr);
  NodeIn nl = load(y0 - 2), nc = load(y0 - 1);
  double R2H = 0, R2w = 0, R2t = 0;  // row r-2's contribution to row r-1
  double R1H = 0, R1w = 0, R1t = 0;  // row r-1's contribution to row r
  double C1H = 0, C1w = 0, C1t = 0;  // row r-1's contribution to itself
  for (int r = y0 - 1; r <= y1; ++r) {
    const NodeIn nr = load(r + 1);
    wb = (wb << 1) | wom(r + 3);
    const bool rin = r >= 0 && r < ny;
    const bool lex = r - 1 >= 0, rex = r + 1 < ny;
    const bool ok = col && rin && nc.H > p.hmin && (!lex || nl.H > p.hmin) &&
                    (!rex || nr.H > p.hmin);
    Vjp3 v{};
    if (ok) {
      const long long m = (long long)r * nx + i;
      v = vjp_local(nl, nc, nr, lex, rex, yib[r], yib[r + 1], yisb[r], tanR ? tanR[r] : 0.0, p,
                    a.lamH[m], a.lamV[m], a.lamU[m]);
    }
    const int j = r - 1;
    if (j >= y0) {
      const bool local = (wb & 0x1FFu) == 0x1FFu;
      if (__ballot(col && !local) != 0 && lane == 0) a.flags[flag_index(blockIdx.x * 64, j, nx)] = 1;
      if (col && local) {
        const long long m = (long long)j * nx + i;
        a.outH[m] = (R2H + C1H) + v.LH;
        a.outV[m] = (R2w + C1w) + v.Lw;
        a.outU[m] = (R2t + C1t) + v.Lt;
      }
    }
    R2H = R1H; R2w = R1w; R2t = R1t;
    R1H = v.RH; R1w = v.Rw; R1t = v.Rt;
    C1H = v.CH; C1w = v.Cw; C1t = v.Ct;
    nl = nc;
    nc = nr;
  }
}

// Shoreline launch: one wavefront per workgroup, grid-stride over chunks of
// 64 flags of the interior launches: the lanes read a chunk at once, and
// each flagged wavefront of it is redone here for its non-local nodes, and
// its flag cleared for the next sweep.
template <int AXIS>
__global__ __launch_bounds__(64) void adjoint_general_kernel(GridDesc g, SweepArgs a, int nwaves,
                                                             int gx) {
  constexpr int kWpb = kAdjBlock / 64;
  const AdjPar p = adj_par(g);
  const int lane = threadIdx.x;
  const int nchunks = (nwaves + 63) / 64;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int wl = c * 64 + lane;
    unsigned long long set = __ballot(wl < nwaves && a.flags[wl] != 0);
    while (set != 0) {
      const int w = c * 64 + (__ffsll((unsigned long long)set) - 1);
      set &= set - 1;
      const int b = w / kWpb, part = w % kWpb;
      const int jrow = b / gx;
      const int i = (b % gx) * kAdjBlock + part * 64 + lane;
      if (i < g.nx) {
        const Line ln = make_line<AXIS>(g, a, i, jrow);
        if (!window_local(ln, AXIS == 0 ? i : jrow, p.hmin)) sweep_node<AXIS>(g, a, ln, p, i, jrow);
      }
      if (lane == 0) a.flags[w] = 0;
    }
  }
}

// Record adjoints of one level: lambda += d(record)/d(state)^T dL/drecord.
// A record is (h - d, u, v) on wet nodes, zeros on dry ones.  One thread per
// gauge node: the first gauge on a node adds the records of every gauge on
// that node, in gauge order (deterministic, no atomics).
__global__ void inject_kernel(GridDesc g, const double* H, const long long* gidx, int ng,
                              const double* rec_adj, double* lamH, double* lamU, double* lamV) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ng) return;
  const long long k = gidx[q];
  for (int r = 0; r < q; ++r)
    if (gidx[r] == k) return;
  if (!(H[k] > g.hmin)) return;
  double aH = lamH[k], aU = lamU[k], aV = lamV[k];
  for (int r = q; r < ng; ++r)
    if (gidx[r] == k) {
      aH += rec_adj[3 * r + 0];
      aU += rec_adj[3 * r + 1];
      aV += rec_adj[3 * r + 2];
    }
  lamH[k] = aH; lamU[k] = aU; lamV[k] = aV;
}

// Adjoint of the initial condition h = max(d + eta, 0) (free-surface
// deformation) with dry nodes zeroed: pass lambda through on wet nodes.
__global__ void initial_adjoint_kernel(GridDesc g, const double* H0, const double* lamH,
                                       const double* lamU, const double* lamV, double* dEta,
                                       double* dU, double* dV, long long N) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const bool wet = H0[k] > g.hmin;
  if (dEta) dEta[k] = wet ? lamH[k] : 0.0;
  if (dU) dU[k] = wet ? lamU[k] : 0.0;
  if (dV) dV[k] = wet ? lamV[k] : 0.0;
}

}  // namespace

int adjoint_flag_count(int nx, int ny) {
  return (nx + kAdjBlock - 1) / kAdjBlock * (kAdjBlock / 64) * ny;
}

hipError_t launch_adjoint_sweep(const GridDesc* gd_host, int axis, const double* preH,
                                const double* preU, const double* preV, const double* lamH,
                                const double* lamU, const double* lamV, double* outH,
                                double* outU, double* outV, unsigned char* flags, hipStream_t s) {
  SweepArgs a{preH, preU, preV, lamH, lamU, lamV, outH, outU, outV, flags};
  const int gx = (gd_host->nx + kAdjBlock - 1) / kAdjBlock;
  const int nwaves = adjoint_flag_count(gd_host->nx, gd_host->ny);
  const int nchunks = (nwaves + 63) / 64;
  const int nb = nchunks < 1024 ? nchunks : 1024;
  if (axis == 0) {
    const dim3 gxs((gd_host->nx + kAdjStrip - 1) / kAdjStrip, gd_host->ny);
    hipLaunchKernelGGL(adjoint_local_x_kernel, gxs, dim3(64), 0, s, *gd_host, a);
    hipLaunchKernelGGL(adjoint_general_kernel<0>, dim3(nb), dim3(64), 0, s, *gd_host, a, nwaves, gx);
  } else {
    // row bands: enough wavefronts to fill the GPU, at least 8 rows each
    const int nbx = (gd_host->nx + 63) / 64;
    long long sg = (long long)nbx * gd_host->ny / 4096;
    const int seg = (int)(sg < 8 ? 8 : (sg > 64 ? 64 : sg));
    const dim3 gys(nbx, (gd_host->ny + seg - 1) / seg);
    hipLaunchKernelGGL(adjoint_local_y_kernel, gys, dim3(64), 0, s, *gd_host, a, seg);
    hipLaunchKernelGGL(adjoint_general_kernel<1>, dim3(nb), dim3(64), 0, s, *gd_host, a, nwaves, gx);
  }
  return hipGetLastError();
}

hipError_t launch_inject(const GridDesc* gd_host, const double* H, const long long* gidx, int ng,
                         const double* rec_adj, double* lamH, double* lamU, double* lamV,
                         hipStream_t s) {
  if (ng <= 0) return hipSuccess;
  const int bs = 64;
  hipLaunchKernelGGL(inject_kernel, dim3((ng + bs - 1) / bs), dim3(bs), 0, s, *gd_host, H, gidx, ng,
                     rec_adj, lamH, lamU, lamV);
  return hipGetLastError();
}

hipError_t launch_initial_adjoint(const GridDesc* gd_host, const double* H0, const double* lamH,
                                  const double* lamU, const double* lamV, double* dEta, double* dU,
                                  double* dV, long long N, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(initial_adjoint_kernel, dim3((unsigned)((N + bs - 1) / bs)), dim3(bs), 0, s,
                     *gd_host, H0, lamH, lamU, lamV, dEta, dU, dV, N);
  return hipGetLastError();
}

}  // namespace clf
