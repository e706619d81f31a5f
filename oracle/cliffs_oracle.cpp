// Cliffs split-step ORACLE: a plain, slow, FP64 CPU implementation of the
// dimensionally split VTCS-2 time step with the moving-cliff wet/dry update
// and the depth-jump preprocessing, written from the paper (Tolkova, Cliffs
// User Manual, arXiv 1410.0753) for testing only.
//
// TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
// CPU-baseline leg may load this library.  It shares no code, header or
// constant generator with the GPU library: every formula below is written
// out here from the paper, in the paper's order and notation, with plain
// loops over rows (x-sweep) and columns (y-sweep).
//
// Paper passages followed:
//   * model equations: section Numerics / Difference Scheme, eq1, eqABC;
//   * dimensional splitting into 1-D problems: eq2A, eq2B;
//   * Riemann invariants p = u + 2 sqrt(gh), q = u - 2 sqrt(gh) and the three
//     convection problems pq1, pq2, pq3;
//   * depth-balanced difference Q(k,j): eqQ;
//   * the update: solver2 (default) and solver1;
//   * state recovery: stateu, stateh;
//   * the inundation cycle (a)-(e): section Inundation algorithm;
//   * depth preprocessing: section Numerical stability, eqs dstab, newdw, newdc,
//     and the depth_ssl defaults (alpha = 2, min depth 0.1 m).
//
// Where the paper is silent, the readings are the ones listed in the design
// notes of this repository (dry threshold H > h_min is wet; tangential
// velocity advected with the solver2 form; mirror-ghost walls half a node
// out; flooding ties; direction-aware velocity cap; H = max(P-M,0)^2/16g;
// arc-length spherical spacing with a tan(lat) continuity source; linear
// time interpolation of forcing; bilinear wet-weighted nesting output).
// Bottom friction is the -alpha_j dt term that solver2 and solver1 carry on
// p and q, with alpha the Manning acceleration g n^2 w |U| / h^(4/3) taken at
// the old time level like every other right-hand-side term (ptaylor), its
// decrement capped at the velocity itself (friction does not reverse the
// flow); a semi-implicit form is kept as an option.  Open (radiating) edges are an
// addition of this repository, not in the paper (see open_ghost).
//
// Floating-point order.  Every expression is written with explicit
// parentheses in the order fixed by the formulation note, compiled with
// -ffp-contract=off, so that an independent implementation following the
// same note can reproduce the results bit for bit.
//
// Parity status: pinned by the CPU test-suite (lake at rest, linear
// single-node pulse closed forms eq:u/eq:et and eq:u2/eq:et2, Lax-Wendroff
// Fourier factor, wave speed sqrt(gH), CFL threshold, mirror symmetry,
// transposition, 1-D reduction, wet-front advance, flooding tie on a
// symmetric sill, preprocessing postcondition, sea-floor deformation,
// friction's one-step closed form and first-order convergence to the decay
// law, open-edge transparency and drainage, restart, complex-step vs finite
// differences).  The paper gives no spherical equations; the spherical form
// is pinned by the lake at rest, the equator limit, the zonal wave speed at
// 45 N (the cos(lat) factor of the x spacing) and the first-order
// convergence of the area-weighted volume sum(h cos(lat)), which the
// tan(lat) continuity source decides.  The momentum equations carry no
// spherical terms (none pinned).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kG = 9.81;
const double kPi = 3.14159265358979323846;

typedef std::complex<double> cplx;

inline double re(double a) { return a; }
inline double re(const cplx& a) { return a.real(); }
inline double sqrt_t(double a) { return std::sqrt(a); }
inline cplx sqrt_t(const cplx& a) { return std::sqrt(a); }
inline double cbrt_t(double a) { return std::cbrt(a); }
inline cplx cbrt_t(const cplx& a) { return std::pow(a, 1.0 / 3.0); }

struct Par {
  double dt, hdt, dt2, hmin, n2, gn2, inv16g, R;
  int itopo, solver, order, sph_metric;
  double dwall;
  int maxout, gout, bndout;
  int fric_form;   // 0: explicit -alpha dt on p and q (solver2); 1: semi-implicit option
  int open_mask;   // open (radiating) edges: 1 W, 2 E, 4 S, 8 N
};

// ---------------------------------------------------------------------------
// Depth preprocessing (Numerical stability: dstab, newdw, newdc).
// Reading: raise wet depths below min_depth to min_depth, then repeat Jacobi
// passes (all rows, then all columns) until nothing changes.  For a wet node
// with both line neighbours present: if max(d_l, d_r)/d > alpha^2 then
//   both neighbours wet  -> d = (sqrt(d_l) + sqrt(d_r))^2 / 4   (newdw)
//   one neighbour dry    -> d = d_w / alpha^2                   (newdc)
// ---------------------------------------------------------------------------
bool ssl_fix(double dl, double dj, double dr, double a2, double* out) {
  if (!(dj > 0.0)) return false;
  double mx = dl > dr ? dl : dr;
  if (!((mx / dj) > a2)) return false;
  bool wl = dl > 0.0, wr = dr > 0.0;
  if (wl && wr) {
    double s = std::sqrt(dl) + std::sqrt(dr);
    *out = (s * s) * 0.25;
    return true;
  }
  if (wl || wr) {
    double dw = wl ? dl : dr;
    *out = dw / a2;
    return true;
  }
  return false;
}

int ssl_run(int nx, int ny, double* d, double alpha, double min_depth) {
  const size_t N = (size_t)nx * ny;
  for (size_t i = 0; i < N; ++i)
    if (d[i] > 0.0 && d[i] < min_depth) d[i] = min_depth;
  const double a2 = alpha * alpha;
  std::vector<double> nd(N);
  for (int pass = 1; pass <= 1000; ++pass) {
    bool changed = false;
    // row-wise (along x)
    std::copy(d, d + N, nd.begin());
    if (nx >= 3) {
      for (int j = 0; j < ny; ++j)
        for (int i = 1; i + 1 < nx; ++i) {
          size_t k = (size_t)j * nx + i;
          double v;
          if (ssl_fix(d[k - 1], d[k], d[k + 1], a2, &v) && v != d[k]) {
            nd[k] = v;
            changed = true;
          }
        }
    }
    std::copy(nd.begin(), nd.end(), d);
    // column-wise (along y)
    if (ny >= 3) {
      for (int j = 1; j + 1 < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          size_t k = (size_t)j * nx + i;
          double v;
          if (ssl_fix(d[k - nx], d[k], d[k + nx], a2, &v) && v != d[k]) {
            nd[k] = v;
            changed = true;
          }
        }
    }
    std::copy(nd.begin(), nd.end(), d);
    if (!changed) return pass;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// One 1-D sweep over a line of n nodes (section Inundation algorithm (a)-(e)
// with solver2 / solver1 as step (d)).  w = normal velocity, t = tangential.
// ib[k] = 1/Delta_{k-1} for k = 0..n (Delta_{-1} = Delta_0, Delta_{n-1} =
// Delta_{n-2}); isb[k] = 1/(Delta_{k-1} + Delta_k).  fac multiplies every
// inverse spacing (spherical row factor, 1 otherwise).  tanR (per node, may
// be null) adds the spherical continuity source (y-sweep only).
// ---------------------------------------------------------------------------
template <class T>
struct Nb {
  T H, w, t;
  double D;
};

template <class T>
T Qhat(const T& lam_a, const T& xi_a, double D_a, const T& lam_b, const T& xi_b,
       double D_b, double Gf, double inv) {
  // eqQ with a = left node, b = right node: Q(b, a)
  T s = lam_b + lam_a;
  T h = 0.5 * s;
  T dx = xi_b - xi_a;
  T m = h * dx;
  double dd = D_b - D_a;
  double gd = Gf * dd;
  T num = m - gd;
  return num * inv;
}

template <class T>
T Qhat_t(const T& lam_a, const T& xi_a, const T& lam_b, const T& xi_b, double inv) {
  // eqQ for pq3 (no depth term)
  T s = lam_b + lam_a;
  T h = 0.5 * s;
  T dx = xi_b - xi_a;
  T m = h * dx;
  return m * inv;
}

template <class T>
T advance(const Par& p, const T& xi, const T& lam, const T& QL, const T& QR, const T& Qc,
          double iS) {
  // solver2: xi - dt/2 (QL + QR) + lam dt^2 (QR - QL)/(Dx_{k-1} + Dx_k)
  // solver1: xi - dt Q(k+1,k-1) + lam dt^2 (QR - QL)/(Dx_{k-1} + Dx_k)
  T a3;
  if (p.solver == 1) {
    T a2 = p.dt * Qc;
    a3 = xi - a2;
  } else {
    T a1 = QL + QR;
    T a2 = p.hdt * a1;
    a3 = xi - a2;
  }
  T b1 = QR - QL;
  T b2 = lam * p.dt2;
  T b3 = b2 * b1;
  T b4 = b3 * iS;
  return a3 + b4;
}

// Open (radiating) edge, a reading of this repository (the paper has no open
// boundary): the neighbour beyond an open edge is a ghost that carries the
// edge node's outgoing Riemann invariant unchanged and the still-water value
// of the incoming one.  Beyond the right end the outgoing invariant is
// p = w + 2c and the incoming one q0 = -2 sqrt(g d); beyond the left end the
// outgoing one is q = w - 2c and the incoming one p0 = 2 sqrt(g d).  The
// ghost's velocity and celerity follow from stateu and c = (p - q)/4; its
// depth and tangential velocity are the edge node's.
template <class T>
void open_ghost(const T& w, const T& c, double D, bool right, T* wg, T* cg) {
  const double c0 = std::sqrt(kG * (D > 0.0 ? D : 0.0));
  T pp, qq;
  if (right) {
    pp = w + 2.0 * c;
    qq = T(-2.0 * c0);
  } else {
    pp = T(2.0 * c0);
    qq = w - 2.0 * c;
  }
  *wg = 0.5 * (pp + qq);
  T cc = 0.25 * (pp - qq);
  if (re(cc) < 0.0) cc = T(0.0);
  *cg = cc;
}

template <class T>
void sweep_line(const Par& p, int n, T* H, T* w, T* t, const double* D, const unsigned char* fixed,
                const double* ib, const double* isb, double fac, const double* tanR,
                bool open_l, bool open_r) {
  std::vector<char> wet0(n), wet1(n);
  std::vector<int> src(n, 0);  // -1 from left, +1 from right, 2 tie, 0 none
  std::vector<T> H1(n), w1(n), t1(n), Hn(n), wn(n), tn(n);
  const T zero = T(0.0);

  // (a) dry marking: H <= h_min is dry; dry nodes carry no water, no velocity
  for (int k = 0; k < n; ++k) {
    wet0[k] = re(H[k]) > p.hmin;
    if (!wet0[k]) {
      H[k] = zero;
      w[k] = zero;
      t[k] = zero;
    }
  }
  // (b) flooding of dry nodes next to wet ones
  for (int k = 0; k < n; ++k) {
    H1[k] = H[k];
    w1[k] = w[k];
    t1[k] = t[k];
    wet1[k] = wet0[k];
    if (wet0[k] || fixed[k]) continue;
    if (p.itopo == 0 && D[k] < p.dwall) continue;  // vertical-wall mode: land never floods
    bool qL = false, qR = false;
    T fL = zero, fR = zero;
    if (k > 0 && wet0[k - 1]) {
      fL = (H[k - 1] - D[k - 1]) + D[k];
      qL = re(fL) > p.hmin;
    }
    if (k + 1 < n && wet0[k + 1]) {
      fR = (H[k + 1] - D[k + 1]) + D[k];
      qR = re(fR) > p.hmin;
    }
    int s = 0;
    if (qL && qR) {
      if (re(fL) > re(fR)) s = -1;
      else if (re(fR) > re(fL)) s = 1;
      else s = 2;
    } else if (qL) {
      s = -1;
    } else if (qR) {
      s = 1;
    }
    if (s == 0) continue;
    src[k] = s;
    wet1[k] = 1;
    H1[k] = T(p.hmin);
    if (s == 2) {
      w1[k] = 0.5 * (w[k - 1] + w[k + 1]);
      t1[k] = 0.5 * (t[k - 1] + t[k + 1]);
    } else {
      w1[k] = w[k + s];
      t1[k] = t[k + s];
    }
  }
  // (c) walls at wet/dry interfaces and grid edges, (d) the update
  for (int k = 0; k < n; ++k) {
    if (fixed[k]) {
      Hn[k] = H1[k];
      wn[k] = w1[k];
      tn[k] = t1[k];
      continue;
    }
    if (!wet1[k]) {
      Hn[k] = zero;
      wn[k] = zero;
      tn[k] = zero;
      continue;
    }
    Nb<T> L, C, Rr;
    C.H = H1[k]; C.w = w1[k]; C.t = t1[k]; C.D = D[k];
    T cC = sqrt_t(kG * C.H), cL, cR;
    if (k > 0 && wet1[k - 1]) {
      L.H = H1[k - 1]; L.w = w1[k - 1]; L.t = t1[k - 1]; L.D = D[k - 1];
      cL = sqrt_t(kG * L.H);
    } else if (k == 0 && open_l) {
      L.H = C.H; L.t = C.t; L.D = C.D;  // open edge ghost (only w and c are used)
      open_ghost(C.w, cC, C.D, false, &L.w, &cL);
    } else {
      L.H = C.H; L.w = -C.w; L.t = C.t; L.D = C.D;  // mirror ghost
      cL = cC;
    }
    if (k + 1 < n && wet1[k + 1]) {
      Rr.H = H1[k + 1]; Rr.w = w1[k + 1]; Rr.t = t1[k + 1]; Rr.D = D[k + 1];
      cR = sqrt_t(kG * Rr.H);
    } else if (k == n - 1 && open_r) {
      Rr.H = C.H; Rr.t = C.t; Rr.D = C.D;
      open_ghost(C.w, cC, C.D, true, &Rr.w, &cR);
    } else {
      Rr.H = C.H; Rr.w = -C.w; Rr.t = C.t; Rr.D = C.D;
      cR = cC;
    }
    const double iL = fac * ib[k];
    const double iR = fac * ib[k + 1];
    const double iS = fac * isb[k];
    // family P: xi = w + 2c, lambda = w + c
    T xP_L = L.w + 2.0 * cL, xP_C = C.w + 2.0 * cC, xP_R = Rr.w + 2.0 * cR;
    T lP_L = L.w + cL, lP_C = C.w + cC, lP_R = Rr.w + cR;
    // family M: xi = w - 2c, lambda = w - c
    T xM_L = L.w - 2.0 * cL, xM_C = C.w - 2.0 * cC, xM_R = Rr.w - 2.0 * cR;
    T lM_L = L.w - cL, lM_C = C.w - cC, lM_R = Rr.w - cR;
    T QPL = Qhat(lP_L, xP_L, L.D, lP_C, xP_C, C.D, kG, iL);
    T QPR = Qhat(lP_C, xP_C, C.D, lP_R, xP_R, Rr.D, kG, iR);
    T QML = Qhat(lM_L, xM_L, L.D, lM_C, xM_C, C.D, kG, iL);
    T QMR = Qhat(lM_C, xM_C, C.D, lM_R, xM_R, Rr.D, kG, iR);
    T QTL = Qhat_t(L.w, L.t, C.w, C.t, iL);
    T QTR = Qhat_t(C.w, C.t, Rr.w, Rr.t, iR);
    T QPc = zero, QMc = zero, QTc = zero;
    if (p.solver == 1) {
      QPc = Qhat(lP_L, xP_L, L.D, lP_R, xP_R, Rr.D, kG, iS);
      QMc = Qhat(lM_L, xM_L, L.D, lM_R, xM_R, Rr.D, kG, iS);
      QTc = Qhat_t(L.w, L.t, Rr.w, Rr.t, iS);
    }
    T Pn = advance(p, xP_C, lP_C, QPL, QPR, QPc, iS);
    T Mn = advance(p, xM_C, lM_C, QML, QMR, QMc, iS);
    T Tn = advance(p, C.t, C.w, QTL, QTR, QTc, iS);
    if (tanR != nullptr && tanR[k] != 0.0) {
      // spherical continuity source +h v tan(lat)/R: p += dt c v tan/R, q -= the same
      T s1 = p.dt * cC;
      T s2 = s1 * C.w;
      T s3 = s2 * tanR[k];
      Pn = Pn + s3;
      Mn = Mn - s3;
    }
    if (p.n2 > 0.0 && p.fric_form == 0) {
      // bottom friction, the -alpha_j dt term of solver2 / solver1 on p and q,
      // with the Manning acceleration alpha = g n^2 w |U| / h^(4/3) at the old
      // time level: alpha dt = f w with f = dt g n^2 |U| / h^(4/3).  Friction
      // cannot reverse the flow, so f is capped at 1 (reading: in thin fast
      // layers the uncapped explicit term overshoots and grows without bound)
      T sp = sqrt_t(C.w * C.w + C.t * C.t);
      T den = C.H * cbrt_t(C.H);
      T f = ((p.dt * p.gn2) * sp) / den;
      if (re(f) > 1.0) f = T(1.0);
      T a = f * C.w;
      Pn = Pn - a;
      Mn = Mn - a;
    }
    // stateu, stateh
    T ws = Pn + Mn;
    T wv = 0.5 * ws;
    T dd = Pn - Mn;
    if (re(dd) < 0.0) dd = zero;
    T Hv = (dd * dd) * p.inv16g;
    if (p.n2 > 0.0 && p.fric_form == 1) {
      // option: semi-implicit Manning on the normal velocity, w' / (1 + dt alpha / w)
      T sp = sqrt_t(C.w * C.w + C.t * C.t);
      T den = C.H * cbrt_t(C.H);
      T fr = (p.dt * p.gn2 * sp) / den;
      wv = wv / (1.0 + fr);
    }
    Hn[k] = Hv;
    wn[k] = wv;
    tn[k] = Tn;
  }
  // (e) limits for newly wet nodes
  for (int k = 0; k < n; ++k) {
    int s = src[k];
    if (s == 0) continue;
    if (s == 2) {
      T a = Hn[k - 1], b = Hn[k + 1];
      T m = re(b) < re(a) ? b : a;
      T cap = 0.5 * m;
      if (re(Hn[k]) > re(cap)) Hn[k] = cap;
      continue;
    }
    int j = k + s;
    T cap = 0.5 * Hn[j];
    if (re(Hn[k]) > re(cap)) Hn[k] = cap;
    if (s == -1) {
      if (re(wn[k]) > re(wn[j])) wn[k] = wn[j];
    } else {
      if (re(wn[k]) < re(wn[j])) wn[k] = wn[j];
    }
  }
  for (int k = 0; k < n; ++k) {
    H[k] = Hn[k];
    w[k] = wn[k];
    t[k] = tn[k];
  }
}

// ---------------------------------------------------------------------------
// The model: grid, metrics, state, sampling.
// ---------------------------------------------------------------------------
struct Enclosed {
  int nx, ny;
  // per side (W, E, S, N): np points, 4 corner node indices, 4 weights
  std::vector<long> idx[4];
  std::vector<double> wt[4];
};

template <class T>
struct Model {
  int nx = 0, ny = 0, coord = 0;
  std::vector<double> x, y, d;
  std::vector<T> H, u, v;
  Par p{};
  int ssl_passes = 0;
  // metrics
  std::vector<double> xfac;        // [ny] row factor on x spacing
  std::vector<double> xib, xisb;   // [nx+1], [nx]
  std::vector<double> yib, yisb;   // [ny+1], [ny]
  std::vector<double> tanR;        // [ny]
  long n = 0;
  bool rec0 = false;
  // maxwave
  std::vector<double> emax, smax;
  // gauges
  std::vector<int> gx, gy;
  std::vector<T> grec;  // [nrec][ng][3]
  std::vector<double> gtime;
  // enclosed grids
  std::vector<Enclosed> enc;
  std::vector<std::vector<T>> srec;  // per grid: [nrec][4 sides concatenated][3][np]
  std::vector<std::vector<double>> stime;
  // forcing
  bool fside[4] = {false, false, false, false};
  std::vector<double> ftime[4], fvals[4];
  int fnp[4] = {0, 0, 0, 0};

  bool one_d() const { return nx == 1 || ny == 1; }
};

void line_metrics(int n, const double* s, double scale, std::vector<double>& ib,
                  std::vector<double>& isb) {
  // Delta_k = scale * (s_{k+1} - s_k); ghost spacings copy the edge ones
  ib.assign(n + 1, 0.0);
  isb.assign(n, 0.0);
  if (n < 2) return;
  std::vector<double> b(n + 1);
  for (int k = 0; k + 1 < n; ++k) b[k + 1] = scale * (s[k + 1] - s[k]);
  b[0] = b[1];
  b[n] = b[n - 1];
  for (int k = 0; k <= n; ++k) ib[k] = 1.0 / b[k];
  for (int k = 0; k < n; ++k) isb[k] = 1.0 / (b[k] + b[k + 1]);
}

template <class T>
void build_metrics(Model<T>& m) {
  const double deg = kPi / 180.0;
  if (m.coord == 1) {
    const double Rd = m.p.R * deg;
    // x: Delta x_{i,j} = (R pi/180 cos(lat_i)) * (lon_{j+1} - lon_j)
    line_metrics(m.nx, m.x.data(), 1.0, m.xib, m.xisb);
    m.xfac.resize(m.ny);
    for (int j = 0; j < m.ny; ++j) m.xfac[j] = 1.0 / (Rd * std::cos(m.y[j] * deg));
    // y: Delta y_i = (R pi/180) (lat_{i+1} - lat_i)
    line_metrics(m.ny, m.y.data(), Rd, m.yib, m.yisb);
    m.tanR.resize(m.ny);
    for (int j = 0; j < m.ny; ++j)
      m.tanR[j] = m.p.sph_metric ? std::tan(m.y[j] * deg) / m.p.R : 0.0;
  } else {
    line_metrics(m.nx, m.x.data(), 1.0, m.xib, m.xisb);
    line_metrics(m.ny, m.y.data(), 1.0, m.yib, m.yisb);
    m.xfac.assign(m.ny, 1.0);
    m.tanR.assign(m.ny, 0.0);
  }
}


template <class T>
bool is_fixed(const Model<T>& m, int i, int j) {
  return (m.fside[0] && i == 0) || (m.fside[1] && i == m.nx - 1) || (m.fside[2] && j == 0) ||
         (m.fside[3] && j == m.ny - 1);
}

// x-sweep: every row is an independent 1-D problem along x (eq2A), with
// w = u and t = v.
template <class T>
void xsweep(Model<T>& m) {
  const int nx = m.nx;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < m.ny; ++j) {
    std::vector<T> H(nx), w(nx), t(nx);
    std::vector<double> D(nx);
    std::vector<unsigned char> fx(nx);
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      H[i] = m.H[k]; w[i] = m.u[k]; t[i] = m.v[k]; D[i] = m.d[k];
      fx[i] = is_fixed(m, i, j);
    }
    sweep_line(m.p, nx, H.data(), w.data(), t.data(), D.data(), fx.data(), m.xib.data(),
               m.xisb.data(), m.xfac[j], nullptr, (m.p.open_mask & 1) != 0,
               (m.p.open_mask & 2) != 0);
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      m.H[k] = H[i]; m.u[k] = w[i]; m.v[k] = t[i];
    }
  }
}

// y-sweep: every column is an independent 1-D problem along y (eq2B), with
// w = v and t = u.
template <class T>
void ysweep(Model<T>& m) {
  const int nx = m.nx, ny = m.ny;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nx; ++i) {
    std::vector<T> H(ny), w(ny), t(ny);
    std::vector<double> D(ny);
    std::vector<unsigned char> fx(ny);
    for (int j = 0; j < ny; ++j) {
      size_t k = (size_t)j * nx + i;
      H[j] = m.H[k]; w[j] = m.v[k]; t[j] = m.u[k]; D[j] = m.d[k];
      fx[j] = is_fixed(m, i, j);
    }
    sweep_line(m.p, ny, H.data(), w.data(), t.data(), D.data(), fx.data(), m.yib.data(),
               m.yisb.data(), 1.0, m.coord == 1 ? m.tanR.data() : nullptr,
               (m.p.open_mask & 4) != 0, (m.p.open_mask & 8) != 0);
    for (int j = 0; j < ny; ++j) {
      size_t k = (size_t)j * nx + i;
      m.H[k] = H[j]; m.v[k] = w[j]; m.u[k] = t[j];
    }
  }
}

// Boundary forcing: linear interpolation in time of the (u, v, eta) series
// onto the outer ring of nodes; applied at the start of a step at t = n dt.
double interp_series(const std::vector<double>& tt, const double* vals, int stride, int q,
                     int np, int pt, double t) {
  const int nt = (int)tt.size();
  auto at = [&](int k) { return vals[(size_t)k * stride + (size_t)q * np + pt]; };
  if (t <= tt[0]) return at(0);
  if (t >= tt[nt - 1]) return at(nt - 1);
  int k = 0;
  while (k + 1 < nt && tt[k + 1] <= t) ++k;
  double a = (t - tt[k]) / (tt[k + 1] - tt[k]);
  double v0 = at(k), v1 = at(k + 1);
  return v0 + a * (v1 - v0);
}

template <class T>
void apply_forcing(Model<T>& m) {
  const double t = (double)m.n * m.p.dt;
  for (int s = 0; s < 4; ++s) {
    if (!m.fside[s]) continue;
    const int np = m.fnp[s];
    for (int k = 0; k < np; ++k) {
      int i, j;
      if (s == 0) { i = 0; j = k; }
      else if (s == 1) { i = m.nx - 1; j = k; }
      else if (s == 2) { i = k; j = 0; }
      else { i = k; j = m.ny - 1; }
      size_t idx = (size_t)j * m.nx + i;
      const int stride = 3 * np;
      double uu = interp_series(m.ftime[s], m.fvals[s].data(), stride, 0, np, k, t);
      double vv = interp_series(m.ftime[s], m.fvals[s].data(), stride, 1, np, k, t);
      double ee = interp_series(m.ftime[s], m.fvals[s].data(), stride, 2, np, k, t);
      double h = m.d[idx] + ee;
      if (h < 0.0) h = 0.0;
      if (h > m.p.hmin) {
        m.H[idx] = T(h); m.u[idx] = T(uu); m.v[idx] = T(vv);
      } else {
        m.H[idx] = T(0.0); m.u[idx] = T(0.0); m.v[idx] = T(0.0);
      }
    }
  }
}

// Sampling.  Maxwave: running maxima of eta and of the current speed over
// wet nodes.  Gauges: (eta, u, v) at nodes.  Enclosed grids: bilinear
// (wet-weighted) values along the four sides.  Dry nodes report zeros.
template <class T>
void update_maxwave(Model<T>& m) {
  const size_t N = (size_t)m.nx * m.ny;
  for (size_t k = 0; k < N; ++k) {
    if (!(re(m.H[k]) > m.p.hmin)) continue;
    double e = re(m.H[k]) - m.d[k];
    if (e > m.emax[k]) m.emax[k] = e;
    double uu = re(m.u[k]), vv = re(m.v[k]);
    double sp = std::sqrt(uu * uu + vv * vv);
    if (sp > m.smax[k]) m.smax[k] = sp;
  }
}

template <class T>
void record_gauges(Model<T>& m) {
  const int ng = (int)m.gx.size();
  for (int g = 0; g < ng; ++g) {
    size_t k = (size_t)m.gy[g] * m.nx + m.gx[g];
    if (re(m.H[k]) > m.p.hmin) {
      m.grec.push_back(m.H[k] - m.d[k]);
      m.grec.push_back(m.u[k]);
      m.grec.push_back(m.v[k]);
    } else {
      m.grec.push_back(T(0.0)); m.grec.push_back(T(0.0)); m.grec.push_back(T(0.0));
    }
  }
  m.gtime.push_back((double)m.n * m.p.dt);
}

template <class T>
void record_series(Model<T>& m) {
  for (size_t e = 0; e < m.enc.size(); ++e) {
    const Enclosed& E = m.enc[e];
    for (int s = 0; s < 4; ++s) {
      const int np = (s < 2) ? E.ny : E.nx;
      std::vector<T> buf((size_t)3 * np, T(0.0));
      for (int k = 0; k < np; ++k) {
        double ws = 0.0;
        T au = T(0.0), av = T(0.0), ae = T(0.0);
        for (int c = 0; c < 4; ++c) {
          long idx = E.idx[s][(size_t)4 * k + c];
          double wgt = E.wt[s][(size_t)4 * k + c];
          if (!(re(m.H[idx]) > m.p.hmin)) continue;
          ws = ws + wgt;
          au = au + wgt * m.u[idx];
          av = av + wgt * m.v[idx];
          ae = ae + wgt * (m.H[idx] - m.d[idx]);
        }
        if (ws > 0.0) {
          buf[k] = au / ws;
          buf[(size_t)np + k] = av / ws;
          buf[(size_t)2 * np + k] = ae / ws;
        }
      }
      m.srec[e].insert(m.srec[e].end(), buf.begin(), buf.end());
    }
    m.stime[e].push_back((double)m.n * m.p.dt);
  }
}

template <class T>
void take_records(Model<T>& m) {
  if (!m.gx.empty() && m.p.gout > 0 && m.n % m.p.gout == 0) record_gauges(m);
  if (!m.enc.empty() && m.p.bndout > 0 && m.n % m.p.bndout == 0) record_series(m);
}

// One split step (eq2A then eq2B, or the reverse on odd steps when the
// alternating order is selected).  1-D grids run only the sweep along
// their one dimension.
template <class T>
void step_once(Model<T>& m) {
  if (!m.rec0 && m.n == 0) {
    take_records(m);
    m.rec0 = true;
  }
  if (m.fside[0] || m.fside[1] || m.fside[2] || m.fside[3]) apply_forcing(m);
  bool yx = (m.p.order == 1) && (m.n % 2 == 1);
  bool dox = m.nx > 1, doy = m.ny > 1;
  if (!yx) {
    if (dox) xsweep(m);
    if (doy) ysweep(m);
  } else {
    if (doy) ysweep(m);
    if (dox) xsweep(m);
  }
  m.n += 1;
  if (m.p.maxout > 0 && m.n % m.p.maxout == 0) update_maxwave(m);
  take_records(m);
}

template <class T>
void reset_state(Model<T>& m) {
  const size_t N = (size_t)m.nx * m.ny;
  m.n = 0;
  m.rec0 = false;
  m.emax.assign(N, 0.0);
  m.smax.assign(N, 0.0);
  m.grec.clear();
  m.gtime.clear();
  for (auto& v : m.srec) v.clear();
  for (auto& v : m.stime) v.clear();
}

template <class T>
void dry_pass(Model<T>& m) {
  const size_t N = (size_t)m.nx * m.ny;
  for (size_t k = 0; k < N; ++k) {
    bool blocked = m.p.itopo == 0 && m.d[k] < m.p.dwall;
    if (!(re(m.H[k]) > m.p.hmin) || blocked) {
      m.H[k] = T(0.0); m.u[k] = T(0.0); m.v[k] = T(0.0);
    }
  }
}

// Initial conditions: a deformation applied to the free surface
// (H = max(d + eta, 0)) or to the sea floor (d <- d - eta, H = max(d_old, 0)),
// plus the initial velocities; nodes at or below h_min are dry.
template <class T>
void set_initial_t(Model<T>& m, const double* eta, const T* etai, const double* u,
                   const double* v, int deform_bottom) {
  const size_t N = (size_t)m.nx * m.ny;
  for (size_t k = 0; k < N; ++k) {
    T e = etai ? etai[k] : T(eta ? eta[k] : 0.0);
    T h;
    if (deform_bottom) {
      h = T(m.d[k] > 0.0 ? m.d[k] : 0.0);
      m.d[k] = m.d[k] - re(e);
    } else {
      h = m.d[k] + e;
      if (re(h) < 0.0) h = T(0.0);
    }
    m.H[k] = h;
    m.u[k] = T(u ? u[k] : 0.0);
    m.v[k] = T(v ? v[k] : 0.0);
  }
  dry_pass(m);
  reset_state(m);
}

template <class T>
int init_model(Model<T>& m, int nx, int ny, int coord, const double* x, const double* y,
               const double* depth, double dt, double hmin, double n2, int itopo, double dwall,
               double ssl_alpha, double ssl_min, int order, int solver, double R, int sph,
               int maxout, int gout, int bndout, int fric_form, int open_mask) {
  if (nx < 1 || ny < 1) return -1;
  if (fric_form != 0 && fric_form != 1) return -1;
  if (open_mask < 0 || open_mask > 15) return -1;
  bool oned = nx == 1 || ny == 1;
  if (oned && nx * ny < 3) return -1;
  if (!oned && (nx < 3 || ny < 3)) return -1;
  if (!(hmin > 0.0) || !(dt > 0.0)) return -1;
  for (int i = 0; i + 1 < nx; ++i)
    if (!(x[i + 1] > x[i])) return -1;
  for (int j = 0; j + 1 < ny; ++j)
    if (!(y[j + 1] > y[j])) return -1;
  m.nx = nx; m.ny = ny; m.coord = coord;
  m.x.assign(x, x + nx);
  m.y.assign(y, y + ny);
  m.d.assign(depth, depth + (size_t)nx * ny);
  Par& p = m.p;
  p.dt = dt;
  p.hdt = 0.5 * dt;
  p.dt2 = dt * dt;
  p.hmin = hmin;
  p.n2 = n2;
  p.gn2 = kG * n2;
  p.inv16g = 1.0 / (16.0 * kG);
  p.R = R;
  p.itopo = itopo;
  p.dwall = dwall;
  p.solver = solver;
  p.order = order;
  p.sph_metric = sph;
  p.maxout = maxout;
  p.gout = gout;
  p.bndout = bndout;
  p.fric_form = fric_form;
  p.open_mask = open_mask;
  if (ssl_alpha > 0.0) {
    m.ssl_passes = ssl_run(nx, ny, m.d.data(), ssl_alpha, ssl_min);
    if (m.ssl_passes < 0) return -2;
  }
  build_metrics(m);
  const size_t N = (size_t)nx * ny;
  m.H.assign(N, T(0.0));
  m.u.assign(N, T(0.0));
  m.v.assign(N, T(0.0));
  for (size_t k = 0; k < N; ++k) m.H[k] = T(m.d[k] > 0.0 ? m.d[k] : 0.0);
  dry_pass(m);
  reset_state(m);
  return 0;
}

template <class T>
double max_cfl(const Model<T>& m) {
  // still-water Courant number sqrt(g d) dt / Delta over wet nodes (both axes)
  double mx = 0.0;
  for (int j = 0; j < m.ny; ++j)
    for (int i = 0; i < m.nx; ++i) {
      double dd = m.d[(size_t)j * m.nx + i];
      if (!(dd > 0.0)) continue;
      double c = std::sqrt(kG * dd) * m.p.dt;
      if (m.nx > 1) {
        double ix = m.xfac[j] * std::max(m.xib[i], m.xib[i + 1]);
        mx = std::max(mx, c * ix);
      }
      if (m.ny > 1) {
        double iy = std::max(m.yib[j], m.yib[j + 1]);
        mx = std::max(mx, c * iy);
      }
    }
  return mx;
}

int add_enclosed(Model<double>& m, Enclosed& E, int nxe, int nye, const double* xe,
                 const double* ye) {
  if (m.one_d() || nxe < 2 || nye < 2) return -1;
  E.nx = nxe;
  E.ny = nye;
  auto locate = [](const std::vector<double>& c, double p, int* i0, double* w) -> bool {
    const int n = (int)c.size();
    if (p < c[0] || p > c[n - 1]) return false;
    int i = 0;
    while (i + 2 < n && c[i + 1] <= p) ++i;
    *i0 = i;
    *w = (p - c[i]) / (c[i + 1] - c[i]);
    return true;
  };
  for (int s = 0; s < 4; ++s) {
    const int np = (s < 2) ? nye : nxe;
    E.idx[s].resize((size_t)4 * np);
    E.wt[s].resize((size_t)4 * np);
    for (int k = 0; k < np; ++k) {
      double px, py;
      if (s == 0) { px = xe[0]; py = ye[k]; }
      else if (s == 1) { px = xe[nxe - 1]; py = ye[k]; }
      else if (s == 2) { px = xe[k]; py = ye[0]; }
      else { px = xe[k]; py = ye[nye - 1]; }
      int i0, j0;
      double wx, wy;
      if (!locate(m.x, px, &i0, &wx) || !locate(m.y, py, &j0, &wy)) return -1;
      long b = (long)j0 * m.nx + i0;
      long id[4] = {b, b + 1, b + m.nx, b + m.nx + 1};
      double wt[4] = {(1.0 - wx) * (1.0 - wy), wx * (1.0 - wy), (1.0 - wx) * wy, wx * wy};
      for (int c = 0; c < 4; ++c) {
        E.idx[s][(size_t)4 * k + c] = id[c];
        E.wt[s][(size_t)4 * k + c] = wt[c];
      }
    }
  }
  return 0;
}

}  // namespace

// ===========================================================================
// C API (ctypes).  All arrays are host arrays, row-major [ny][nx].
// ===========================================================================
extern "C" {

typedef Model<double> OraModel;

// Thread count of the row / column loops (timing only; results do not
// depend on it).  n <= 0 leaves the OpenMP default.  Returns the count in use.
int ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void* ora_create(int nx, int ny, int coord, const double* x, const double* y, const double* depth,
                 double dt, double hmin, double n2, int itopo, double dwall, double ssl_alpha,
                 double ssl_min, int order, int solver, double R, int sph, int maxout, int gout,
                 int bndout, int fric_form, int open_mask, int* status) {
  OraModel* m = new OraModel();
  int rc = init_model(*m, nx, ny, coord, x, y, depth, dt, hmin, n2, itopo, dwall, ssl_alpha,
                      ssl_min, order, solver, R, sph, maxout, gout, bndout, fric_form, open_mask);
  *status = rc;
  if (rc != 0) {
    delete m;
    return nullptr;
  }
  return m;
}

void ora_destroy(void* h) { delete (OraModel*)h; }
int ora_ssl_passes(void* h) { return ((OraModel*)h)->ssl_passes; }
double ora_max_cfl(void* h) { return max_cfl(*(OraModel*)h); }

void ora_get_depth(void* h, double* d) {
  OraModel* m = (OraModel*)h;
  std::copy(m->d.begin(), m->d.end(), d);
}

int ora_set_initial(void* h, const double* eta, const double* u, const double* v, int deform) {
  set_initial_t(*(OraModel*)h, eta, (const double*)nullptr, u, v, deform);
  return 0;
}

int ora_set_raw_state(void* h, const double* H, const double* u, const double* v, long n) {
  OraModel* m = (OraModel*)h;
  const size_t N = (size_t)m->nx * m->ny;
  std::copy(H, H + N, m->H.begin());
  std::copy(u, u + N, m->u.begin());
  std::copy(v, v + N, m->v.begin());
  m->n = n;
  m->rec0 = n > 0;  // the record of step n was taken when step n was reached
  return 0;
}

void ora_get_raw_state(void* h, double* H, double* u, double* v) {
  OraModel* m = (OraModel*)h;
  std::copy(m->H.begin(), m->H.end(), H);
  std::copy(m->u.begin(), m->u.end(), u);
  std::copy(m->v.begin(), m->v.end(), v);
}

void ora_get_state(void* h, double* eta, double* u, double* v, unsigned char* wet) {
  OraModel* m = (OraModel*)h;
  const size_t N = (size_t)m->nx * m->ny;
  for (size_t k = 0; k < N; ++k) {
    bool w = m->H[k] > m->p.hmin;
    if (eta) eta[k] = w ? m->H[k] - m->d[k] : 0.0;
    if (u) u[k] = w ? m->u[k] : 0.0;
    if (v) v[k] = w ? m->v[k] : 0.0;
    if (wet) wet[k] = w ? 1 : 0;
  }
}

long ora_step_count(void* h) { return ((OraModel*)h)->n; }

int ora_step(void* h, int nsteps) {
  OraModel* m = (OraModel*)h;
  for (int s = 0; s < nsteps; ++s) step_once(*m);
  return 0;
}

// One sweep only (axis 0 = x, 1 = y): no forcing, no sampling, no counter.
int ora_sweep(void* h, int axis) {
  OraModel* m = (OraModel*)h;
  if (axis == 0) xsweep(*m);
  else ysweep(*m);
  return 0;
}

int ora_set_gauges(void* h, int n, const int* ix, const int* iy) {
  OraModel* m = (OraModel*)h;
  for (int g = 0; g < n; ++g)
    if (ix[g] < 0 || ix[g] >= m->nx || iy[g] < 0 || iy[g] >= m->ny) return -1;
  m->gx.assign(ix, ix + n);
  m->gy.assign(iy, iy + n);
  m->grec.clear();
  m->gtime.clear();
  return 0;
}

int ora_num_gauge_records(void* h) { return (int)((OraModel*)h)->gtime.size(); }

void ora_read_gauges(void* h, double* out, double* times) {
  OraModel* m = (OraModel*)h;
  std::copy(m->grec.begin(), m->grec.end(), out);
  std::copy(m->gtime.begin(), m->gtime.end(), times);
}

void ora_read_maxwave(void* h, double* emax, double* smax) {
  OraModel* m = (OraModel*)h;
  std::copy(m->emax.begin(), m->emax.end(), emax);
  std::copy(m->smax.begin(), m->smax.end(), smax);
}

int ora_add_enclosed(void* h, int nx, int ny, const double* x, const double* y) {
  OraModel* m = (OraModel*)h;
  Enclosed E;
  if (add_enclosed(*m, E, nx, ny, x, y) != 0) return -1;
  m->enc.push_back(E);
  m->srec.emplace_back();
  m->stime.emplace_back();
  return (int)m->enc.size() - 1;
}

int ora_num_series_records(void* h, int id) {
  return (int)((OraModel*)h)->stime[id].size();
}

// vals: [nrec][3][np] for the requested side (0 W, 1 E, 2 S, 3 N)
void ora_read_series(void* h, int id, int side, double* vals, double* times) {
  OraModel* m = (OraModel*)h;
  const Enclosed& E = m->enc[id];
  const size_t per = (size_t)3 * (2 * E.ny + 2 * E.nx);
  size_t off = 0;
  for (int s = 0; s < side; ++s) off += (size_t)3 * ((s < 2) ? E.ny : E.nx);
  const size_t np3 = (size_t)3 * ((side < 2) ? E.ny : E.nx);
  const size_t nrec = m->stime[id].size();
  for (size_t r = 0; r < nrec; ++r)
    std::copy(m->srec[id].begin() + r * per + off, m->srec[id].begin() + r * per + off + np3,
              vals + r * np3);
  std::copy(m->stime[id].begin(), m->stime[id].end(), times);
}

// side: 0 W, 1 E, 2 S, 3 N; vals [nt][3][np], (u, v, eta) per point
int ora_set_forcing(void* h, int side, int nt, const double* t, const double* vals) {
  OraModel* m = (OraModel*)h;
  if (side < 0 || side > 3 || nt < 1) return -1;
  int np = (side < 2) ? m->ny : m->nx;
  for (int k = 0; k + 1 < nt; ++k)
    if (!(t[k + 1] > t[k])) return -1;
  m->fside[side] = true;
  m->fnp[side] = np;
  m->ftime[side].assign(t, t + nt);
  m->fvals[side].assign(vals, vals + (size_t)nt * 3 * np);
  return 0;
}

// Standalone preprocessing: returns the number of passes, -1 if not converged.
int ora_ssl(int nx, int ny, double* d, double alpha, double min_depth) {
  return ssl_run(nx, ny, d, alpha, min_depth);
}

// Complex-step derivative of the gauge misfit
//   L = 1/2 sum_{records} sum_g (eta_g - obs)^2
// along the direction deta of the initial surface: the model is rerun with
// the complex initial surface eta + i h deta (free-surface deformation,
// zero velocities).  Comparisons use real parts, so every branch follows the
// real run.  Returns L and dL = Im(L)/h.
int ora_cs_gauge_loss(void* h, const double* eta, const double* deta, double hstep, int nsteps,
                      const double* obs, double* L, double* dL) {
  OraModel* r = (OraModel*)h;
  Model<cplx> m;
  m.nx = r->nx; m.ny = r->ny; m.coord = r->coord;
  m.x = r->x; m.y = r->y; m.d = r->d; m.p = r->p;
  m.xfac = r->xfac; m.xib = r->xib; m.xisb = r->xisb;
  m.yib = r->yib; m.yisb = r->yisb; m.tanR = r->tanR;
  m.gx = r->gx; m.gy = r->gy;
  const size_t N = (size_t)m.nx * m.ny;
  m.H.assign(N, cplx(0.0)); m.u.assign(N, cplx(0.0)); m.v.assign(N, cplx(0.0));
  std::vector<cplx> e(N);
  for (size_t k = 0; k < N; ++k) e[k] = cplx(eta[k], hstep * deta[k]);
  set_initial_t(m, nullptr, e.data(), nullptr, nullptr, 0);
  for (int s = 0; s < nsteps; ++s) step_once(m);
  const size_t nrec = m.gtime.size(), ng = m.gx.size();
  cplx acc(0.0);
  for (size_t q = 0; q < nrec; ++q)
    for (size_t g = 0; g < ng; ++g) {
      cplx dv = m.grec[(q * ng + g) * 3] - obs[q * ng + g];
      acc += 0.5 * dv * dv;
    }
  *L = acc.real();
  *dL = acc.imag() / hstep;
  return (int)nrec;
}

// Complex-step derivative of a weighted misfit of every gauge record,
//   L = sum over records q, gauges g, components c of 0.5 w_c (rec - obs)^2
// with components (eta, u, v), along a direction (deta, du, dv) of the
// initial surface (free-surface deformation) and velocities.  Velocities of
// dry nodes are zero, as after any initial condition.  obs: [nrec][ng][3].
int ora_cs_record_loss(void* h, const double* eta, const double* u, const double* v,
                       const double* deta, const double* du, const double* dv, double hstep,
                       int nsteps, const double* obs, const double* w, double* L, double* dL) {
  OraModel* r = (OraModel*)h;
  Model<cplx> m;
  m.nx = r->nx; m.ny = r->ny; m.coord = r->coord;
  m.x = r->x; m.y = r->y; m.d = r->d; m.p = r->p;
  m.xfac = r->xfac; m.xib = r->xib; m.xisb = r->xisb;
  m.yib = r->yib; m.yisb = r->yisb; m.tanR = r->tanR;
  m.gx = r->gx; m.gy = r->gy;
  const size_t N = (size_t)m.nx * m.ny;
  m.H.assign(N, cplx(0.0)); m.u.assign(N, cplx(0.0)); m.v.assign(N, cplx(0.0));
  std::vector<cplx> e(N);
  for (size_t k = 0; k < N; ++k) e[k] = cplx(eta[k], hstep * deta[k]);
  set_initial_t(m, nullptr, e.data(), nullptr, nullptr, 0);
  for (size_t k = 0; k < N; ++k)
    if (re(m.H[k]) > 0.0) {  // wet after the dry pass (dry nodes hold h = 0)
      m.u[k] = cplx(u[k], hstep * du[k]);
      m.v[k] = cplx(v[k], hstep * dv[k]);
    }
  for (int s = 0; s < nsteps; ++s) step_once(m);
  const size_t nrec = m.gtime.size(), ng = m.gx.size();
  cplx acc(0.0);
  for (size_t q = 0; q < nrec; ++q)
    for (size_t g = 0; g < ng; ++g)
      for (int c = 0; c < 3; ++c) {
        cplx dvv = m.grec[(q * ng + g) * 3 + c] - obs[(q * ng + g) * 3 + c];
        acc += 0.5 * w[c] * dvv * dvv;
      }
  *L = acc.real();
  *dL = acc.imag() / hstep;
  return (int)nrec;
}

}  // extern "C"
