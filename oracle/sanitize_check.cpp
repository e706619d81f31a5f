// Memory and undefined-behaviour check of the oracle (test infrastructure).
// Built with -fsanitize=address,undefined together with cliffs_oracle.cpp and
// run by tests/test_oracle_sanitized.py: every entry point of the C API is
// exercised on small grids (Cartesian with land, spherical, 1-D along each
// axis, friction in both forms, open edges, solver1, alternate order, wall
// mode, gauges, enclosed grids, forcing, restart, complex step).  A
// sanitizer report, or a non-finite result, makes the program exit non-zero.
#include <cmath>
#include <cstdio>
#include <vector>

extern "C" {
int ora_set_threads(int n);
void* ora_create(int nx, int ny, int coord, const double* x, const double* y, const double* depth,
                 double dt, double hmin, double n2, int itopo, double dwall, double ssl_alpha,
                 double ssl_min, int order, int solver, double R, int sph, int maxout, int gout,
                 int bndout, int fric_form, int open_mask, int* status);
void ora_destroy(void* h);
int ora_ssl_passes(void* h);
double ora_max_cfl(void* h);
void ora_get_depth(void* h, double* d);
int ora_set_initial(void* h, const double* eta, const double* u, const double* v, int deform);
int ora_set_raw_state(void* h, const double* H, const double* u, const double* v, long n);
void ora_get_raw_state(void* h, double* H, double* u, double* v);
void ora_get_state(void* h, double* eta, double* u, double* v, unsigned char* wet);
long ora_step_count(void* h);
int ora_step(void* h, int nsteps);
int ora_sweep(void* h, int axis);
int ora_set_gauges(void* h, int n, const int* ix, const int* iy);
int ora_num_gauge_records(void* h);
void ora_read_gauges(void* h, double* out, double* times);
void ora_read_maxwave(void* h, double* emax, double* smax);
int ora_add_enclosed(void* h, int nx, int ny, const double* x, const double* y);
int ora_num_series_records(void* h, int id);
void ora_read_series(void* h, int id, int side, double* vals, double* times);
int ora_set_forcing(void* h, int side, int nt, const double* t, const double* vals);
int ora_ssl(int nx, int ny, double* d, double alpha, double min_depth);
int ora_cs_gauge_loss(void* h, const double* eta, const double* deta, double hstep, int nsteps,
                      const double* obs, double* L, double* dL);
int ora_cs_record_loss(void* h, const double* eta, const double* u, const double* v,
                       const double* deta, const double* du, const double* dv, double hstep,
                       int nsteps, const double* obs, const double* w, double* L, double* dL);
}

namespace {

int failures = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "check failed: %s\n", what);
    ++failures;
  }
}

bool all_finite(const std::vector<double>& a) {
  for (double v : a)
    if (!std::isfinite(v)) return false;
  return true;
}

// One scenario: a basin with a coast on the west, a bump of water, and every
// output read back.
void scenario(int nx, int ny, int coord, int solver, int order, double n2, int itopo,
              bool extras, int fric_form = 0, int open_mask = 0) {
  std::vector<double> x(nx), y(ny), d((size_t)nx * ny), eta((size_t)nx * ny, 0.0);
  const double dx = coord ? 1.0 / 60.0 : 200.0;
  for (int i = 0; i < nx; ++i) x[i] = (coord ? 150.0 : 0.0) + i * dx;
  for (int j = 0; j < ny; ++j) y[j] = (coord ? 20.0 : 0.0) + j * dx;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      d[k] = (nx > 1 ? 60.0 * (i - 0.2 * nx) / nx : 30.0) + 3.0 * std::sin(0.3 * j);
      const double r2 = std::pow((i - 0.6 * nx) / 4.0, 2) + std::pow((j - 0.5 * ny) / 4.0, 2);
      eta[k] = 0.5 * std::exp(-r2);
    }
  int st = 0;
  void* h = ora_create(nx, ny, coord, x.data(), y.data(), d.data(), coord ? 2.0 : 1.0, 0.1, n2,
                       itopo, 0.5, 2.0, 0.1, order, solver, 6371000.0, 1, 1, 2, 1, fric_form,
                       open_mask, &st);
  check(h != nullptr && st == 0, "create");
  if (!h) return;
  check(ora_max_cfl(h) < 1.0 && ora_ssl_passes(h) >= 0, "diagnostics");
  std::vector<double> dd((size_t)nx * ny);
  ora_get_depth(h, dd.data());
  check(ora_set_initial(h, eta.data(), nullptr, nullptr, 0) == 0, "set_initial");
  std::vector<int> gx = {nx / 2, nx - 1, 0}, gy = {ny / 2, 0, ny - 1};
  check(ora_set_gauges(h, 3, gx.data(), gy.data()) == 0, "gauges");
  if (extras && nx > 8 && ny > 8) {
    std::vector<double> ex(6), ey(5);
    for (int i = 0; i < 6; ++i) ex[i] = x[2] + i * 0.5 * dx;
    for (int j = 0; j < 5; ++j) ey[j] = y[2] + j * 0.5 * dx;
    check(ora_add_enclosed(h, 6, 5, ex.data(), ey.data()) == 0, "enclosed");
    std::vector<double> t = {0.0, 100.0}, vals(2 * 3 * (size_t)ny, 0.01);
    check(ora_set_forcing(h, 0, 2, t.data(), vals.data()) == 0, "forcing");
  }
  check(ora_step(h, 30) == 0, "step");
  if (nx > 1) check(ora_sweep(h, 0) == 0, "sweep x");
  if (ny > 1) check(ora_sweep(h, 1) == 0, "sweep y");
  std::vector<double> H((size_t)nx * ny), u(H.size()), v(H.size()), e(H.size());
  std::vector<unsigned char> wet(H.size());
  ora_get_raw_state(h, H.data(), u.data(), v.data());
  ora_get_state(h, e.data(), u.data(), v.data(), wet.data());
  check(all_finite(H) && all_finite(e) && all_finite(u), "finite state");
  const long n = ora_step_count(h);
  check(ora_set_raw_state(h, H.data(), u.data(), v.data(), n) == 0, "restart");
  check(ora_step(h, 5) == 0, "step after restart");
  const int nrec = ora_num_gauge_records(h);
  std::vector<double> rec((size_t)nrec * 3 * 3), times(nrec);
  ora_read_gauges(h, rec.data(), times.data());
  check(all_finite(rec), "finite gauges");
  std::vector<double> emax(H.size()), smax(H.size());
  ora_read_maxwave(h, emax.data(), smax.data());
  check(all_finite(emax) && all_finite(smax), "finite maxwave");
  if (extras && nx > 8 && ny > 8) {
    const int ns = ora_num_series_records(h, 0);
    std::vector<double> sv((size_t)ns * 3 * 6), stt(ns);
    ora_read_series(h, 0, 2, sv.data(), stt.data());
    check(all_finite(sv), "finite series");
  }
  ora_destroy(h);
}

void complex_step() {
  const int nx = 16, ny = 12;
  std::vector<double> x(nx), y(ny), d((size_t)nx * ny, 40.0), eta(d.size()), de(d.size(), 0.01),
      z(d.size(), 0.0);
  for (int i = 0; i < nx; ++i) x[i] = i * 100.0;
  for (int j = 0; j < ny; ++j) y[j] = j * 100.0;
  for (size_t k = 0; k < eta.size(); ++k) eta[k] = 0.1 * std::sin(0.7 * k);
  int st = 0;
  void* h = ora_create(nx, ny, 0, x.data(), y.data(), d.data(), 1.0, 0.1, 0.0, 1, 0.0, 2.0, 0.1,
                       0, 2, 6371000.0, 1, 1, 1, 1, 0, 0, &st);
  std::vector<int> gx = {3, 9}, gy = {4, 7};
  ora_set_gauges(h, 2, gx.data(), gy.data());
  std::vector<double> obs(11 * 2 * 3, 0.0), w = {1.0, 0.5, 0.5};
  double L = 0, dL = 0;
  ora_cs_gauge_loss(h, eta.data(), de.data(), 1e-30, 10, obs.data(), &L, &dL);
  check(std::isfinite(L) && std::isfinite(dL), "complex-step gauge loss");
  ora_cs_record_loss(h, eta.data(), z.data(), z.data(), de.data(), de.data(), de.data(), 1e-30, 10,
                     obs.data(), w.data(), &L, &dL);
  check(std::isfinite(L) && std::isfinite(dL), "complex-step record loss");
  ora_destroy(h);
}

}  // namespace

int main() {
  ora_set_threads(2);
  scenario(40, 30, 0, 2, 0, 0.0, 1, true);     // Cartesian, land, nesting, forcing
  scenario(40, 30, 1, 2, 1, 0.0, 1, true);     // spherical, alternate order
  scenario(40, 30, 0, 1, 0, 0.0009, 1, false); // solver1, friction
  scenario(40, 30, 1, 2, 0, 0.0009, 1, false, 1, 0);  // semi-implicit friction option
  scenario(40, 30, 0, 2, 0, 0.0, 1, false, 0, 15);    // open edges
  scenario(50, 1, 0, 2, 0, 0.0, 1, false, 0, 3);      // open ends of a 1-D line
  scenario(40, 30, 0, 2, 0, 0.0, 0, false);    // wall mode
  scenario(50, 1, 0, 2, 0, 0.0, 1, false);     // 1-D along x
  scenario(1, 50, 0, 2, 0, 0.0, 1, false);     // 1-D along y
  scenario(3, 3, 0, 2, 0, 0.0, 1, false);      // smallest 2-D grid
  complex_step();
  std::vector<double> spike = {0.0, 16.0, 1.0, 16.0, -2.0};
  check(ora_ssl(5, 1, spike.data(), 2.0, 0.1) >= 0, "preprocessing");
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  return failures ? 1 : 0;
}
