// Drives every C entry point of the oracle on small inputs; built with the
// address and undefined-behaviour sanitizers by a CPU test, which expects
// "ok" and a clean exit (any out-of-bounds access, leak of an uninitialised
// value into a branch the sanitizers see, or undefined arithmetic aborts).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int32_t oracle_velocity_set(int32_t q, int32_t* c, double* w);
int32_t oracle_moment_basis(int32_t q, double* M, double* Minv, int32_t* group);
int32_t oracle_equilibrium(int32_t q, double rho, const double* u, double* feq);
int32_t oracle_collide(int32_t q, const double* f, double omega, int32_t mode, double* fstar, double* gamma,
                       double* ds, double* dh);
int32_t oracle_collide_z(int32_t q, const double* f_ri, double omega, int32_t mode, double* fstar_ri,
                         double* gamma_ri);
int32_t oracle_run(int32_t q, int32_t n, int32_t steps, double omega, int32_t mode, double* f, double* gamma_stats,
                   int32_t threads);
int32_t oracle_run_z(int32_t q, int32_t n, int32_t steps, double omega, int32_t mode, double* f_ri, int32_t threads);
int32_t oracle_init_field(int32_t q, int64_t ncell, const double* u, double* f);
int32_t oracle_init_field_z(int32_t q, int64_t ncell, const double* u_ri, double* f_ri);
int32_t oracle_max_threads(void);
}

static int fails = 0;

static void expect(bool cond, const char* what, int q) {
  if (!cond) {
    std::printf("FAILED (q = %d): %s\n", q, what);
    ++fails;
  }
}

int main() {
  std::mt19937_64 gen(7);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  const double omega = 1.9;
  for (int q : {27, 19}) {
    std::vector<int32_t> c(3 * q), group(q);
    std::vector<double> w(q), M(q * q), Minv(q * q);
    expect(oracle_velocity_set(q, c.data(), w.data()) != 0, "velocity set", q);
    expect(oracle_moment_basis(q, M.data(), Minv.data(), group.data()) != 0, "moment basis", q);
    // one cell: perturbed equilibrium through the three collision modes
    const double u[3] = {0.03, -0.02, 0.01};
    std::vector<double> f(q), fs(q), ds(q), dh(q);
    expect(oracle_equilibrium(q, 1.0, u, f.data()) != 0, "equilibrium", q);
    for (int i = 0; i < q; ++i) f[i] *= 1.0 + 0.005 * U(gen);
    for (int mode = 0; mode < 3; ++mode) {
      double gamma = 0.0;
      expect(oracle_collide(q, f.data(), omega, mode, fs.data(), &gamma, ds.data(), dh.data()) != 0, "collide", q);
      expect(std::isfinite(gamma), "finite gamma", q);
    }
    std::vector<double> fz(2 * q), fsz(2 * q), gz(2);
    for (int i = 0; i < q; ++i) {
      fz[2 * i] = f[i];
      fz[2 * i + 1] = i == 3 ? 1e-30 : 0.0;
    }
    for (int mode : {0, 2})
      expect(oracle_collide_z(q, fz.data(), omega, mode, fsz.data(), gz.data()) != 0, "complex collide", q);
    // a small lattice: fields, runs in every mode, complex run
    const int n = 8;
    const int64_t ncell = int64_t(n) * n * n;
    std::vector<double> uf(3 * ncell), field(ncell * q), stats(3 * 3);
    for (double& v : uf) v = 0.02 * U(gen);
    expect(oracle_init_field(q, ncell, uf.data(), field.data()) != 0, "init field", q);
    for (int mode = 0; mode < 3; ++mode) {
      std::vector<double> g = field;
      expect(oracle_run(q, n, 3, omega, mode, g.data(), stats.data(), 2) != 0, "run", q);
      for (double v : g) expect(std::isfinite(v), "finite populations", q);
    }
    std::vector<double> uz(2 * 3 * ncell, 0.0), fzf(2 * ncell * q);
    for (int64_t k = 0; k < 3 * ncell; ++k) uz[2 * k] = uf[k];
    expect(oracle_init_field_z(q, ncell, uz.data(), fzf.data()) != 0, "complex init field", q);
    for (int mode : {0, 2}) {
      std::vector<double> gz2 = fzf;
      expect(oracle_run_z(q, n, 2, omega, mode, gz2.data(), 2) != 0, "complex run", q);
    }
    expect(oracle_run_z(q, n, 1, omega, 1, fzf.data(), 2) == 0, "complex run rejects BGK mode", q);
  }
  expect(oracle_velocity_set(15, nullptr, nullptr) == 0, "unknown lattice", 15);
  expect(oracle_max_threads() >= 1, "threads", 0);
  if (fails == 0) std::printf("ok\n");
  return fails == 0 ? 0 : 1;
}
