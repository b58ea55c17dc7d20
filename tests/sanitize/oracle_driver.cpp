// Sanitizer driver for the CPU oracle (test infrastructure): the oracle's
// source compiled into this program with AddressSanitizer and
// UndefinedBehaviorSanitizer, run over every configuration it supports on
// tiny ragged grids (2D/3D; PLM minmod, van Leer, WENO-Z; HLL, HLLD; SSP-RK2,
// SSP-RK3; FP64 and mixed; both edge averages; GLM cleaning; the tangent and
// the operation counter). Exit status 0 when every call returns 0 and every
// value is finite; any memory or undefined-behaviour error aborts.
#include "../../oracle/mhd_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

// A smooth magnetised state with a staggered, divergence-free field (from a
// vector potential A_z = a cos(2 pi x) cos(2 pi y) plus a uniform field).
std::vector<double> make_state(int dim, int nx, int ny, int nz, bool glm) {
  const size_t n = (size_t)nx * ny * nz;
  const int nf = glm ? 9 : 8;
  std::vector<double> U((size_t)nf * n);
  const double pi = 3.14159265358979323846, dx = 1.0 / nx, dy = 1.0 / ny, dz = 1.0 / nz;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t c = ((size_t)k * ny + j) * nx + i;
        const double x = (i + 0.5) * dx, y = (j + 0.5) * dy, z = (k + 0.5) * dz;
        const double rho = 1.0 + 0.2 * std::sin(2 * pi * (x + 0.3 * y + 0.1 * z));
        const double vx = 0.3 * std::sin(2 * pi * y), vy = 0.2 * std::cos(2 * pi * x);
        const double vz = dim == 3 ? 0.1 * std::sin(2 * pi * (x + z)) : 0.05;
        const double p = 1.0 + 0.1 * std::cos(2 * pi * (x - y));
        auto az = [&](double xe, double ye) { return 0.05 * std::cos(2 * pi * xe) * std::cos(2 * pi * ye); };
        const double xl = i * dx, yl = j * dy;
        // staggered faces: b_x at (i-1/2, j), b_y at (i, j-1/2)
        const double bx = 0.4 + (az(xl, yl + dy) - az(xl, yl)) / dy;
        const double by = 0.1 - (az(xl + dx, yl) - az(xl, yl)) / dx;
        const double bz = 0.2;
        U[0 * n + c] = rho;
        U[1 * n + c] = rho * vx;
        U[2 * n + c] = rho * vy;
        U[3 * n + c] = rho * vz;
        U[4 * n + c] = p / (5.0 / 3.0 - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                       0.5 * (bx * bx + by * by + bz * bz);
        U[5 * n + c] = bx;
        U[6 * n + c] = by;
        U[7 * n + c] = bz;
        if (glm) U[8 * n + c] = 0.01 * std::sin(2 * pi * x);
      }
  return U;
}

bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

}  // namespace

int main() {
  int failures = 0, runs = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int lim = 0; lim <= 2; ++lim)
      for (int rs = 0; rs <= 1; ++rs)
        for (int prec = 0; prec <= 1; ++prec)
          for (int integ = 0; integ <= 1; ++integ)
            for (int mode = 0; mode <= 2; ++mode) {  // CT + UCT-HLL, CT + UCT-HLLD, GLM
              if (lim == 2 && prec == 1) continue;
              const int nx = 9, ny = 7, nz = dim == 3 ? 6 : 1;
              OCfg c{};
              c.dim = dim; c.nx = nx; c.ny = ny; c.nz = nz;
              c.xmin = 0; c.xmax = 1; c.ymin = 0; c.ymax = 1; c.zmin = 0; c.zmax = 1;
              c.gamma = 5.0 / 3.0; c.cfl = 0.3; c.limiter = lim; c.riemann = rs;
              c.precision = prec; c.nthreads = 2; c.integrator = integ;
              c.emf = mode == 1 ? 1 : 0;
              const bool glm = mode == 2;
              std::vector<double> U = make_state(dim, nx, ny, nz, glm);
              std::vector<double> dts(2);
              const int rc = glm ? oracle_glm_run(&c, U.data(), 2, dts.data())
                                 : oracle_run(&c, U.data(), 2, dts.data());
              ++runs;
              if (rc != 0 || !finite_all(U) || !finite_all(dts)) {
                std::fprintf(stderr, "fail: dim %d lim %d rs %d prec %d integ %d mode %d rc %d\n",
                             dim, lim, rs, prec, integ, mode, rc);
                ++failures;
              }
              if (!glm && prec == 0 && lim < 2 && integ == 0) {  // tangent and counter
                std::vector<double> V = make_state(dim, nx, ny, nz, false), dV(V.size(), 1e-3);
                if (oracle_step_jvp(&c, V.data(), dV.data(), 1e-3, 1.0) != 0 ||
                    !finite_all(V) || !finite_all(dV))
                  ++failures;
                long long ops[16];
                std::vector<double> W = make_state(dim, nx, ny, nz, false);
                if (oracle_count_ops(&c, W.data(), ops) != 0) ++failures;
                runs += 2;
              }
            }
  std::printf("oracle sanitizer driver: %d runs, %d failures\n", runs, failures);
  return failures ? 1 : 0;
}
