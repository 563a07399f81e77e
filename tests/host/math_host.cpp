// Host build of the device math (hweno_math.h), driven from
// tests/test_host_math.py: each input line is
//   <op> <prec> <a> <b> <c> <d> <e> <f>
// op 'r': hw_plus(fm, f0, fp, Hm, H0, Hp) with the reconstruction weights;
// op 'l': limit1(um, u0, up, vm, vp, h = f, 1/h) with the limiter weights;
// prec 'd' or 'f'.  The weights come first on the command line:
//   math_host g0 g1 g2 d0 d1 d2 eps
// One result per line, printed with 17 significant digits.
#include <cstdio>
#include <cstdlib>

#include "../../paper_2207_05258_amd/csrc/hweno_math.h"

using namespace hweno;

template <typename T>
static Weights<T> weights(double a, double b, double c, double eps) {
  return Weights<T>{T(a), T(b), T(c), T(eps), T(a) + T(b) + T(c)};
}

template <typename T>
static double run(char op, const double* v, const double* g, double eps) {
  if (op == 'r')
    return double(hw_plus<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), T(v[5]),
                             weights<T>(g[0], g[1], g[2], eps)));
  const T h = T(v[5]);
  return double(limit1<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), h, T(1) / h,
                          weights<T>(g[3], g[4], g[5], eps)));
}

int main(int argc, char** argv) {
  if (argc != 8) {
    std::fprintf(stderr, "usage: math_host g0 g1 g2 d0 d1 d2 eps\n");
    return 2;
  }
  double g[6];
  for (int i = 0; i < 6; ++i) g[i] = std::atof(argv[1 + i]);
  const double eps = std::atof(argv[7]);
  char op, prec;
  double v[6];
  while (std::scanf(" %c %c %lf %lf %lf %lf %lf %lf", &op, &prec, &v[0], &v[1], &v[2], &v[3],
                    &v[4], &v[5]) == 8) {
    const double r = prec == 'd' ? run<double>(op, v, g, eps) : run<float>(op, v, g, eps);
    std::printf("%.17g\n", r);
  }
  return 0;
}
