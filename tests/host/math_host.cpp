// Host build of the device math (hweno_math.h, hweno_adjoint.h), driven from
// tests/test_host_math.py.  The weights come first on the command line:
//   math_host g0 g1 g2 d0 d1 d2 eps gamma
// then each input line is <op> <prec> <values...>, prec 'd' or 'f':
//   r  fm f0 fp Hm H0 Hp           hw_plus with the reconstruction weights
//   l  um u0 up vm vp h            limit1 with the limiter weights
//   p  U[4] Dn[4] Dt[4]            2D Euler point_fluxes: F, A Dn, A Dt
//   e  UL[4] UR[4] x[4]            Roe-averaged eigen-system: L x, then R (L x)
//   R  fm f0 fp Hm H0 Hp           hw_plus_vjp with a unit adjoint: the gradient
//   L  um u0 up vm vp h            limit1_vjp with a unit adjoint: the gradient
//   P  U Dn Dt gF gA gB (4 each)   point_fluxes_vjp: gU, gDn, gDt
//   c  um u0 up vm vp (4 each) h    2D Euler characteristic limiter (normal frame)
//   C  um u0 up vm vp (4 each) h g  its reverse with the adjoint g (4): gum gu0 gup gvm gvp
// and prints its results on one line, 17 significant digits each.
#include <cstdio>
#include <cstdlib>

#include "../../paper_2207_05258_amd/csrc/hweno_adjoint.h"

using namespace hweno;

static double g[6], eps, gam;

template <typename T>
static Weights<T> weights(int o) {
  return Weights<T>{T(g[o]), T(g[o + 1]), T(g[o + 2]), T(eps), T(g[o]) + T(g[o + 1]) + T(g[o + 2])};
}

template <typename T>
static void run(char op, const double* v) {
  if (op == 'r') {
    std::printf("%.17g\n", double(hw_plus<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), T(v[5]),
                                             weights<T>(0))));
  } else if (op == 'l') {
    const T h = T(v[5]);
    std::printf("%.17g\n", double(limit1<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), h,
                                            T(1) / h, weights<T>(3))));
  } else if (op == 'p') {
    Consts<T> k{};
    k.gm1 = T(gam - 1.0);
    k.gam = T(gam);
    T U[4], Dn[4], Dt[4], F[4], A[4], B[4];
    for (int c = 0; c < 4; ++c) U[c] = T(v[c]), Dn[c] = T(v[4 + c]), Dt[c] = T(v[8 + c]);
    point_fluxes<T, PH_EULER, 4, true>(U, Dn, Dt, k, T(0), F, A, B);
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(F[c]));
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(A[c]));
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(B[c]));
    std::printf("\n");
  } else if (op == 'R') {
    T gr[6] = {};
    hw_plus_vjp<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), T(v[5]), weights<T>(0), T(1), gr[0],
                   gr[1], gr[2], gr[3], gr[4], gr[5]);
    for (int i = 0; i < 6; ++i) std::printf("%.17g ", double(gr[i]));
    std::printf("\n");
  } else if (op == 'L') {
    T gr[5] = {};
    const T h = T(v[5]);
    limit1_vjp<T>(T(v[0]), T(v[1]), T(v[2]), T(v[3]), T(v[4]), h, T(1) / h, weights<T>(3), T(1),
                  gr[0], gr[1], gr[2], gr[3], gr[4]);
    for (int i = 0; i < 5; ++i) std::printf("%.17g ", double(gr[i]));
    std::printf("\n");
  } else if (op == 'P') {
    Consts<T> k{};
    k.gm1 = T(gam - 1.0);
    k.gam = T(gam);
    T in[24], gU[4] = {}, gDn[4] = {}, gDt[4] = {};
    for (int i = 0; i < 24; ++i) in[i] = T(v[i]);
    point_fluxes_vjp<T, PH_EULER, 4, true>(in, in + 4, in + 8, k, T(0), in + 12, in + 16, in + 20,
                                           gU, gDn, gDt);
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(gU[c]));
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(gDn[c]));
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(gDt[c]));
    std::printf("\n");
  } else if (op == 'c' || op == 'C') {
    T st[5][4], out[4], g[5][4] = {};
    for (int q = 0; q < 5; ++q)
      for (int c = 0; c < 4; ++c) st[q][c] = T(v[4 * q + c]);
    const T h = T(v[20]);
    if (op == 'c') {
      limit_char<T, 4>(st[0], st[1], st[2], st[3], st[4], h, T(1) / h, weights<T>(3), T(gam - 1.0), out);
      for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(out[c]));
    } else {
      T gout[4];
      for (int c = 0; c < 4; ++c) gout[c] = T(v[21 + c]);
      limit_char_vjp<T, 4>(st[0], st[1], st[2], st[3], st[4], h, T(1) / h, weights<T>(3),
                           T(gam - 1.0), gout, g[0], g[1], g[2], g[3], g[4]);
      for (int q = 0; q < 5; ++q)
        for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(g[q][c]));
    }
    std::printf("\n");
  } else {
    T UL[4], UR[4], x[4], w[4], y[4];
    for (int c = 0; c < 4; ++c) UL[c] = T(v[c]), UR[c] = T(v[4 + c]), x[c] = T(v[8 + c]);
    Eigen<T, 4> e;
    e.roe(UL, UR, T(gam - 1.0));
    e.project(x, w);
    e.back(w, y);
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(w[c]));
    for (int c = 0; c < 4; ++c) std::printf("%.17g ", double(y[c]));
    std::printf("\n");
  }
}

int main(int argc, char** argv) {
  if (argc != 9) {
    std::fprintf(stderr, "usage: math_host g0 g1 g2 d0 d1 d2 eps gamma\n");
    return 2;
  }
  for (int i = 0; i < 6; ++i) g[i] = std::atof(argv[1 + i]);
  eps = std::atof(argv[7]);
  gam = std::atof(argv[8]);
  char op, prec;
  while (std::scanf(" %c %c", &op, &prec) == 2) {
    const int n = (op == 'r' || op == 'l' || op == 'R' || op == 'L') ? 6
                  : op == 'P' ? 24 : op == 'c' ? 21 : op == 'C' ? 25 : 12;
    double v[25];
    for (int i = 0; i < n; ++i)
      if (std::scanf("%lf", &v[i]) != 1) return 3;
    if (prec == 'd')
      run<double>(op, v);
    else
      run<float>(op, v);
  }
  return 0;
}
