// CPU check of the kernels' FFT plans (pl_fft.hpp): for every transform
// length of the library, the P cooperating threads of one transform are run
// one after another -- each thread's stage computation on its W values,
// then the exchange between stages through a plain array -- and the result
// is compared with the DFT written out as a sum (long double).  Also checks
// that every exchange and the last-to-first permutation move each element
// exactly once.  Prints one line per case; exit status 1 on a failure.
#include "pl_fft.hpp"

#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

using namespace pl;
using V = std::vector<std::vector<cx<double>>>;

static bool g_ok = true;

template <class PL, int S, bool INV>
void stage(V& v, const cx<double>* tw) {
  for (int t = 0; t < PL::P; ++t) stage_compute<PL, S, INV>(v[t].data(), t, tw);
}

// move outputs of stage S-1 (positions out_pos) to inputs of stage S
// (positions in_pos); every element must be written exactly once
template <class PL, int SA, int RA, int SB, int RB, bool OUT_A>
void permute(V& v, const char* what) {
  std::vector<cx<double>> buf(PL::N);
  std::vector<int> seen(PL::N, 0);
  for (int t = 0; t < PL::P; ++t)
    for (int q = 0; q < PL::W / RA; ++q)
      for (int m = 0; m < RA; ++m) {
        const int e = OUT_A ? out_pos<PL, SA>(t, q, m) : in_pos<PL, SA>(t, q, m);
        buf[e] = v[t][q * RA + m];
        ++seen[e];
      }
  for (int e = 0; e < PL::N; ++e)
    if (seen[e] != 1) {
      std::printf("N=%d %s: element %d written %d times\n", PL::N, what, e, seen[e]);
      g_ok = false;
    }
  for (int t = 0; t < PL::P; ++t)
    for (int q = 0; q < PL::W / RB; ++q)
      for (int r = 0; r < RB; ++r) v[t][q * RB + r] = buf[in_pos<PL, SB>(t, q, r)];
}

template <int N, bool INV>
void check(double tol) {
  using PL = Plan<N>;
  constexpr int RL = LastStage<PL>::R;
  std::vector<cx<double>> tw(N);
  for (int e = 0; e < N; ++e) tw[e] = {std::cos(2.0 * M_PI * e / N), -std::sin(2.0 * M_PI * e / N)};
  std::mt19937 gen(1000 + N);
  std::normal_distribution<double> nd;
  std::vector<std::complex<double>> x(N);
  for (auto& z : x) z = {nd(gen), nd(gen)};
  V v(PL::P, std::vector<cx<double>>(PL::W));
  for (int t = 0; t < PL::P; ++t)
    for (int q = 0; q < PL::W / PL::R0; ++q)
      for (int r = 0; r < PL::R0; ++r) {
        const auto z = x[in_pos<PL, 0>(t, q, r)];
        v[t][q * PL::R0 + r] = {z.real(), z.imag()};
      }
  stage<PL, 0, INV>(v, tw.data());
  if constexpr (PL::NS > 1) {
    permute<PL, 0, StageInfo<PL, 0>::R, 1, StageInfo<PL, 1>::R, true>(v, "exchange 0->1");
    stage<PL, 1, INV>(v, tw.data());
  }
  if constexpr (PL::NS > 2) {
    permute<PL, 1, StageInfo<PL, 1>::R, 2, StageInfo<PL, 2>::R, true>(v, "exchange 1->2");
    stage<PL, 2, INV>(v, tw.data());
  }
  std::vector<std::complex<double>> y(N);
  for (int t = 0; t < PL::P; ++t)
    for (int q = 0; q < PL::W / RL; ++q)
      for (int m = 0; m < RL; ++m) {
        const auto c = v[t][q * RL + m];
        y[out_pos<PL, PL::NS - 1>(t, q, m)] = {c.x, c.y};
      }
  long double err = 0, nrm = 0;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < N; ++k) {
    std::complex<long double> s = 0;
    for (int n = 0; n < N; ++n) {
      const long double ph = (INV ? 2 : -2) * pi * (long double)((long)n * k % N) / N;
      s += std::complex<long double>(x[n].real(), x[n].imag()) * std::complex<long double>(std::cos(ph), std::sin(ph));
    }
    const std::complex<long double> d = s - std::complex<long double>(y[k].real(), y[k].imag());
    err = std::max(err, std::abs(d));
    nrm = std::max(nrm, std::abs(s));
  }
  const double rel = (double)(err / nrm);
  const bool ok = rel <= tol;
  g_ok = g_ok && ok;
  std::printf("N=%d P=%d W=%d radices %d %d %d %s: max error %.2e of max |X| %s\n", N, PL::P, PL::W, PL::R0, PL::R1,
              PL::R2, INV ? "inverse" : "forward", rel, ok ? "ok" : "FAIL");
  // the inverse-then-forward hand-over: last-stage slots back to stage-0 slots
  if constexpr (!INV) permute<PL, PL::NS - 1, RL, 0, PL::R0, true>(v, "last to first");
}

template <int N>
void both(double tol) {
  check<N, false>(tol);
  check<N, true>(tol);
}

int main() {
  const double tol = 1e-14;
  both<8>(tol);
  both<12>(tol);
  both<16>(tol);
  both<24>(tol);
  both<32>(tol);
  both<48>(tol);
  both<64>(tol);
  both<96>(tol);
  both<128>(tol);
  both<192>(tol);
  both<256>(tol);
  both<512>(tol);
  return g_ok ? 0 : 1;
}
