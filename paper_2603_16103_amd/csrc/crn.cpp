// Shared Monte Carlo draws of one simplification pass (Appendix A: common
// random numbers across candidate pairs).  The paper names no generator; the
// draws are keyed by (seed, pass, draw, component) through the published
// SplitMix64 output function and turned into normals by Box-Muller.
#include <cmath>
#include <cstdint>

namespace ng {

namespace {

// SplitMix64 (Steele, Lea, Flood 2014): the output for state x.
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform(uint64_t seed, int round, int s, int c) {
  const uint64_t h = splitmix64(splitmix64(splitmix64(seed) ^ (uint64_t)(int64_t)round) ^
                                (uint64_t)(8 * (int64_t)s + c));
  return (double)(h >> 11) * 0x1.0p-53;
}

}  // namespace

void crn_host(uint64_t seed, int round, int S, float* out) {
  const double two_pi = 2.0 * M_PI;
  for (int s = 0; s < S; ++s) {
    const double u = uniform(seed, round, s, 0);
    const double u1 = uniform(seed, round, s, 1);
    const double u2 = uniform(seed, round, s, 2);
    const double u3 = uniform(seed, round, s, 3);
    const double u4 = uniform(seed, round, s, 4);
    const double r1 = std::sqrt(-2.0 * std::log(1.0 - u1));
    const double r2 = std::sqrt(-2.0 * std::log(1.0 - u3));
    out[4 * s + 0] = (float)u;
    out[4 * s + 1] = (float)(r1 * std::cos(two_pi * u2));
    out[4 * s + 2] = (float)(r1 * std::sin(two_pi * u2));
    out[4 * s + 3] = (float)(r2 * std::cos(two_pi * u4));
  }
}

}  // namespace ng
