// Host replays of the device schedules (the library's tpd_debug_emulate*
// entry points) against the binary64 oracle, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_sanitizers_host.py: every
// index map, tile decode, LDS exchange and list/compaction buffer of the
// replays, and the oracle's own buffers, run under the sanitizers.  The
// build replays complex128 only (TPD_EMULATE_COMPLEX128_ONLY); complex64
// replays are checked by the regular test-suite.  Prints
// one line per check and exits nonzero on the first mismatch.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tpd.h"

extern "C" {
int oracle_tpd_recursive(const double* A, int n, double* out, uint64_t* live, uint64_t* ops);
int oracle_tpd_iterative_mt(const double* A, int n, double* out, uint64_t* live, int threads);
int oracle_tpd_partial(const double* A, int n, const uint64_t* req, size_t m, double* out);
int oracle_synthesize(const double* w, int n, double* A);
}

namespace {

using cd = std::complex<double>;

struct Rng {  // splitmix64
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    const double u = uniform() + 1e-300, v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
  }
};

int failures = 0;
void report(const char* what, bool ok) {
  std::printf("%s %s\n", ok ? "ok" : "FAIL", what);
  if (!ok) ++failures;
}

std::vector<cd> gaussian(int n, uint64_t seed, bool hermitian) {
  Rng r{seed};
  const size_t d = (size_t)1 << n;
  std::vector<cd> A(d * d);
  for (auto& z : A) z = cd(r.normal(), r.normal());
  if (hermitian)
    for (size_t i = 0; i < d; ++i)
      for (size_t j = i; j < d; ++j) {
        const cd h = (A[i * d + j] + std::conj(A[j * d + i])) * 0.5;
        A[i * d + j] = h;
        A[j * d + i] = std::conj(h);
      }
  return A;
}

std::vector<cd> oracle(const std::vector<cd>& A, int n) {
  std::vector<cd> w((size_t)1 << (2 * n));
  if (oracle_tpd_recursive((const double*)A.data(), n, (double*)w.data(), nullptr, nullptr) != 0) ++failures;
  return w;
}

bool same_bits(const cd* a, const cd* b, size_t m) {
  for (size_t i = 0; i < m; ++i)
    if (!(a[i].real() == b[i].real() && a[i].imag() == b[i].imag())) return false;
  return true;
}

uint64_t spread(uint64_t v) {
  uint64_t r = 0;
  for (int b = 0; b < 32; ++b) r |= ((v >> b) & 1u) << (2 * b);
  return r;
}
// matrix layout (row h, column l) -> canonical order
std::vector<cd> matrix_to_canonical(const std::vector<cd>& m, int n) {
  const uint64_t d = (uint64_t)1 << n;
  std::vector<cd> c(m.size());
  for (uint64_t h = 0; h < d; ++h)
    for (uint64_t l = 0; l < d; ++l) c[(spread(h) << 1) | spread(l)] = m[h * d + l];
  return c;
}

void dense_checks() {
  for (int n = 0; n <= 9; ++n) {
    const auto A = gaussian(n, 100 + n, false);
    const auto ref = oracle(A, n);
    const size_t m = ref.size();
    std::vector<cd> out(m, cd(NAN, NAN));
    char name[96];
    std::snprintf(name, sizeof name, "complex128 n=%d canonical, bitwise Algorithm 1", n);
    report(name, tpd_debug_emulate(A.data(), n, out.data(), TPD_C128, 0, 0) == TPD_SUCCESS &&
                     same_bits(out.data(), ref.data(), m));
    std::vector<cd> ip = A;
    std::snprintf(name, sizeof name, "complex128 n=%d matrix layout in place", n);
    report(name, tpd_debug_emulate(ip.data(), n, ip.data(), TPD_C128, TPD_FLAG_LAYOUT_MATRIX, 1) == TPD_SUCCESS &&
                     same_bits(matrix_to_canonical(ip, n).data(), ref.data(), m));
  }
}

void tuned_and_chunked_checks() {
  const int n = 10;
  const auto A = gaussian(n, 7, false);
  const auto ref = oracle(A, n);
  for (int db = 3; db <= 5; ++db)
    for (int cb = 0; cb <= 3; cb += 3)
      for (int w = 0; w <= (cb ? 3 : 0); w += (w ? 1 : 2)) {
        std::vector<cd> out(ref.size(), cd(NAN, NAN));
        char name[96];
        std::snprintf(name, sizeof name, "n=10 tile width 2^%d chunk bits %d window %d", db, cb, w);
        report(name, tpd_debug_emulate_tuned(A.data(), n, out.data(), TPD_C128, 0, 0, db, 4, cb, w) == TPD_SUCCESS &&
                         same_bits(out.data(), ref.data(), ref.size()));
      }
}

// the transverse-field Ising chain, section "Results": weights -1 on Z_i Z_i+1
// and -g on X_i, assembled by the oracle's synthesis
std::vector<cd> tfim_weights(int n, double g) {
  std::vector<cd> w((size_t)1 << (2 * n), cd(0, 0));
  for (int i = 0; i + 1 < n; ++i) w[(uint64_t)15 << (2 * (n - 2 - i))] = -1.0;  // Z Z at sites i, i+1
  for (int i = 0; i < n; ++i) w[(uint64_t)1 << (2 * (n - 1 - i))] = -g;          // X at site i
  return w;
}

void hermitian_pruning_checks() {
  for (int n : {9, 10}) {
    const auto w = tfim_weights(n, 0.5);
    std::vector<cd> H((size_t)1 << (2 * n));
    if (oracle_synthesize((const double*)w.data(), n, (double*)H.data()) != 0) ++failures;
    std::vector<cd> out(w.size(), cd(NAN, NAN));
    char name[96];
    std::snprintf(name, sizeof name, "TFIM n=%d Hermitian mode, pruned tiles, canonical", n);
    report(name, tpd_debug_emulate(H.data(), n, out.data(), TPD_C128, TPD_FLAG_HERMITIAN, 0) == TPD_SUCCESS &&
                     same_bits(out.data(), w.data(), w.size()));
    std::vector<cd> ip = H;
    std::snprintf(name, sizeof name, "TFIM n=%d Hermitian mode, pruned tiles, matrix layout in place", n);
    report(name, tpd_debug_emulate(ip.data(), n, ip.data(), TPD_C128, TPD_FLAG_HERMITIAN | TPD_FLAG_LAYOUT_MATRIX,
                                   1) == TPD_SUCCESS &&
                     same_bits(matrix_to_canonical(ip, n).data(), w.data(), w.size()));
  }
}

void partial_checks() {
  const int n = 10;
  const auto A = gaussian(n, 11, true);
  Rng r{12};
  std::vector<uint64_t> req(700);
  for (auto& q : req) q = r.next() % ((uint64_t)1 << (2 * n));
  std::vector<cd> ref(req.size()), vals(req.size()), work((size_t)1 << (2 * n), cd(NAN, NAN));
  if (oracle_tpd_partial((const double*)A.data(), n, req.data(), req.size(), (double*)ref.data()) != 0) ++failures;
  report("partial n=10, 700 requests, bitwise Algorithm 3",
         tpd_debug_emulate_partial(A.data(), n, work.data(), req.data(), req.size(), vals.data(), TPD_C128, 0, 0) ==
                 TPD_SUCCESS &&
             same_bits(vals.data(), ref.data(), ref.size()));
  bool ok = tpd_debug_emulate_partial(A.data(), n, work.data(), req.data(), req.size(), vals.data(), TPD_C128,
                                      TPD_FLAG_HERMITIAN, 0) == TPD_SUCCESS;
  for (size_t i = 0; i < req.size() && ok; ++i) ok = vals[i].real() == ref[i].real() && vals[i].imag() == 0.0;
  report("partial n=10 Hermitian mode: real parts bitwise, imaginary parts 0", ok);
}

void compact_check() {
  const int n = 8;
  Rng r{21};
  std::vector<cd> c((size_t)1 << (2 * n));
  for (auto& z : c) z = r.uniform() < 0.05 ? cd(r.normal(), r.normal()) : cd(0, 0);
  std::vector<uint64_t> q(c.size());
  std::vector<cd> w(c.size());
  uint64_t total = 0;
  bool ok = tpd_debug_emulate_compact(c.data(), n, TPD_C128, 0, 0.0, q.data(), w.data(), c.size(), &total) ==
            TPD_SUCCESS;
  uint64_t k = 0;
  for (uint64_t i = 0; i < c.size() && ok; ++i)
    if (c[i] != cd(0, 0)) ok = k < total && q[k] == i && w[k] == c[i], ++k;
  report("compaction n=8 equals the ordered selection", ok && k == total);
}

void synth_check() {
  const int n = 6;
  Rng r{31};
  std::vector<cd> w((size_t)1 << (2 * n));
  for (auto& z : w) z = cd((double)(int)(r.next() % 17) - 8.0, (double)(int)(r.next() % 17) - 8.0);
  std::vector<cd> ref(w.size()), out(w.size(), cd(NAN, NAN));
  if (oracle_synthesize((const double*)w.data(), n, (double*)ref.data()) != 0) ++failures;
  report("synthesis n=6 integer weights exact",
         tpd_debug_emulate_synth(w.data(), n, out.data(), TPD_C128, 0, 0) == TPD_SUCCESS &&
             same_bits(out.data(), ref.data(), ref.size()));
}

void batched_check() {
  std::vector<std::vector<cd>> mats, outs;
  std::vector<int> ns;
  for (int k = 0; k < 30; ++k) {
    const int n = k % 10;
    ns.push_back(n);
    mats.push_back(gaussian(n, 400 + k, k % 2 == 1));
    outs.emplace_back((size_t)1 << (2 * n), cd(NAN, NAN));
  }
  std::vector<const void*> in(mats.size());
  std::vector<void*> out(mats.size());
  for (size_t k = 0; k < mats.size(); ++k) {
    in[k] = mats[k].data();
    out[k] = outs[k].data();
  }
  for (int code = 0; code < 3; ++code) {
    // the same shape code for every n (code 2 exists for n >= 3 only)
    int codes[10];
    for (int n = 0; n < 10; ++n) codes[n] = (code == 2 && n < 3) ? 0 : code;
    for (auto& o : outs) std::fill(o.begin(), o.end(), cd(NAN, NAN));
    bool ok = tpd_debug_emulate_batched(in.data(), ns.data(), (int)ns.size(), out.data(), TPD_C128, 0, codes) ==
              TPD_SUCCESS;
    for (size_t k = 0; k < mats.size() && ok; ++k) {
      const auto ref = oracle(mats[k], ns[k]);
      ok = same_bits(outs[k].data(), ref.data(), ref.size());
    }
    char name[96];
    std::snprintf(name, sizeof name, "batched 30 matrices n=0..9, shape code %d, bitwise Algorithm 1", code);
    report(name, ok);
  }
}

void oracle_mt_check() {
  const int n = 9;
  const auto A = gaussian(n, 55, true);
  const auto ref = oracle(A, n);
  std::vector<cd> w(ref.size());
  report("oracle Algorithm 2 on 4 threads equals Algorithm 1",
         oracle_tpd_iterative_mt((const double*)A.data(), n, (double*)w.data(), nullptr, 4) == 0 &&
             same_bits(w.data(), ref.data(), ref.size()));
}

}  // namespace

int main() {
  dense_checks();
  tuned_and_chunked_checks();
  hermitian_pruning_checks();
  partial_checks();
  compact_check();
  synth_check();
  batched_check();
  oracle_mt_check();
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
