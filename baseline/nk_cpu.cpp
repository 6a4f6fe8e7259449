// The straightforward O(n·k) CPU transforms of the paper, multi-threaded with
// OpenMP: a reported baseline for the GPU library, not its checker.
//
//   zeta    (§3 Eq. zeta-fast, Alg. 3): chain-wise prefix sums P = V f, then
//           g(x) = Σ_j P[niv_j(x)] over the finite entries (U P).
//   Möbius  (§3, Alg. 4 scheduled by Alg. 5): y'(x) = g(x) − Σ_{j ≠ chain(x)}
//           y'(niv_j(x)) level by level, every level's elements in parallel;
//           then f(x) = y'(x) − y'(element below x in its chain) (V^{-1}).
//
// Data: function matrices [n, B] row-major in node order; chains given by the
// chain-major numbering (chain c owns rows chain_off[c] .. chain_off[c+1],
// bottom first, node_of_row maps a row to its element); niv as a dense [n, k]
// matrix of rows in that numbering (-1 = none), the same dense map the GPU
// library keeps.  Float data is float32 with float64 accumulation; int64 wraps
// modulo 2^64 (unsigned arithmetic).  Loops are parallel over chains x column
// blocks (scan), rows (gather) and the rows of a level (Möbius).
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

template <typename T> struct Acc;
template <> struct Acc<float> { using A = double; };
template <> struct Acc<int64_t> { using A = uint64_t; };

constexpr int64_t CB = 16;  // columns per scan task

template <typename T>
void zeta_impl(int64_t n, int64_t k, int64_t B, const int32_t* chain_off, const int32_t* node_of_row,
               const int32_t* niv_rows, const T* f, T* g, typename Acc<T>::A* P) {
  using A = typename Acc<T>::A;
  const int64_t ncb = (B + CB - 1) / CB;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int64_t c = 0; c < k; ++c)
    for (int64_t cb = 0; cb < ncb; ++cb) {
      const int64_t b0 = cb * CB, b1 = std::min(B, b0 + CB);
      A acc[CB];
      for (int64_t b = b0; b < b1; ++b) acc[b - b0] = A(0);
      for (int64_t r = chain_off[c]; r < chain_off[c + 1]; ++r) {
        const T* fr = f + (int64_t)node_of_row[r] * B;
        A* pr = P + r * B;
        for (int64_t b = b0; b < b1; ++b) {
          acc[b - b0] += (A)fr[b];
          pr[b] = acc[b - b0];
        }
      }
    }
#pragma omp parallel
  {
    std::vector<A> s(B);
#pragma omp for schedule(dynamic, 256)
    for (int64_t r = 0; r < n; ++r) {
      std::fill(s.begin(), s.end(), A(0));
      const int32_t* nv = niv_rows + r * k;
      for (int64_t j = 0; j < k; ++j) {
        const int32_t t = nv[j];
        if (t < 0) continue;
        const A* pt = P + (int64_t)t * B;
        for (int64_t b = 0; b < B; ++b) s[b] += pt[b];
      }
      T* gr = g + (int64_t)node_of_row[r] * B;
      for (int64_t b = 0; b < B; ++b) gr[b] = (T)s[b];
    }
  }
}

template <typename T>
void mobius_impl(int64_t n, int64_t k, int64_t B, const int32_t* chain_of_row, const int32_t* chain_off,
                 const int32_t* node_of_row, const int32_t* niv_rows, const int32_t* lev_ptr,
                 const int32_t* lev_rows, int64_t nlev, const T* g, T* f, typename Acc<T>::A* Y) {
  using A = typename Acc<T>::A;
  for (int64_t l = 0; l < nlev; ++l) {
#pragma omp parallel
    {
      std::vector<A> s(B);
#pragma omp for schedule(dynamic, 64)
      for (int64_t i = lev_ptr[l]; i < lev_ptr[l + 1]; ++i) {
        const int64_t r = lev_rows[i];
        const T* gr = g + (int64_t)node_of_row[r] * B;
        for (int64_t b = 0; b < B; ++b) s[b] = (A)gr[b];
        const int32_t* nv = niv_rows + r * k;
        for (int64_t j = 0; j < k; ++j) {
          const int32_t t = nv[j];
          if (t < 0 || t == r) continue;
          const A* yt = Y + (int64_t)t * B;
          for (int64_t b = 0; b < B; ++b) s[b] -= yt[b];
        }
        A* yr = Y + r * B;
        for (int64_t b = 0; b < B; ++b) yr[b] = s[b];
      }
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    const bool first = r == chain_off[chain_of_row[r]];
    const A* yr = Y + r * B;
    T* fr = f + (int64_t)node_of_row[r] * B;
    for (int64_t b = 0; b < B; ++b) fr[b] = (T)(first ? yr[b] : yr[b] - yr[b - B]);
  }
}

double median(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  const size_t m = v.size() / 2;
  return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
}

template <typename Fn>
double time_median(Fn fn, int reps, double* each) {
  fn();  // one warm-up
  std::vector<double> t;
  for (int i = 0; i < reps; ++i) {
    const auto a = std::chrono::steady_clock::now();
    fn();
    const auto b = std::chrono::steady_clock::now();
    t.push_back(std::chrono::duration<double>(b - a).count());
    if (each) each[i] = t.back();
  }
  return median(t);
}

}  // namespace

extern "C" {

// Threads the next calls use (0: OpenMP's default).  Returns the count in effect.
int nk_set_threads(int threads) {
  if (threads > 0) omp_set_num_threads(threads);
  return omp_get_max_threads();
}

// dtype 0 = int64, 1 = float32.  work: n * B accumulators (8 bytes each).
int nk_zeta(int dtype, int64_t n, int64_t k, int64_t B, const int32_t* chain_off, const int32_t* node_of_row,
            const int32_t* niv_rows, const void* f, void* g, void* work) {
  if (n < 0 || k < 0 || B < 1) return 1;
  if (dtype == 0)
    zeta_impl<int64_t>(n, k, B, chain_off, node_of_row, niv_rows, (const int64_t*)f, (int64_t*)g, (uint64_t*)work);
  else if (dtype == 1)
    zeta_impl<float>(n, k, B, chain_off, node_of_row, niv_rows, (const float*)f, (float*)g, (double*)work);
  else
    return 1;
  return 0;
}

int nk_mobius(int dtype, int64_t n, int64_t k, int64_t B, const int32_t* chain_of_row, const int32_t* chain_off,
              const int32_t* node_of_row, const int32_t* niv_rows, const int32_t* lev_ptr, const int32_t* lev_rows,
              int64_t nlev, const void* g, void* f, void* work) {
  if (n < 0 || k < 0 || B < 1 || nlev < 0) return 1;
  if (dtype == 0)
    mobius_impl<int64_t>(n, k, B, chain_of_row, chain_off, node_of_row, niv_rows, lev_ptr, lev_rows, nlev,
                         (const int64_t*)g, (int64_t*)f, (uint64_t*)work);
  else if (dtype == 1)
    mobius_impl<float>(n, k, B, chain_of_row, chain_off, node_of_row, niv_rows, lev_ptr, lev_rows, nlev,
                       (const float*)g, (float*)f, (double*)work);
  else
    return 1;
  return 0;
}

// The median of `reps` timed calls after one warm-up (std::chrono::steady_clock),
// seconds; each[i] (nullable, reps entries) receives every timed call.
double nk_time_zeta(int dtype, int64_t n, int64_t k, int64_t B, const int32_t* chain_off, const int32_t* node_of_row,
                    const int32_t* niv_rows, const void* f, void* g, void* work, int reps, double* each) {
  return time_median([&] { nk_zeta(dtype, n, k, B, chain_off, node_of_row, niv_rows, f, g, work); }, reps, each);
}

double nk_time_mobius(int dtype, int64_t n, int64_t k, int64_t B, const int32_t* chain_of_row,
                      const int32_t* chain_off, const int32_t* node_of_row, const int32_t* niv_rows,
                      const int32_t* lev_ptr, const int32_t* lev_rows, int64_t nlev, const void* g, void* f,
                      void* work, int reps, double* each) {
  return time_median([&] {
    nk_mobius(dtype, n, k, B, chain_of_row, chain_off, node_of_row, niv_rows, lev_ptr, lev_rows, nlev, g, f, work);
  }, reps, each);
}

}  // extern "C"
