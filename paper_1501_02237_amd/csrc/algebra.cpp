// Host prologue of the degree path: rank, component count and a small
// saturated kernel basis of an integer exponent matrix, in checked int64.
//
// Section 2 of the paper obtains the point set from the Smith form P A Q = D:
// the bottom n - r rows of the unimodular P span the integer kernel lattice,
// and the degree is k! Vol(conv{0, columns of P_0}) (Proposition "degree").
// Any unimodular transform with A U = [H | 0] gives the same lattice in the
// last k columns of U, and any basis change of that lattice leaves the
// volume unchanged, so the library computes U by Euclid-style column
// reduction (repeatedly subtract the nearest multiple of the smallest entry
// of the row) and keeps the kernel columns short by pairwise Gauss
// (Lagrange) reduction after every row.  The number of components |prod d_j|
// (Proposition "topological") is the gcd of the r x r minors of A, which is
// |det| of the triangular form of H reached by row-Euclid steps.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "bdeg_internal.hpp"

namespace bdeg {
namespace {

struct Overflow {};

inline int64_t ck_mul(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_mul_overflow(a, b, &r)) throw Overflow();
  return r;
}
inline int64_t ck_add(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_add_overflow(a, b, &r)) throw Overflow();
  return r;
}
inline int64_t ck_sub(int64_t a, int64_t b) {
  int64_t r;
  if (__builtin_sub_overflow(a, b, &r)) throw Overflow();
  return r;
}
inline int64_t iabs(int64_t a) {
  if (a == INT64_MIN) throw Overflow();
  return a < 0 ? -a : a;
}
inline int64_t floor_div(int64_t a, int64_t b) { // b > 0
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) q--;
  return q;
}
// nearest integer to a / b (b != 0), ties toward +infinity
inline int64_t round_div(int64_t a, int64_t b) {
  if (b < 0) {
    a = ck_sub(0, a);
    b = ck_sub(0, b);
  }
  return floor_div(ck_add(ck_mul(2, a), b), ck_mul(2, b));
}

// Column-major working matrix W = [A ; I_n]: col[c][row], rows 0..m-1 hold
// A U, rows m..m+n-1 hold U.
struct Work {
  int m, n;
  std::vector<std::vector<int64_t>> col;
  void axpy(int c, int64_t q, int d) { // col c -= q * col d
    if (q == 0) return;
    auto &x = col[c];
    const auto &y = col[d];
    for (size_t i = 0; i < x.size(); i++) x[i] = ck_sub(x[i], ck_mul(q, y[i]));
  }
  int64_t udot(int a, int b) const { // dot of the U parts
    int64_t s = 0;
    for (int i = m; i < m + n; i++) s = ck_add(s, ck_mul(col[a][i], col[b][i]));
    return s;
  }
};

// Pairwise Gauss reduction of columns [lo, n) by their U parts.  Every step
// subtracts an integer multiple of one column from another (unimodular) and
// strictly shortens it, so the loop ends.
void pairwise_reduce(Work &W, int lo) {
  const int n = W.n;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int a = lo; a < n; a++)
      for (int b = lo; b < n; b++) {
        if (a == b) continue;
        int64_t bb = W.udot(b, b);
        if (bb == 0) continue;
        int64_t q = round_div(W.udot(a, b), bb);
        if (q == 0) continue;
        // ||a - q b||^2 = aa - 2 q ab + q^2 bb < aa  <=>  q (q bb - 2 ab) < 0
        int64_t ab = W.udot(a, b);
        if (ck_mul(q, ck_sub(ck_mul(q, bb), ck_mul(2, ab))) < 0) {
          W.axpy(a, q, b);
          changed = true;
        }
      }
  }
}

} // namespace

KernelPoints kernel_points(const int64_t *A, int m, int n) {
  KernelPoints kp;
  kp.m = m;
  kp.n = n;
  try {
    Work W;
    W.m = m;
    W.n = n;
    W.col.assign(n, std::vector<int64_t>(m + n, 0));
    for (int c = 0; c < n; c++) {
      for (int i = 0; i < m; i++) W.col[c][i] = A[(size_t)i * n + c];
      W.col[c][m + c] = 1;
    }
    int r = 0;
    for (int i = 0; i < m && r < n; i++) {
      for (;;) {
        int best = -1, nz = 0;
        for (int c = r; c < n; c++) {
          int64_t v = W.col[c][i];
          if (v == 0) continue;
          nz++;
          if (best < 0 || iabs(v) < iabs(W.col[best][i])) best = c;
        }
        if (nz <= 1) break;
        for (int c = r; c < n; c++)
          if (c != best && W.col[c][i] != 0) W.axpy(c, round_div(W.col[c][i], W.col[best][i]), best);
      }
      int piv = -1;
      for (int c = r; c < n; c++)
        if (W.col[c][i] != 0) { piv = c; break; }
      if (piv < 0) continue; // row i depends on earlier rows
      std::swap(W.col[piv], W.col[r]);
      r++;
      pairwise_reduce(W, r);
    }
    kp.rank = r;
    kp.k = n - r;
    if (r < m) kp.flags |= BDEG_F_NEEDS_CONSISTENCY;

    // components: row-Euclid on H = rows 0..m-1 of the pivot columns 0..r-1
    std::vector<std::vector<int64_t>> H(m, std::vector<int64_t>(r));
    for (int i = 0; i < m; i++)
      for (int c = 0; c < r; c++) H[i][c] = W.col[c][i];
    u128 comps = 1;
    for (int t = 0; t < r; t++) {
      for (;;) {
        int best = -1, nz = 0;
        for (int i = t; i < m; i++) {
          if (H[i][t] == 0) continue;
          nz++;
          if (best < 0 || iabs(H[i][t]) < iabs(H[best][t])) best = i;
        }
        if (nz <= 1) break;
        for (int i = t; i < m; i++)
          if (i != best && H[i][t] != 0) {
            int64_t q = round_div(H[i][t], H[best][t]);
            for (int c = t; c < r; c++) H[i][c] = ck_sub(H[i][c], ck_mul(q, H[best][c]));
          }
      }
      int piv = -1;
      for (int i = t; i < m; i++)
        if (H[i][t] != 0) { piv = i; break; }
      if (piv < 0) throw Overflow(); // cannot happen: H has full column rank r
      std::swap(H[piv], H[t]);
      u128 d = (u128)iabs(H[t][t]);
      if (comps > (~(u128)0) / d) throw Overflow();
      comps *= d;
    }
    kp.comps = comps;

    // points: origin, then row i of the kernel basis (columns r..n-1 of U)
    const int k = kp.k;
    kp.pts.assign((size_t)(n + 1) * k, 0);
    for (int i = 0; i < n; i++)
      for (int c = 0; c < k; c++) {
        int64_t v = W.col[r + c][m + i];
        if (v > INT32_MAX || v < -INT32_MAX) throw Overflow();
        kp.pts[(size_t)(i + 1) * k + c] = (int32_t)v;
      }
  } catch (Overflow &) {
    kp.status = BDEG_E_OVERFLOW;
  }
  return kp;
}

// Hadamard bound on every minor the device path forms.  A spatial residual at
// depth t is a (t+2) x (t+2) determinant with rows (1, p_j) over t+1 chosen
// coordinates, so |.| <= prod over its rows of sqrt(1 + |p_j|^2) <= Hs, the
// product over the k+1 largest such factors.  A height residual expands along
// the height column into at most k+1 height differences times such minors:
// |.| <= (k+1) * span * Hs.  The device keeps spatial values in int32 and
// splits heights as H1 * 2^31 + H0 so that every product is 32 x 32 -> 64 bits;
// sums of two such products must fit int64, so it needs Hs < 2^31 and
// (k+1) * span * Hs < 2^60.
//
// The same minors are also bounded column-wise (Hadamard on columns): the
// all-ones column has norm <= sqrt(k+1) and coordinate column i has norm
// <= sqrt(k+1) * max_j |p_ji|, so Hs^2 <= (k+1)^(k+1) * prod_i max(1, M_i)^2.
// The smaller of the two certificates is used; point sets that are long in a
// few directions only (a lattice with one long basis vector) pass the second.
bool device_bounds_ok(const int32_t *pts, int N, int k, uint64_t height_span, int spatial_bits, int height_bits) {
  const u128 lim = (u128)1 << (2 * spatial_bits);
  // row-wise: product of the k+1 largest (1 + |p_j|^2)
  std::vector<u128> f(N);
  for (int j = 0; j < N; j++) {
    u128 s = 1;
    for (int i = 0; i < k; i++) {
      int64_t v = pts[(size_t)j * k + i];
      s += (u128)(v * v);
    }
    f[j] = s;
  }
  std::sort(f.begin(), f.end(), [](u128 a, u128 b) { return a > b; });
  u128 h2_rows = 1;
  for (int j = 0; j < std::min(N, k + 1) && h2_rows < lim; j++) {
    if (f[j] != 0 && h2_rows > lim / f[j]) h2_rows = lim;
    else h2_rows *= f[j];
  }
  // column-wise: (k+1)^(k+1) * prod_i max(1, M_i)^2
  u128 h2_cols = 1;
  for (int i = 0; i <= k && h2_cols < lim; i++) {
    u128 f2 = (u128)(k + 1);
    if (i < k) {
      int64_t mx = 1;
      for (int j = 0; j < N; j++) mx = std::max<int64_t>(mx, std::abs((int64_t)pts[(size_t)j * k + i]));
      f2 *= (u128)(mx * mx);
    }
    if (h2_cols > lim / f2) h2_cols = lim;
    else h2_cols *= f2;
  }
  const u128 h2 = std::min(h2_rows, h2_cols);
  if (h2 >= lim) return false;
  // ((k+1) * span)^2 * Hs^2 < 2^(2 height_bits)
  u128 ks = (u128)(k + 1) * (u128)(height_span ? height_span : 1);
  if (ks >= ((u128)1 << height_bits)) return false;
  u128 ks2 = ks * ks;
  const u128 lim2 = (u128)1 << (2 * height_bits);
  if (h2 != 0 && ks2 > lim2 / h2) return false;
  return true;
}

} // namespace bdeg
