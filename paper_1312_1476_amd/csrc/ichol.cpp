// Incomplete-Cholesky factorisation for Proposition 1 with M = L L^T, F = L (Section 5.2), host side.
//
// Left-looking, column by column, on C = Q + shift diag(Q):
//   l_jj = sqrt(c_jj - sum_{k<j} l_jk^2),  l_ij = (c_ij - sum_{k<j} l_ik l_jk) / l_jj  (i > j),
// the numerator of an off-diagonal entry being dropped (before the division, so later columns see the
// zero) when droptol >= 0 and |numerator| < droptol ||Q[:, j]||_2, or, when droptol < 0 (IC(0)), where
// Q_ij = 0.  A non-positive pivot restarts the factorisation with the next shift of 0, 1e-3, 2e-3, ...
// The columns k that touch row j are kept on linked lists keyed by their next row (the classical
// left-looking sparse scheme), with a dense accumulator for column j.
//
// The triangular solves run level by level: forward (L y = b) row i waits for the rows j < i of its
// row of L, backward (L^T x = y) for the rows j > i of its row of L^T; rows of one level are independent.
#include "ichol.hpp"

#include <algorithm>
#include <cmath>

namespace gmrf {

namespace {

// One attempt at a fixed shift; false on breakdown.
bool factor_shifted(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, double droptol, double shift,
                    const std::vector<double>& colnorm, std::vector<std::vector<std::pair<int32_t, double>>>& cols,
                    std::vector<double>& diag) {
  cols.assign((size_t)n, {});
  diag.assign((size_t)n, 0.0);
  std::vector<double> w((size_t)n, 0.0);
  std::vector<int64_t> mark((size_t)n, -1), orig((size_t)n, -1);
  std::vector<int32_t> head((size_t)n, -1), link((size_t)n, -1);
  std::vector<size_t> nextpos((size_t)n, 0);
  std::vector<int32_t> pattern;
  for (int64_t j = 0; j < n; ++j) {
    pattern.clear();
    // column j of the lower triangle of C: row j's entries with column >= j (Q symmetric)
    for (int64_t e = rp[j]; e < rp[j + 1]; ++e) {
      const int64_t i = ci[e];
      if (i < j) continue;
      if (mark[(size_t)i] != j) {
        mark[(size_t)i] = j;
        w[(size_t)i] = 0.0;
        pattern.push_back((int32_t)i);
      }
      w[(size_t)i] += (i == j) ? va[e] * (1.0 + shift) : va[e];
      if (va[e] != 0.0) orig[(size_t)i] = j;
    }
    if (mark[(size_t)j] != j) {
      mark[(size_t)j] = j;
      w[(size_t)j] = 0.0;
      pattern.push_back((int32_t)j);
    }
    // subtract l_ik l_jk for every column k < j with l_jk != 0
    int32_t k = head[(size_t)j];
    head[(size_t)j] = -1;
    while (k >= 0) {
      const int32_t knext = link[(size_t)k];
      auto& ck = cols[(size_t)k];
      const double ljk = ck[nextpos[(size_t)k]].second;
      for (size_t p = nextpos[(size_t)k]; p < ck.size(); ++p) {
        const int64_t i = ck[p].first;
        if (mark[(size_t)i] != j) {
          mark[(size_t)i] = j;
          w[(size_t)i] = 0.0;
          pattern.push_back((int32_t)i);
        }
        w[(size_t)i] -= ck[p].second * ljk;
      }
      if (++nextpos[(size_t)k] < ck.size()) {
        const int32_t i2 = ck[nextpos[(size_t)k]].first;
        link[(size_t)k] = head[(size_t)i2];
        head[(size_t)i2] = k;
      }
      k = knext;
    }
    const double piv = w[(size_t)j];
    if (!(piv > 0.0) || !std::isfinite(piv)) return false;
    const double d = std::sqrt(piv);
    diag[(size_t)j] = d;
    std::sort(pattern.begin(), pattern.end());
    auto& cj = cols[(size_t)j];
    for (int32_t i : pattern) {
      if (i <= j) continue;
      const double num = w[(size_t)i];
      const bool keep = droptol < 0.0 ? (orig[(size_t)i] == j) : (std::fabs(num) >= droptol * colnorm[(size_t)j]);
      if (keep && num != 0.0) cj.emplace_back(i, num / d);
    }
    if (!cj.empty()) {
      nextpos[(size_t)j] = 0;
      const int32_t i2 = cj[0].first;
      link[(size_t)j] = head[(size_t)i2];
      head[(size_t)i2] = (int32_t)j;
    }
  }
  return true;
}

void levels(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, bool forward,
            std::vector<int32_t>& lvl_ptr, std::vector<int32_t>& lvl_rows) {
  std::vector<int32_t> lev((size_t)n, 0);
  int32_t nlev = 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = forward ? t : n - 1 - t;
    int32_t l = 0;
    for (int64_t e = rp[(size_t)i]; e < rp[(size_t)i + 1]; ++e) l = std::max(l, lev[(size_t)ci[(size_t)e]] + 1);
    lev[(size_t)i] = l;
    nlev = std::max(nlev, l + 1);
  }
  lvl_ptr.assign((size_t)nlev + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++lvl_ptr[(size_t)lev[(size_t)i] + 1];
  for (int32_t l = 0; l < nlev; ++l) lvl_ptr[(size_t)l + 1] += lvl_ptr[(size_t)l];
  lvl_rows.assign((size_t)n, 0);
  std::vector<int32_t> fill(lvl_ptr.begin(), lvl_ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i) lvl_rows[(size_t)fill[(size_t)lev[(size_t)i]]++] = (int32_t)i;
}

}  // namespace

bool ichol_factor(int64_t n, const int64_t* rp, const int32_t* ci, const double* va, double droptol, IcholHost& out) {
  std::vector<double> colnorm((size_t)n, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    double s = 0.0;
    for (int64_t e = rp[j]; e < rp[j + 1]; ++e) s += va[e] * va[e];
    colnorm[(size_t)j] = std::sqrt(s);
  }
  std::vector<std::vector<std::pair<int32_t, double>>> cols;
  std::vector<double> diag;
  bool ok = false;
  double shift = 0.0;
  for (int attempt = 0; attempt <= 31 && !ok; ++attempt) {
    shift = attempt == 0 ? 0.0 : 1e-3 * std::ldexp(1.0, attempt - 1);
    ok = factor_shifted(n, rp, ci, va, droptol, shift, colnorm, cols, diag);
  }
  if (!ok) return false;
  out.n = n;
  out.shift = shift;
  out.diag = diag;
  out.logdet_M = 0.0;
  for (double d : diag) out.logdet_M += 2.0 * std::log(d);
  // L^T by rows = L by columns (strictly upper part)
  out.urp.assign((size_t)n + 1, 0);
  for (int64_t j = 0; j < n; ++j) out.urp[(size_t)j + 1] = out.urp[(size_t)j] + (int64_t)cols[(size_t)j].size();
  out.uci.resize((size_t)out.urp[(size_t)n]);
  out.uva.resize((size_t)out.urp[(size_t)n]);
  for (int64_t j = 0; j < n; ++j) {
    int64_t p = out.urp[(size_t)j];
    for (const auto& e : cols[(size_t)j]) {
      out.uci[(size_t)p] = e.first;
      out.uva[(size_t)p] = e.second;
      ++p;
    }
  }
  // L by rows (strictly lower part): transpose, rows in increasing column order
  out.lrp.assign((size_t)n + 1, 0);
  for (int64_t j = 0; j < n; ++j)
    for (const auto& e : cols[(size_t)j]) ++out.lrp[(size_t)e.first + 1];
  for (int64_t i = 0; i < n; ++i) out.lrp[(size_t)i + 1] += out.lrp[(size_t)i];
  out.lci.resize((size_t)out.lrp[(size_t)n]);
  out.lva.resize((size_t)out.lrp[(size_t)n]);
  std::vector<int64_t> fill(out.lrp.begin(), out.lrp.end() - 1);
  for (int64_t j = 0; j < n; ++j)
    for (const auto& e : cols[(size_t)j]) {
      const int64_t p = fill[(size_t)e.first]++;
      out.lci[(size_t)p] = (int32_t)j;
      out.lva[(size_t)p] = e.second;
    }
  levels(n, out.lrp, out.lci, true, out.flev_ptr, out.flev_rows);
  levels(n, out.urp, out.uci, false, out.blev_ptr, out.blev_rows);
  return true;
}

}  // namespace gmrf
