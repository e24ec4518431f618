// Host-side tuning logic (plain C++, no device code).
//
// Section 2.4 of the paper tunes the critical separation r_crit while the
// simulation runs: the GPU time of the gravity calculation is treated as a
// function of r_crit and minimised with Brent's method, and the minimum keeps
// being perturbed because the best value drifts as the system evolves.
//
// BrentMin is Brent's minimisation without derivatives on a bracket [a, b]
// (golden-section steps, parabolic interpolation through the three best
// points when it is safe; R. P. Brent, Algorithms for Minimization without
// Derivatives, 1973, ch. 5) written as an ask/tell state machine: ask() is the
// point to evaluate next, tell(f) hands back the measured value.  So each
// evaluation can be one timed step of a running simulation.
#pragma once

#include <cmath>
#include <utility>
#include <vector>

namespace gothic {

struct BrentMin {
  double a = 0, b = 1;          // current bracket of the minimum
  double x = 0, w = 0, v = 0;   // best point, second best, previous second best
  double fx = 0, fw = 0, fv = 0;
  double d = 0, e = 0;          // last step and the one before
  double xatol = 1e-5;
  double next = 0;              // point whose value is awaited
  int nfev = 0, maxfev = 500;
  bool converged = false;

  static constexpr double kGold = 0.3819660112501051;   // (3 - sqrt 5) / 2
  static double sqrt_eps() { return std::sqrt(2.2e-16); }

  void start(double lo, double hi, double tol, int max_evals) {
    a = lo;
    b = hi;
    xatol = tol;
    maxfev = max_evals;
    nfev = 0;
    converged = false;
    d = e = 0.0;
    next = a + kGold * (b - a);
  }

  double ask() const { return next; }
  bool done() const { return converged || nfev >= maxfev; }
  double best() const { return nfev > 0 ? x : next; }
  double best_value() const { return fx; }

  void tell(double f) {
    const double u = next;
    if (nfev++ == 0) {
      x = w = v = u;
      fx = fw = fv = f;
    } else if (f <= fx) {  // u is the new best: shrink towards it
      if (u >= x) a = x; else b = x;
      v = w; fv = fw;
      w = x; fw = fx;
      x = u; fx = f;
    } else {               // keep x, shrink away from u
      if (u < x) a = u; else b = u;
      if (f <= fw || w == x) {
        v = w; fv = fw;
        w = u; fw = f;
      } else if (f <= fv || v == x || v == w) {
        v = u; fv = f;
      }
    }
    plan();
  }

 private:
  static double sgn1(double t) { return t > 0 ? 1.0 : (t < 0 ? -1.0 : 1.0); }

  // choose the next point, or declare convergence
  void plan() {
    const double xm = 0.5 * (a + b);
    const double tol1 = sqrt_eps() * std::fabs(x) + xatol / 3.0;
    const double tol2 = 2.0 * tol1;
    if (std::fabs(x - xm) <= tol2 - 0.5 * (b - a)) {
      converged = true;
      next = x;
      return;
    }
    bool golden = true;
    if (std::fabs(e) > tol1) {
      // parabola through (x, fx), (w, fw), (v, fv): its vertex is x + p / q
      double r = (x - w) * (fx - fv);
      double q = (x - v) * (fx - fw);
      double p = (x - v) * q - (x - w) * r;
      q = 2.0 * (q - r);
      if (q > 0.0) p = -p;
      q = std::fabs(q);
      const double e_old = e;
      e = d;
      // accept only a step inside the bracket and smaller than half the one
      // before last (otherwise the parabola is not converging)
      if (std::fabs(p) < std::fabs(0.5 * q * e_old) && p > q * (a - x) && p < q * (b - x)) {
        d = p / q;
        const double u = x + d;
        if (u - a < tol2 || b - u < tol2) d = tol1 * sgn1(xm - x);
        golden = false;
      }
    }
    if (golden) {
      e = (x >= xm) ? a - x : b - x;
      d = kGold * e;
    }
    next = x + sgn1(d) * std::fmax(std::fabs(d), tol1);
  }
};

// Online tuning of one quantity from measurements of the running program:
// Brent on [lo, hi]; after convergence a new search follows over a bracket a
// quarter as wide as [lo, hi], centred on the best point (clipped to [lo,
// hi]): the perturbation that keeps the value tracking a moving optimum.
struct OnlineTuner {
  BrentMin bm;
  double lo = 0, hi = 1, tol = 0.1;
  int max_evals = 30;
  double best = 0;      // best point of the last finished search
  bool have_best = false;
  int searches = 0;

  void init(double lo_, double hi_, double tol_, int max_evals_) {
    lo = lo_;
    hi = hi_;
    tol = tol_;
    max_evals = max_evals_;
    have_best = false;
    searches = 0;
    bm.start(lo, hi, tol, max_evals);
  }
  double current() const { return bm.ask(); }
  void observe(double f) {
    bm.tell(f);
    if (bm.done()) {
      best = bm.best();
      have_best = true;
      ++searches;
      const double h = 0.125 * (hi - lo);
      double a = best - h, b = best + h;
      if (a < lo) a = lo;
      if (b > hi) b = hi;
      bm.start(a, b, tol, max_evals);
    }
  }
};

// Group shape per sub-step class.  A block time step changes the number of
// i-particles from step to step by orders of magnitude, and the best number
// of threads sharing one i-particle (S) depends on it (Section 3.4, Fig. 7);
// the paper fixes S and names choosing it per step as future work (Section
// 4).  Here a group of G i-particles is walked by W lanes (the walk width,
// the paper's T_sub of Table 2) with S = W / G lanes each, so a shape is a
// pair (G, W).  The candidates are timed round-robin,
// `rounds` walks each (interleaved, so a tree that ages between rebuilds
// weighs on every candidate alike), and the smallest mean walk time wins.
struct GroupPicker {
  // candidate shapes: group size G with one group per wave64 (W = 64), and
  // G with walk width W < 64 (64 / W groups walked side by side in a wave)
  static constexpr int kCand = 8;
  static constexpr int kSizes[kCand] = {8, 16, 32, 64, 4, 8, 8, 16};
  static constexpr int kWidths[kCand] = {64, 64, 64, 64, 16, 16, 32, 32};
  int rounds = 2;
  double sum[kCand] = {};
  int count[kCand] = {};
  int next = 0;     // candidate timed next
  int chosen = -1;  // index of the winner once every candidate is timed

  void init(int rounds_) {
    rounds = rounds_ < 1 ? 1 : rounds_;
    for (int k = 0; k < kCand; ++k) {
      sum[k] = 0.0;
      count[k] = 0;
    }
    next = 0;
    chosen = -1;
  }
  bool decided() const { return chosen >= 0; }
  int current() const { return kSizes[decided() ? chosen : next]; }
  int current_width() const { return kWidths[decided() ? chosen : next]; }
  void choose(int G, int W = 64) {  // fixed from outside
    for (int k = 0; k < kCand; ++k)
      if (kSizes[k] == G && kWidths[k] == W) chosen = k;
  }
  void observe(double t) {
    if (decided()) return;
    sum[next] += t;
    ++count[next];
    next = (next + 1) % kCand;
    if (next == 0 && count[kCand - 1] >= rounds) {
      int b = 0;
      for (int k = 1; k < kCand; ++k)
        if (sum[k] / count[k] < sum[b] / count[b]) b = k;
      chosen = b;
    }
  }
};

// Tree-rebuild interval (Section 2.6 and Appendix C of the paper).  Reusing
// the last tree saves its construction time t_make, while the walk time
// t_walk^(i) of the i-th step on the same tree grows as the tree drifts from
// the particle distribution.  The mean cost per step over n steps,
// (t_make + sum_i t_walk^(i)) / n, is minimised with three growth models fitted
// by least squares to the walk times measured since the last rebuild:
//   linear     t_walk^(i) = t1 + (i-1) dt               optimum n^2 = 2 t_make / dt
//   power law  t_walk^(i) = t1 r^(i-1)                  (n ln r - 1) r^n = (r-1) t_make/t1 - 1
//   parabolic  t_walk^(i) = t1 + (i-1) b + (i-1)^2 a    n^2 (b/2 + (4n-3) a/6) = t_make
// and the model with the smallest reduced chi^2 (unit weights; nu = m-2 or
// m-3) decides.  Each optimum condition is solved for n in [1, n_max] by
// bisection where the model has a minimum (dt > 0; r > 1; (2n-1) a + b >= 0),
// otherwise n_max.
struct RebuildModels {
  enum Kind { kNone = -1, kLinear = 0, kPower = 1, kParabolic = 2 };
  double t_make = 0.0;
  std::vector<double> tw;  // t_walk^(1..m) since the last rebuild
  double n_max = 64.0;

  void rebuilt(double make) {
    t_make = make;
    tw.clear();
  }
  void sample(double walk) { tw.push_back(walk); }

  struct Fit {
    int kind = kNone;
    double p0 = 0, p1 = 0, p2 = 0;  // t1, slope-or-ratio, curvature
    double chi2nu = HUGE_VAL;
    double n_opt = 0;
  };

  // model value at step i (1-based)
  static double model(const Fit &f, double i) {
    const double x = i - 1.0;
    if (f.kind == kLinear) return f.p0 + x * f.p1;
    if (f.kind == kPower) return f.p0 * std::pow(f.p1, x);
    return f.p0 + x * f.p1 + x * x * f.p2;
  }

  double chi2nu(const Fit &f, int dof_params) const {
    const int m = (int)tw.size();
    double c = 0.0;
    for (int i = 0; i < m; ++i) {
      const double r = model(f, i + 1.0) - tw[i];
      c += r * r;
    }
    return c / (double)(m - dof_params);
  }

  // increasing g on [1, n_max]: smallest n with g(n) >= 0 (bisection)
  template <class G>
  double solve_increasing(G g) const {
    double lo = 1.0, hi = n_max;
    if (g(lo) >= 0.0) return lo;
    if (g(hi) < 0.0) return hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (g(mid) >= 0.0) hi = mid; else lo = mid;
    }
    return hi;
  }

  Fit fit_linear() const {
    Fit f;
    const int m = (int)tw.size();
    if (m < 3) return f;
    double sx = 0, st = 0;
    for (int i = 0; i < m; ++i) { sx += i; st += tw[i]; }
    const double xb = sx / m, tb = st / m;
    double sxx = 0, sxt = 0;
    for (int i = 0; i < m; ++i) {
      sxx += (i - xb) * (i - xb);
      sxt += (i - xb) * (tw[i] - tb);
    }
    f.kind = kLinear;
    f.p1 = sxt / sxx;
    f.p0 = tb - f.p1 * xb;
    f.chi2nu = chi2nu(f, 2);
    f.n_opt = f.p1 > 0.0 ? std::fmin(std::fmax(std::sqrt(2.0 * t_make / f.p1), 1.0), n_max)
                         : n_max;
    return f;
  }

  Fit fit_power() const {
    Fit f;
    const int m = (int)tw.size();
    if (m < 3) return f;
    for (double t : tw)
      if (!(t > 0.0)) return f;
    double sx = 0, sl = 0;
    for (int i = 0; i < m; ++i) { sx += i; sl += std::log(tw[i]); }
    const double xb = sx / m, lb = sl / m;
    double sxx = 0, sxl = 0;
    for (int i = 0; i < m; ++i) {
      sxx += (i - xb) * (i - xb);
      sxl += (i - xb) * (std::log(tw[i]) - lb);
    }
    const double lr = sxl / sxx;
    f.kind = kPower;
    f.p1 = std::exp(lr);
    f.p0 = std::exp(lb - lr * xb);
    f.chi2nu = chi2nu(f, 2);
    if (f.p1 > 1.0) {
      const double r = f.p1, rhs = (r - 1.0) * t_make / f.p0 - 1.0;
      f.n_opt = solve_increasing([&](double n) { return (n * lr - 1.0) * std::pow(r, n) - rhs; });
    } else {
      f.n_opt = n_max;
    }
    return f;
  }

  Fit fit_parabolic() const {
    Fit f;
    const int m = (int)tw.size();
    if (m < 4) return f;
    // normal equations for t = c0 + c1 x + c2 x^2, x = i - 1
    double S[5] = {0, 0, 0, 0, 0}, T[3] = {0, 0, 0};
    for (int i = 0; i < m; ++i) {
      double xp = 1.0;
      for (int k = 0; k < 5; ++k) {
        S[k] += xp;
        if (k < 3) T[k] += xp * tw[i];
        xp *= i;
      }
    }
    double A[3][4] = {{S[0], S[1], S[2], T[0]}, {S[1], S[2], S[3], T[1]},
                      {S[2], S[3], S[4], T[2]}};
    for (int col = 0; col < 3; ++col) {  // Gaussian elimination, partial pivoting
      int piv = col;
      for (int r = col + 1; r < 3; ++r)
        if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
      for (int k = 0; k < 4; ++k) std::swap(A[col][k], A[piv][k]);
      if (A[col][col] == 0.0) return f;
      for (int r = 0; r < 3; ++r) {
        if (r == col) continue;
        const double q = A[r][col] / A[col][col];
        for (int k = col; k < 4; ++k) A[r][k] -= q * A[col][k];
      }
    }
    f.kind = kParabolic;
    f.p0 = A[0][3] / A[0][0];
    f.p1 = A[1][3] / A[1][1];
    f.p2 = A[2][3] / A[2][2];
    f.chi2nu = chi2nu(f, 3);
    const double a = f.p2, b = f.p1;
    auto g = [&](double n) { return n * n * (0.5 * b + (4.0 * n - 3.0) * a / 6.0) - t_make; };
    // g' = n ((2n - 1) a + b): g increases exactly where the extremum would be
    // a minimum; search that part of [1, n_max]
    double lo = 1.0, hi = n_max;
    if (a > 0.0) {
      lo = std::fmax(lo, 0.5 * (1.0 - b / a));
    } else if (a < 0.0) {
      hi = std::fmin(hi, 0.5 * (1.0 - b / a));
    } else if (b < 0.0) {
      hi = 0.0;  // constant or decreasing walk time: no minimum
    }
    if (lo > hi || g(hi) < 0.0) {
      f.n_opt = n_max;
    } else if (g(lo) >= 0.0) {
      f.n_opt = lo;
    } else {
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (g(mid) >= 0.0) hi = mid; else lo = mid;
      }
      f.n_opt = hi;
    }
    return f;
  }

  // the model with the smallest reduced chi^2
  Fit best() const {
    Fit b;
    for (const Fit &f : {fit_linear(), fit_power(), fit_parabolic()})
      if (f.kind != kNone && f.chi2nu < b.chi2nu) b = f;
    return b;
  }

  // rebuild before the next step?
  bool due() const {
    const double m = (double)tw.size();
    if (m >= n_max) return true;
    const Fit f = best();
    return f.kind != kNone && m >= f.n_opt;
  }
};

}  // namespace gothic
