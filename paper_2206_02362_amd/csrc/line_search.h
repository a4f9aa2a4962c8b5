// More-Thuente line search (J. J. More and D. J. Thuente, "Line search
// algorithms with guaranteed sufficient decrease", ACM TOMS 20(3), 1994), the
// step-length rule of the L-BFGS outer loop (Section 3).  Host code only.
//
// Looks along a descent direction for a step a with
//   phi(a) <= phi(0) + ftol a phi'(0)   and   |phi'(a)| <= gtol |phi'(0)|
// (the strong Wolfe conditions).  Reverse communication: start() and next()
// return kEvaluate with `stp` set to the step whose phi and phi' the caller
// supplies to next(); kConverged means `stp` satisfies both conditions,
// kWarning that the search ended without them (interval below xtol, rounding,
// or a step bound reached), kError that the arguments are invalid.
//
// The search keeps an interval [stx, sty] known to contain acceptable steps
// once `bracketed` is set, and extrapolates (between 1.1 and 4 times the last
// increase) until then.  While no trial step has shown sufficient decrease
// with a nonnegative slope it works on psi(a) = phi(a) - a ftol phi'(0).  Each
// new trial comes from safeguarded cubic and quadratic interpolation of the
// two endpoints (`interpolate`); when the interval fails to shrink by a third
// over two trials, the next trial is its midpoint.
//
// Provenance: the formulas of the trial steps (the cubic and quadratic
// interpolants, their safeguards and the constants 1.1, 4.0 and 0.66) are
// those of MINPACK-2's dcsrch / dcstep, the reference implementation of the
// method, kept expression for expression (same parenthesization, same
// variable names) because the tests require MINPACK's trial steps one for
// one; the reverse-communication structure and the shared cubic helper are
// this file's own.
#pragma once

#include <algorithm>
#include <cmath>

namespace fw {

struct MoreThuente {
  enum Status { kEvaluate, kConverged, kWarning, kError };

  double ftol = 1e-4, gtol = 0.9, xtol = 1e-14, stpmin = 0.0, stpmax = 1e10;
  double stp = 0.0;

  Status start(double stp0, double phi0, double dphi0) {
    if (!(stp0 >= stpmin && stp0 <= stpmax) || !(dphi0 < 0.0) || ftol < 0.0 || gtol < 0.0 || xtol < 0.0 ||
        stpmin < 0.0 || stpmax < stpmin)
      return kError;
    stp = stp0;
    finit_ = phi0;
    ginit_ = dphi0;
    gtest_ = ftol * dphi0;
    bracketed_ = false;
    psi_ = true;
    width_ = stpmax - stpmin;
    width1_ = 2.0 * width_;
    stx_ = sty_ = 0.0;
    fx_ = fy_ = phi0;
    gx_ = gy_ = dphi0;
    lo_ = 0.0;
    hi_ = stp0 + kUp * stp0;
    return kEvaluate;
  }

  Status next(double f, double g) {
    const double ftest = finit_ + stp * gtest_;
    if (psi_ && f <= ftest && g >= 0.0) psi_ = false;
    const bool stalled = (bracketed_ && (stp <= lo_ || stp >= hi_)) ||
                         (bracketed_ && hi_ - lo_ <= xtol * hi_) ||
                         (stp == stpmax && f <= ftest && g <= gtest_) ||
                         (stp == stpmin && (f > ftest || g >= gtest_));
    if (f <= ftest && std::fabs(g) <= gtol * -ginit_) return kConverged;
    if (stalled) return kWarning;

    if (psi_ && f <= fx_ && f > ftest) {
      // interpolate psi, then map the endpoint values back to phi
      double fx = fx_ - stx_ * gtest_, fy = fy_ - sty_ * gtest_, gx = gx_ - gtest_, gy = gy_ - gtest_;
      interpolate(fx, gx, fy, gy, f - stp * gtest_, g - gtest_);
      fx_ = fx + stx_ * gtest_;
      fy_ = fy + sty_ * gtest_;
      gx_ = gx + gtest_;
      gy_ = gy + gtest_;
    } else {
      interpolate(fx_, gx_, fy_, gy_, f, g);
    }
    if (bracketed_) {
      if (std::fabs(sty_ - stx_) >= kShrink * width1_) stp = stx_ + 0.5 * (sty_ - stx_);
      width1_ = width_;
      width_ = std::fabs(sty_ - stx_);
      lo_ = std::min(stx_, sty_);
      hi_ = std::max(stx_, sty_);
    } else {
      lo_ = stp + kLow * (stp - stx_);
      hi_ = stp + kUp * (stp - stx_);
    }
    stp = std::min(std::max(stp, stpmin), stpmax);
    if (bracketed_ && (stp <= lo_ || stp >= hi_ || hi_ - lo_ <= xtol * hi_)) stp = stx_;
    return kEvaluate;
  }

 private:
  static constexpr double kLow = 1.1, kUp = 4.0, kShrink = 0.66;
  double finit_ = 0, ginit_ = 0, gtest_ = 0;
  bool bracketed_ = false, psi_ = true;
  double width_ = 0, width1_ = 0;
  double stx_ = 0, fx_ = 0, gx_ = 0, sty_ = 0, fy_ = 0, gy_ = 0;
  double lo_ = 0, hi_ = 0;

  // cubic through (a, fa, ga) and (b, fb, gb): returns the minimizer's offset
  // ratio r with the step a + r (b - a); `clamp` allows a negative radicand
  static double cubic_ratio(double a, double fa, double ga, double b, double fb, double gb, bool clamp, bool flip) {
    const double theta = 3.0 * (fa - fb) / (b - a) + ga + gb;
    const double s = std::max(std::fabs(theta), std::max(std::fabs(ga), std::fabs(gb)));
    double rad = (theta / s) * (theta / s) - (ga / s) * (gb / s);
    if (clamp) rad = std::max(0.0, rad);
    double gamma = s * std::sqrt(rad);
    if (flip) gamma = -gamma;
    const double p = (gamma - ga) + theta;
    const double q = ((gamma - ga) + gamma) + gb;
    return p / q;
  }

  // One safeguarded trial step from the endpoints (stx, fx, gx), (sty, fy, gy)
  // and the trial (stp, f, g); updates the interval and `stp`.
  void interpolate(double &fx, double &gx, double &fy, double &gy, double f, double g) {
    const double sgnd = g * (gx / std::fabs(gx));
    double next;
    if (f > fx) {
      // higher value: the minimum lies between stx and stp
      const double rc = cubic_ratio(stx_, fx, gx, stp, f, g, false, stp < stx_);
      const double stpc = stx_ + rc * (stp - stx_);
      const double stpq = stx_ + ((gx / ((fx - f) / (stp - stx_) + gx)) / 2.0) * (stp - stx_);
      next = std::fabs(stpc - stx_) < std::fabs(stpq - stx_) ? stpc : stpc + (stpq - stpc) / 2.0;
      bracketed_ = true;
    } else if (sgnd < 0.0) {
      // slopes of opposite sign: the minimum lies between stx and stp
      const double rc = cubic_ratio(stp, f, g, stx_, fx, gx, false, stp > stx_);
      const double stpc = stp + rc * (stx_ - stp);
      const double stpq = stp + (g / (g - gx)) * (stx_ - stp);
      next = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
      bracketed_ = true;
    } else if (std::fabs(g) < std::fabs(gx)) {
      // same sign, smaller slope magnitude: the cubic may have no minimizer
      // in the direction of stx; its step then goes to the interval bound
      const double theta = 3.0 * (fx - f) / (stp - stx_) + gx + g;
      const double s = std::max(std::fabs(theta), std::max(std::fabs(gx), std::fabs(g)));
      double gamma = s * std::sqrt(std::max(0.0, (theta / s) * (theta / s) - (gx / s) * (g / s)));
      if (stp > stx_) gamma = -gamma;
      const double p = (gamma - g) + theta;
      const double q = (gamma + (gx - g)) + gamma;
      const double r = p / q;
      double stpc;
      if (r < 0.0 && gamma != 0.0) stpc = stp + r * (stx_ - stp);
      else stpc = stp > stx_ ? hi_ : lo_;
      const double stpq = stp + (g / (g - gx)) * (stx_ - stp);
      if (bracketed_) {
        next = std::fabs(stpc - stp) < std::fabs(stpq - stp) ? stpc : stpq;
        const double cap = stp + kShrink * (sty_ - stp);
        next = stp > stx_ ? std::min(cap, next) : std::max(cap, next);
      } else {
        next = std::fabs(stpc - stp) > std::fabs(stpq - stp) ? stpc : stpq;
        next = std::max(lo_, std::min(hi_, next));
      }
    } else {
      // same sign, no smaller slope: use the far endpoint, or extrapolate
      if (bracketed_) {
        const double rc = cubic_ratio(stp, f, g, sty_, fy, gy, false, stp > sty_);
        next = stp + rc * (sty_ - stp);
      } else {
        next = stp > stx_ ? hi_ : lo_;
      }
    }
    // new interval: the lower value stays at stx
    if (f > fx) {
      sty_ = stp;
      fy = f;
      gy = g;
    } else {
      if (sgnd < 0.0) {
        sty_ = stx_;
        fy = fx;
        gy = gx;
      }
      stx_ = stp;
      fx = f;
      gx = g;
    }
    stp = next;
  }
};

}  // namespace fw
