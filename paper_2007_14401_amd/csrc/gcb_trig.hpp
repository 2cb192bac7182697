// sin and cos by Cody-Waite additive reduction by pi/2 with a two-part
// constant (first part 33 significant bits, so k * kPio2Hi is exact for
// |k| < 2^20, i.e. |x| below about 1.6e6) and Taylor polynomials of degree
// 19 (sin) and 20 (cos) on [-pi/4, pi/4] in Horner form: within one unit in
// the last place of the correctly rounded values away from their zeros.
// The curved-spacetime metric takes sin and cos of theta with it, the
// gyro-phase option of the guiding-center step the phase advance of a step.
#pragma once

#include <type_traits>

#include "gcb_common.hpp"

namespace gcb {

constexpr double kPio2Hi = 1.57079632673412561417e+00;
constexpr double kPio2Lo = 6.07710050650619224932e-11;
constexpr double kTrigPi = 3.141592653589793;

// binary64: the full polynomial; binary32: the reduction in binary64 and
// the polynomials to degree 11/12, which reach binary32 precision
template <typename R>
GCB_HD void sincos_poly(double th, R& sn, R& cs) {
    const double k = floor(th * (2.0 / kTrigPi) + 0.5);
    const double yd = (th - k * kPio2Hi) - k * kPio2Lo;
    const R y = (R)yd;
    const R z = y * y;
    R ps, pc;
    if constexpr (std::is_same<R, float>::value) {
        ps = (R)(-1.0 / 39916800.0);
        ps = ps * z + (R)(1.0 / 362880.0);
        ps = ps * z + (R)(-1.0 / 5040.0);
        ps = ps * z + (R)(1.0 / 120.0);
        ps = ps * z + (R)(-1.0 / 6.0);
        pc = (R)(1.0 / 479001600.0);
        pc = pc * z + (R)(-1.0 / 3628800.0);
        pc = pc * z + (R)(1.0 / 40320.0);
        pc = pc * z + (R)(-1.0 / 720.0);
        pc = pc * z + (R)(1.0 / 24.0);
        pc = pc * z + (R)(-1.0 / 2.0);
    } else {
        ps = -1.0 / 121645100408832000.0;              // -1/19!
        ps = ps * z + 1.0 / 355687428096000.0;         // 1/17!
        ps = ps * z + -1.0 / 1307674368000.0;          // -1/15!
        ps = ps * z + 1.0 / 6227020800.0;              // 1/13!
        ps = ps * z + -1.0 / 39916800.0;               // -1/11!
        ps = ps * z + 1.0 / 362880.0;                  // 1/9!
        ps = ps * z + -1.0 / 5040.0;                   // -1/7!
        ps = ps * z + 1.0 / 120.0;                     // 1/5!
        ps = ps * z + -1.0 / 6.0;                      // -1/3!
        pc = 1.0 / 2432902008176640000.0;              // 1/20!
        pc = pc * z + -1.0 / 6402373705728000.0;       // -1/18!
        pc = pc * z + 1.0 / 20922789888000.0;          // 1/16!
        pc = pc * z + -1.0 / 87178291200.0;            // -1/14!
        pc = pc * z + 1.0 / 479001600.0;               // 1/12!
        pc = pc * z + -1.0 / 3628800.0;                // -1/10!
        pc = pc * z + 1.0 / 40320.0;                   // 1/8!
        pc = pc * z + -1.0 / 720.0;                    // -1/6!
        pc = pc * z + 1.0 / 24.0;                      // 1/4!
        pc = pc * z + -1.0 / 2.0;                      // -1/2!
    }
    const R s = y + (y * z) * ps;
    const R c = (R)1 + z * pc;
    const int q = (int)((long long)k & 3);
    sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    cs = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}

}  // namespace gcb
