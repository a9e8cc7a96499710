// Host construction of the integer acceptance tables, in binary128.
//
// Sec. 2.1 of the paper precomputes the Metropolis factor for every possible
// energy change; App. C builds its random-number tables with GNU quadmath.
// Here the factors are turned into uint32 thresholds for the test r <= thr on
// a uniform 32-bit r:
//
//   thr = ceil(2^32 * min(1, e^{-x})) - 1,   so   P(r <= thr) = ceil(2^32 p)/2^32,
//
// the first 32-bit number not below the exact probability.  x is evaluated
// from the exact double inputs in binary128 (113-bit significand), far
// beyond the 32 bits the comparison keeps.
//
//   Metropolis, slot g:  x = 4k(2 - n_s) + 4kp_g(1 - n_t),
//                        k = beta/L_tau, kp_g = -1/2 ln tanh(beta Gamma_g/L_tau)
//   exchange, pair g:    x = 4 m (kp_g - kp_{g+1}) for Bt[g+1]-Bt[g] = -4m,
//                        m = 1..len while the threshold is positive (0 after).
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

namespace {

constexpr uint32_t kU32Max = 0xFFFFFFFFu;

uint32_t threshold_of_exponent(__float128 x) {
    if (x <= 0) return kU32Max;
    __float128 v = ceilq(ldexpq(expq(-x), 32)) - 1;
    if (v <= 0) return 0;
    if (v >= (__float128)kU32Max) return kU32Max;
    return (uint32_t)v;
}

__float128 time_coupling(double beta, uint32_t L_tau, double gamma) {
    __float128 arg = (__float128)beta * (__float128)gamma / (__float128)L_tau;
    return -logq(tanhq(arg)) / 2;
}

void set_err(char* err, size_t n, const char* msg) {
    if (err && n) {
        std::snprintf(err, n, "%s", msg);
    }
}

}  // namespace

// Returns 0 on success, -1 on invalid input, -2 if an exchange table would
// need more than `cap` entries.  thr: [N][15] (n_s*3 + n_t); eq/len: [N-1];
// sw: [(N-1)*cap], pair g's entries at g*cap.
extern "C" int qsg_tables_build_host(double beta, uint32_t L_tau, uint32_t N,
                                     const double* gamma, uint32_t cap,
                                     uint32_t* thr, uint8_t* eq, uint32_t* len,
                                     uint32_t* sw, char* err, size_t errlen) {
    if (!(beta > 0) || !std::isfinite(beta) || L_tau == 0 || N == 0 || !gamma) {
        set_err(err, errlen, "tables: invalid beta, L_tau, n_gamma or ladder");
        return -1;
    }
    for (uint32_t g = 0; g < N; ++g) {
        if (!(gamma[g] > 0) || !std::isfinite(gamma[g])) {
            set_err(err, errlen, "tables: Gamma values must be finite and > 0");
            return -1;
        }
        if (g + 1 < N && !(gamma[g] <= gamma[g + 1])) {
            set_err(err, errlen, "tables: ladder must be non-decreasing");
            return -1;
        }
    }
    const __float128 k = (__float128)beta / (__float128)L_tau;
    for (uint32_t g = 0; g < N; ++g) {
        const __float128 kp = time_coupling(beta, L_tau, gamma[g]);
        for (int ns = 0; ns < 5; ++ns)
            for (int nt = 0; nt < 3; ++nt) {
                __float128 x = 4 * k * (2 - ns) + 4 * kp * (1 - nt);
                if (thr) thr[g * 15 + ns * 3 + nt] = threshold_of_exponent(x);
            }
    }
    for (uint32_t g = 0; g + 1 < N; ++g) {
        if (gamma[g] == gamma[g + 1]) {
            if (eq) eq[g] = 1;
            if (len) len[g] = 0;
            continue;
        }
        if (eq) eq[g] = 0;
        const __float128 d = time_coupling(beta, L_tau, gamma[g]) -
                             time_coupling(beta, L_tau, gamma[g + 1]);
        uint32_t m = 1;
        for (;; ++m) {
            uint32_t v = threshold_of_exponent(4 * (__float128)m * d);
            if (v == 0) break;
            if (m > cap) {
                set_err(err, errlen, "tables: exchange table longer than swap_table_cap");
                return -2;
            }
            if (sw) sw[(size_t)g * cap + (m - 1)] = v;
        }
        if (len) len[g] = m - 1;
        if (sw)
            for (uint32_t i = m - 1; i < cap; ++i) sw[(size_t)g * cap + i] = 0;
    }
    return 0;
}
