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
//   Metropolis, slot g:  x = 4k_g(2 - n_s) + 4kp_g(1 - n_t)
//   exchange, pair g:    x = 4 m (c_g - c_{g+1}) for D = -4m, m = 1..len while
//                        the threshold is positive (0 after), D the change of
//                        the exchanged energy.
//
// Two forms.  Transverse-field ladder (the Trotter form with separate space
// and time couplings): k_g = beta/L_tau, kp_g = -1/2 ln tanh(beta Gamma_g/L_tau),
// c = kp, D from the time bonds.  Coupling ladder (Sec. 1, Eqs. (2)-(3): one
// coupling k on every bond, the paper's own PT variable): k_g = kp_g = c_g =
// the listed k, D from all bonds.
#include <quadmath.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

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

// Tables from per-slot couplings: ks (space), kt (time) and c (exchange),
// with equal[g] when slots g and g+1 carry the same ladder value.
int build_tables(uint32_t N, const __float128* ks, const __float128* kt, const __float128* c,
                 const uint8_t* equal, uint32_t cap, uint32_t* thr, uint8_t* eq, uint32_t* len,
                 uint32_t* sw, char* err, size_t errlen) {
    for (uint32_t g = 0; g < N; ++g)
        for (int ns = 0; ns < 5; ++ns)
            for (int nt = 0; nt < 3; ++nt) {
                __float128 x = 4 * ks[g] * (2 - ns) + 4 * kt[g] * (1 - nt);
                if (thr) thr[g * 15 + ns * 3 + nt] = threshold_of_exponent(x);
            }
    for (uint32_t g = 0; g + 1 < N; ++g) {
        if (equal[g]) {
            if (eq) eq[g] = 1;
            if (len) len[g] = 0;
            continue;
        }
        if (eq) eq[g] = 0;
        const __float128 d = c[g] - c[g + 1];
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

}  // namespace

// Transverse-field ladder.  Returns 0 on success, -1 on invalid input, -2 if
// an exchange table would need more than `cap` entries.  thr: [N][15]
// (n_s*3 + n_t); eq/len: [N-1]; sw: [(N-1)*cap], pair g's entries at g*cap.
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
    std::vector<__float128> ks(N), kt(N);
    std::vector<uint8_t> equal(N, 0);
    for (uint32_t g = 0; g < N; ++g) {
        ks[g] = (__float128)beta / (__float128)L_tau;
        kt[g] = time_coupling(beta, L_tau, gamma[g]);
        equal[g] = g + 1 < N && gamma[g] == gamma[g + 1];
    }
    return build_tables(N, ks.data(), kt.data(), kt.data(), equal.data(),
                        cap, thr, eq, len, sw, err, errlen);
}

// Coupling ladder: k_g on every bond of slot g, non-increasing in g (the
// paper lists its k values in decreasing order, App. C), so the transverse
// field -ln tanh(k)/(2k) (Sec. 1) ascends with the slot as in the other form.
extern "C" int qsg_tables_build_host_k(uint32_t N, const double* k, uint32_t cap, uint32_t* thr,
                                       uint8_t* eq, uint32_t* len, uint32_t* sw, char* err,
                                       size_t errlen) {
    if (N == 0 || !k) {
        set_err(err, errlen, "tables: invalid n_gamma or ladder");
        return -1;
    }
    for (uint32_t g = 0; g < N; ++g) {
        if (!(k[g] > 0) || !std::isfinite(k[g])) {
            set_err(err, errlen, "tables: k values must be finite and > 0");
            return -1;
        }
        if (g + 1 < N && !(k[g] >= k[g + 1])) {
            set_err(err, errlen, "tables: k ladder must be non-increasing");
            return -1;
        }
    }
    std::vector<__float128> kk(N);
    std::vector<uint8_t> equal(N, 0);
    for (uint32_t g = 0; g < N; ++g) {
        kk[g] = (__float128)k[g];
        equal[g] = g + 1 < N && k[g] == k[g + 1];
    }
    return build_tables(N, kk.data(), kk.data(), kk.data(), equal.data(),
                        cap, thr, eq, len, sw, err, errlen);
}
