// C ABI of the transfer-matrix product and its Lanczos driver (declared in
// include/qsg.h; paper: Sec. 2.2, the EDQSG code; App. D, the parity-aware
// basis).  The product runs in the kernels of qsg_transfer.hip; the Lanczos
// steps run on the device too (product, dot products, updates), and only
// the tridiagonal projection (at most max_iter numbers) is solved on the
// host, by Sturm-sequence bisection and inverse iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/qsg.h"
#include "qsg_corr_mix.h"
#include "qsg_transfer.h"

namespace {

using qsg::TmParams;

constexpr uint32_t kMaxLanczos = 4096;
constexpr uint32_t kMaxLengths = 4096;  // Euclidean lengths per correlation call

#define TM_HIP(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return qsg::report_error(QSG_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

qsg_status make_params(const qsg_tm_desc* d, TmParams& P) {
    if (!d) return qsg::report_error(QSG_E_INVALID, "null transfer-matrix descriptor");
    if (d->L > QSG_TM_MAX_L)
        return qsg::report_error(QSG_E_UNSUPPORTED, "L = %u: a sector vector of 2^%u doubles does "
                                 "not fit one device here (L <= %u)", d->L, d->L * d->L - 1,
                                 QSG_TM_MAX_L);
    if (d->L < 2) return qsg::report_error(QSG_E_INVALID, "L = %u < 2", d->L);
    if (d->parity != 1 && d->parity != -1)
        return qsg::report_error(QSG_E_INVALID, "parity %d is not +1 or -1", d->parity);
    if (!std::isfinite(d->k) || !std::isfinite(d->k_perp))
        return qsg::report_error(QSG_E_INVALID, "couplings must be finite");
    std::memset(&P, 0, sizeof P);
    const uint32_t L = d->L, V = L * L;
    P.L = L;
    P.n = V - 1;
    for (uint32_t j = 0; j < V; ++j) {
        if ((d->jx[j] != 1 && d->jx[j] != -1) || (d->jy[j] != 1 && d->jy[j] != -1))
            return qsg::report_error(QSG_E_INVALID, "coupling of site %u is not +-1", j);
        const uint32_t x1 = j % L, x2 = j / L, bit = 1u << j;
        (x1 + 1 < L ? P.not_last_col : P.last_col) |= bit;
        (x2 + 1 < L ? P.not_last_row : P.last_row) |= bit;
        if (d->jx[j] < 0) P.jxm |= bit;
        if (d->jy[j] < 0) P.jym |= bit;
    }
    P.all = (V == 32) ? ~0u : ((1u << V) - 1);
    const double kp = d->k_perp;
    P.jp = 1.0 / (1.0 + std::exp(-2.0 * kp));  // e^kp / (e^kp + e^-kp)
    P.jm = 1.0 / (1.0 + std::exp(2.0 * kp));   // e^-kp / (e^kp + e^-kp)
    P.jm_last = d->parity * P.jm;
    for (uint32_t u = 0; u <= 2 * V; ++u)  // Bsp = 2 L^2 - 2 u
        P.wtab[u] = std::exp(0.5 * d->k * (double)(2.0 * V - 2.0 * u));
    return QSG_OK;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[0..m-1) (Sturm sequence).
uint32_t count_below(const std::vector<double>& a, const std::vector<double>& b, uint32_t m,
                     double x, double tiny) {
    uint32_t cnt = 0;
    double q = 1.0;
    for (uint32_t i = 0; i < m; ++i) {
        q = a[i] - x - (i ? b[i - 1] * b[i - 1] / q : 0.0);
        if (std::fabs(q) < tiny) q = -tiny;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// Eigenvalue number i (ascending) by bisection inside the Gershgorin bounds.
double bisect(const std::vector<double>& a, const std::vector<double>& b, uint32_t m, uint32_t i,
              double lo, double hi, double tiny) {
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(a, b, m, mid, tiny) > i) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Solve (T - theta) z = z in place: Gaussian elimination with partial
// pivoting of the tridiagonal matrix (U gains a second superdiagonal).
void shifted_solve(const std::vector<double>& a, const std::vector<double>& b, uint32_t m,
                   double theta, double tiny, std::vector<double>& z) {
    std::vector<double> d(m), lo(m, 0.0), up(m, 0.0), up2(m, 0.0);
    std::vector<char> swapped(m, 0);
    for (uint32_t i = 0; i < m; ++i) {
        d[i] = a[i] - theta;
        if (i + 1 < m) lo[i] = up[i] = b[i];
    }
    for (uint32_t i = 0; i + 1 < m; ++i) {
        if (std::fabs(d[i]) >= std::fabs(lo[i])) {
            if (std::fabs(d[i]) < tiny) d[i] = tiny;
            const double f = lo[i] / d[i];
            lo[i] = f;
            d[i + 1] -= f * up[i];
        } else {  // rows i and i+1 exchanged
            const double di = d[i], dn = d[i + 1], ui = up[i];
            const double f = di / lo[i];
            d[i] = lo[i];
            lo[i] = f;
            up[i] = dn;
            d[i + 1] = ui - f * dn;
            if (i + 2 < m) {
                up2[i] = up[i + 1];
                up[i + 1] = -f * up[i + 1];
            }
            swapped[i] = 1;
        }
    }
    if (std::fabs(d[m - 1]) < tiny) d[m - 1] = tiny;
    for (uint32_t i = 0; i + 1 < m; ++i) {
        if (swapped[i]) std::swap(z[i], z[i + 1]);
        z[i + 1] -= lo[i] * z[i];
    }
    for (int64_t i = (int64_t)m - 1; i >= 0; --i) {
        double s = z[i];
        if (i + 1 < (int64_t)m) s -= up[i] * z[i + 1];
        if (i + 2 < (int64_t)m) s -= up2[i] * z[i + 2];
        z[i] = s / d[i];
    }
}

// Unit eigenvector of the tridiagonal matrix for the eigenvalue theta
// (inverse iteration from a constant vector).
std::vector<double> tri_vector(const std::vector<double>& a, const std::vector<double>& b,
                               uint32_t m, double theta, double tiny) {
    std::vector<double> z(m, 1.0);
    for (int it = 0; it < 3; ++it) {
        shifted_solve(a, b, m, theta, tiny, z);
        double nrm = 0.0;
        for (double v : z) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0) || !std::isfinite(nrm)) break;
        for (double& v : z) v /= nrm;
    }
    return z;
}

// Entries of the Walsh-Hadamard transform of v^2 that the ground-state
// correlations need (App. E): a set S of sites has R_S = W[S without the
// last site] / W[0].  Ordered pairs and quadruples of sites reduce to the
// set met an odd number of times (empty, a pair, a quadruple), so
//   Q2 = V + 2 sum_pairs R^2,
//   Q4 = 3V^2 - 2V + (12V - 16) sum_pairs R^2 + 24 sum_quadruples R^2,
//   F  = V + sum_pairs R^2 [cos(2 pi dx1 / L) + cos(2 pi dx2 / L)].
// Weights per entry: (Q2, Q4, F).
struct CorrTable {
    std::vector<uint32_t> mask;
    std::vector<double> w;
    double q2 = 0, q4 = 0, f = 0;  // the empty set's terms
};

CorrTable corr_table(uint32_t L) {
    CorrTable t;
    const uint32_t V = L * L, last = V - 1;
    auto bits = [&](std::initializer_list<uint32_t> s) {
        uint32_t m = 0;
        for (uint32_t i : s)
            if (i != last) m |= 1u << i;
        return m;
    };
    const double two_pi = 6.283185307179586476925286766559;
    for (uint32_t x = 0; x < V; ++x)
        for (uint32_t y = x + 1; y < V; ++y) {
            t.mask.push_back(bits({x, y}));
            const double dx1 = (double)(x % L) - (double)(y % L);
            const double dx2 = (double)(x / L) - (double)(y / L);
            t.w.insert(t.w.end(), {2.0, 12.0 * V - 16.0,
                                   std::cos(two_pi * dx1 / L) + std::cos(two_pi * dx2 / L)});
        }
    for (uint32_t a = 0; a < V; ++a)
        for (uint32_t b = a + 1; b < V; ++b)
            for (uint32_t c = b + 1; c < V; ++c)
                for (uint32_t d = c + 1; d < V; ++d) {
                    t.mask.push_back(bits({a, b, c, d}));
                    t.w.insert(t.w.end(), {0.0, 24.0, 0.0});
                }
    t.q2 = V;
    t.q4 = 3.0 * V * V - 2.0 * V;
    t.f = V;
    return t;
}

size_t corr_entries(uint32_t L) {
    const size_t V = (size_t)L * L;
    return V * (V - 1) / 2 + V * (V - 1) * (V - 2) * (V - 3) / 24;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

uint64_t qsg_tm_dim(uint32_t L) {
    return (L >= 2 && L <= QSG_TM_MAX_L) ? (uint64_t)1 << (L * L - 1) : 0;
}

qsg_status qsg_tm_apply(const qsg_tm_desc* d, const double* d_in, double* d_out, void* hip_stream) {
    TmParams P;
    if (qsg_status st = make_params(d, P)) return st;
    if (!d_in || !d_out) return qsg::report_error(QSG_E_INVALID, "null vector");
    TM_HIP(qsg::launch_tm_apply(P, d_in, d_out, static_cast<hipStream_t>(hip_stream)));
    return QSG_OK;
}

size_t qsg_tm_lanczos_workspace_bytes(uint32_t L, uint32_t max_iter) {
    const uint64_t N = qsg_tm_dim(L);
    if (!N || max_iter == 0 || max_iter > kMaxLanczos) return 0;
    const size_t doubles = (size_t)(max_iter + 2) * N + (size_t)(max_iter + 1) * qsg::kTmDotBlocks +
                           2 * (size_t)(max_iter + 1) + 2 + max_iter;
    return doubles * sizeof(double);
}

qsg_status qsg_tm_lanczos(const qsg_tm_desc* d, uint32_t max_iter, uint32_t n_eig, double tol,
                          uint64_t seed, void* d_ws, size_t ws_bytes, double* eigs, double* resid,
                          uint32_t* iters, double* d_vec, void* hip_stream) {
    TmParams P;
    if (qsg_status st = make_params(d, P)) return st;
    const size_t N = (size_t)qsg_tm_dim(d->L);
    if (max_iter == 0 || max_iter > kMaxLanczos || n_eig == 0 || n_eig > max_iter || n_eig > N)
        return qsg::report_error(QSG_E_INVALID, "need 1 <= n_eig <= max_iter <= %u and n_eig <= %zu",
                                 kMaxLanczos, N);
    if (!(tol >= 0)) return qsg::report_error(QSG_E_INVALID, "tolerance must be >= 0");
    if (!eigs || !resid || !iters || !d_ws) return qsg::report_error(QSG_E_INVALID, "null buffer");
    if (ws_bytes < qsg_tm_lanczos_workspace_bytes(d->L, max_iter))
        return qsg::report_error(QSG_E_BUFFER, "workspace needs %zu bytes",
                                 qsg_tm_lanczos_workspace_bytes(d->L, max_iter));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* V = static_cast<double*>(d_ws);                     // [max_iter + 1][N]
    double* w = V + (size_t)(max_iter + 1) * N;                 // [N]
    double* partial = w + N;                                    // [max_iter + 1][dot blocks]
    double* h = partial + (size_t)(max_iter + 1) * qsg::kTmDotBlocks;
    double* h2 = h + (max_iter + 1);
    double* nrm = h2 + (max_iter + 1);                          // [2]
    double* y = nrm + 2;                                        // [max_iter]

    TM_HIP(qsg::launch_tm_random(w, N, seed, s));
    TM_HIP(qsg::launch_tm_dots(w, 1, N, w, partial, nrm, s));
    TM_HIP(qsg::launch_tm_scale(w, N, nrm, V, s));

    std::vector<double> alpha, beta;  // the projection: diagonal, off-diagonal
    std::vector<double> theta, est;
    std::vector<double> y0;
    uint32_t m = 0;
    for (uint32_t j = 0; j < max_iter; ++j) {
        double* vj = V + (size_t)j * N;
        TM_HIP(qsg::launch_tm_apply(P, vj, w, s));
        // classical Gram-Schmidt against every basis vector, twice
        TM_HIP(qsg::launch_tm_dots(V, j + 1, N, w, partial, h, s));
        TM_HIP(qsg::launch_tm_update(V, j + 1, N, h, w, s));
        TM_HIP(qsg::launch_tm_dots(V, j + 1, N, w, partial, h2, s));
        TM_HIP(qsg::launch_tm_update(V, j + 1, N, h2, w, s));
        TM_HIP(qsg::launch_tm_dots(w, 1, N, w, partial, nrm, s));
        double hj[2], nr;
        TM_HIP(hipMemcpyAsync(&hj[0], h + j, sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipMemcpyAsync(&hj[1], h2 + j, sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipMemcpyAsync(&nr, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
        TM_HIP(hipStreamSynchronize(s));
        alpha.push_back(hj[0] + hj[1]);
        const double bj = std::sqrt(nr);
        m = j + 1;
        // Ritz values of the projection, largest first, and residual estimates
        double glo = std::numeric_limits<double>::infinity(), ghi = -glo;
        for (uint32_t i = 0; i < m; ++i) {
            const double r = (i ? std::fabs(beta[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(beta[i]) : 0.0);
            glo = std::min(glo, alpha[i] - r);
            ghi = std::max(ghi, alpha[i] + r);
        }
        const double scale = std::max(std::fabs(glo), std::fabs(ghi));
        const double tiny = std::max(scale, 1e-300) * 1e-300;
        const uint32_t nf = std::min(n_eig, m);
        theta.assign(nf, 0.0);
        est.assign(nf, 0.0);
        const double pad = 1e-14 * scale + tiny;
        for (uint32_t i = 0; i < nf; ++i) {
            theta[i] = bisect(alpha, beta, m, m - 1 - i, glo - pad, ghi + pad, tiny);
            const std::vector<double> z = tri_vector(alpha, beta, m, theta[i], tiny);
            est[i] = bj * std::fabs(z[m - 1]);
            if (i == 0) y0 = z;
        }
        const bool exhausted = bj <= 1e-12 * scale;
        bool converged = nf == n_eig;
        for (uint32_t i = 0; i < nf && converged; ++i)
            converged = est[i] <= tol * std::fabs(theta[0]);
        if (exhausted || converged) break;
        beta.push_back(bj);
        if (j + 1 < max_iter) TM_HIP(qsg::launch_tm_scale(w, N, nrm, V + (size_t)(j + 1) * N, s));
    }
    for (uint32_t i = 0; i < n_eig; ++i) {
        const bool have = i < theta.size();
        eigs[i] = have ? theta[i] : std::numeric_limits<double>::quiet_NaN();
        resid[i] = have ? est[i] : std::numeric_limits<double>::quiet_NaN();
    }
    *iters = m;
    if (d_vec) {
        TM_HIP(hipMemcpyAsync(y, y0.data(), m * sizeof(double), hipMemcpyHostToDevice, s));
        TM_HIP(qsg::launch_tm_combine(V, m, N, y, d_vec, s));
        TM_HIP(hipStreamSynchronize(s));
    }
    return QSG_OK;
}

size_t qsg_tm_correlations_workspace_bytes(uint32_t L) {
    const uint64_t N = qsg_tm_dim(L);
    if (!N) return 0;
    const size_t E = corr_entries(L);
    return align256(N * sizeof(double)) + align256(E * sizeof(uint32_t)) +
           align256(3 * E * sizeof(double)) + align256(4 * sizeof(double));
}

qsg_status qsg_tm_correlations(uint32_t L, const double* d_vec, void* d_ws, size_t ws_bytes,
                               double* out, void* hip_stream) {
    if (L > QSG_TM_MAX_L)
        return qsg::report_error(QSG_E_UNSUPPORTED, "L = %u > %u", L, QSG_TM_MAX_L);
    if (L < 2) return qsg::report_error(QSG_E_INVALID, "L = %u < 2", L);
    if (!d_vec || !d_ws || !out) return qsg::report_error(QSG_E_INVALID, "null buffer");
    if (ws_bytes < qsg_tm_correlations_workspace_bytes(L))
        return qsg::report_error(QSG_E_BUFFER, "workspace needs %zu bytes",
                                 qsg_tm_correlations_workspace_bytes(L));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t N = (size_t)qsg_tm_dim(L);
    const CorrTable t = corr_table(L);
    const uint32_t E = (uint32_t)t.mask.size();
    char* base = static_cast<char*>(d_ws);
    double* W = reinterpret_cast<double*>(base);
    uint32_t* mask = reinterpret_cast<uint32_t*>(base + align256(N * sizeof(double)));
    double* w = reinterpret_cast<double*>(reinterpret_cast<char*>(mask) +
                                          align256(E * sizeof(uint32_t)));
    double* sums = reinterpret_cast<double*>(reinterpret_cast<char*>(w) +
                                             align256(3 * (size_t)E * sizeof(double)));
    TmParams P;
    std::memset(&P, 0, sizeof P);
    P.L = L;
    P.n = L * L - 1;
    TM_HIP(qsg::launch_tm_wht_squares(P, d_vec, W, s));
    TM_HIP(hipMemcpyAsync(mask, t.mask.data(), E * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TM_HIP(hipMemcpyAsync(w, t.w.data(), 3 * (size_t)E * sizeof(double), hipMemcpyHostToDevice, s));
    TM_HIP(qsg::launch_tm_corr(W, mask, w, E, sums, s));
    double h[3];
    TM_HIP(hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    out[0] = t.q2 + h[0];
    out[1] = t.q4 + h[1];
    out[2] = t.f + h[2];
    return QSG_OK;
}


size_t qsg_tm_correlations_lt_workspace_bytes(uint32_t L, uint32_t n) {
    const uint64_t N = qsg_tm_dim(L);
    if (!N || n == 0 || n > kMaxLengths) return 0;
    const size_t E = corr_entries(L);
    return 2 * align256(N * sizeof(double)) + align256(E * sizeof(uint32_t)) +
           align256(3 * E * sizeof(double)) + 2 * align256(3 * (size_t)n * sizeof(double));
}

qsg_status qsg_tm_correlations_lt(uint32_t L, const double* d_even, const double* d_odd,
                                  double lambda_even, double lambda_odd, const uint32_t* l_taus,
                                  uint32_t n, void* d_ws, size_t ws_bytes, double* out,
                                  void* hip_stream) {
    if (L > QSG_TM_MAX_L)
        return qsg::report_error(QSG_E_UNSUPPORTED, "L = %u > %u", L, QSG_TM_MAX_L);
    if (L < 2) return qsg::report_error(QSG_E_INVALID, "L = %u < 2", L);
    if (n == 0 || n > kMaxLengths)
        return qsg::report_error(QSG_E_INVALID, "%u lengths (1 .. %u)", n, kMaxLengths);
    if (!d_even || !d_odd || !l_taus || !d_ws || !out)
        return qsg::report_error(QSG_E_INVALID, "null buffer");
    if (!(lambda_even > 0.0) || !(lambda_odd > 0.0) || !std::isfinite(lambda_even) ||
        !std::isfinite(lambda_odd))
        return qsg::report_error(QSG_E_INVALID, "eigenvalues %g, %g are not positive and finite",
                                 lambda_even, lambda_odd);
    if (ws_bytes < qsg_tm_correlations_lt_workspace_bytes(L, n))
        return qsg::report_error(QSG_E_BUFFER, "workspace needs %zu bytes",
                                 qsg_tm_correlations_lt_workspace_bytes(L, n));
    // odd weight per length: 1 / (1 + (lambda_even / lambda_odd)^L_tau)
    std::vector<double> w_odd(n);
    const double log_ratio = std::log(lambda_even) - std::log(lambda_odd);
    for (uint32_t i = 0; i < n; ++i)
        w_odd[i] = l_taus[i] == 0 ? 0.0 : 1.0 / (1.0 + std::exp(l_taus[i] * log_ratio));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t N = (size_t)qsg_tm_dim(L);
    const CorrTable t = corr_table(L);
    const uint32_t E = (uint32_t)t.mask.size();
    char* base = static_cast<char*>(d_ws);
    double* We = reinterpret_cast<double*>(base);
    double* Wo = reinterpret_cast<double*>(base + align256(N * sizeof(double)));
    uint32_t* mask = reinterpret_cast<uint32_t*>(base + 2 * align256(N * sizeof(double)));
    double* w = reinterpret_cast<double*>(reinterpret_cast<char*>(mask) +
                                          align256(E * sizeof(uint32_t)));
    double* wodd = reinterpret_cast<double*>(reinterpret_cast<char*>(w) +
                                             align256(3 * (size_t)E * sizeof(double)));
    double* sums = reinterpret_cast<double*>(reinterpret_cast<char*>(wodd) +
                                             align256(3 * (size_t)n * sizeof(double)));
    TmParams P;
    std::memset(&P, 0, sizeof P);
    P.L = L;
    P.n = L * L - 1;
    TM_HIP(qsg::launch_tm_wht_squares(P, d_even, We, s));
    TM_HIP(qsg::launch_tm_wht_squares(P, d_odd, Wo, s));
    TM_HIP(hipMemcpyAsync(mask, t.mask.data(), E * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TM_HIP(hipMemcpyAsync(w, t.w.data(), 3 * (size_t)E * sizeof(double), hipMemcpyHostToDevice, s));
    TM_HIP(hipMemcpyAsync(wodd, w_odd.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
    TM_HIP(qsg::launch_tm_corr_mixed(We, Wo, mask, w, E, wodd, n, sums, s));
    std::vector<double> h(3 * (size_t)n);
    TM_HIP(hipMemcpyAsync(h.data(), sums, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < n; ++i) {
        out[3 * i] = t.q2 + h[3 * i];
        out[3 * i + 1] = t.q4 + h[3 * i + 1];
        out[3 * i + 2] = t.f + h[3 * i + 2];
    }
    return QSG_OK;
}

}  // extern "C"
