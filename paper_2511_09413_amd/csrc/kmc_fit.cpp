// Relaxation time of a decay curve (declared in include/kmc.h, kmc_fit_decay).
//
// After the polarising bias is removed the fraction of ions in the first
// decile decays as one exponential towards an asymptote shared by every run
// (main text section 4, relaxation decay; SI S5).  The relaxation time of a
// sampled curve is that of the least-squares single exponential
//     m(t) ~ C + A exp(-(t - t0)/tau).
// Host-side binary64 arithmetic on a few thousand samples: the fit is
// parameterised by the decay rate k = T/tau in the window time u = (t - t0)/T
// (T the window's largest |t - t0|), model g(u) = C + A exp(-k u), and solved
// by Gauss-Newton steps on the normal equations.  The sensitivities
// d tau / d m_i come from the implicit-function theorem on the stationarity
// condition J^T r = 0 of the same parameterisation:
//     (J^T J - sum_i r_i H_i) d(C, A, k)/d m_i = J_i,   d tau = -(T / k^2) dk.
#include "../../include/kmc.h"

#include <cmath>
#include <string>
#include <vector>

namespace kmc {
kmc_status record_error(kmc_status s, const std::string &msg);
}

namespace {

// Solve the 3x3 system M x = b by Gaussian elimination with partial pivoting;
// false if M is singular to working precision.
bool solve3(double M[3][3], double b[3], double x[3]) {
    double a[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) a[i][j] = M[i][j];
        a[i][3] = b[i];
    }
    double scale = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) scale = std::fmax(scale, std::fabs(a[i][j]));
    if (!(scale > 0.0)) return false;
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
        if (std::fabs(a[piv][col]) <= 1e-300 + 1e-15 * scale) return false;
        if (piv != col)
            for (int j = 0; j < 4; ++j) std::swap(a[piv][j], a[col][j]);
        for (int r = col + 1; r < 3; ++r) {
            const double f = a[r][col] / a[col][col];
            for (int j = col; j < 4; ++j) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = a[i][3];
        for (int j = i + 1; j < 3; ++j) s -= a[i][j] * x[j];
        x[i] = s / a[i][i];
    }
    return true;
}

struct Curve {
    std::vector<double> u, m;  // window time (t - t0)/T and the samples
};

double sum_sq(const Curve &cv, const double p[3]) {
    double s = 0.0;
    for (size_t i = 0; i < cv.u.size(); ++i) {
        const double r = cv.m[i] - (p[0] + p[1] * std::exp(-p[2] * cv.u[i]));
        s += r * r;
    }
    return s;
}

// Normal-equation pieces at p: JtJ, Jt r and (optionally) sum_i r_i H_i.
void normal_terms(const Curve &cv, const double p[3], double JtJ[3][3], double Jtr[3], double RH[3][3]) {
    for (int i = 0; i < 3; ++i) {
        Jtr[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
            JtJ[i][j] = 0.0;
            if (RH) RH[i][j] = 0.0;
        }
    }
    for (size_t n = 0; n < cv.u.size(); ++n) {
        const double u = cv.u[n], e = std::exp(-p[2] * u);
        const double r = cv.m[n] - (p[0] + p[1] * e);
        const double J[3] = {1.0, e, -p[1] * u * e};
        for (int i = 0; i < 3; ++i) {
            Jtr[i] += J[i] * r;
            for (int j = 0; j < 3; ++j) JtJ[i][j] += J[i] * J[j];
        }
        if (RH) {
            // d2g/dA dk = -u e, d2g/dk2 = A u^2 e; the rest vanish
            RH[1][2] += r * (-u * e);
            RH[2][1] += r * (-u * e);
            RH[2][2] += r * (p[1] * u * u * e);
        }
    }
}

}  // namespace

extern "C" kmc_status kmc_fit_decay(const double *t, const double *m, int64_t n, double t0, double *params,
                                    double *weights) {
    using kmc::record_error;
    if (!t || !m || !params) return record_error(KMC_EINVAL, "t, m and params must not be NULL");
    if (n < 4) return record_error(KMC_EINVAL, "the decay fit needs at least 4 samples");
    if (!std::isfinite(t0)) return record_error(KMC_EINVAL, "t0 must be finite");
    double T = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(t[i]) || !std::isfinite(m[i])) return record_error(KMC_EINVAL, "samples must be finite");
        T = std::fmax(T, std::fabs(t[i] - t0));
    }
    if (!(T > 0.0)) return record_error(KMC_EINVAL, "every sample time equals t0");
    Curve cv;
    cv.u.resize((size_t)n);
    cv.m.assign(m, m + n);
    for (int64_t i = 0; i < n; ++i) cv.u[(size_t)i] = (t[i] - t0) / T;

    // starting point: the caller's, or the asymptote from the last tenth of
    // the window, the amplitude at the first sample and the rate from the
    // first sample within 1/e of the asymptote
    double p[3];
    if (std::isfinite(params[0]) && std::isfinite(params[1]) && std::isfinite(params[2]) && params[2] > 0.0) {
        p[0] = params[0];
        p[1] = params[1];
        p[2] = T / params[2];
    } else {
        const int64_t tail = n / 10 > 0 ? n / 10 : 1;
        double c = 0.0;
        for (int64_t i = n - tail; i < n; ++i) c += m[i];
        c /= (double)tail;
        p[0] = c;
        p[1] = m[0] - c;
        double u_e = 1.0 / 3.0;
        for (int64_t i = 0; i < n; ++i)
            if (std::fabs(m[i] - c) < std::fabs(m[0] - c) / std::exp(1.0) && cv.u[(size_t)i] > 0.0) {
                u_e = cv.u[(size_t)i];
                break;
            }
        p[2] = 1.0 / u_e;
    }

    double s = sum_sq(cv, p), prev = INFINITY;
    bool done = false;
    for (int it = 0; it < 500 && !done; ++it) {
        double JtJ[3][3], Jtr[3], d[3];
        normal_terms(cv, p, JtJ, Jtr, nullptr);
        if (!solve3(JtJ, Jtr, d)) return record_error(KMC_EUNSUPPORTED, "decay fit: singular normal equations");
        double rel = 0.0;
        for (int i = 0; i < 3; ++i) rel = std::fmax(rel, std::fabs(d[i]) / std::fmax(std::fabs(p[i]), 1e-300));
        if (rel < 1e-6) {
            // near the minimum the residual sum is flat to rounding: full
            // steps while they shrink
            if (rel >= prev) break;
            for (int i = 0; i < 3; ++i) p[i] += d[i];
            prev = rel;
            done = rel < 1e-15;
            continue;
        }
        double lam = 1.0, q[3], sq = 0.0;
        for (;;) {
            for (int i = 0; i < 3; ++i) q[i] = p[i] + lam * d[i];
            if (q[2] > 0.0 && (sq = sum_sq(cv, q)) <= s) break;
            lam *= 0.5;
            if (lam < 1e-12) return record_error(KMC_EUNSUPPORTED, "decay fit: no descent step");
        }
        for (int i = 0; i < 3; ++i) p[i] = q[i];
        s = sq;
        if (it == 499) return record_error(KMC_EUNSUPPORTED, "decay fit did not converge");
    }
    if (!(p[2] > 0.0) || !std::isfinite(p[0]) || !std::isfinite(p[1]))
        return record_error(KMC_EUNSUPPORTED, "decay fit left the domain tau > 0");

    if (weights) {
        double JtJ[3][3], Jtr[3], RH[3][3], M[3][3];
        normal_terms(cv, p, JtJ, Jtr, RH);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = JtJ[i][j] - RH[i][j];
        // the k row of M^-1 (M symmetric): solve M z = e_k, then dk/dm_i = z . J_i
        double ek[3] = {0.0, 0.0, 1.0}, z[3];
        if (!solve3(M, ek, z)) return record_error(KMC_EUNSUPPORTED, "decay fit: singular sensitivity system");
        const double dtau_dk = -T / (p[2] * p[2]);
        for (int64_t i = 0; i < n; ++i) {
            const double u = cv.u[(size_t)i], e = std::exp(-p[2] * u);
            weights[i] = dtau_dk * (z[0] + z[1] * e + z[2] * (-p[1] * u * e));
        }
    }
    params[0] = p[0];
    params[1] = p[1];
    params[2] = T / p[2];
    return KMC_OK;
}
