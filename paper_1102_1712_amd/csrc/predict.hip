// Eq. 3: per-coefficient linear prediction of the next projection's initial
// coefficients from the last L solved ones, and the least-squares fit of its
// coefficients on a training sequence.  Host code (K x L scalars per
// projection); no device memory.
#include <math.h>
#include <string.h>

#include "pcasolve.h"

namespace {

constexpr int MAX_L = 8;

bool finite_all(const double *v, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

}  // namespace

extern "C" int pcas_predict(int32_t K, int32_t L, const double *coeffs, const double *history,
                            int32_t n_hist, double *w_out) {
    if (K < 1 || K > PCAS_MAX_K || L < 1 || L > MAX_L || n_hist < L) return PCAS_EINVAL;
    if (!coeffs || !history || !w_out) return PCAS_EINVAL;
    if (!finite_all(coeffs, (long)K * L) || !finite_all(history, (long)n_hist * K))
        return PCAS_ENONFINITE;
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int l = 1; l <= L; ++l) acc += coeffs[k * L + (l - 1)] * history[(long)(n_hist - l) * K + k];
        w_out[k] = acc;
    }
    return PCAS_OK;
}

// For each coefficient k: minimise sum_{t=L}^{T-1} (w[t][k] - sum_l c_l w[t-l][k])^2
// over c by a QR factorisation of the (T - L) x L lagged matrix (modified
// Gram-Schmidt, done twice for orthogonality), then back substitution.
extern "C" int pcas_fit_predictor(int32_t T, int32_t K, int32_t L, const double *w_train,
                                  double *coeffs_out) {
    if (K < 1 || K > PCAS_MAX_K || L < 1 || L > MAX_L || T <= L) return PCAS_EINVAL;
    if (!w_train || !coeffs_out) return PCAS_EINVAL;
    if (!finite_all(w_train, (long)T * K)) return PCAS_ENONFINITE;
    const int m = T - L;
    double *Q = new double[(size_t)m * L];
    double *rhs = new double[m];
    int status = PCAS_OK;
    for (int k = 0; k < K && status == PCAS_OK; ++k) {
        // column l-1 holds w[t - l][k] for t = L .. T-1
        for (int l = 1; l <= L; ++l)
            for (int i = 0; i < m; ++i) Q[(size_t)(l - 1) * m + i] = w_train[(long)(L + i - l) * K + k];
        for (int i = 0; i < m; ++i) rhs[i] = w_train[(long)(L + i) * K + k];
        double R[MAX_L][MAX_L];
        memset(R, 0, sizeof(R));
        for (int j = 0; j < L && status == PCAS_OK; ++j) {
            double *qj = Q + (size_t)j * m;
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < j; ++i) {
                    const double *qi = Q + (size_t)i * m;
                    double d = 0.0;
                    for (int t = 0; t < m; ++t) d += qi[t] * qj[t];
                    for (int t = 0; t < m; ++t) qj[t] -= d * qi[t];
                    R[i][j] += d;
                }
            double nrm = 0.0;
            for (int t = 0; t < m; ++t) nrm += qj[t] * qj[t];
            nrm = sqrt(nrm);
            if (!(nrm > 0.0)) {
                status = PCAS_ESINGULAR;
                break;
            }
            R[j][j] = nrm;
            for (int t = 0; t < m; ++t) qj[t] /= nrm;
        }
        if (status != PCAS_OK) break;
        // R c = Q^T rhs
        double qtb[MAX_L];
        for (int j = 0; j < L; ++j) {
            const double *qj = Q + (size_t)j * m;
            double d = 0.0;
            for (int t = 0; t < m; ++t) d += qj[t] * rhs[t];
            qtb[j] = d;
        }
        // a column whose residual after the others is negligible makes the
        // fit ill-posed (e.g. a constant sequence for L = 2)
        double rmax = 0.0;
        for (int j = 0; j < L; ++j) rmax = fmax(rmax, fabs(R[j][j]));
        for (int j = 0; j < L; ++j)
            if (!(fabs(R[j][j]) > 1e-12 * rmax)) status = PCAS_ESINGULAR;
        if (status != PCAS_OK) break;
        for (int j = L - 1; j >= 0; --j) {
            double v = qtb[j];
            for (int i = j + 1; i < L; ++i) v -= R[j][i] * coeffs_out[k * L + i];
            coeffs_out[k * L + j] = v / R[j][j];
        }
    }
    delete[] Q;
    delete[] rhs;
    return status;
}
