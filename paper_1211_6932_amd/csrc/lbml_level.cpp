// lbml_level.cpp -- host FP64 level model of the learned initialiser (include/lbml.h):
// the Chebyshev tensor basis of the four features and its ridge-regularised
// least-squares fit by Householder QR.  No device code.
#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "lbml.h"

namespace lbmp {
lb_status abi_fail(lb_status st, const std::string& msg);
}  // namespace lbmp

namespace {

using lbmp::abi_fail;

constexpr int kFeatures = LBML_IN;
constexpr int kDeg[kFeatures] = {2, 6, 3, 1};  // a, T/T_c, u = 1/R, nu_g/nu_l
constexpr int kTerms = LBML_LEVEL_TERMS;
static_assert((kDeg[0] + 1) * (kDeg[1] + 1) * (kDeg[2] + 1) * (kDeg[3] + 1) == kTerms, "term count");
constexpr double kRidge = 1e-12;
constexpr int32_t kMaxFitRows = 262144;

// The fitted variable of feature f: R enters as u = 1/R.
double variable(const double* x, int f) { return f == 2 ? 1.0 / x[2] : x[f]; }

bool row_ok(const double* x)
{
    for (int f = 0; f < kFeatures; ++f)
        if (!std::isfinite(x[f])) return false;
    return x[2] > 0.0;
}

// One row of the basis matrix (column ((i * 7 + j) * 4 + k) * 2 + l).
void basis_row(const lbml_level_model& m, const double* x, double* row)
{
    double T[kFeatures][7];
    for (int f = 0; f < kFeatures; ++f) {
        double z = 0.0;
        if (m.hi[f] > m.lo[f]) {
            z = 2.0 * (variable(x, f) - m.lo[f]) / (m.hi[f] - m.lo[f]) - 1.0;
            z = std::fmin(1.0, std::fmax(-1.0, z));
        }
        T[f][0] = 1.0;
        T[f][1] = z;
        for (int n = 2; n <= kDeg[f]; ++n) T[f][n] = 2.0 * z * T[f][n - 1] - T[f][n - 2];
    }
    int c = 0;
    for (int i = 0; i <= kDeg[0]; ++i)
        for (int j = 0; j <= kDeg[1]; ++j)
            for (int k = 0; k <= kDeg[2]; ++k)
                for (int l = 0; l <= kDeg[3]; ++l) row[c++] = T[0][i] * T[1][j] * T[2][k] * T[3][l];
}

// Least-squares solution of the column-major rows x p system M c = b by Householder
// QR (M and b are overwritten).  False if a diagonal of R vanishes.
bool householder_solve(std::vector<double>& M, std::vector<double>& b, long long rows, int p, double* c)
{
    std::vector<double> diag(p);
    for (int j = 0; j < p; ++j) {
        double* col = M.data() + (long long)j * rows;
        double norm2 = 0.0;
        for (long long r = j; r < rows; ++r) norm2 += col[r] * col[r];
        const double norm = std::sqrt(norm2);
        if (!(norm > 0.0)) return false;
        const double alpha = col[j] > 0.0 ? -norm : norm;
        // v = col[j:] - alpha e_j, stored in place; v^T v = 2 norm (norm + |col[j]|)
        col[j] -= alpha;
        const double vtv = 2.0 * norm * (norm + std::fabs(col[j] + alpha));
        for (int q = j + 1; q < p; ++q) {
            double* cq = M.data() + (long long)q * rows;
            double s = 0.0;
            for (long long r = j; r < rows; ++r) s += col[r] * cq[r];
            const double f = 2.0 * s / vtv;
            for (long long r = j; r < rows; ++r) cq[r] -= f * col[r];
        }
        double s = 0.0;
        for (long long r = j; r < rows; ++r) s += col[r] * b[r];
        const double f = 2.0 * s / vtv;
        for (long long r = j; r < rows; ++r) b[r] -= f * col[r];
        diag[j] = alpha;
    }
    for (int j = p - 1; j >= 0; --j) {
        double s = b[j];
        for (int q = j + 1; q < p; ++q) s -= M[(long long)q * rows + j] * c[q];
        c[j] = s / diag[j];
    }
    return true;
}

}  // namespace

extern "C" {

lb_status lbml_level_fit(const double* x, const double* y, int32_t n, lbml_level_model* model)
{
    if (!x || !y || !model) return abi_fail(LB_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxFitRows) return abi_fail(LB_EINVAL, "lbml_level_fit: need 1 <= n <= 262144 rows");
    for (int32_t i = 0; i < n; ++i) {
        if (!row_ok(x + (long long)i * kFeatures)) return abi_fail(LB_EINVAL, "features must be finite with R > 0");
        if (!std::isfinite(y[i])) return abi_fail(LB_EINVAL, "targets must be finite");
    }
    lbml_level_model m{};
    for (int f = 0; f < kFeatures; ++f) {
        m.lo[f] = m.hi[f] = variable(x, f);
        for (int32_t i = 1; i < n; ++i) {
            const double v = variable(x + (long long)i * kFeatures, f);
            m.lo[f] = std::fmin(m.lo[f], v);
            m.hi[f] = std::fmax(m.hi[f], v);
        }
    }
    const long long rows = (long long)n + kTerms;
    std::vector<double> M, b;
    try {
        M.assign((size_t)rows * kTerms, 0.0);
        b.assign((size_t)rows, 0.0);
    } catch (const std::bad_alloc&) {
        return abi_fail(LB_ENOMEM, "lbml_level_fit: host working matrix could not be allocated");
    }
    double row[kTerms];
    double trace = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        basis_row(m, x + (long long)i * kFeatures, row);
        for (int c = 0; c < kTerms; ++c) {
            M[(size_t)c * rows + i] = row[c];
            trace += row[c] * row[c];
        }
        b[i] = y[i];
    }
    const double ridge = std::sqrt(kRidge * trace / kTerms);
    for (int c = 0; c < kTerms; ++c) M[(size_t)c * rows + n + c] = ridge;
    if (!householder_solve(M, b, rows, kTerms, m.coef)) return abi_fail(LB_EINVAL, "lbml_level_fit: singular system");
    for (int c = 0; c < kTerms; ++c)
        if (!std::isfinite(m.coef[c])) return abi_fail(LB_EINVAL, "lbml_level_fit: non-finite coefficients");
    *model = m;
    return LB_OK;
}

lb_status lbml_level_eval(const lbml_level_model* model, const double* x, int32_t n, double* y)
{
    if (!model || (n > 0 && (!x || !y))) return abi_fail(LB_EINVAL, "NULL argument");
    if (n < 0 || n > (1 << 30)) return abi_fail(LB_EINVAL, "lbml_level_eval: need 0 <= n <= 2^30");
    double row[kTerms];
    for (int32_t i = 0; i < n; ++i) {
        const double* xi = x + (long long)i * kFeatures;
        if (!row_ok(xi)) return abi_fail(LB_EINVAL, "features must be finite with R > 0");
        basis_row(*model, xi, row);
        double s = 0.0;
        for (int c = 0; c < kTerms; ++c) s += model->coef[c] * row[c];
        y[i] = s;
    }
    return LB_OK;
}

}  // extern "C"
