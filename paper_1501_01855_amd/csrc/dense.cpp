// Small dense complex linear algebra on the host (see dense.h).
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace ovl {
namespace dense {

void eigh(int n, const std::vector<zc> &Ain, std::vector<double> &evals, std::vector<zc> &Vout)
{
    std::vector<zc> A = Ain;
    std::vector<zc> V(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    // symmetrise (inputs assembled from inexact vectors are Hermitian only to rounding)
    for (int i = 0; i < n; ++i) {
        A[i * n + i] = zc(A[i * n + i].real(), 0.0);
        for (int j = i + 1; j < n; ++j) {
            const zc h = 0.5 * (A[i * n + j] + std::conj(A[j * n + i]));
            A[i * n + j] = h;
            A[j * n + i] = std::conj(h);
        }
    }
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::abs(A[i]));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(A[p * n + q]);
        if (std::sqrt(off) <= 1e-17 * (scale > 0 ? scale : 1.0) * n) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const zc apq = A[p * n + q];
                const double r = std::abs(apq);
                if (r <= 1e-300) continue;
                const zc ph = apq / r;   // e^{i phi}
                const double app = A[p * n + p].real(), aqq = A[q * n + q].real();
                // real rotation for [[app, r], [r, aqq]] after the phase change
                const double theta = (aqq - app) / (2.0 * r);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // G = diag(1, conj(ph)) [[c, s], [-s, c]] acting on columns p, q:
                //   G_pp = c, G_pq = s, G_qp = -s conj(ph), G_qq = c conj(ph)
                const zc gpp = c, gpq = s, gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
                // A <- A G (columns)
                for (int k = 0; k < n; ++k) {
                    const zc akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = akp * gpp + akq * gqp;
                    A[k * n + q] = akp * gpq + akq * gqq;
                }
                // A <- G^H A (rows)
                for (int k = 0; k < n; ++k) {
                    const zc apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = std::conj(gpp) * apk + std::conj(gqp) * aqk;
                    A[q * n + k] = std::conj(gpq) * apk + std::conj(gqq) * aqk;
                }
                A[p * n + q] = 0.0;
                A[q * n + p] = 0.0;
                A[p * n + p] = zc(A[p * n + p].real(), 0.0);
                A[q * n + q] = zc(A[q * n + q].real(), 0.0);
                for (int k = 0; k < n; ++k) {
                    const zc vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = vkp * gpp + vkq * gqp;
                    V[k * n + q] = vkp * gpq + vkq * gqq;
                }
            }
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return A[a * n + a].real() < A[b * n + b].real(); });
    evals.resize(n);
    Vout.assign(n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        evals[k] = A[order[k] * n + order[k]].real();
        for (int i = 0; i < n; ++i) Vout[i * n + k] = V[i * n + order[k]];
    }
}

bool cholesky_upper(int n, const std::vector<zc> &A, std::vector<zc> &R)
{
    R.assign(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(R[k * n + j]);
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double rjj = std::sqrt(d);
        R[j * n + j] = rjj;
        for (int i = j + 1; i < n; ++i) {
            zc s = A[j * n + i];
            for (int k = 0; k < j; ++k) s -= std::conj(R[k * n + j]) * R[k * n + i];
            R[j * n + i] = s / rjj;
        }
    }
    return true;
}

std::vector<zc> inv_upper(int n, const std::vector<zc> &R)
{
    std::vector<zc> X(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        X[j * n + j] = 1.0 / R[j * n + j];
        for (int i = j - 1; i >= 0; --i) {
            zc s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += R[i * n + k] * X[k * n + j];
            X[i * n + j] = -s / R[i * n + i];
        }
    }
    return X;
}

std::vector<zc> matmul(int m, int k, int n, const std::vector<zc> &A, const std::vector<zc> &B)
{
    std::vector<zc> C(m * n, 0.0);
    for (int i = 0; i < m; ++i)
        for (int l = 0; l < k; ++l) {
            const zc a = A[i * k + l];
            for (int j = 0; j < n; ++j) C[i * n + j] += a * B[l * n + j];
        }
    return C;
}

std::vector<zc> matmul_ah(int k, int m, int n, const std::vector<zc> &A, const std::vector<zc> &B)
{
    std::vector<zc> C(m * n, 0.0);
    for (int l = 0; l < k; ++l)
        for (int i = 0; i < m; ++i) {
            const zc a = std::conj(A[l * m + i]);
            for (int j = 0; j < n; ++j) C[i * n + j] += a * B[l * n + j];
        }
    return C;
}

}  // namespace dense
}  // namespace ovl
