// Host construction of the Gauss rules used by the kernels.
//
// Nodes are the zeros of the orthonormal polynomials, located by scanning for
// sign changes, refined by bisection and a Newton step; weights are the
// Christoffel numbers 1 / sum_{j<n} p_j(x_i)^2 of the orthonormal family.
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "bmd_internal.hpp"

namespace bmd {
namespace {

// Orthonormal Hermite polynomials for the weight exp(-x^2):
// p_0 = pi^(-1/4), p_{j+1} = sqrt(2/(j+1)) x p_j - sqrt(j/(j+1)) p_{j-1}.
void hermite_values(int n, double x, double* p) {
    p[0] = std::pow(M_PI, -0.25);
    if (n >= 1) p[1] = std::sqrt(2.0) * x * p[0];
    for (int j = 1; j < n; ++j)
        p[j + 1] = std::sqrt(2.0 / (j + 1)) * x * p[j] - std::sqrt(static_cast<double>(j) / (j + 1)) * p[j - 1];
}

// Orthonormal Legendre polynomials on [-1, 1]: sqrt((2j+1)/2) P_j with
// (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}.
void legendre_values(int n, double x, double* p) {
    std::vector<double> P(n + 2);
    P[0] = 1.0;
    if (n >= 1) P[1] = x;
    for (int j = 1; j < n; ++j) P[j + 1] = ((2.0 * j + 1.0) * x * P[j] - j * P[j - 1]) / (j + 1.0);
    for (int j = 0; j <= n; ++j) p[j] = std::sqrt((2.0 * j + 1.0) / 2.0) * P[j];
}

template <typename F>
void zeros_and_weights(int n, double lo, double hi, double step, F values, double* x, double* w) {
    std::vector<double> p(n + 2);
    auto pn = [&](double t) {
        values(n, t, p.data());
        return p[n];
    };
    int found = 0;
    double a = lo, fa = pn(a);
    while (a < hi && found < n) {
        double b = a + step, fb = pn(b);
        if ((fa < 0.0) != (fb < 0.0)) {
            double l = a, r = b, fl = fa;
            for (int it = 0; it < 200 && r - l > 0.0; ++it) {
                double mid = 0.5 * (l + r);
                if (mid <= l || mid >= r) break;
                double fm = pn(mid);
                if ((fm < 0.0) == (fl < 0.0)) { l = mid; fl = fm; } else { r = mid; }
            }
            x[found++] = 0.5 * (l + r);
        }
        a = b;
        fa = fb;
    }
    for (int i = 0; i < found; ++i) {
        values(n, x[i], p.data());
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += p[j] * p[j];
        w[i] = 1.0 / s;
    }
}

}  // namespace

namespace {

// Rules are pure functions of n: build each once per process.
std::mutex g_rule_mutex;
std::map<int, std::vector<double>> g_hermite, g_legendre;

template <typename Build>
void cached(std::map<int, std::vector<double>>& cache, int n, double* x, double* w, Build build) {
    std::lock_guard<std::mutex> lock(g_rule_mutex);
    auto it = cache.find(n);
    if (it == cache.end()) {
        std::vector<double> r(2 * n);
        build(n, r.data(), r.data() + n);
        it = cache.emplace(n, std::move(r)).first;
    }
    for (int i = 0; i < n; ++i) {
        x[i] = it->second[i];
        w[i] = it->second[n + i];
    }
}

}  // namespace

void gauss_hermite_prob(int n, double* x, double* w) {
    cached(g_hermite, n, x, w, [](int n_, double* xx, double* ww) {
        // zeros of the degree-n Hermite polynomial lie in |x| < sqrt(2n+1) and are
        // at least ~pi/sqrt(2n+1) apart: scan in quarters of that spacing
        const double R = std::sqrt(2.0 * n_ + 1.0) + 1.0;
        zeros_and_weights(n_, -R, R, 0.25 * M_PI / std::sqrt(2.0 * n_ + 1.0), hermite_values, xx, ww);
        // weight exp(-x^2)  ->  standard normal density: z = sqrt(2) x, w / sqrt(pi)
        for (int i = 0; i < n_; ++i) {
            xx[i] *= std::sqrt(2.0);
            ww[i] /= std::sqrt(M_PI);
        }
    });
}

void gauss_legendre(int n, double* x, double* w) {
    cached(g_legendre, n, x, w, [](int n_, double* xx, double* ww) {
        // the outermost zeros are about (2.4/(n+1/2))^2/2 from +-1; scan finer than that
        zeros_and_weights(n_, -1.0, 1.0, 0.25 / ((n_ + 1.0) * (n_ + 1.0)), legendre_values, xx, ww);
    });
}

void gl_table(double* out) {
    static const int sizes[8] = {4, 6, 8, 10, 12, 16, 20, 24};
    int off = 0;
    for (int s = 0; s < 8; ++s) {
        int n = sizes[s];
        gauss_legendre(n, out + off, out + off + n);
        off += 2 * n;
    }
}

}  // namespace bmd
