// Host-side discretisation data (see basis.hpp).  Roots are found by bracketing sign changes on a
// fine grid and bisecting to machine precision, which needs no linear-algebra library.
#include "basis.hpp"

#include <algorithm>
#include <cmath>
#include <functional>

namespace sg {

void legendre(int n, double x, double* p, double* dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid off the end points
    if (std::fabs(1.0 - x * x) > 1e-300) *dp = n * (p0 - x * p1) / (1.0 - x * x);
    else *dp = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
}

// All roots of f in the open interval (a, b), assuming they are simple and separated by more than
// (b - a) / 20000.
static std::vector<double> roots_in(const std::function<double(double)>& f, double a, double b) {
    const int N = 20000;
    std::vector<double> out;
    double xl = a, fl = f(a + 1e-15);
    for (int i = 1; i <= N; ++i) {
        double xr = a + (b - a) * i / N;
        if (i == N) xr = b - 1e-15;
        double fr = f(xr);
        if (fl == 0.0) {
            out.push_back(xl);
        } else if (fl * fr < 0.0) {
            double lo = xl, hi = xr, flo = fl;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = f(mid);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            out.push_back(0.5 * (lo + hi));
        }
        xl = xr;
        fl = fr;
    }
    return out;
}

std::vector<double> gauss_points(int n, std::vector<double>* weights) {
    auto f = [n](double x) { double p, dp; legendre(n, x, &p, &dp); return p; };
    std::vector<double> r = roots_in(f, -1.0, 1.0);
    std::vector<double> x(n), w(n);
    for (int i = 0; i < n; ++i) {
        double p, dp;
        legendre(n, r[i], &p, &dp);
        x[i] = 0.5 * (r[i] + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - r[i] * r[i]) * dp * dp);
    }
    if (weights) *weights = w;
    return x;
}

std::vector<double> gll_points(int k) {
    std::vector<double> x;
    x.push_back(0.0);
    if (k >= 2) {
        auto f = [k](double t) { double p, dp; legendre(k, t, &p, &dp); return dp; };
        for (double r : roots_in(f, -1.0, 1.0)) x.push_back(0.5 * (r + 1.0));
    }
    x.push_back(1.0);
    return x;
}

std::vector<double> right_radau_points(int r) {
    // roots of P_{r+1}(s) - P_r(s) on [-1, 1]; s = 1 is always one of them
    auto f = [r](double s) {
        double a, da, b, db;
        legendre(r + 1, s, &a, &da);
        legendre(r, s, &b, &db);
        return a - b;
    };
    std::vector<double> x;
    for (double s : roots_in(f, -1.0, 1.0)) x.push_back(0.5 * (s + 1.0));
    x.push_back(1.0);
    return x;
}

double lagrange_value(const std::vector<double>& nodes, int a, double x) {
    double v = 1.0;
    for (size_t j = 0; j < nodes.size(); ++j)
        if ((int)j != a) v *= (x - nodes[j]) / (nodes[a] - nodes[j]);
    return v;
}

double lagrange_deriv(const std::vector<double>& nodes, int a, double x) {
    double s = 0.0;
    for (size_t k = 0; k < nodes.size(); ++k) {
        if ((int)k == a) continue;
        double t = 1.0 / (nodes[a] - nodes[k]);
        for (size_t j = 0; j < nodes.size(); ++j)
            if ((int)j != a && j != k) t *= (x - nodes[j]) / (nodes[a] - nodes[j]);
        s += t;
    }
    return s;
}

bool time_matrices(int r, double tau, std::vector<double>* At, std::vector<double>* Bt_diag) {
    const int n = r + 1;
    std::vector<double> nodes = right_radau_points(r);
    if ((int)nodes.size() != n) return false;
    std::vector<double> qw;
    std::vector<double> qx = gauss_points(r + 2, &qw);
    At->assign(n * n, 0.0);
    Bt_diag->assign(n, 0.0);
    double bmax = 0.0, boff = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0.0, b = 0.0;
            for (size_t q = 0; q < qx.size(); ++q) {
                a += qw[q] * lagrange_deriv(nodes, j, qx[q]) * lagrange_value(nodes, i, qx[q]);
                b += qw[q] * lagrange_value(nodes, j, qx[q]) * lagrange_value(nodes, i, qx[q]);
            }
            a += lagrange_value(nodes, j, 0.0) * lagrange_value(nodes, i, 0.0);
            (*At)[i * n + j] = a;
            if (i == j) { (*Bt_diag)[i] = tau * b; bmax = std::max(bmax, std::fabs(b)); }
            else boff = std::max(boff, std::fabs(b));
        }
    return boff <= 1e-12 * bmax;
}

std::vector<std::vector<int>> total_degree_set(int M, int p) {
    std::vector<std::vector<int>> out;
    std::vector<int> cur(M, 0);
    std::function<void(int, int)> rec = [&](int k, int remaining) {
        if (k == M - 1) {
            cur[k] = remaining;
            out.push_back(cur);
            return;
        }
        for (int a = remaining; a >= 0; --a) {
            cur[k] = a;
            rec(k + 1, remaining - a);
        }
    };
    for (int deg = 0; deg <= p; ++deg) rec(0, deg);
    return out;
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

double hermite_triple_1d(int a, int b, int c) {
    int tot = a + b + c;
    if (tot % 2) return 0.0;
    int s = tot / 2;
    if (s < a || s < b || s < c) return 0.0;
    return std::sqrt(factorial(a) * factorial(b) * factorial(c)) /
           (factorial(s - a) * factorial(s - b) * factorial(s - c));
}

// He_n(x) / sqrt(n!) by the three-term recurrence He_{n+1} = x He_n - n He_{n-1}.
double hermite_normalized(int n, double x) {
    double hm = 1.0, h = x;
    if (n == 0) return 1.0;
    double fact = 1.0;
    for (int k = 1; k < n; ++k) {
        const double hn = x * h - k * hm;
        hm = h;
        h = hn;
    }
    for (int k = 2; k <= n; ++k) fact *= k;
    return h / std::sqrt(fact);
}

namespace {
bool check_modes(int M, int n_mu, const int* mu, Coupling* out, std::string* err) {
    out->affine = true;
    out->mu0 = -1;
    for (int k = 0; k < n_mu; ++k) {
        int deg = 0;
        for (int m = 0; m < M; ++m) {
            if (mu[k * M + m] < 0) { *err = "negative entry in coef_mu"; return false; }
            deg += mu[k * M + m];
        }
        if (deg == 0 && out->mu0 < 0) out->mu0 = k;
        if (deg > 1) out->affine = false;
        // a repeated multi-index would be summed by the coupling lists but not by the register-resident
        // affine path, which keeps one coefficient row per e_m: reject it
        for (int j = 0; j < k; ++j) {
            bool same = true;
            for (int m = 0; m < M && same; ++m) same = mu[j * M + m] == mu[k * M + m];
            if (same) { *err = deg == 0 ? "coef_mu lists mu = 0 twice" : "coef_mu lists a multi-index twice"; return false; }
        }
    }
    if (out->mu0 < 0) { *err = "coef_mu must contain mu = 0"; return false; }
    return true;
}
}  // namespace

bool build_sample_coupling(int M, int n_samples, const double* xi, int n_mu, const int* mu, Coupling* out,
                           std::string* err) {
    out->n_xi = n_samples;
    out->n_mu = n_mu;
    out->ptr.assign(1, 0);
    out->beta.clear();
    out->w.clear();
    if (!check_modes(M, n_mu, mu, out, err)) return false;
    for (int s = 0; s < n_samples; ++s)
        for (int k = 0; k < n_mu; ++k) {
            double v = 1.0;
            for (int m = 0; m < M; ++m) v *= hermite_normalized(mu[k * M + m], xi[(size_t)s * M + m]);
            out->beta.push_back(s);
            out->w.push_back(v);
            out->ptr.push_back((int)out->beta.size());
        }
    return true;
}

bool build_batch_coupling(int M, int n_members, const int* degrees, const double* scale, int n_mu, const int* mu,
                          Coupling* out, std::vector<int>* offsets, std::string* err) {
    out->n_mu = n_mu;
    out->ptr.assign(1, 0);
    out->beta.clear();
    out->w.clear();
    if (!check_modes(M, n_mu, mu, out, err)) return false;
    offsets->assign(1, 0);
    for (int j = 0; j < n_members; ++j) {
        if (degrees[j] < 0) { *err = "negative member degree"; return false; }
        if (scale[(size_t)j * n_mu + out->mu0] != 1.0) { *err = "member scale of mu = 0 must be 1"; return false; }
        const auto idx = total_degree_set(M, degrees[j]);
        const int off = offsets->back();
        for (size_t a = 0; a < idx.size(); ++a)
            for (int k = 0; k < n_mu; ++k) {
                const double sc = scale[(size_t)j * n_mu + k];
                for (size_t b = 0; b < idx.size(); ++b) {
                    double v = sc;
                    for (int m = 0; m < M && v != 0.0; ++m) v *= hermite_triple_1d(mu[k * M + m], idx[a][m], idx[b][m]);
                    if (v != 0.0) {
                        out->beta.push_back(off + (int)b);
                        out->w.push_back(v);
                    }
                }
                out->ptr.push_back((int)out->beta.size());
            }
        offsets->push_back(off + (int)idx.size());
    }
    out->n_xi = offsets->back();
    return true;
}

bool build_coupling(int M, int p, int n_mu, const int* mu, Coupling* out, std::string* err) {
    auto idx = total_degree_set(M, p);
    const int n_xi = (int)idx.size();
    out->n_xi = n_xi;
    out->n_mu = n_mu;
    out->ptr.assign(1, 0);
    out->beta.clear();
    out->w.clear();
    if (!check_modes(M, n_mu, mu, out, err)) return false;
    for (int a = 0; a < n_xi; ++a)
        for (int k = 0; k < n_mu; ++k) {
            for (int b = 0; b < n_xi; ++b) {
                double v = 1.0;
                for (int m = 0; m < M && v != 0.0; ++m) v *= hermite_triple_1d(mu[k * M + m], idx[a][m], idx[b][m]);
                if (v != 0.0) {
                    out->beta.push_back(b);
                    out->w.push_back(v);
                }
            }
            out->ptr.push_back((int)out->beta.size());
        }
    return true;
}

}  // namespace sg
