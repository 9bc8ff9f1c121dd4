// Host-side planning for the TDSLDA kernels (plain C++, no HIP): radix
// factorisation of the lattice sides, Stockham twiddle tables, full W_n
// tables, and the bfloat16 split of the 1D spectral kinetic matrix used by
// the matrix-core form.  Kept free of device code so that it can also be
// compiled by an ordinary C++ compiler for host-side tests.
#pragma once

#include <cmath>
#include <cstring>
#include <vector>

namespace lise {

#ifndef LISE_PLAN_HAVE_DEVICE_TYPES
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};
constexpr int kMaxStages = 7;
struct AxisPlan {
    int n;
    int nst;
    int radix[kMaxStages];
    int p[kMaxStages];
    int tw[kMaxStages];
};
#endif

namespace plan {

// Radices of a mixed-radix Stockham transform of length n: as many 8s as
// possible (two 4s for 2^4, a 4 or a 2 for the remainder), then 3s and 5s.

inline bool factorize(int n, int* radix, int* nst) {
    if (n < 1) return false;
    int e2 = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++e2; }
    std::vector<int> r;
    // powers of two: prefer radix 8, then a 4-4 or 4 or 2 remainder
    int rem = e2;
    while (rem >= 3 && !(rem == 4)) { r.push_back(8); rem -= 3; }
    if (rem == 4) { r.push_back(4); r.push_back(4); rem = 0; }
    if (rem == 2) { r.push_back(4); rem = 0; }
    if (rem == 1) { r.push_back(2); rem = 0; }
    while (m % 3 == 0) { r.push_back(3); m /= 3; }
    while (m % 5 == 0) { r.push_back(5); m /= 5; }
    if (m != 1) return false;
    if ((int)r.size() > kMaxStages) return false;
    *nst = (int)r.size();
    for (size_t i = 0; i < r.size(); ++i) radix[i] = r[i];
    return true;
}

// Build the plan of one axis and append its twiddles (double precision,
// angles reduced exactly: 2 pi (q k mod (pR)) / (pR)).
inline bool make_plan(int n, AxisPlan* pl, std::vector<cpx<double>>* tw) {
    std::memset(pl, 0, sizeof(*pl));
    pl->n = n;
    if (!factorize(n, pl->radix, &pl->nst)) return false;
    int p = 1;
    for (int s = 0; s < pl->nst; ++s) {
        const int R = pl->radix[s];
        pl->p[s] = p;
        pl->tw[s] = (int)tw->size();
        const long long pr = (long long)p * R;
        for (int k = 0; k < p; ++k)
            for (int q = 1; q < R; ++q) {
                const long long num = ((long long)q * k) % pr;
                const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)num / (long double)pr;
                cpx<double> w;
                w.re = (double)cosl(ang);
                w.im = (double)sinl(ang);
                tw->push_back(w);
            }
        p *= R;
    }
    return true;
}


// W_n^j = exp(-2 pi i j / n), j < n, appended to tw; returns the offset.
inline int full_table(int n, std::vector<cpx<double>>* tw) {
    const int off = (int)tw->size();
    for (int j = 0; j < n; ++j) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
        cpx<double> w;
        w.re = (double)cosl(ang);
        w.im = (double)sinl(ang);
        tw->push_back(w);
    }
    return off;
}

inline bool mfma_side(int n) { return n == 16 || n == 32 || n == 48 || n == 64; }

// float -> bfloat16 bits, round to nearest even (host side)
inline unsigned short host_bf16(float f) {
    unsigned u;
    std::memcpy(&u, &f, 4);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
inline float host_bf16_value(unsigned short h) {
    unsigned u = ((unsigned)h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// bf16 hi/lo parts of the 1D spectral kinetic matrix
// T[n][m] = (1/N) sum_k (k^2/2) cos(k (n - m) a), k in FFT order.
inline std::vector<unsigned short> kinetic_matrix_bf16(int n, double a) {
    std::vector<unsigned short> out(2 * (size_t)n * n);
    const long double pi = 3.14159265358979323846264338327950288L;
    for (int r = 0; r < n; ++r)
        for (int m = 0; m < n; ++m) {
            long double acc = 0.0L;
            for (int j = 0; j < n; ++j) {
                const int js = (2 * j < n) ? j : j - n;
                const long double k = 2.0L * pi * js / ((long double)n * a);
                acc += 0.5L * k * k * cosl(k * (long double)(r - m) * a);
            }
            const float v = (float)(acc / n);
            const unsigned short hi = host_bf16(v);
            const unsigned short lo = host_bf16(v - host_bf16_value(hi));
            out[(size_t)r * n + m] = hi;
            out[(size_t)n * n + (size_t)r * n + m] = lo;
        }
    return out;
}

// K of the cubic-lattice coupling renormalisation (Eq. geff_3D):
// (12/pi) * integral over [0, pi/4] of ln(1 + 1/cos^2 t) dt, composite Simpson
// rule on 4096 panels in long double (smooth integrand: error far below 1e-16).
inline long double lattice_K() {
    const long double pi = 3.141592653589793238462643383279502884L;
    const int n = 4096;
    const long double h = (pi / 4.0L) / n;
    auto f = [](long double t) {
        const long double c = cosl(t);
        return log1pl(1.0L / (c * c));
    };
    long double s = f(0.0L) + f(pi / 4.0L);
    for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0L : 2.0L) * f(i * h);
    return 12.0L / pi * (s * h / 3.0L);
}

// Coupling g used in Delta = -g kappa: the bare g, or with regularisation the
// g_eff of 1/g_eff = 1/g - m* K / (4 pi^2 hbar^2) * (pi / a) with m* = hbar = 1.
// Returns false when 1/g_eff is zero (divergent coupling) or g is zero.
inline bool effective_coupling(double g, double a, int regularize, double* out) {
    if (!regularize) {
        *out = g;
        return true;
    }
    if (g == 0.0 || !(a > 0.0)) return false;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double inv = 1.0L / g - lattice_K() / (4.0L * pi * a);
    if (inv == 0.0L) return false;
    *out = (double)(1.0L / inv);
    return true;
}

}  // namespace plan
}  // namespace lise
