// C wrappers over the library's host planning header, for CPU-only tests.
#include <vector>
#include "lise_plan.hpp"

using namespace lise;

extern "C" int hp_plan(int n, int* nst, int* radix, int* p, int* twoff, double* tw, int cap) {
    AxisPlan pl;
    std::vector<cpx<double>> t;
    if (!plan::make_plan(n, &pl, &t)) return -1;
    *nst = pl.nst;
    for (int s = 0; s < pl.nst; ++s) {
        radix[s] = pl.radix[s];
        p[s] = pl.p[s];
        twoff[s] = pl.tw[s];
    }
    if ((int)t.size() > cap) return -2;
    for (size_t i = 0; i < t.size(); ++i) {
        tw[2 * i] = t[i].re;
        tw[2 * i + 1] = t[i].im;
    }
    return (int)t.size();
}

extern "C" int hp_full_table(int n, double* tw) {
    std::vector<cpx<double>> t;
    plan::full_table(n, &t);
    for (size_t i = 0; i < t.size(); ++i) {
        tw[2 * i] = t[i].re;
        tw[2 * i + 1] = t[i].im;
    }
    return (int)t.size();
}

extern "C" void hp_kinetic_bf16(int n, double a, unsigned short* out) {
    std::vector<unsigned short> k = plan::kinetic_matrix_bf16(n, a);
    for (size_t i = 0; i < k.size(); ++i) out[i] = k[i];
}
