// Device code of the TDSLDA step for gfx950 (MI355X).
//
// The kinetic operator T = F^{-1} (|k|^2/2) F of Sec. "Discretization" has a
// symbol that is a sum over axes, k^2 = kx^2 + ky^2 + kz^2, so
//     T f = F_xy^{-1} [(kx^2 + ky^2)/2 F_xy f] + F_z^{-1} [kz^2/2 F_z f],
// exactly (the transforms along the other axes cancel).  The step is built
// from two kernels per Hamiltonian application:
//   * kz_kernel: the z-axis term on xz-tiles (coalesced rows of x), written
//     to a scratch buffer G;
//   * kp_kernel: per xy-plane, the 2D FFT term in LDS, plus G, plus the local
//     mixing of Eq. (tdslda) with V = U + U_ext and Delta, followed by the
//     mode's epilogue (Taylor term, ABM phase 1 or ABM phase 2) and the
//     float64 partial sums of the densities of Eq. (rho_t, nu_t).
// When a whole lattice cube fits in LDS, kp_kernel also does the z axis and
// G is not used ("fused" mode).
//
// FFTs are self-sorting mixed-radix Stockham transforms (radices 2,3,4,5,8)
// ping-ponging between two LDS buffers, one radix-R butterfly per thread per
// stage.  Forward uses exp(-2 pi i/n), inverse exp(+2 pi i/n) unnormalised;
// the 1/n factors are folded into the k^2 multiply.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lise {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) {
    cpx<T> c;
    c.re = r;
    c.im = i;
    return c;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T>
__device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return mk(a.re, -a.im); }
// Loads and stores of the state arrays can carry the nontemporal hint (the
// `nt` bit of global_load/global_store).  Where one instruction of a wave
// covers whole 128-byte lines the hint raised bandwidth (a plain 1-read +
// 1-write stream on gfx950: 5.4 -> 6.2 TB/s); where it covers parts of lines
// (a 20-point plane row spread over 4 lanes) the next instruction fetched the
// rest of the line again and the plane kernel ran up to 2.3x slower.  So each
// kernel passes NT from its own access pattern.  Fields, twiddles and density
// partials, which are reused, never take the hint.  LISE_STREAM_HINT=0 turns
// the hint off everywhere.
#ifndef LISE_STREAM_HINT
#define LISE_STREAM_HINT 1
#endif
template <typename T>
struct vec2_of;
template <>
struct vec2_of<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct vec2_of<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
// The state arrays, fields and partial sums live in device global memory.
// Pointers that a kernel reads from a descriptor table in memory (the batched
// kernels) are generic to the compiler, which then emits flat instructions;
// those also count against the LDS wait counter, so every wait for LDS data
// would wait for outstanding memory traffic as well.  The accessors below
// state the global address space explicitly (a no-op on the address).
template <typename P>
__device__ __forceinline__ const __attribute__((address_space(1))) P* gptr(const P* p) {
    return (const __attribute__((address_space(1))) P*)p;
}
template <typename P>
__device__ __forceinline__ __attribute__((address_space(1))) P* gptr(P* p) {
    return (__attribute__((address_space(1))) P*)p;
}
template <typename P>
__device__ __forceinline__ P ldg(const P* p) {
    return *gptr(p);
}
template <typename P>
__device__ __forceinline__ void stg(P* p, P v) {
    *gptr(p) = v;
}

template <typename T, bool NT>
__device__ __forceinline__ cpx<T> ld_hint(const cpx<T>* p) {
    typedef typename vec2_of<T>::type V;
    const __attribute__((address_space(1))) V* q = reinterpret_cast<const __attribute__((address_space(1))) V*>(gptr(p));
    V v;
    if constexpr (NT && LISE_STREAM_HINT) v = __builtin_nontemporal_load(q);
    else v = *q;
    return mk(T(v.x), T(v.y));
}
template <typename T, bool NT>
__device__ __forceinline__ void st_hint(cpx<T>* p, cpx<T> v) {
    typedef typename vec2_of<T>::type V;
    __attribute__((address_space(1))) V* q = reinterpret_cast<__attribute__((address_space(1))) V*>(gptr(p));
    V w;
    w.x = v.re;
    w.y = v.im;
    if constexpr (NT && LISE_STREAM_HINT) __builtin_nontemporal_store(w, q);
    else *q = w;
}

// multiply by i * sigma, sigma = +1 or -1
template <typename T, int SIG>
__device__ __forceinline__ cpx<T> mul_isig(cpx<T> a) {
    return SIG > 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
}

// ---------------------------------------------------------------------------
// FFT plan of one axis: radices of the stages and, per stage, the product p
// of the earlier radices and the offset of its twiddles in the table.  The
// twiddles of stage s are w(k, q) = exp(-2 pi i q k / (p R)), k < p,
// 1 <= q < R, stored at tw[off + k (R-1) + q - 1].
constexpr int kMaxStages = 7;
struct AxisPlan {
    int n;
    int nst;
    int radix[kMaxStages];
    int p[kMaxStages];
    int tw[kMaxStages];
};

// Lines of a batch of 1D transforms inside an LDS buffer.  Line L starts at
// (L / lsub) * ls_out + (L % lsub) * ls_in; its elements are es apart.
// lines_fast = 1 assigns consecutive threads to consecutive lines (strided
// axes), 0 to consecutive butterflies of one line (the contiguous axis).
struct LineMap {
    int nlines, lsub, ls_in, ls_out, es, lines_fast;
};

// Small DFTs of size R on registers: b_s = sum_q a_q exp(SIG 2 pi i q s / R).
template <typename T, int R, int SIG>
struct SmallDft;

template <typename T, int SIG>
struct SmallDft<T, 2, SIG> {
    static __device__ __forceinline__ void run(cpx<T>* a) {
        cpx<T> t = a[0] - a[1];
        a[0] = a[0] + a[1];
        a[1] = t;
    }
};

template <typename T, int SIG>
struct SmallDft<T, 3, SIG> {
    static __device__ __forceinline__ void run(cpx<T>* a) {
        const T c = T(-0.5);
        const T s = T(0.86602540378443864676372317075294);  // sqrt(3)/2
        cpx<T> t1 = a[1] + a[2];
        cpx<T> t2 = a[0] + c * t1;
        cpx<T> t3 = mul_isig<T, SIG>(s * (a[1] - a[2]));
        a[0] = a[0] + t1;
        a[1] = t2 + t3;
        a[2] = t2 - t3;
    }
};

template <typename T, int SIG>
struct SmallDft<T, 4, SIG> {
    static __device__ __forceinline__ void run(cpx<T>* a) {
        cpx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
        cpx<T> s13 = a[1] + a[3], d13 = mul_isig<T, SIG>(a[1] - a[3]);
        a[0] = s02 + s13;
        a[2] = s02 - s13;
        a[1] = d02 + d13;
        a[3] = d02 - d13;
    }
};

template <typename T, int SIG>
struct SmallDft<T, 5, SIG> {
    static __device__ __forceinline__ void run(cpx<T>* a) {
        // cos(2pi/5) = (sqrt5-1)/4, cos(4pi/5) = -(sqrt5+1)/4,
        // sin(2pi/5) = sqrt(10+2sqrt5)/4, sin(4pi/5) = sqrt(10-2sqrt5)/4
        const T c1 = T(0.30901699437494742410229341718282);
        const T c2 = T(-0.80901699437494742410229341718282);
        const T s1 = T(0.95105651629515357211643933337938);
        const T s2 = T(0.58778525229247312916870595463907);
        cpx<T> p14 = a[1] + a[4], m14 = a[1] - a[4];
        cpx<T> p23 = a[2] + a[3], m23 = a[2] - a[3];
        cpx<T> r1 = a[0] + c1 * p14 + c2 * p23;
        cpx<T> r2 = a[0] + c2 * p14 + c1 * p23;
        cpx<T> i1 = mul_isig<T, SIG>(s1 * m14 + s2 * m23);
        cpx<T> i2 = mul_isig<T, SIG>(s2 * m14 - s1 * m23);
        a[0] = a[0] + p14 + p23;
        a[1] = r1 + i1;
        a[4] = r1 - i1;
        a[2] = r2 + i2;
        a[3] = r2 - i2;
    }
};

template <typename T, int SIG>
struct SmallDft<T, 8, SIG> {
    static __device__ __forceinline__ void run(cpx<T>* a) {
        // even/odd split into two DFT-4s, then the radix-2 combination with
        // w8^k = exp(SIG 2 pi i k / 8).
        cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
        cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
        SmallDft<T, 4, SIG>::run(e);
        SmallDft<T, 4, SIG>::run(o);
        const T h = T(0.70710678118654752440084436210485);  // 1/sqrt2
        cpx<T> o1 = h * (o[1] + mul_isig<T, SIG>(o[1]));     // w8^1 = (1 + i SIG)/sqrt2
        cpx<T> o2 = mul_isig<T, SIG>(o[2]);                  // w8^2 = i SIG
        cpx<T> o3 = h * (mul_isig<T, SIG>(o[3]) - o[3]);     // w8^3 = (-1 + i SIG)/sqrt2
        a[0] = e[0] + o[0];
        a[4] = e[0] - o[0];
        a[1] = e[1] + o1;
        a[5] = e[1] - o1;
        a[2] = e[2] + o2;
        a[6] = e[2] - o2;
        a[3] = e[3] + o3;
        a[7] = e[3] - o3;
    }
};

// One Stockham stage of radix R over all lines of a LineMap:
//   inputs  x[i + q m], m = n / R, twiddled by w(k, q), k = i mod p,
//   outputs y[(i / p) p R + k + s p] = DFT_R of the twiddled inputs.
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                          int n, int p, const cpx<T>* __restrict__ tw,
                                          const LineMap lm, int tid, int nth) {
    const int m = n / R;
    const int total = lm.nlines * m;
    for (int t = tid; t < total; t += nth) {
        int L, i;
        if (lm.lines_fast) {
            L = t % lm.nlines;
            i = t / lm.nlines;
        } else {
            i = t % m;
            L = t / m;
        }
        const int base = (L / lm.lsub) * lm.ls_out + (L % lm.lsub) * lm.ls_in;
        const int k = i % p;
        cpx<T> a[R];
#pragma unroll
        for (int q = 0; q < R; ++q) a[q] = src[base + (i + q * m) * lm.es];
        if (p > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                cpx<T> w = tw[k * (R - 1) + (q - 1)];
                if (INV) w.im = -w.im;
                a[q] = a[q] * w;
            }
        }
        SmallDft<T, R, INV ? 1 : -1>::run(a);
        const int j = (i / p) * p * R + k;
#pragma unroll
        for (int s = 0; s < R; ++s) dst[base + (j + s * p) * lm.es] = a[s];
    }
}

// Full 1D transform along one axis; returns the buffer holding the result.
template <typename T, bool INV>
__device__ cpx<T>* fft_axis(cpx<T>* src, cpx<T>* dst, const AxisPlan& pl,
                            const cpx<T>* __restrict__ tw, const LineMap lm, int tid, int nth) {
    for (int s = 0; s < pl.nst; ++s) {
        const int R = pl.radix[s];
        const int p = pl.p[s];
        const cpx<T>* t = tw + pl.tw[s];
        switch (R) {
            case 2: fft_stage<T, 2, INV>(src, dst, pl.n, p, t, lm, tid, nth); break;
            case 3: fft_stage<T, 3, INV>(src, dst, pl.n, p, t, lm, tid, nth); break;
            case 4: fft_stage<T, 4, INV>(src, dst, pl.n, p, t, lm, tid, nth); break;
            case 5: fft_stage<T, 5, INV>(src, dst, pl.n, p, t, lm, tid, nth); break;
            default: fft_stage<T, 8, INV>(src, dst, pl.n, p, t, lm, tid, nth); break;
        }
        __syncthreads();
        cpx<T>* x = src;
        src = dst;
        dst = x;
    }
    return src;
}

__device__ __forceinline__ int signed_mode(int i, int n) { return (2 * i < n) ? i : i - n; }

// ---------------------------------------------------------------------------
// Kernel arguments

enum KpMode { KP_APPLY = 0, KP_ABM1 = 1, KP_ABM2 = 2, KP_KINETIC = 3, KP_ETA = 4, KP_ETAXY = 5 };

template <typename T>
struct KPArgs {
    int nx, ny, nz, C, npair;
    int zb;          // xy-planes per workgroup (nz when fused)
    int jg;          // qpwfs walked by one workgroup
    int kcount;      // qpwfs in this launch
    long long j0;    // first qpwf (global index) of this launch
    int fused;       // 1: z axis in LDS too, G unused
    AxisPlan px, py, pz;
    const cpx<T>* tw;
    T cx, cy, cz;    // k_a^2 / 2 / (transform size) = c_a * m_a^2
    const double* V;
    const double* D;  // complex, interleaved
    double mu_a[2], mu_b[2];
    int sgn[2], ca[2], cb[2];
    double w;         // density weight of a pair
    const cpx<T>* in;
    const cpx<T>* G;  // indexed by the qpwf index within the launch
    // KP_APPLY
    cpx<T>* out;
    cpx<T>* acc;
    cpx<T>* deriv;
    int acc_from_in;
    double coef_re, coef_im;
    // KP_ABM1: in = y_n, a1 = y_{n-1} -> Y, a2 = y'_{n-1}, a3 = y'_{n-2},
    //          a4 = y'_{n-3} -> m, a5 = p_n - c_n (read only), a6 -> y'_n
    // KP_ABM2: in = m, a1 = Y -> y_{n+1}, a5 = p_n - c_n -> p_{n+1} - c_{n+1}
    cpx<T>* a1;
    cpx<T>* a2;
    cpx<T>* a3;
    cpx<T>* a4;
    cpx<T>* a5;
    cpx<T>* a6;
    double dt;
    double* dpart;    // [slot][3][N] float64 density partial sums
    int dens_src;     // 0: none, 1: the produced vector (m, y_{n+1}, acc or out)
    int accumulate;   // 0: store partials, 1: add to them
    double* epart;    // KP_KINETIC, KP_ETA: one float64 per workgroup
    // per global qpwf: the instantaneous quasiparticle energy eta_j of
    // Eq. (sp_en), subtracted from H in every mode that applies H (null: off)
    const double* eta;
    // KP_KINETIC on the register-FFT plane kernel, optional: per workgroup the
    // Parseval sums over the v components of (m_x, m_y) |F_xy v|^2 (signed
    // plane-wave indices, Nyquist index 0), for the total current
    double* ppart;
    // ABM phases of the plane kernel with the z-term computed in the kernel:
    // the kinetic operator along z as a dense real symmetric nz x nz matrix
    // (row-major; null where the z-term comes from the z-axis kernel)
    const T* tzm;
};

// ---------------------------------------------------------------------------
// Epilogue of one point shared by the plane kernels: local mixing of
// Eq. (tdslda) with V = U + U_ext and Delta, the mode's update, and the
// float64 density accumulation of the vector the mode produces.
//
// The ABM phases use an exact re-association of Eq. (p), (m), (c), (y) that
// lets phase 2 read only m, Y, d_n = p_n - c_n (and the z-term G):
//   phase 1: s = (y_n + y_{n-1})/2,
//            c~ = s + dt/48 (51 y'_n + 3 y'_{n-1} + y'_{n-2})   (c without m'),
//            Y = p - c~ = dt/48 (68 y'_n - 102 y'_{n-1} + 68 y'_{n-2} - 17 y'_{n-3}),
//            m = c~ + Y - 161/170 d_n   (= p - 161/170 d_n);
//   phase 2: with k = 17 dt / 48 and m' = -i H m,
//            d_{n+1} = p - c = Y - k m',
//            y_{n+1} = c + 9/170 (p - c) = p - 161/170 d_{n+1}
//                    = m + 161/170 (d_n - d_{n+1}).
// Y is formed from the derivatives directly and y_{n+1} as m plus a small
// correction, so no quantity of the size of y is cancelled and no float32
// weights have to add up to one.  Phase 1 stores y'_n over y'_{n-4}, m over
// y'_{n-3} and Y over y_{n-1} (d_n stays); phase 2 stores y_{n+1} over Y and
// d_{n+1} over d_n.

//
// KP_ETA accumulates Re(f^* H f) of the pair (the summand of eta_j); with
// phase removal on (a.eta set) the other modes apply H - eta_j (ej) instead
// of H.

template <typename T, int MODE, bool HASG, bool NT>
__device__ __forceinline__ void point_epilogue(const KPArgs<T>& a, int pr, cpx<T> Ta, cpx<T> Tb, cpx<T> fa, cpx<T> fb,
                                               long long ea, long long eb, long long rpt, long long ga, long long gb,
                                               cpx<T> coef, T cdt, T ej,
                                               double& dn, double& dkr, double& dki, double& ekin) {
    // Every load of the point is issued before any arithmetic, so that one
    // round trip to memory serves the z-term, the fields and the ABM history.
    cpx<T> Ga = mk(T(0), T(0)), Gb = mk(T(0), T(0));
    if constexpr (HASG) {
        Ga = ld_hint<T, NT>(a.G + ga);
        Gb = ld_hint<T, NT>(a.G + gb);
    }
    if constexpr (MODE == KP_KINETIC) {
        Tb = Tb + Gb;
        ekin += a.w * (double(fb.re) * double(Tb.re) + double(fb.im) * double(Tb.im));
        return;
    }
    const double Vd = ldg(a.V + rpt);
    const double Dre = ldg(a.D + 2 * rpt), Dim = ldg(a.D + 2 * rpt + 1);
    cpx<T> h1a, h1b, h2a, h2b, h3a, h3b, h4a, h4b, h5a, h5b;
    if constexpr (MODE == KP_ABM1) {
        h1a = ld_hint<T, NT>(a.a1 + ea); h1b = ld_hint<T, NT>(a.a1 + eb);
        h2a = ld_hint<T, NT>(a.a2 + ea); h2b = ld_hint<T, NT>(a.a2 + eb);
        h3a = ld_hint<T, NT>(a.a3 + ea); h3b = ld_hint<T, NT>(a.a3 + eb);
        h4a = ld_hint<T, NT>(a.a4 + ea); h4b = ld_hint<T, NT>(a.a4 + eb);
        h5a = ld_hint<T, NT>(a.a5 + ea); h5b = ld_hint<T, NT>(a.a5 + eb);
    } else if constexpr (MODE == KP_ABM2) {
        h1a = ld_hint<T, NT>(a.a1 + ea); h1b = ld_hint<T, NT>(a.a1 + eb);
        h5a = ld_hint<T, NT>(a.a5 + ea); h5b = ld_hint<T, NT>(a.a5 + eb);
    }
    Ta = Ta + Ga;
    Tb = Tb + Gb;
    const T sg = T(a.sgn[pr]);
    const T Vr = T(Vd);
    const cpx<T> Dl = mk(sg * T(Dre), sg * T(Dim));
    const T mua = T(a.mu_a[pr]), mub = T(a.mu_b[pr]);
    // H u = (h - mu_a) u + s Delta v ;  H v = s Delta^* u - (h - mu_b) v
    cpx<T> Ha = Ta + (Vr - mua) * fa + Dl * fb;
    cpx<T> Hb = conjg(Dl) * fa - (Tb + (Vr - mub) * fb);
    if constexpr (MODE == KP_ETA) {
        ekin += double(fa.re) * double(Ha.re) + double(fa.im) * double(Ha.im) + double(fb.re) * double(Hb.re) +
                double(fb.im) * double(Hb.im);
        return;
    }
    if (a.eta) {
        Ha = Ha - ej * fa;
        Hb = Hb - ej * fb;
    }
    cpx<T> va, vb;   // vector whose densities are accumulated
    if constexpr (MODE == KP_APPLY) {
        const cpx<T> oa = coef * Ha, ob = coef * Hb;
        if (a.deriv) {
            a.deriv[ea] = mk(Ha.im, -Ha.re);
            a.deriv[eb] = mk(Hb.im, -Hb.re);
        }
        va = oa;
        vb = ob;
        if (a.acc) {
            const cpx<T> pa = a.acc_from_in ? fa : a.acc[ea];
            const cpx<T> pb = a.acc_from_in ? fb : a.acc[eb];
            va = pa + oa;
            vb = pb + ob;
            a.acc[ea] = va;
            a.acc[eb] = vb;
        }
        if (a.out) {
            a.out[ea] = oa;
            a.out[eb] = ob;
        }
    } else if constexpr (MODE == KP_ABM1) {
        const cpx<T> da = mk(Ha.im, -Ha.re), db = mk(Hb.im, -Hb.re);   // y'_n = -i H y_n
        const cpx<T> sa = T(0.5) * (fa + h1a), sb = T(0.5) * (fb + h1b);
        const cpx<T> Ya = cdt * (T(68) * da - T(102) * h2a + T(68) * h3a - T(17) * h4a);
        const cpx<T> Yb = cdt * (T(68) * db - T(102) * h2b + T(68) * h3b - T(17) * h4b);
        const cpx<T> ca = sa + cdt * (T(51) * da + T(3) * h2a + h3a);
        const cpx<T> cb = sb + cdt * (T(51) * db + T(3) * h2b + h3b);
        va = (ca + Ya) - T(161.0 / 170.0) * h5a;   // m = p - 161/170 d_n
        vb = (cb + Yb) - T(161.0 / 170.0) * h5b;
        st_hint<T, NT>(a.a6 + ea, da);
        st_hint<T, NT>(a.a6 + eb, db);
        st_hint<T, NT>(a.a4 + ea, va);
        st_hint<T, NT>(a.a4 + eb, vb);
        st_hint<T, NT>(a.a1 + ea, Ya);
        st_hint<T, NT>(a.a1 + eb, Yb);
    } else {   // KP_ABM2: in = m, a1 = Y -> y_{n+1}, a5 = d_n -> d_{n+1}
        const cpx<T> ma = mk(Ha.im, -Ha.re), mb = mk(Hb.im, -Hb.re);   // m' = -i H m
        const T k = T(17) * cdt;
        const cpx<T> ra = h1a - k * ma, rb = h1b - k * mb;             // d_{n+1}
        va = fa + T(161.0 / 170.0) * (h5a - ra);                        // y_{n+1}
        vb = fb + T(161.0 / 170.0) * (h5b - rb);
        st_hint<T, NT>(a.a1 + ea, va);
        st_hint<T, NT>(a.a1 + eb, vb);
        st_hint<T, NT>(a.a5 + ea, ra);
        st_hint<T, NT>(a.a5 + eb, rb);
    }
    if (a.dens_src) {
        const double br = double(vb.re), bi = double(vb.im);
        const double ar = double(va.re), ai = double(va.im);
        dn += a.w * (br * br + bi * bi);
        const double hs = 0.5 * a.w * double(a.sgn[pr]);
        dkr += hs * (br * ar + bi * ai);   // Re(conj(b) a)
        dki += hs * (br * ai - bi * ar);   // Im(conj(b) a)
    }
}

template <typename T, int MODE, int PPT>
__global__ void __launch_bounds__(256) kp_kernel(const KPArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* bufA = reinterpret_cast<cpx<T>*>(smem_raw);
    const int nth = blockDim.x;
    const int tid = threadIdx.x;
    const int nxy = a.nx * a.ny;
    const int P = a.zb * nxy;                  // points of one component in this WG
    cpx<T>* bufB = bufA + 2 * P;
    const int z0 = blockIdx.x * a.zb;
    const long long N = (long long)nxy * a.nz;
    const int jbeg = blockIdx.y * a.jg;
    const int jend = min(a.kcount, jbeg + a.jg);

    double dn[PPT], dkr[PPT], dki[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) dn[i] = dkr[i] = dki[i] = 0.0;
    double ekin = 0.0;

    const T cdt = T(a.dt / 48.0);
    const cpx<T> coef = mk(T(a.coef_re), T(a.coef_im));

    // line maps of the three axes over the two LDS planes-stacks
    const LineMap lmx = {2 * a.zb * a.ny, 2 * a.zb * a.ny, a.nx, 0, 1, 0};
    const LineMap lmy = {2 * a.zb * a.nx, a.nx, 1, nxy, a.nx, 1};
    const LineMap lmz = {2 * nxy, nxy, 1, a.nz * nxy, nxy, 1};

    for (int jl = jbeg; jl < jend; ++jl) {
        const long long jgl = a.j0 + jl;
        const T ej = a.eta ? T(a.eta[jgl]) : T(0);
        for (int pr = 0; pr < a.npair; ++pr) {
            const long long offa = ((jgl * a.C + a.ca[pr]) * a.nz + z0) * (long long)nxy;
            const long long offb = ((jgl * a.C + a.cb[pr]) * a.nz + z0) * (long long)nxy;
            cpx<T> fa[PPT], fb[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int q = tid + i * nth;
                if (q < P) {
                    fa[i] = a.in[offa + q];
                    fb[i] = a.in[offb + q];
                    bufA[q] = fa[i];
                    bufA[P + q] = fb[i];
                }
            }
            __syncthreads();
            // forward transforms (x, y, and z when fused)
            cpx<T>* r = fft_axis<T, false>(bufA, bufB, a.px, a.tw, lmx, tid, nth);
            cpx<T>* o = (r == bufA) ? bufB : bufA;
            r = fft_axis<T, false>(r, o, a.py, a.tw, lmy, tid, nth);
            o = (r == bufA) ? bufB : bufA;
            if (a.fused) {
                r = fft_axis<T, false>(r, o, a.pz, a.tw, lmz, tid, nth);
                o = (r == bufA) ? bufB : bufA;
            }
            // multiply by k^2/2 divided by the transform size
            for (int e = tid; e < 2 * P; e += nth) {
                const int q = e % P;
                const int x = q % a.nx;
                const int y = (q / a.nx) % a.ny;
                const int mx = signed_mode(x, a.nx), my = signed_mode(y, a.ny);
                T f = a.cx * T(mx * mx) + a.cy * T(my * my);
                if (a.fused) {
                    const int mz = signed_mode(q / nxy, a.nz);
                    f += a.cz * T(mz * mz);
                }
                r[e] = f * r[e];
            }
            __syncthreads();
            if (a.fused) {
                r = fft_axis<T, true>(r, o, a.pz, a.tw, lmz, tid, nth);
                o = (r == bufA) ? bufB : bufA;
            }
            r = fft_axis<T, true>(r, o, a.py, a.tw, lmy, tid, nth);
            o = (r == bufA) ? bufB : bufA;
            r = fft_axis<T, true>(r, o, a.px, a.tw, lmx, tid, nth);

            const long long lofa = (((long long)jl * a.C + a.ca[pr]) * a.nz + z0) * nxy;
            const long long lofb = (((long long)jl * a.C + a.cb[pr]) * a.nz + z0) * nxy;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int q = tid + i * nth;
                if (q >= P) continue;
                const cpx<T> Ta = r[q], Tb = r[P + q];
                if (a.fused)
                    point_epilogue<T, MODE, false, false>(a, pr, Ta, Tb, fa[i], fb[i], offa + q, offb + q,
                                                   (long long)z0 * nxy + q, 0, 0, coef, cdt, ej, dn[i], dkr[i],
                                                   dki[i], ekin);
                else
                    point_epilogue<T, MODE, true, false>(a, pr, Ta, Tb, fa[i], fb[i], offa + q, offb + q,
                                                  (long long)z0 * nxy + q, lofa + q, lofb + q, coef, cdt, ej, dn[i],
                                                  dkr[i], dki[i], ekin);
            }
            __syncthreads();
        }
    }
    if (MODE == KP_KINETIC || MODE == KP_ETA) {
        // workgroup reduction of the kinetic (or eta) partial sum
        double* red = reinterpret_cast<double*>(smem_raw);
        red[tid] = ekin;
        __syncthreads();
        for (int s = nth / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) a.epart[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
        return;
    }
    if (a.dens_src) {
        double* base = a.dpart + (long long)blockIdx.y * 3 * N + (long long)z0 * nxy;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int q = tid + i * nth;
            if (q >= P) continue;
            if (a.accumulate) {
                base[q] += dn[i];
                base[N + q] += dkr[i];
                base[2 * N + q] += dki[i];
            } else {
                base[q] = dn[i];
                base[N + q] = dkr[i];
                base[2 * N + q] = dki[i];
            }
        }
    }
}

// eta_j = a^3 sum over the nblk plane blocks of qpwf j (fixed order), one
// thread per qpwf; part[j * nblk + b] comes from the KP_ETA launch (jg = 1).
__global__ void __launch_bounds__(256) eta_reduce_kernel(const double* __restrict__ part, int nblk, int k,
                                                         double a3, double* __restrict__ eta) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(long long)j * nblk + b];
    eta[j] = a3 * s;
}

// eta_j = a^3 (sum of the nblk plane partials + sum of the nez z-kinetic
// partials of qpwf j), one workgroup per qpwf, fixed-order sums (strided per
// thread, then a tree): the cheap eta pass of the register-FFT kernels.
__global__ void __launch_bounds__(256) eta_reduce2_kernel(const double* __restrict__ part, int nblk,
                                                          const double* __restrict__ ezpart, long long nez,
                                                          double a3, double* __restrict__ eta) {
    __shared__ double red[256];
    const int j = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (long long i = t; i < nez; i += 256) s += ezpart[(long long)j * nez + i];
    for (int b = t; b < nblk; b += 256) s += part[(long long)j * nblk + b];
    red[t] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) eta[j] = a3 * red[0];
}

// ---------------------------------------------------------------------------
// z-axis kinetic term on xz-tiles: G = F_z^{-1} [kz^2/2 F_z f] / nz

template <typename T>
struct KZArgs {
    int nx, ny, nz, C, yb;
    long long j0;
    AxisPlan pz;
    const cpx<T>* tw;
    T cz;
    const cpx<T>* in;
    cpx<T>* G;
};

template <typename T>
__global__ void __launch_bounds__(256) kz_kernel(const KZArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* bufA = reinterpret_cast<cpx<T>*>(smem_raw);
    const int row = a.yb * a.nx;             // points of one z-row of the tile
    const int P = a.nz * row;
    cpx<T>* bufB = bufA + P;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int y0 = blockIdx.x * a.yb;
    const long long jc = blockIdx.y;         // local qpwf * C + component
    const long long nxy = (long long)a.nx * a.ny;
    const long long gbase = ((a.j0 * a.C + jc) * a.nz) * nxy + (long long)y0 * a.nx;
    const long long lbase = (jc * a.nz) * nxy + (long long)y0 * a.nx;
    for (int e = tid; e < P; e += nth) {
        const int z = e / row, rr = e % row;
        bufA[e] = a.in[gbase + z * nxy + rr];
    }
    __syncthreads();
    const LineMap lm = {row, row, 1, 0, row, 1};
    cpx<T>* r = fft_axis<T, false>(bufA, bufB, a.pz, a.tw, lm, tid, nth);
    cpx<T>* o = (r == bufA) ? bufB : bufA;
    for (int e = tid; e < P; e += nth) {
        const int mz = signed_mode(e / row, a.nz);
        r[e] = (a.cz * T(mz * mz)) * r[e];
    }
    __syncthreads();
    r = fft_axis<T, true>(r, o, a.pz, a.tw, lm, tid, nth);
    for (int e = tid; e < P; e += nth) {
        const int z = e / row, rr = e % row;
        a.G[lbase + z * nxy + rr] = r[e];
    }
}

// ---------------------------------------------------------------------------
// Boost of Eq. (kick): u -> e^{i chi} u, v -> e^{-i chi} v.  phase[r] holds
// e^{i chi(r)} in float64; components below nu are u, the rest v.

template <typename T>
__global__ void __launch_bounds__(256) kick_kernel(cpx<T>* __restrict__ state, const double* __restrict__ phase,
                                                   long long N, int C, int nu, long long total) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e % N;
        const int c = (int)((e / N) % C);
        const double pr = phase[2 * r], pi = (c < nu ? 1.0 : -1.0) * phase[2 * r + 1];
        const cpx<T> v = state[e];
        const double vr = double(v.re), vi = double(v.im);
        state[e] = mk(T(vr * pr - vi * pi), T(vr * pi + vi * pr));
    }
}

__global__ void __launch_bounds__(256) phase_kernel(const double* __restrict__ chi, long long N,
                                                    double* __restrict__ phase) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    double s, c;
    sincos(chi[r], &s, &c);
    phase[2 * r] = c;
    phase[2 * r + 1] = s;
}

// ---------------------------------------------------------------------------
// Current density of Eq. (j): j = -w sum_k Im(v_k^* grad v_k) with spectral
// first derivatives F^{-1}[i k F v] (N/2 mode of an even axis zeroed).  Each
// workgroup walks jg qpwfs and writes float64 partial sums per slot into
// jpart[slot][axis][N]; a fixed-order sum over the slots follows.

template <typename T>
struct CurArgs {
    int nx, ny, nz, C, yb, jg;
    long long M;
    int nv, v0;            // v components: v0 .. v0 + nv - 1
    double w;
    AxisPlan px, py, pz;
    const cpx<T>* tw;
    T fx, fy, fz;          // 2 pi / (L_a n_a): derivative factor per signed mode
    const cpx<T>* in;
    double* jpart;
};

template <typename T>
__device__ __forceinline__ T deriv_factor(int m, int n, T f) {
    return (2 * m == n) ? T(0) : f * T(signed_mode(m, n));
}

// x and y components from one xy-plane in LDS (PPT points per thread)
template <typename T, int PPT>
__global__ void __launch_bounds__(256) current_xy_kernel(const CurArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    const int nxy = a.nx * a.ny;
    cpx<T>* bufA = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* bufB = bufA + nxy;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int z = blockIdx.x;
    const long long N = (long long)nxy * a.nz;
    const long long j0 = (long long)blockIdx.y * a.jg;
    const long long j1 = min(a.M, j0 + a.jg);
    const LineMap lmx = {a.ny, a.ny, a.nx, 0, 1, 0};
    const LineMap lmy = {a.nx, a.nx, 1, 0, a.nx, 1};
    double jx[PPT], jy[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) jx[i] = jy[i] = 0.0;
    for (long long j = j0; j < j1; ++j) {
        for (int cv = 0; cv < a.nv; ++cv) {
            const long long off = ((j * a.C + a.v0 + cv) * a.nz + z) * (long long)nxy;
            cpx<T> f[PPT];
            for (int ax = 0; ax < 2; ++ax) {
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    const int q = tid + i * nth;
                    if (q < nxy) {
                        if (ax == 0) f[i] = a.in[off + q];
                        bufA[q] = f[i];
                    }
                }
                __syncthreads();
                const LineMap& lm = ax == 0 ? lmx : lmy;
                const AxisPlan& pl = ax == 0 ? a.px : a.py;
                cpx<T>* r = fft_axis<T, false>(bufA, bufB, pl, a.tw, lm, tid, nth);
                cpx<T>* o = (r == bufA) ? bufB : bufA;
                for (int e = tid; e < nxy; e += nth) {
                    const int m = ax == 0 ? e % a.nx : e / a.nx;
                    const T k = ax == 0 ? deriv_factor<T>(m, a.nx, a.fx) : deriv_factor<T>(m, a.ny, a.fy);
                    r[e] = mk(-k * r[e].im, k * r[e].re);   // i k F v
                }
                __syncthreads();
                r = fft_axis<T, true>(r, o, pl, a.tw, lm, tid, nth);
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    const int q = tid + i * nth;
                    if (q < nxy) {
                        const cpx<T> d = r[q];
                        // Im(conj(f) d)
                        const double im = double(f[i].re) * double(d.im) - double(f[i].im) * double(d.re);
                        if (ax == 0) jx[i] -= a.w * im;
                        else jy[i] -= a.w * im;
                    }
                }
                __syncthreads();
            }
        }
    }
    double* base = a.jpart + (long long)blockIdx.y * 3 * N + (long long)z * nxy;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int q = tid + i * nth;
        if (q < nxy) {
            base[q] = jx[i];
            base[N + q] = jy[i];
        }
    }
}

// z component on tiles of yb rows by nz planes (layout [z][row])
template <typename T, int PPT>
__global__ void __launch_bounds__(256) current_z_kernel(const CurArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    const int row = a.yb * a.nx;
    const int P = a.nz * row;
    cpx<T>* bufA = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* bufB = bufA + P;
    const int tid = threadIdx.x, nth = blockDim.x;
    const long long nxy = (long long)a.nx * a.ny;
    const long long N = nxy * a.nz;
    const int y0 = blockIdx.x * a.yb;
    const long long j0 = (long long)blockIdx.y * a.jg;
    const long long j1 = min(a.M, j0 + a.jg);
    const LineMap lm = {row, row, 1, 0, row, 1};
    double jz[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) jz[i] = 0.0;
    for (long long j = j0; j < j1; ++j) {
        for (int cv = 0; cv < a.nv; ++cv) {
            const long long off = ((j * a.C + a.v0 + cv) * a.nz) * nxy + (long long)y0 * a.nx;
            cpx<T> f[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int e = tid + i * nth;
                if (e < P) {
                    const int zz = e / row, rr = e % row;
                    f[i] = a.in[off + zz * nxy + rr];
                    bufA[e] = f[i];
                }
            }
            __syncthreads();
            cpx<T>* r = fft_axis<T, false>(bufA, bufB, a.pz, a.tw, lm, tid, nth);
            cpx<T>* o = (r == bufA) ? bufB : bufA;
            for (int e = tid; e < P; e += nth) {
                const T k = deriv_factor<T>(e / row, a.nz, a.fz);
                r[e] = mk(-k * r[e].im, k * r[e].re);
            }
            __syncthreads();
            r = fft_axis<T, true>(r, o, a.pz, a.tw, lm, tid, nth);
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int e = tid + i * nth;
                if (e < P) {
                    const cpx<T> d = r[e];
                    jz[i] -= a.w * (double(f[i].re) * double(d.im) - double(f[i].im) * double(d.re));
                }
            }
            __syncthreads();
        }
    }
    double* base = a.jpart + (long long)blockIdx.y * 3 * N + 2 * N + (long long)y0 * a.nx;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int e = tid + i * nth;
        if (e < P) {
            const int zz = e / row, rr = e % row;
            base[zz * nxy + rr] = jz[i];
        }
    }
}

// out[e] = sum over slots of part[slot][e], e < n3 (fixed order)
__global__ void __launch_bounds__(256) slot_sum_kernel(const double* __restrict__ part, int nslots, long long n3,
                                                       double* __restrict__ out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n3) return;
    double s = 0.0;
    for (int k = 0; k < nslots; ++k) s += part[(long long)k * n3 + e];
    out[e] = s;
}

// ---------------------------------------------------------------------------
// Densities straight from a state (no Hamiltonian), one thread per point,
// each thread walking jg qpwfs; partial sums per slot.

template <typename T>
__global__ void __launch_bounds__(256) dens_partial_kernel(const cpx<T>* __restrict__ in, int C, long long N,
                                                           long long M, int jg, double w,
                                                           double* __restrict__ dpart) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const long long j0 = (long long)blockIdx.y * jg;
    const long long j1 = min(M, j0 + jg);
    double n = 0.0, kr = 0.0, ki = 0.0;
    for (long long j = j0; j < j1; ++j) {
        for (int pr = 0; pr < C / 2; ++pr) {
            const int ca = (C == 2) ? 0 : pr;
            const int cb = (C == 2) ? 1 : 3 - pr;
            const double s = (pr == 0) ? 1.0 : -1.0;
            const cpx<T> u = in[(j * C + ca) * N + r];
            const cpx<T> v = in[(j * C + cb) * N + r];
            const double br = double(v.re), bi = double(v.im), ar = double(u.re), ai = double(u.im);
            n += w * (br * br + bi * bi);
            kr += 0.5 * w * s * (br * ar + bi * ai);
            ki += 0.5 * w * s * (br * ai - bi * ar);
        }
    }
    double* base = dpart + (long long)blockIdx.y * 3 * N;
    base[r] = n;
    base[N + r] = kr;
    base[2 * N + r] = ki;
}

// One system's part of a batched density pass (dens_partial_kernel on a
// table): the vector v (M qpwfs of C components of N points), slots of jgd
// qpwfs, weight w.
template <typename T>
struct DensDesc {
    const cpx<T>* v;
    long long N, M;
    int C, jgd;
    double w;
    double* dpart;
    long long bx;   // workgroups along the points: ceil(N / 256)
};

// Every system of a group in one launch: blks[s] is the first workgroup of
// system s (blks[nsys] = gridDim.x); within a system, workgroup b takes the
// points of block b % bx of slot b / bx.
template <typename T>
__global__ void __launch_bounds__(256) dens_batch_kernel(const DensDesc<T>* __restrict__ tab,
                                                         const long long* __restrict__ blks, int nsys) {
    int lo = 0, hi = nsys;
    const long long b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blks[mid] <= b) lo = mid;
        else hi = mid;
    }
    const DensDesc<T>& d = tab[lo];
    const long long lb = b - blks[lo];
    const long long slot = lb / d.bx;
    const long long r = (lb - slot * d.bx) * blockDim.x + threadIdx.x;
    if (r >= d.N) return;
    const long long j0 = slot * d.jgd;
    const long long j1 = min(d.M, j0 + d.jgd);
    double n = 0.0, kr = 0.0, ki = 0.0;
    for (long long j = j0; j < j1; ++j) {
        for (int pr = 0; pr < d.C / 2; ++pr) {
            const int ca = (d.C == 2) ? 0 : pr;
            const int cb = (d.C == 2) ? 1 : 3 - pr;
            const double s = (pr == 0) ? 1.0 : -1.0;
            const cpx<T> u = ld_hint<T, false>(d.v + (j * d.C + ca) * d.N + r);
            const cpx<T> v = ld_hint<T, false>(d.v + (j * d.C + cb) * d.N + r);
            const double br = double(v.re), bi = double(v.im), ar = double(u.re), ai = double(u.im);
            n += d.w * (br * br + bi * bi);
            kr += 0.5 * d.w * s * (br * ar + bi * ai);
            ki += 0.5 * d.w * s * (br * ai - bi * ar);
        }
    }
    double* base = d.dpart + slot * 3 * d.N;
    stg(base + r, n);
    stg(base + d.N + r, kr);
    stg(base + 2 * d.N + r, ki);
}

// ---------------------------------------------------------------------------
// Sum of the density partials (fixed order: deterministic), optional average
// with another density set (series-expansion corrector), and the local
// fields U + U_ext and Delta.

struct FieldParams {
    int nx, ny, nz;
    double a;
    double beta, g;
    int frozen;
    double U0, D0re, D0im;
    double extA, extw, r0x, r0y, r0z, t_on;
};

__device__ __forceinline__ double ext_ramp(const FieldParams& f, double t) {
    if (f.t_on > 0.0 && t < f.t_on) {
        const double s = sin(M_PI * fmax(t, 0.0) / (2.0 * f.t_on));
        return s * s;
    }
    return 1.0;
}

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

__device__ __forceinline__ double ext_potential(const FieldParams& f, long long r, double ramp) {
    if (f.extA == 0.0) return 0.0;
    const int x = int(r % f.nx);
    const int y = int((r / f.nx) % f.ny);
    const int z = int(r / ((long long)f.nx * f.ny));
    const double dx = min_image(x * f.a - f.r0x, f.nx * f.a);
    const double dy = min_image(y * f.a - f.r0y, f.ny * f.a);
    const double dz = min_image(z * f.a - f.r0z, f.nz * f.a);
    const double d2 = dz * dz + dy * dy + dx * dx;
    return f.extA * ramp * exp(-d2 / (2.0 * f.extw * f.extw));
}

// The time comes from device memory (tdev[0] + toff) so that a captured
// graph of whole steps stays valid on every replay.
// A workgroup takes kFieldPts consecutive points; its kFieldGroups waves sum
// the slots g, g + kFieldGroups, ... of those points (coalesced rows of the
// slot array), and the first wave adds the group sums in order g = 0, 1, ...
// (a fixed order: bitwise reproducible), then forms the fields.
constexpr int kFieldPts = 64;
constexpr int kFieldGroups = 16;
// blk: the workgroup's block of kFieldPts points within the system
__device__ __forceinline__ void fields_body(
    const double* __restrict__ dpart, int nslots, long long N, const double* __restrict__ avg_with,
    double* __restrict__ dens_out, double* __restrict__ V, double* __restrict__ D, const FieldParams& fp,
    const double* __restrict__ tdev, double toff, int* __restrict__ bad, long long blk) {
    __shared__ double part[3][kFieldGroups][kFieldPts];
    const int pt = threadIdx.x % kFieldPts, g = threadIdx.x / kFieldPts;
    const long long r = blk * kFieldPts + pt;
    if (nslots > 0) {
        double n = 0.0, kr = 0.0, ki = 0.0;
        if (r < N) {
            for (int s = g; s < nslots; s += kFieldGroups) {
                const double* b = dpart + (long long)s * 3 * N;
                n += b[r];
                kr += b[N + r];
                ki += b[2 * N + r];
            }
        }
        part[0][g][pt] = n;
        part[1][g][pt] = kr;
        part[2][g][pt] = ki;
        __syncthreads();
    }
    if (g != 0 || r >= N) return;
    const double t = tdev[0] + toff;
    double n, kr, ki;
    if (nslots > 0) {
        n = kr = ki = 0.0;
        for (int h = 0; h < kFieldGroups; ++h) {
            n += part[0][h][pt];
            kr += part[1][h][pt];
            ki += part[2][h][pt];
        }
    } else {
        n = dens_out[r];
        kr = dens_out[N + r];
        ki = dens_out[2 * N + r];
    }
    if (avg_with) {
        n = 0.5 * (n + avg_with[r]);
        kr = 0.5 * (kr + avg_with[N + r]);
        ki = 0.5 * (ki + avg_with[2 * N + r]);
    }
    if (!(isfinite(n) && isfinite(kr) && isfinite(ki))) atomicOr(bad, 1);
    dens_out[r] = n;
    dens_out[N + r] = kr;
    dens_out[2 * N + r] = ki;
    double U;
    double dre, dim;
    if (fp.frozen) {
        U = fp.U0;
        dre = fp.D0re;
        dim = fp.D0im;
    } else {
        const double c = cbrt(n);
        U = fp.beta * c * c;
        dre = -fp.g * kr;
        dim = -fp.g * ki;
    }
    V[r] = U + ext_potential(fp, r, ext_ramp(fp, t));
    D[2 * r] = dre;
    D[2 * r + 1] = dim;
}

__global__ void __launch_bounds__(kFieldPts * kFieldGroups) fields_kernel(
    const double* __restrict__ dpart, int nslots, long long N, const double* __restrict__ avg_with,
    double* __restrict__ dens_out, double* __restrict__ V, double* __restrict__ D, FieldParams fp,
    const double* __restrict__ tdev, double toff, int* __restrict__ bad) {
    fields_body(dpart, nslots, N, avg_with, dens_out, V, D, fp, tdev, toff, bad, (long long)blockIdx.x);
}

// One system's part of a batched density reduction + fields launch.
struct FieldsDesc {
    const double* dpart;
    int nslots;
    long long N;
    double* dens;
    double* V;
    double* D;
    FieldParams fp;
    const double* tdev;
    int* bad;
};

// Every system of a batch in one launch: blks[s] is the first workgroup of
// system s (blks[nsys] = gridDim.x).  No averaging (ABM phases only).
__global__ void __launch_bounds__(kFieldPts * kFieldGroups) fields_batch_kernel(
    const FieldsDesc* __restrict__ tab, const long long* __restrict__ blks, int nsys, double toff) {
    int lo = 0, hi = nsys;
    const long long b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blks[mid] <= b) lo = mid;
        else hi = mid;
    }
    const FieldsDesc& d = tab[lo];
    fields_body(d.dpart, d.nslots, d.N, nullptr, d.dens, d.V, d.D, d.fp, d.tdev, toff, d.bad, b - blks[lo]);
}

// Observables of the fields: per-block partial sums of
// [n, n x, n y, n z, 3/5 beta n^{5/3}, g |kappa|^2, U_ext n, |Delta| n].
constexpr int kNObs = 8;
__global__ void __launch_bounds__(256) obs_fields_kernel(const double* __restrict__ dens,
                                                         const double* __restrict__ D, long long N,
                                                         FieldParams fp, double t,
                                                         double* __restrict__ part) {
    __shared__ double red[kNObs][256];
    const int tid = threadIdx.x;
    double acc[kNObs] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double ramp = ext_ramp(fp, t);
    for (long long r = (long long)blockIdx.x * blockDim.x + tid; r < N; r += (long long)gridDim.x * blockDim.x) {
        const double n = dens[r], kr = dens[N + r], ki = dens[2 * N + r];
        const int x = int(r % fp.nx);
        const int y = int((r / fp.nx) % fp.ny);
        const int z = int(r / ((long long)fp.nx * fp.ny));
        const double c = cbrt(n);
        acc[0] += n;
        acc[1] += n * (x * fp.a);
        acc[2] += n * (y * fp.a);
        acc[3] += n * (z * fp.a);
        acc[4] += 0.6 * fp.beta * c * c * c * c * c;
        acc[5] += fp.g * (kr * kr + ki * ki);
        acc[6] += ext_potential(fp, r, ramp) * n;
        acc[7] += sqrt(D[2 * r] * D[2 * r] + D[2 * r + 1] * D[2 * r + 1]) * n;
    }
    for (int k = 0; k < kNObs; ++k) red[k][tid] = acc[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < kNObs; ++k) red[k][tid] += red[k][tid + s];
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < kNObs; ++k) part[blockIdx.x * kNObs + k] = red[k][0];
}

// Norm of each qpwf: sum over components and points of |psi|^2 (float64).
template <typename T>
__global__ void __launch_bounds__(256) norm_kernel(const cpx<T>* __restrict__ in, long long per,
                                                   double* __restrict__ norms) {
    __shared__ double red[256];
    const long long j = blockIdx.x;
    const cpx<T>* p = in + j * per;
    double s = 0.0;
    for (long long e = threadIdx.x; e < per; e += blockDim.x) {
        const double re = double(p[e].re), im = double(p[e].im);
        s += re * re + im * im;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) norms[j] = red[0];
}

// Squared norm of one component of each qpwf, sum over points of |psi_c|^2
// (float64): workgroup b takes component c = cbeg + b % ncomp_sum of qpwf
// j = b / ncomp_sum and writes out[b] (spin-resolved particle numbers).
template <typename T>
__global__ void __launch_bounds__(256) comp_norm_kernel(const cpx<T>* __restrict__ in, int C, int cbeg, int nc,
                                                        long long N, double* __restrict__ out) {
    __shared__ double red[256];
    const long long b = blockIdx.x;
    const long long j = b / nc;
    const int c = cbeg + (int)(b % nc);
    const cpx<T>* p = in + (j * C + c) * N;
    double s = 0.0;
    for (long long e = threadIdx.x; e < N; e += blockDim.x) {
        const double re = double(p[e].re), im = double(p[e].im);
        s += re * re + im * im;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
}

// Precision conversion between the float64 interface and the state.
template <typename TO, typename TI>
__global__ void __launch_bounds__(256) convert_kernel(const cpx<TI>* __restrict__ in, cpx<TO>* __restrict__ out,
                                                      long long n) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const cpx<TI> v = in[e];
        out[e] = mk(TO(v.re), TO(v.im));
    }
}

// Advance the device-side time of a system by dt (one thread).
__global__ void tick_kernel(double* __restrict__ t, double dt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) t[0] = t[0] + dt;
}

// t_n -> t_n + dt for the device-side times of n systems
__global__ void tick_batch_kernel(double* const* __restrict__ t, int n, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t[i][0] = t[i][0] + dt;
}

__global__ void __launch_bounds__(256) zero_kernel(double* __restrict__ p, long long n) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

}  // namespace lise
