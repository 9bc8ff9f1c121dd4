// Size-specialised kernels of the TDSLDA step for the lattice sides that
// occur in practice (8, 16, 20, 24, 32, 48, 64): the FFTs run in registers.
//
// z axis (kz_fast): one thread per z-column holds the whole column (N
//   values) and does forward FFT, the kz^2/2 multiply and the inverse FFT in
//   registers; consecutive lanes take consecutive x, so every load and store
//   of a wave is one contiguous run.
//
// xy planes (kp_fast): an N-point line is split over L lanes (4, 8 or 16),
//   lane s holding elements s + L q (q < P = N/L).  Forward transform:
//     A_s[k1] = DFT_P over q of x[s + L q]          (registers)
//     B_s[k1] = A_s[k1] * W_N^{s k1}                 (per-lane twiddle)
//     X[k1 + P k2] = DFT_L over s of B_s[k1]        (radix-2 exchanges across
//                                                    lanes: DPP, ds_swizzle)
//   after which lane s holds X[k1 + P bitrev(s)].  The inverse
//   runs the same steps backwards, so frequency order never has to be
//   restored.  Rows are transformed first, one LDS transpose gives columns,
//   the k^2 multiply sits between the forward and inverse column transforms,
//   and a second transpose returns rows for the inverse x transform, whose
//   output feeds the local mixing and ABM epilogue straight from registers
//   (or, where L points of a row are less than a 128-byte line, through LDS
//   in natural order: see kp_fast).
//
// ABM phases with the z-term inside the plane kernel (kp_fast_zd): the z
//   kernel's transform pair is the dense real symmetric matrix T_z, applied
//   to the z-columns of the input (read through L2) by the workgroups of
//   the planes themselves, so the step needs no z-term scratch.
//
// pz_kernel: the z part of the total current by Parseval, for observables.
#pragma once

#include "lise_device.hpp"

namespace lise {

// ---------------------------------------------------------------------------
// compile-time radix plan (same rule as the host planner)
struct RadixList {
    int cnt;
    int r[8];
};

constexpr RadixList radix_list(int N) {
    RadixList L{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    int m = N, e2 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++e2;
    }
    while (e2 >= 3 && e2 != 4) {
        L.r[L.cnt++] = 8;
        e2 -= 3;
    }
    if (e2 == 4) {
        L.r[L.cnt++] = 4;
        L.r[L.cnt++] = 4;
        e2 = 0;
    }
    if (e2 == 2) L.r[L.cnt++] = 4;
    if (e2 == 1) L.r[L.cnt++] = 2;
    while (m % 3 == 0) {
        L.r[L.cnt++] = 3;
        m /= 3;
    }
    while (m % 5 == 0) {
        L.r[L.cnt++] = 5;
        m /= 5;
    }
    return L;
}

constexpr int radix_prod(int N, int S) {
    RadixList L = radix_list(N);
    int p = 1;
    for (int i = 0; i < S; ++i) p *= L.r[i];
    return p;
}

// Register Stockham FFT of size N.  tab holds W_TN^j = exp(-2 pi i j/TN)
// with TN = N * TS, so W_N^j = tab[j * TS].
template <typename T, int N, int TS, bool INV, int S = 0>
struct RegFft {
    static __device__ __forceinline__ void run(cpx<T>* x, const cpx<T>* __restrict__ tab) {
        constexpr RadixList L = radix_list(N);
        if constexpr (S < L.cnt) {
            constexpr int R = L.r[S];
            constexpr int p = radix_prod(N, S);
            constexpr int m = N / R;
            cpx<T> y[N];
#pragma unroll
            for (int i = 0; i < m; ++i) {
                const int k = i % p;
                cpx<T> a[R];
#pragma unroll
                for (int q = 0; q < R; ++q) a[q] = x[i + q * m];
                if (k != 0) {
#pragma unroll
                    for (int q = 1; q < R; ++q) {
                        cpx<T> w = tab[((q * k * (N / (p * R))) % N) * TS];
                        if (INV) w.im = -w.im;
                        a[q] = a[q] * w;
                    }
                }
                SmallDft<T, R, INV ? 1 : -1>::run(a);
                const int j = (i / p) * p * R + k;
#pragma unroll
                for (int s = 0; s < R; ++s) y[j + s * p] = a[s];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) x[i] = y[i];
            RegFft<T, N, TS, INV, S + 1>::run(x, tab);
        }
    }
};

// ---------------------------------------------------------------------------
// Lane exchanges: partner lane s ^ D.  D = 1, 2 use DPP quad_perm
// ([1,0,3,2] and [2,3,0,1]); D = 4, 8, 16 use ds_swizzle in bit mode
// (and-mask 0x1f, xor-mask D), which stays inside groups of 32 lanes.
constexpr int kQuadXor1 = 0xB1;
constexpr int kQuadXor2 = 0x4E;

template <int D>
__device__ __forceinline__ int xchg_i(int v) {
    if constexpr (D == 1) return __builtin_amdgcn_mov_dpp(v, kQuadXor1, 0xF, 0xF, false);
    else if constexpr (D == 2) return __builtin_amdgcn_mov_dpp(v, kQuadXor2, 0xF, 0xF, false);
    else return __builtin_amdgcn_ds_swizzle(v, 0x1F | (D << 10));
}
template <int D>
__device__ __forceinline__ float xchg(float v) { return __int_as_float(xchg_i<D>(__float_as_int(v))); }
template <int D>
__device__ __forceinline__ double xchg(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = xchg_i<D>((int)(b & 0xffffffffLL));
    const int hi = xchg_i<D>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int D, typename T>
__device__ __forceinline__ cpx<T> xchg(cpx<T> v) {
    return mk(xchg<D>(v.re), xchg<D>(v.im));
}

__host__ __device__ constexpr int bitrev(int s, int L) {
    int r = 0;
    for (int b = 1; b < L; b <<= 1) r = (r << 1) | ((s & b) ? 1 : 0);
    return r;
}

// Radix-2 decimation-in-frequency stages across lanes, partner distance D
// down to 1.  tab holds W_N^j; W_{2D}^j = tab[j N / (2D)].
template <typename T, int P, int L, int D>
struct LaneDif {
    static __device__ __forceinline__ void run(cpx<T>* x, const cpx<T>* __restrict__ tab, int s) {
        if constexpr (D >= 1) {
            constexpr int N = L * P;
            const bool up = (s & D) != 0;
            cpx<T> w = mk(T(1), T(0));
            if constexpr (D > 1) w = tab[(s & (D - 1)) * (N / (2 * D))];
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                const cpx<T> p = xchg<D>(x[k1]);
                cpx<T> d = p - x[k1];
                if constexpr (D > 1) d = d * w;
                x[k1] = up ? d : x[k1] + p;
            }
            LaneDif<T, P, L, D / 2>::run(x, tab, s);
        }
    }
};

// Radix-2 decimation-in-time stages across lanes (inverse transform), partner
// distance D up to L/2; the upper element is twiddled by W_{2D}^{-j} first.
template <typename T, int P, int L, int D>
struct LaneDit {
    static __device__ __forceinline__ void run(cpx<T>* x, const cpx<T>* __restrict__ tab, int s) {
        if constexpr (D < L) {
            constexpr int N = L * P;
            const bool up = (s & D) != 0;
            cpx<T> w = mk(T(1), T(0));
            if constexpr (D > 1) w = conjg(tab[(s & (D - 1)) * (N / (2 * D))]);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                cpx<T> v = x[k1];
                if constexpr (D > 1) v = up ? v * w : v;
                const cpx<T> p = xchg<D>(v);
                x[k1] = up ? p - v : v + p;
            }
            LaneDit<T, P, L, 2 * D>::run(x, tab, s);
        }
    }
};

// Forward line transform of N = L*P points over L lanes: x[q] = element
// s + L q on entry, X[k1 + P bitrev(s)] at x[k1] on exit.
template <typename T, int P, int L>
__device__ __forceinline__ void lane_fwd(cpx<T>* x, const cpx<T>* __restrict__ tab, int s) {
    RegFft<T, P, L, false>::run(x, tab);
#pragma unroll
    for (int k1 = 1; k1 < P; ++k1) x[k1] = x[k1] * tab[s * k1];
    LaneDif<T, P, L, L / 2>::run(x, tab, s);
}

// Inverse of lane_fwd, unnormalised: N * element s + L q at x[q] on exit.
template <typename T, int P, int L>
__device__ __forceinline__ void lane_inv(cpx<T>* x, const cpx<T>* __restrict__ tab, int s) {
    LaneDit<T, P, L, 1>::run(x, tab, s);
#pragma unroll
    for (int k1 = 1; k1 < P; ++k1) x[k1] = x[k1] * conjg(tab[s * k1]);
    RegFft<T, P, L, true>::run(x, tab);
}

// lanes per line of the plane kernel: enough that a lane holds at most 2
// points of a line where the side allows, capped at 16 (more waves per SIMD:
// 32 x 32 planes measured 2.5% faster in float64, 15% in float32 than 4 points)
#ifndef LISE_PLANE_MAXP_F64
#define LISE_PLANE_MAXP_F64 2
#endif
#ifndef LISE_PLANE_MAXP_F32
#define LISE_PLANE_MAXP_F32 2
#endif

// esz: bytes of the real type (8 = float64, 4 = float32)
__host__ __device__ constexpr int plane_lanes_of(int esz, int N) {
    const int maxp = esz == 8 ? LISE_PLANE_MAXP_F64 : LISE_PLANE_MAXP_F32;
    int L = 4;
    while (N / L > maxp && L < 16 && N % (2 * L) == 0) L *= 2;
    return L;
}

// nontemporal hints in the plane kernel: one load instruction of a wave reads
// L consecutive points of each of its rows, so the hint is taken only where
// those L points and a whole row are multiples of a 128-byte line (every
// instruction then covers whole lines)
__host__ __device__ constexpr bool plane_stream_hint_of(int esz, int N) {
    return (plane_lanes_of(esz, N) * 2 * esz) % 128 == 0 && (N * 2 * esz) % 128 == 0;
}

template <typename T, int N>
constexpr bool plane_stream_hint() {
    return plane_stream_hint_of((int)sizeof(T), N);
}

template <typename T, int N>
constexpr int plane_lanes() {
    return plane_lanes_of((int)sizeof(T), N);
}

// one xy-plane per workgroup: L lanes per row, rounded up to whole waves
__host__ __device__ constexpr int plane_block_of(int esz, int N) {
    return (plane_lanes_of(esz, N) * N + 63) / 64 * 64;
}

template <typename T, int N>
constexpr int plane_block() {
    return plane_block_of((int)sizeof(T), N);
}

// ---------------------------------------------------------------------------
// z axis: one thread per column, the column in registers.

template <typename T>
struct KZFastArgs {
    long long ncols;     // K * C * nx * ny columns in this launch
    long long nxy;
    long long j0;
    int C;
    T cz;                // (2 pi^2 / L_z^2) / nz
    const cpx<T>* tw;    // W_nz^j, j < nz
    const cpx<T>* in;
    cpx<T>* G;
    // optional: per thread, +-sum_z Re(x^* T_z x) = +-sum_k cz m^2 |X_k|^2
    // (Parseval; + for the u components c < nu, - for v), for the eta pass
    double* ezpart;
    int nu;
};

// col: the column of this thread within the launch's K * C * nx * ny columns
template <typename T, int NZ, bool NT>
__device__ __forceinline__ void kz_fast_body(const KZFastArgs<T>& a, const long long col) {
    __shared__ cpx<T> tab[NZ];
    for (int i = threadIdx.x; i < NZ; i += blockDim.x) tab[i] = ld_hint<T, false>(a.tw + i);
    __syncthreads();
    if (col >= a.ncols) return;
    const long long jc = col / a.nxy, r = col - jc * a.nxy;
    const cpx<T>* src = a.in + (a.j0 * a.C + jc) * NZ * a.nxy + r;
    cpx<T>* dst = a.G + jc * NZ * a.nxy + r;
    cpx<T> x[NZ];
#pragma unroll
    for (int z = 0; z < NZ; ++z) x[z] = ld_hint<T, NT>(src + z * a.nxy);
    RegFft<T, NZ, 1, false>::run(x, tab);
    double e = 0.0;
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
        const int m = (2 * z < NZ) ? z : z - NZ;
        const T f = a.cz * T(m * m);
        if (a.ezpart) e += double(f) * (double(x[z].re) * double(x[z].re) + double(x[z].im) * double(x[z].im));
        x[z] = f * x[z];
    }
    if (a.ezpart) a.ezpart[col] = (int)(jc % a.C) < a.nu ? e : -e;
    RegFft<T, NZ, 1, true>::run(x, tab);
#pragma unroll
    for (int z = 0; z < NZ; ++z) st_hint<T, NT>(dst + z * a.nxy, x[z]);
}

template <typename T, int NZ, bool NT>
__global__ void __launch_bounds__(256) kz_fast(const KZFastArgs<T> a) {
    kz_fast_body<T, NZ, NT>(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// z axis with a column split over L adjacent lanes (lane s holds z = s + L q,
// q < NZ / L): the line transform of the plane kernel (lane_fwd / lane_inv)
// along z.  A wave reads L contiguous runs of 64 / L columns per load; the
// column needs NZ / L registers pairs instead of NZ.
#ifndef LISE_KZ_LANES
#define LISE_KZ_LANES 1
#endif

// a column of nz points over L lanes: L divides nz and each lane keeps >= 2 points
__host__ __device__ constexpr bool kz_lanes_valid(int nz, int L) {
    return L == 1 || (nz % L == 0 && nz / L >= 2);
}

// default lanes per column
__host__ __device__ constexpr int kz_lanes_of(int nz) {
    return (LISE_KZ_LANES > 1 && kz_lanes_valid(nz, LISE_KZ_LANES)) ? LISE_KZ_LANES : 1;
}

template <int NZ>
constexpr int kz_lanes() {
    return kz_lanes_of(NZ);
}

// t: the thread index within the launch (L threads per column)
template <typename T, int NZ, int L, bool NT>
__device__ __forceinline__ void kz_lanes_body(const KZFastArgs<T>& a, const long long t) {
    constexpr int P = NZ / L;
    __shared__ cpx<T> tab[NZ];
    for (int i = threadIdx.x; i < NZ; i += blockDim.x) tab[i] = ld_hint<T, false>(a.tw + i);
    __syncthreads();
    const long long col = t / L;
    const int s = (int)(t % L);
    // the L lanes of a column are adjacent and L divides 64: a column is
    // either wholly inside the launch or wholly outside
    if (col >= a.ncols) return;
    const long long jc = col / a.nxy, r = col - jc * a.nxy;
    const cpx<T>* src = a.in + (a.j0 * a.C + jc) * NZ * a.nxy + r;
    cpx<T>* dst = a.G + jc * NZ * a.nxy + r;
    cpx<T> x[P];
#pragma unroll
    for (int q = 0; q < P; ++q) x[q] = ld_hint<T, NT>(src + (s + L * q) * a.nxy);
    lane_fwd<T, P, L>(x, tab, s);
    const int brs = bitrev(s, L);
    double e = 0.0;
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
        const int kz = k1 + P * brs;
        const int m = (2 * kz < NZ) ? kz : kz - NZ;
        const T f = a.cz * T(m * m);
        if (a.ezpart) e += double(f) * (double(x[k1].re) * double(x[k1].re) + double(x[k1].im) * double(x[k1].im));
        x[k1] = f * x[k1];
    }
    if (a.ezpart) a.ezpart[t] = (int)(jc % a.C) < a.nu ? e : -e;
    lane_inv<T, P, L>(x, tab, s);
#pragma unroll
    for (int q = 0; q < P; ++q) st_hint<T, NT>(dst + (s + L * q) * a.nxy, x[q]);
}

template <typename T, int NZ, int L, bool NT>
__global__ void __launch_bounds__(256) kz_lanes_kernel(const KZFastArgs<T> a) {
    kz_lanes_body<T, NZ, L, NT>(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Systems of one z side advanced by one launch: tab[s] describes system s,
// blks[s] is its first workgroup (blks[nsys] = gridDim.x); a system's threads
// start at a workgroup boundary, so every workgroup belongs to one system.
__device__ __forceinline__ int batch_find_ll(const long long* __restrict__ blks, int nsys, long long b) {
    int lo = 0, hi = nsys;   // blks[lo] <= b < blks[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blks[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T, int NZ, int L, bool NT>
__global__ void __launch_bounds__(256) kz_fast_batch(const KZFastArgs<T>* __restrict__ tab,
                                                     const long long* __restrict__ blks, int nsys) {
    const int s = batch_find_ll(blks, nsys, (long long)blockIdx.x);
    const long long t = ((long long)blockIdx.x - blks[s]) * blockDim.x + threadIdx.x;
    if constexpr (L > 1)
        kz_lanes_body<T, NZ, L, NT>(tab[s], t);
    else
        kz_fast_body<T, NZ, NT>(tab[s], t);
}

// Total current along z by Parseval (Eq. j summed over the lattice): per
// column of a v component, sum_kz m_z |F_z v|^2 with the signed plane-wave
// index m_z (Nyquist index 0, as for every odd derivative), summed over the
// workgroup's 256 columns in a fixed order.  One thread per column, the
// column in registers; u columns contribute nothing.
template <typename T, int NZ>
__global__ void __launch_bounds__(256) pz_kernel(const KZFastArgs<T> a, double* __restrict__ part) {
    __shared__ cpx<T> tab[NZ];
    __shared__ double red[256];
    for (int i = threadIdx.x; i < NZ; i += blockDim.x) tab[i] = ld_hint<T, false>(a.tw + i);
    __syncthreads();
    const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (col < a.ncols) {
        const long long jc = col / a.nxy, r = col - jc * a.nxy;
        if ((int)(jc % a.C) >= a.nu) {
            const cpx<T>* src = a.in + (a.j0 * a.C + jc) * NZ * a.nxy + r;
            cpx<T> x[NZ];
#pragma unroll
            for (int z = 0; z < NZ; ++z) x[z] = src[z * a.nxy];
            RegFft<T, NZ, 1, false>::run(x, tab);
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                const int m = (2 * z < NZ) ? z : (2 * z == NZ ? 0 : z - NZ);
                e += double(m) * (double(x[z].re) * double(x[z].re) + double(x[z].im) * double(x[z].im));
            }
        }
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Current density of Eq. (j) on the register-FFT path (sides up to 32):
// j_a = -w sum_j sum_v Im(v^* d_a v), with the spectral first derivative along
// one axis (1D forward transform, i k_a with the Nyquist index zeroed, 1D
// inverse; the factor f carries 2 pi / L_a and the 1/n of the round trip).
// Each thread accumulates over the qpwfs of its slot group (blockIdx.y) and
// writes jpart[slot][axis][N]; a fixed-order slot sum follows.

// x: the rows of an xy-plane over L lanes (the plane kernel's lane order), one
// workgroup per z-plane and slot group.
template <typename T, int N>
__global__ void __launch_bounds__((plane_block<T, N>())) jx_fast(const CurArgs<T> a, const cpx<T>* __restrict__ twN) {
    constexpr int L = plane_lanes<T, N>();
    constexpr int P = N / L;
    __shared__ cpx<T> tab[N];
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += blockDim.x) tab[i] = twN[i];
    __syncthreads();
    if (tid >= L * N) return;   // no barrier follows
    const int row = tid / L, s = tid % L, brs = bitrev(s, L);
    const int z = blockIdx.x;
    constexpr long long nxy = (long long)N * N;
    const long long N3 = nxy * a.nz;
    const long long j0 = (long long)blockIdx.y * a.jg;
    const long long j1 = min(a.M, j0 + a.jg);
    double jx[P];
#pragma unroll
    for (int q = 0; q < P; ++q) jx[q] = 0.0;
    for (long long j = j0; j < j1; ++j) {
        for (int cv = 0; cv < a.nv; ++cv) {
            const cpx<T>* src = a.in + ((j * a.C + a.v0 + cv) * a.nz + z) * nxy + row * N;
            cpx<T> f[P], d[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                f[q] = src[s + L * q];
                d[q] = f[q];
            }
            lane_fwd<T, P, L>(d, tab, s);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                const T k = deriv_factor<T>(k1 + P * brs, N, a.fx);
                d[k1] = mk(-k * d[k1].im, k * d[k1].re);   // i k F v
            }
            lane_inv<T, P, L>(d, tab, s);
#pragma unroll
            for (int q = 0; q < P; ++q)
                jx[q] -= a.w * (double(f[q].re) * double(d[q].im) - double(f[q].im) * double(d[q].re));
        }
    }
    double* out = a.jpart + (long long)blockIdx.y * 3 * N3 + (long long)z * nxy + row * N;
#pragma unroll
    for (int q = 0; q < P; ++q) out[s + L * q] = jx[q];
}

// y and z: one thread per line along the axis, the transformed line in
// registers and its accumulators in LDS; consecutive threads take consecutive x (or xy
// points), so each load of a wave is one contiguous run.  Line t starts at
// (t / inner) * outer + t % inner; its NA points are es apart.
constexpr int kJLineThreads = 128;
template <typename T, int NA>
__global__ void __launch_bounds__(kJLineThreads) jline_fast(const CurArgs<T> a, const cpx<T>* __restrict__ twA,
                                                             long long nlines, long long inner, long long outer,
                                                             long long es, T fa, int axis) {
    __shared__ cpx<T> tab[NA];
    __shared__ double acc[NA * kJLineThreads];
    const int tid = threadIdx.x;
    for (int i = tid; i < NA; i += blockDim.x) tab[i] = twA[i];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i * kJLineThreads + tid] = 0.0;
    __syncthreads();
    const long long t = (long long)blockIdx.x * kJLineThreads + tid;
    if (t >= nlines) return;   // no barrier follows
    const long long base = (t / inner) * outer + t % inner;
    const long long N3 = (long long)a.nx * a.ny * a.nz;
    const long long j0 = (long long)blockIdx.y * a.jg;
    const long long j1 = min(a.M, j0 + a.jg);
#pragma unroll 1
    for (long long j = j0; j < j1; ++j) {
#pragma unroll 1
        for (int cv = 0; cv < a.nv; ++cv) {
            const cpx<T>* src = a.in + (j * a.C + a.v0 + cv) * N3 + base;
            cpx<T> d[NA];
#pragma unroll
            for (int i = 0; i < NA; ++i) d[i] = src[i * es];
            RegFft<T, NA, 1, false>::run(d, tab);
#pragma unroll
            for (int m = 0; m < NA; ++m) {
                const T k = deriv_factor<T>(m, NA, fa);
                d[m] = mk(-k * d[m].im, k * d[m].re);
            }
            RegFft<T, NA, 1, true>::run(d, tab);
            // v itself is read again (just fetched: a cache hit) instead of
            // holding a second copy of the line in registers
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const cpx<T> f = src[i * es];
                acc[i * kJLineThreads + tid] -=
                    a.w * (double(f.re) * double(d[i].im) - double(f.im) * double(d[i].re));
            }
        }
    }
    double* out = a.jpart + (long long)blockIdx.y * 3 * N3 + (long long)axis * N3 + base;
#pragma unroll
    for (int i = 0; i < NA; ++i) out[i * es] = acc[i * kJLineThreads + tid];
}

// ---------------------------------------------------------------------------
// xy planes of a square lattice side N; one workgroup per z-plane and group
// of jg qpwfs; a row of the plane is spread over L lanes (lane s holds the
// points s + L q).
//
// Global memory order.  Where L points of a row fill whole 128-byte lines
// (plane_stream_hint), every lane reads and writes its own points of the
// state arrays directly.  Elsewhere (NAT: N = 20 on 4 lanes, N = 16, 24 on 8
// lanes in float32, N = 8, 20 in float64) a wave instruction in that order
// would touch 32-64 bytes of many lines, which measured at 3.0-4.3 TB/s
// against 4.9-5.5 for whole lines.  There the workgroup reads x in natural
// order (thread t: points t + i * nth of the plane) into LDS, the row
// transform takes its points from LDS, and after the inverse
// row transform the result goes back to LDS so that the epilogue runs in
// natural order as well: every global access of the kernel is then a
// contiguous run of the wave's width, so these accesses carry the
// nontemporal hint as well (16^3 float32 1.03 -> 0.89 ms per step, 20^3
// 4.13 -> 4.02).  Taking this path for float32 32^3 and 48^3 too (whole
// lines already) measured no faster.
__host__ __device__ constexpr bool plane_natural_of(int esz, int N) {
    return !plane_stream_hint_of(esz, N);
}

template <typename T, int N>
constexpr bool plane_natural() {
    return plane_natural_of((int)sizeof(T), N);
}

template <typename T, int N>
constexpr size_t kp_fast_lds() {
    return (size_t)(N + 2 * N * (N + 1) + (plane_natural<T, N>() ? 2 * N * N : 0)) * sizeof(cpx<T>);
}

#ifndef LISE_KP_MIN_WAVES
#define LISE_KP_MIN_WAVES 1
#endif

// the local part of <f|H f> at one point rpt of the lattice (forward-only
// eta pass): (V - mu_a)|u|^2 - (V - mu_b)|v|^2 + 2 s Re(Delta u^* v)
template <typename T>
__device__ __forceinline__ double eta_local(const KPArgs<T>& a, int pr, double sg, long long rpt, cpx<T> u, cpx<T> v) {
    const double V = a.V[rpt];
    const double Dr = sg * a.D[2 * rpt], Di = sg * a.D[2 * rpt + 1];
    const double ur = double(u.re), ui = double(u.im);
    const double vr = double(v.re), vi = double(v.im);
    return (V - a.mu_a[pr]) * (ur * ur + ui * ui) - (V - a.mu_b[pr]) * (vr * vr + vi * vi) +
           2.0 * (Dr * (ur * vr + ui * vi) - Di * (ur * vi - ui * vr));
}

// The body of the plane kernel: `a` describes one system, `by` is the
// workgroup row (group of jg qpwfs) within that system's launch.
template <typename T, int N, int MODE>
__device__ __forceinline__ void kp_fast_body(const KPArgs<T>& a, const cpx<T>* __restrict__ twN, const int by) {
    constexpr int L = plane_lanes<T, N>();
    constexpr int P = N / L;
    constexpr bool NT = plane_stream_hint<T, N>();
    constexpr bool NAT = plane_natural<T, N>();
    constexpr int LD = N + 1;
    constexpr int NTH = plane_block<T, N>();
    constexpr int NN = N * N;
    constexpr int PN = NAT ? (NN + NTH - 1) / NTH : P;   // points per thread in the epilogue
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tab = reinterpret_cast<cpx<T>*>(smem_raw);
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    for (int i = tid; i < N; i += nth) tab[i] = ld_hint<T, false>(twN + i);
    const int z = blockIdx.x;
    const bool act = tid < L * N;   // lanes of the row transforms
    cpx<T>* La = tab + N;
    cpx<T>* Lb = La + N * LD;
    cpx<T>* Xa = Lb + N * LD;        // natural-order copy of x (NAT only)
    cpx<T>* Xb = Xa + NN;
    const int row = tid / L;
    const int s = tid % L;
    const int brs = bitrev(s, L);
    constexpr long long nxy = (long long)N * N;
    const long long N3 = nxy * a.nz;
    const int jbeg = by * a.jg;
    const int jend = min(a.kcount, jbeg + a.jg);
    const T cdt = T(a.dt / 48.0);
    const cpx<T> coef = mk(T(a.coef_re), T(a.coef_im));
    double dn[PN], dkr[PN], dki[PN];
#pragma unroll
    for (int q = 0; q < PN; ++q) dn[q] = dkr[q] = dki[q] = 0.0;
    double ekin = 0.0;
    double pxs = 0.0, pys = 0.0;   // KP_KINETIC with a.ppart: total-current sums
    __syncthreads();

    for (int jl = jbeg; jl < jend; ++jl) {
        const long long jgl = a.j0 + jl;
        const T ej = a.eta ? T(a.eta[jgl]) : T(0);
        for (int pr = 0; pr < a.npair; ++pr) {
            const long long offa = ((jgl * a.C + a.ca[pr]) * a.nz + z) * nxy;
            const long long offb = ((jgl * a.C + a.cb[pr]) * a.nz + z) * nxy;
            cpx<T> xa[P], xb[P], fa[P], fb[P];
            if constexpr (NAT) {
#pragma unroll
                for (int i = 0; i < PN; ++i) {
                    const int p = tid + i * NTH;
                    if (p < NN) {
                        Xa[p] = ld_hint<T, true>(a.in + offa + p);
                        Xb[p] = ld_hint<T, true>(a.in + offb + p);
                    }
                }
                __syncthreads();
            }
            if (act) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    if constexpr (NAT) {
                        xa[q] = Xa[row * N + s + L * q];
                        xb[q] = Xb[row * N + s + L * q];
                    } else {
                        fa[q] = ld_hint<T, NT>(a.in + offa + row * N + s + L * q);
                        fb[q] = ld_hint<T, NT>(a.in + offb + row * N + s + L * q);
                        xa[q] = fa[q];
                        xb[q] = fb[q];
                    }
                }
                lane_fwd<T, P, L>(xa, tab, s);
                lane_fwd<T, P, L>(xb, tab, s);
#pragma unroll
                for (int k1 = 0; k1 < P; ++k1) {
                    La[(k1 + P * brs) * LD + row] = xa[k1];
                    Lb[(k1 + P * brs) * LD + row] = xb[k1];
                }
            }
            __syncthreads();
            if (act) {
                const int col = row;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    xa[q] = La[col * LD + s + L * q];
                    xb[q] = Lb[col * LD + s + L * q];
                }
                lane_fwd<T, P, L>(xa, tab, s);
                lane_fwd<T, P, L>(xb, tab, s);
                const int mx = (2 * col < N) ? col : col - N;
                const T fx = a.cx * T(mx * mx);
#pragma unroll
                for (int k1 = 0; k1 < P; ++k1) {
                    const int ky = k1 + P * brs;
                    const int my = (2 * ky < N) ? ky : ky - N;
                    const T f = fx + a.cy * T(my * my);
                    if constexpr (MODE == KP_ETAXY) {
                        // Parseval: sum_r f^* T_xy f = sum_k (k^2/2 / nxy) |F|^2; H has -T on v
                        ekin += double(f) * (double(xa[k1].re) * double(xa[k1].re) + double(xa[k1].im) * double(xa[k1].im) -
                                             double(xb[k1].re) * double(xb[k1].re) - double(xb[k1].im) * double(xb[k1].im));
                    } else {
                        if constexpr (MODE == KP_KINETIC) {
                            // Parseval for the total current: sum_r Im(v^* d_x v) = sum_k k_x |F v|^2 / nxy
                            // with the Nyquist index of the odd derivative zeroed
                            if (a.ppart) {
                                const double b2 = double(xb[k1].re) * double(xb[k1].re) +
                                                  double(xb[k1].im) * double(xb[k1].im);
                                pxs += (2 * mx == -N ? 0 : mx) * b2;
                                pys += (2 * my == -N ? 0 : my) * b2;
                            }
                        }
                        xa[k1] = f * xa[k1];
                        xb[k1] = f * xb[k1];
                    }
                }
                if constexpr (MODE != KP_ETAXY) {
                    lane_inv<T, P, L>(xa, tab, s);
                    lane_inv<T, P, L>(xb, tab, s);
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        La[col * LD + s + L * q] = xa[q];
                        Lb[col * LD + s + L * q] = xb[q];
                    }
                }
            }
            __syncthreads();
            if constexpr (MODE == KP_ETAXY) {
                // the local part of <f|H f> from the point values: (V - mu_a)|u|^2
                // - (V - mu_b)|v|^2 + 2 s Re(Delta u^* v)
                const double sg = double(a.sgn[pr]);
                if constexpr (NAT) {
#pragma unroll
                    for (int i = 0; i < PN; ++i) {
                        const int p = tid + i * NTH;
                        if (p < NN) ekin += eta_local(a, pr, sg, (long long)z * nxy + p, Xa[p], Xb[p]);
                    }
                    __syncthreads();   // Xa, Xb are rewritten by the next pair
                } else if (act) {
#pragma unroll
                    for (int q = 0; q < P; ++q)
                        ekin += eta_local(a, pr, sg, (long long)z * nxy + row * N + s + L * q, fa[q], fb[q]);
                }
                continue;   // the next pair reuses La, Lb only after the barrier above
            }
            if (act) {
#pragma unroll
                for (int k1 = 0; k1 < P; ++k1) {
                    xa[k1] = La[(k1 + P * brs) * LD + row];
                    xb[k1] = Lb[(k1 + P * brs) * LD + row];
                }
                lane_inv<T, P, L>(xa, tab, s);
                lane_inv<T, P, L>(xb, tab, s);
            }
            if constexpr (NAT) {
                // the xy-term to LDS in natural order (La, Lb hold N x N
                // points there), then the epilogue in natural order
                __syncthreads();
                if (act) {
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        La[row * N + s + L * q] = xa[q];
                        Lb[row * N + s + L * q] = xb[q];
                    }
                }
                __syncthreads();
                const long long lofa = (((long long)jl * a.C + a.ca[pr]) * a.nz + z) * nxy;
                const long long lofb = (((long long)jl * a.C + a.cb[pr]) * a.nz + z) * nxy;
#pragma unroll
                for (int i = 0; i < PN; ++i) {
                    const int p = tid + i * NTH;
                    if (p < NN)
                        point_epilogue<T, MODE, true, true>(a, pr, La[p], Lb[p], Xa[p], Xb[p], offa + p, offb + p,
                                                             (long long)z * nxy + p, lofa + p, lofb + p, coef, cdt, ej,
                                                             dn[i], dkr[i], dki[i], ekin);
                }
            } else if (act) {
                const long long lofa = (((long long)jl * a.C + a.ca[pr]) * a.nz + z) * nxy;
                const long long lofb = (((long long)jl * a.C + a.cb[pr]) * a.nz + z) * nxy;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int pt = row * N + s + L * q;
                    // the plane kernels never run fused: the z-term is always in G
                    const long long ea = offa + pt, eb = offb + pt;
                    point_epilogue<T, MODE, true, NT>(a, pr, xa[q], xb[q], fa[q], fb[q], ea, eb, (long long)z * nxy + pt,
                                                      lofa + pt, lofb + pt, coef, cdt, ej, dn[q], dkr[q], dki[q], ekin);
                }
            }
            __syncthreads();
        }
        if constexpr (MODE == KP_ETAXY) {
            // one partial sum per wave and qpwf (fixed-order butterfly; lane 0
            // holds the wave's sum), [qpwf][plane block][wave]
            double v = ekin;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if ((tid & 63) == 0) a.epart[((long long)jl * gridDim.x + blockIdx.x) * (nth >> 6) + (tid >> 6)] = v;
            ekin = 0.0;
        }
    }
    if constexpr (MODE == KP_ETAXY) return;
    if (MODE == KP_KINETIC || MODE == KP_ETA) {
        double* red = reinterpret_cast<double*>(smem_raw);
        const long long wg = (long long)by * gridDim.x + blockIdx.x;
        const int nsum = (MODE == KP_KINETIC && a.ppart) ? 3 : 1;
        for (int v = 0; v < nsum; ++v) {
            red[tid] = v == 0 ? ekin : (v == 1 ? pxs : pys);
            __syncthreads();
            int st = 1;
            while (st < nth) st <<= 1;
            for (st >>= 1; st > 0; st >>= 1) {
                if (tid < st && tid + st < nth) red[tid] += red[tid + st];
                __syncthreads();
            }
            if (tid == 0) {
                if (v == 0) a.epart[wg] = red[0];
                else a.ppart[2 * wg + v - 1] = red[0];
            }
            __syncthreads();
        }
        return;
    }
    if constexpr (NAT) {
        if (a.dens_src) {
            double* base = a.dpart + (long long)by * 3 * N3 + (long long)z * nxy;
#pragma unroll
            for (int i = 0; i < PN; ++i) {
                const int p = tid + i * NTH;
                if (p >= NN) continue;
                if (a.accumulate) {
                    stg(base + p, ldg(base + p) + dn[i]);
                    stg(base + N3 + p, ldg(base + N3 + p) + dkr[i]);
                    stg(base + 2 * N3 + p, ldg(base + 2 * N3 + p) + dki[i]);
                } else {
                    stg(base + p, dn[i]);
                    stg(base + N3 + p, dkr[i]);
                    stg(base + 2 * N3 + p, dki[i]);
                }
            }
        }
    } else if (a.dens_src && act) {
        double* base = a.dpart + (long long)by * 3 * N3 + (long long)z * nxy;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int pt = row * N + s + L * q;
            if (a.accumulate) {
                stg(base + pt, ldg(base + pt) + dn[q]);
                stg(base + N3 + pt, ldg(base + N3 + pt) + dkr[q]);
                stg(base + 2 * N3 + pt, ldg(base + 2 * N3 + pt) + dki[q]);
            } else {
                stg(base + pt, dn[q]);
                stg(base + N3 + pt, dkr[q]);
                stg(base + 2 * N3 + pt, dki[q]);
            }
        }
    }
}

template <typename T, int N, int MODE>
__global__ void __launch_bounds__((plane_block<T, N>()), LISE_KP_MIN_WAVES) kp_fast(const KPArgs<T> a, const cpx<T>* __restrict__ twN) {
    kp_fast_body<T, N, MODE>(a, twN, (int)blockIdx.y);
}

// ---------------------------------------------------------------------------
// The ABM phases with the z-term inside the plane kernel (z_dense).  The
// kinetic operator along z is the real symmetric nz x nz matrix T_z (the z
// kernel's transform, multiply, inverse transform written out), so the
// z-term of a point is a dot product with its z-column.  One workgroup takes
// kZdPlanes consecutive planes of its jg qpwfs: per qpwf and pair it reads
// the z-columns at its points once and forms the z-terms of all its planes
// in registers, then runs the xy transforms and the epilogue plane by plane.
// The columns of a qpwf are read by nz / kZdPlanes workgroups; the launch
// puts those on one XCD (xcd_plane_task) so that all but the first read hit
// L2.  No z-axis kernel and no z-term scratch: 14 state arrays per ABM step
// from HBM instead of 20.  Whole-line plane rows with at most two points per
// lane (float64 sides 16, 32; float32 side 32).

#ifndef LISE_ZD_PLANES
#define LISE_ZD_PLANES 4
#endif
#ifndef LISE_ZD_UNROLL
#define LISE_ZD_UNROLL 4
#endif
#ifndef LISE_ZD_XCD
#define LISE_ZD_XCD 1
#endif
constexpr int kZdPlanes = LISE_ZD_PLANES;

__host__ __device__ constexpr bool zd_side(int esz, int N) {
    return N <= 32 && N % kZdPlanes == 0 && !plane_natural_of(esz, N) && N / plane_lanes_of(esz, N) <= 2;
}

// dynamic LDS: twiddles, the two padded row-transform planes, kZdPlanes rows
// of T_z, and the float64 density sums of the workgroup's planes
template <typename T, int N>
constexpr size_t kpzd_lds() {
    return (size_t)(N + 2 * N * (N + 1)) * sizeof(cpx<T>) + (size_t)kZdPlanes * N * sizeof(T) +
           (size_t)kZdPlanes * 3 * N * N * sizeof(double);
}

// Workgroup b of a launch of nt x R tasks (nt plane tasks per row) -> (plane
// task, row).  The dispatcher deals consecutive workgroups to the eight XCDs
// in turn, so workgroup b runs on XCD b % 8; here the nt tasks of one row
// (the same jg qpwfs, hence the same z-columns) are consecutive workgroups
// of one XCD.  Rows beyond the last multiple of 8 map in plain order.  The
// map is a bijection for any R, so results do not depend on where a
// workgroup runs.
__device__ __forceinline__ void xcd_plane_task(int b, int nt, int R, int& task, int& row) {
    const int R8 = R & ~7;
    const int head = nt * R8;
    if (b < head) {
        const int x = b & 7, o = b >> 3;
        row = (o / nt) * 8 + x;
        task = o % nt;
    } else {
        const int r = b - head;
        row = R8 + r / nt;
        task = r % nt;
    }
}

template <typename T, int N, int MODE>
__device__ __forceinline__ void kpzd_body(const KPArgs<T>& a, const cpx<T>* __restrict__ twN, const int by,
                                          const int z0) {
    static_assert(MODE == KP_ABM1 || MODE == KP_ABM2, "in-kernel z-term in the ABM phases only");
    static_assert(zd_side((int)sizeof(T), N), "whole-line plane rows, at most two points per lane");
    constexpr int PZ = kZdPlanes;
    constexpr int L = plane_lanes<T, N>();
    constexpr int P = N / L;
    constexpr bool NT = plane_stream_hint<T, N>();
    constexpr int LD = N + 1;
    constexpr int NN = N * N;
    constexpr long long nxy = NN;
    constexpr long long N3 = nxy * N;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tab = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* La = tab + N;
    cpx<T>* Lb = La + N * LD;
    T* tzr = reinterpret_cast<T*>(Lb + N * LD);            // rows z0 .. z0 + PZ - 1 of T_z
    double* Dl = reinterpret_cast<double*>(tzr + PZ * N);  // [PZ][3][NN] density sums
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    for (int i = tid; i < N; i += nth) tab[i] = ld_hint<T, false>(twN + i);
    for (int i = tid; i < PZ * N; i += nth) tzr[i] = ldg(a.tzm + (long long)z0 * N + i);
    if (a.dens_src)
        for (int i = tid; i < PZ * 3 * NN; i += nth) Dl[i] = 0.0;
    const int row = tid / L;
    const int s = tid % L;
    const int brs = bitrev(s, L);
    const int jbeg = by * a.jg;
    const int jend = min(a.kcount, jbeg + a.jg);
    const T cdt = T(a.dt / 48.0);
    const cpx<T> coef = mk(T(0), T(0));
    double ekin = 0.0;
    __syncthreads();
    for (int jl = jbeg; jl < jend; ++jl) {
        const long long jgl = a.j0 + jl;
        for (int pr = 0; pr < a.npair; ++pr) {
            const long long cola = (jgl * a.C + a.ca[pr]) * N3;
            const long long colb = (jgl * a.C + a.cb[pr]) * N3;
            // the z-terms of the PZ planes at this thread's points: one pass
            // over the z-columns, summed in the order z' = 0, 1, ...
            cpx<T> Ga[PZ][P], Gb[PZ][P];
#pragma unroll
            for (int pl = 0; pl < PZ; ++pl)
#pragma unroll
                for (int q = 0; q < P; ++q) Ga[pl][q] = Gb[pl][q] = mk(T(0), T(0));
#pragma unroll LISE_ZD_UNROLL
            for (int zz = 0; zz < N; ++zz) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int pt = row * N + s + L * q;
                    const cpx<T> u = ld_hint<T, false>(a.in + cola + zz * nxy + pt);
                    const cpx<T> v = ld_hint<T, false>(a.in + colb + zz * nxy + pt);
#pragma unroll
                    for (int pl = 0; pl < PZ; ++pl) {
                        const T t = tzr[pl * N + zz];
                        Ga[pl][q] = mk(Ga[pl][q].re + t * u.re, Ga[pl][q].im + t * u.im);
                        Gb[pl][q] = mk(Gb[pl][q].re + t * v.re, Gb[pl][q].im + t * v.im);
                    }
                }
            }
#pragma unroll
            for (int pl = 0; pl < PZ; ++pl) {
                const int z = z0 + pl;
                const long long offa = cola + z * nxy, offb = colb + z * nxy;
                cpx<T> xa[P], xb[P], fa[P], fb[P];
                // the plane's own points (just read with the columns: cache hits)
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    fa[q] = ld_hint<T, false>(a.in + offa + row * N + s + L * q);
                    fb[q] = ld_hint<T, false>(a.in + offb + row * N + s + L * q);
                    xa[q] = fa[q];
                    xb[q] = fb[q];
                }
                // rows: forward transform along x, transposed into LDS
                lane_fwd<T, P, L>(xa, tab, s);
                lane_fwd<T, P, L>(xb, tab, s);
#pragma unroll
                for (int k1 = 0; k1 < P; ++k1) {
                    La[(k1 + P * brs) * LD + row] = xa[k1];
                    Lb[(k1 + P * brs) * LD + row] = xb[k1];
                }
                __syncthreads();
                {
                    // columns (fixed kx): forward along y, multiply by
                    // (c_x m_x^2 + c_y m_y^2), inverse along y
                    const int col = row;
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        xa[q] = La[col * LD + s + L * q];
                        xb[q] = Lb[col * LD + s + L * q];
                    }
                    lane_fwd<T, P, L>(xa, tab, s);
                    lane_fwd<T, P, L>(xb, tab, s);
                    const int mx = (2 * col < N) ? col : col - N;
                    const T fx = a.cx * T(mx * mx);
#pragma unroll
                    for (int k1 = 0; k1 < P; ++k1) {
                        const int ky = k1 + P * brs;
                        const int my = (2 * ky < N) ? ky : ky - N;
                        const T f = fx + a.cy * T(my * my);
                        xa[k1] = f * xa[k1];
                        xb[k1] = f * xb[k1];
                    }
                    lane_inv<T, P, L>(xa, tab, s);
                    lane_inv<T, P, L>(xb, tab, s);
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        La[col * LD + s + L * q] = xa[q];
                        Lb[col * LD + s + L * q] = xb[q];
                    }
                }
                __syncthreads();
                // rows: inverse along x, then the epilogue at the thread's points
#pragma unroll
                for (int k1 = 0; k1 < P; ++k1) {
                    xa[k1] = La[(k1 + P * brs) * LD + row];
                    xb[k1] = Lb[(k1 + P * brs) * LD + row];
                }
                lane_inv<T, P, L>(xa, tab, s);
                lane_inv<T, P, L>(xb, tab, s);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int pt = row * N + s + L * q;
                    double dn = 0.0, dkr = 0.0, dki = 0.0;
                    point_epilogue<T, MODE, false, NT>(a, pr, xa[q] + Ga[pl][q], xb[q] + Gb[pl][q], fa[q], fb[q],
                                                       offa + pt, offb + pt, (long long)z * nxy + pt, 0, 0, coef, cdt,
                                                       T(0), dn, dkr, dki, ekin);
                    if (a.dens_src) {
                        double* d = Dl + pl * 3 * NN + pt;   // this thread's point only
                        d[0] += dn;
                        d[NN] += dkr;
                        d[2 * NN] += dki;
                    }
                }
                __syncthreads();   // La, Lb are rewritten by the next plane
            }
        }
    }
    if (a.dens_src) {
#pragma unroll
        for (int pl = 0; pl < PZ; ++pl) {
            double* base = a.dpart + (long long)by * 3 * N3 + (long long)(z0 + pl) * nxy;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int pt = row * N + s + L * q;
                const double* d = Dl + pl * 3 * NN + pt;
                if (a.accumulate) {
                    stg(base + pt, ldg(base + pt) + d[0]);
                    stg(base + N3 + pt, ldg(base + N3 + pt) + d[NN]);
                    stg(base + 2 * N3 + pt, ldg(base + 2 * N3 + pt) + d[2 * NN]);
                } else {
                    stg(base + pt, d[0]);
                    stg(base + N3 + pt, d[NN]);
                    stg(base + 2 * N3 + pt, d[2 * NN]);
                }
            }
        }
    }
}

// a one-dimensional grid of (N / kZdPlanes) plane tasks x R rows
template <typename T, int N, int MODE>
__global__ void __launch_bounds__((plane_block<T, N>())) kp_fast_zd(const KPArgs<T> a, const cpx<T>* __restrict__ twN,
                                                                   int R) {
    int task, row;
    if constexpr (LISE_ZD_XCD) {
        xcd_plane_task((int)blockIdx.x, N / kZdPlanes, R, task, row);
    } else {
        row = (int)blockIdx.x / (N / kZdPlanes);
        task = (int)blockIdx.x % (N / kZdPlanes);
    }
    kpzd_body<T, N, MODE>(a, twN, row, task * kZdPlanes);
}

// Systems of one lattice side advanced by one launch: tab[s] describes system
// s (its buffers, fields, functional and qpwf count), rows[s] is the first
// workgroup row of system s (rows[nsys] = gridDim.y).  Each workgroup finds
// its system by bisection over rows; all its threads take the same branch.
__device__ __forceinline__ int batch_find(const int* __restrict__ rows, int nsys, int y) {
    int lo = 0, hi = nsys;   // rows[lo] <= y < rows[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rows[mid] <= y) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T, int N, int MODE>
__global__ void __launch_bounds__((plane_block<T, N>()), LISE_KP_MIN_WAVES)
    kp_fast_batch(const KPArgs<T>* __restrict__ tab, const int* __restrict__ rows, int nsys,
                  const cpx<T>* __restrict__ twN) {
    const int s = batch_find(rows, nsys, (int)blockIdx.y);
    kp_fast_body<T, N, MODE>(tab[s], twN, (int)blockIdx.y - rows[s]);
}

}  // namespace lise
