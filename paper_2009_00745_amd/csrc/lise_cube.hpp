// Single-pass ABM kernel for lattices whose whole cube of a component pair
// fits in a CU's LDS (cubic side 8, 16 or 20; 16 only in float64).
//
// The two-pass schedule (z-axis kernel, then the plane kernel) writes the
// z-term of every qpwf to HBM and reads it back: 20 state arrays per ABM step
// against 14 that the re-associated Eq. (p)-(y) needs.  Here one workgroup
// takes one qpwf pair (u, v) at a time: both component cubes go to LDS, the
// kinetic operator T = F^-1 (k^2/2) F runs as five passes of line transforms
// (x forward, y forward, z forward-multiply-inverse, y inverse, x inverse;
// each thread one line of N points in registers per pass), and the ABM
// epilogue runs in natural order on T u, T v from LDS.  Phase 1 then moves 9
// arrays per qpwf (6 reads, 3 writes) and phase 2 5 (3 reads, 2 writes).
//
// LDS layout of a cube: [z][y][x] with x-rows padded to N + 1 points, so that
// the x-line pass (consecutive threads on consecutive rows) spreads over the
// banks; the y- and z-line passes take consecutive x in consecutive threads.
// The point values u, v of the epilogue are kept in registers from the load
// (KEEP) or read again from global memory where registers are short.
#pragma once

#include "lise_fast.hpp"

namespace lise {

__host__ __device__ constexpr int cube_row(int N) { return N + 1; }
__host__ __device__ constexpr int cube_comp(int N) { return N * N * (N + 1); }

// threads of one workgroup: one line per thread per pass (2 N^2 lines of a
// pair; 20^3 has 800 lines on 1024 threads)
__host__ __device__ constexpr int cube_threads_of(int esz, int N) {
    return N == 8 ? 128 : 1024;
}

// keep the point values of u, v in registers (else read them again)
__host__ __device__ constexpr bool cube_keep_of(int esz, int N) { return N <= 8; }

__host__ __device__ constexpr bool cube_side(int esz, int N) { return N == 8 || N == 16 || (N == 20 && esz == 4); }

// where the single-pass kernel is the default (measured faster than the two
// kernels: side 8 in both precisions, 16 and 20 in float32)
__host__ __device__ constexpr bool cube_auto_of(int esz, int N) { return N == 8 || (esz == 4 && (N == 16 || N == 20)); }

// float64 density accumulators of the epilogue points in registers (else the
// kernel leaves the densities to a separate pass over the vector it wrote:
// one more array read per phase, and registers for the transforms instead)
__host__ __device__ constexpr bool cube_dens_in_of(int esz, int N) { return N == 8 || (N == 16 && esz == 4); }

// dynamic LDS of the kernel: twiddles + two padded cubes
__host__ __device__ constexpr size_t cube_lds_of(int esz, int N) {
    return (size_t)(N + 2 * cube_comp(N)) * 2 * esz;
}

template <typename T, int N>
__device__ __forceinline__ void cube_line(cpx<T>* __restrict__ L, const cpx<T>* __restrict__ tab, int t, int axis,
                                          bool inv, const KPArgs<T>& a) {
    constexpr int NN = N * N, RW = cube_row(N), PL = N * RW, CS = cube_comp(N);
    const int comp = t / NN, rem = t - comp * NN;
    int base, step;
    if (axis == 0) {          // x-lines: (z, y) = rem
        base = comp * CS + (rem / N) * PL + (rem % N) * RW;
        step = 1;
    } else if (axis == 1) {   // y-lines: (z, x) = rem
        base = comp * CS + (rem / N) * PL + (rem % N);
        step = RW;
    } else {                  // z-lines: (y, x) = rem
        base = comp * CS + (rem / N) * RW + (rem % N);
        step = PL;
    }
    cpx<T> x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = L[base + i * step];
    if (axis == 2) {
        // x and y are already in frequency order here (natural order out of
        // the Stockham transforms); multiply by k^2 / 2 / N^3 between the
        // forward and inverse z transforms (Nyquist kept: even derivative)
        const int kx = rem % N, ky = rem / N;
        const int mx = (2 * kx < N) ? kx : kx - N;
        const int my = (2 * ky < N) ? ky : ky - N;
        const T fxy = a.cx * T(mx * mx) + a.cy * T(my * my);
        RegFft<T, N, 1, false>::run(x, tab);
#pragma unroll
        for (int z = 0; z < N; ++z) {
            const int mz = (2 * z < N) ? z : z - N;
            x[z] = (fxy + a.cz * T(mz * mz)) * x[z];
        }
        RegFft<T, N, 1, true>::run(x, tab);
    } else if (inv) {
        RegFft<T, N, 1, true>::run(x, tab);
    } else {
        RegFft<T, N, 1, false>::run(x, tab);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) L[base + i * step] = x[i];
}

// One workgroup row `by` of qpwfs (jg of them); MODE is KP_ABM1 or KP_ABM2.
// a.cx, a.cy, a.cz carry (2 pi^2 / L_a^2) / N^3.
// ap is __restrict__: the kernel's stores through the state pointers never
// modify the descriptor, so its fields stay in scalar registers (the batched
// kernel reads it from a device table)
template <typename T, int N, int MODE>
__device__ __forceinline__ void kc_fast_body(const KPArgs<T>* __restrict__ ap, const cpx<T>* __restrict__ twN,
                                             const int by) {
    const KPArgs<T>& a = *ap;
    static_assert(MODE == KP_ABM1 || MODE == KP_ABM2, "single-pass kernel of the ABM phases");
    constexpr int NTH = cube_threads_of((int)sizeof(T), N);
    constexpr bool KEEP = cube_keep_of((int)sizeof(T), N);
    constexpr int NN = N * N, N3 = N * N * N, RW = cube_row(N), PL = N * RW, CS = cube_comp(N);
    constexpr int PN = (N3 + NTH - 1) / NTH;
    constexpr int KN = KEEP ? PN : 1;
    constexpr bool DIN = cube_dens_in_of((int)sizeof(T), N);
    constexpr int DN = DIN ? PN : 1;
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* tab = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* L = tab + N;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += NTH) tab[i] = ld_hint<T, false>(twN + i);
    const int jbeg = by * a.jg;
    const int jend = min(a.kcount, jbeg + a.jg);
    const T cdt = T(a.dt / 48.0);
    const cpx<T> coef = mk(T(0), T(0));
    double dn[DN], dkr[DN], dki[DN];
#pragma unroll
    for (int q = 0; q < DN; ++q) dn[q] = dkr[q] = dki[q] = 0.0;
    double ekin = 0.0;
    __syncthreads();
    for (int jl = jbeg; jl < jend; ++jl) {
        const long long jgl = a.j0 + jl;
        const T ej = a.eta ? T(a.eta[jgl]) : T(0);
        for (int pr = 0; pr < a.npair; ++pr) {
            const long long offa = (jgl * a.C + a.ca[pr]) * N3;
            const long long offb = (jgl * a.C + a.cb[pr]) * N3;
            cpx<T> fa[KN], fb[KN];
#pragma unroll
            for (int i = 0; i < PN; ++i) {
                int p = tid + i * NTH;
                // recomputed per qpwf rather than hoisted out of the qpwf loop
                // (the hoisted per-point offsets did not fit in registers)
                asm volatile("" : "+v"(p));
                if (p < N3) {
                    // read once when kept; read again later otherwise (no
                    // nontemporal hint then, so that the second read can hit)
                    const cpx<T> u = ld_hint<T, KEEP>(a.in + offa + p);
                    const cpx<T> v = ld_hint<T, KEEP>(a.in + offb + p);
                    const int l = (p / NN) * PL + ((p / N) % N) * RW + p % N;
                    L[l] = u;
                    L[CS + l] = v;
                    if constexpr (KEEP) {
                        fa[i] = u;
                        fb[i] = v;
                    }
                }
            }
            __syncthreads();
            // passes: x, y forward; z forward-multiply-inverse; y, x inverse
            const bool act = tid < 2 * NN;
#pragma unroll 1
            for (int pass = 0; pass < 5; ++pass) {
                const int axis = pass < 3 ? pass : 4 - pass;
                int t = tid;
                asm volatile("" : "+v"(t));
                if (act) cube_line<T, N>(L, tab, t, axis, pass > 2, a);
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < PN; ++i) {
                int p = tid + i * NTH;
                asm volatile("" : "+v"(p));
                if (p < N3) {
                    const int l = (p / NN) * PL + ((p / N) % N) * RW + p % N;
                    cpx<T> u, v;
                    if constexpr (KEEP) {
                        u = fa[i];
                        v = fb[i];
                    } else {
                        u = ld_hint<T, false>(a.in + offa + p);
                        v = ld_hint<T, false>(a.in + offb + p);
                    }
                    point_epilogue<T, MODE, false, true>(a, pr, L[l], L[CS + l], u, v, offa + p, offb + p, p, 0, 0,
                                                         coef, cdt, ej, dn[DIN ? i : 0], dkr[DIN ? i : 0],
                                                         dki[DIN ? i : 0], ekin);
                }
                // one point's loads in flight at a time per thread: the
                // workgroup's 16 waves keep enough requests in flight, and
                // hoisting the loads of every point spilled registers
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();   // the cubes are rewritten by the next pair
        }
    }
    if (DIN && a.dens_src) {
        double* base = a.dpart + (long long)by * 3 * N3;
#pragma unroll
        for (int i = 0; i < PN; ++i) {
            const int p = tid + i * NTH;
            if (p >= N3) continue;
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
}

// Systems of one lattice side in one launch (see kp_fast_batch).  A single
// system runs the same kernel on a one-entry table (put_desc_kernel writes
// it on the stream), so that a system stepped alone and in a batch execute
// identical code and round identically.
template <typename T, int N, int MODE>
__global__ void __launch_bounds__((cube_threads_of((int)sizeof(T), N)))
    kc_fast_batch(const KPArgs<T>* __restrict__ tab, const int* __restrict__ rows, int nsys,
                  const cpx<T>* __restrict__ twN) {
    const int s = batch_find(rows, nsys, (int)blockIdx.y);
    kc_fast_body<T, N, MODE>(tab + s, twN, (int)blockIdx.y - rows[s]);
}

template <typename T>
__global__ void put_desc_kernel(const KPArgs<T> a, int nrows, KPArgs<T>* __restrict__ dst, int* __restrict__ rows) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *dst = a;
        rows[0] = 0;
        rows[1] = nrows;
    }
}

}  // namespace lise
