// Split-bf16 MFMA form of the xy-plane kinetic term (float32 state).
//
// Along one axis the spectral kinetic operator F^{-1} (k^2/2) F is the dense
// real symmetric N x N matrix of the DVR second derivative of Sec.
// "Discretization" (Eq. d2, times -1/2).  For a square plane F (rows y,
// columns x) the transverse kinetic term is therefore two dense products,
//     T_xy F = F T_x + T_y F,
// which run on the matrix cores.  Each float32 operand is split into two
// bfloat16 parts, a = a_hi + a_lo, and a b is formed as
// a_hi b_hi + a_hi b_lo + a_lo b_hi with float32 accumulation (the a_lo b_lo
// term, ~2^-16 relative, is dropped).  The z term comes from the register FFT
// kernel as in the other forms.
//
// v_mfma_f32_16x16x16bf16_1k, one 64-lane wave per 16 x 16 output tile
// (two tiles of one tile-row for the 64 x 64 plane):
//   A[i][k]: lane l holds i = l % 16, k = 4 (l / 16) + t, t < 4
//   B[k][j]: lane l holds j = l % 16, k = 4 (l / 16) + t
//   D[i][j]: lane l, register r holds i = 4 (l / 16) + r, j = l % 16
#pragma once

#include "lise_device.hpp"

namespace lise {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float f) {
    const unsigned u = __float_as_uint(f);
    return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

// element t of the hi and lo fragments from one float
__device__ __forceinline__ void split_bf16(float f, bf16x4& hi, bf16x4& lo, int t) {
    const short h = bf16_bits(f);
    hi[t] = h;
    lo[t] = bf16_bits(f - bf16_value(h));
}

__device__ __forceinline__ f32x4 mfma3(bf16x4 ah, bf16x4 al, bf16x4 bh, bf16x4 bl, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    return c;
}

// output tiles per wave (two tiles of one tile-row for the 64 x 64 plane, so
// that a workgroup has at most 8 waves and a wave may use 256 registers)
template <int N>
constexpr int mfma_tpw() {
    return N >= 64 ? 2 : 1;
}

template <int N>
constexpr int mfma_block() {
    return 64 * (N / 16) * (N / 16) / mfma_tpw<N>();
}

template <int N>
constexpr size_t kp_mfma_lds() {
    return (size_t)2 * N * (N + 1) * sizeof(cpx<float>);
}

// Dhl: bfloat16 bits of the kinetic matrix, hi part [N][N] then lo part.
template <int N, int MODE>
__global__ void __launch_bounds__((mfma_block<N>())) kp_mfma(const KPArgs<float> a,
                                                            const short* __restrict__ Dhl) {
    constexpr int NT = N / 16;
    constexpr int TPW = mfma_tpw<N>();
    constexpr int LD = N + 1;
    extern __shared__ unsigned char smem_raw[];
    cpx<float>* Fa = reinterpret_cast<cpx<float>*>(smem_raw);
    cpx<float>* Fb = Fa + N * LD;
    const short* Dh = Dhl;
    const short* Dl = Dhl + N * N;
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int ty = wave / (NT / TPW), tx0 = (wave % (NT / TPW)) * TPW;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    const int z = blockIdx.x;
    constexpr long long nxy = (long long)N * N;
    const long long N3 = nxy * a.nz;
    const int jbeg = blockIdx.y * a.jg;
    const int jend = min(a.kcount, jbeg + a.jg);
    const float cdt = float(a.dt / 48.0);
    const cpx<float> coef = mk(float(a.coef_re), float(a.coef_im));
    double dn[4 * TPW], dkr[4 * TPW], dki[4 * TPW];
#pragma unroll
    for (int r = 0; r < 4 * TPW; ++r) dn[r] = dkr[r] = dki[r] = 0.0;
    double ekin = 0.0;

    for (int jl = jbeg; jl < jend; ++jl) {
        const long long jgl = a.j0 + jl;
        const float ej = a.eta ? float(a.eta[jgl]) : 0.0f;
        for (int pr = 0; pr < a.npair; ++pr) {
            const long long offa = ((jgl * a.C + a.ca[pr]) * a.nz + z) * nxy;
            const long long offb = ((jgl * a.C + a.cb[pr]) * a.nz + z) * nxy;
            for (int e = tid; e < N * N; e += nth) {
                const int y = e / N, x = e - y * N;
                Fa[y * LD + x] = ld_hint<float, true>(a.in + offa + e);
                Fb[y * LD + x] = ld_hint<float, true>(a.in + offb + e);
            }
            __syncthreads();
            f32x4 ar[TPW], ai[TPW], br[TPW], bi[TPW];
#pragma unroll
            for (int u = 0; u < TPW; ++u) ar[u] = ai[u] = br[u] = bi[u] = f32x4{0, 0, 0, 0};
#pragma unroll 1
            for (int kk = 0; kk < NT; ++kk) {
                // x product: C[y][x] += sum_k F[y][k] T[k][x]; the F fragment
                // (rows of tile-row ty) is shared by the wave's tiles
                bf16x4 far_h, far_l, fai_h, fai_l, fbr_h, fbr_l, fbi_h, fbi_l, d_h, d_l;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 16 * kk + lk + t;
                    const cpx<float> u = Fa[(16 * ty + li) * LD + k];
                    const cpx<float> v = Fb[(16 * ty + li) * LD + k];
                    split_bf16(u.re, far_h, far_l, t);
                    split_bf16(u.im, fai_h, fai_l, t);
                    split_bf16(v.re, fbr_h, fbr_l, t);
                    split_bf16(v.im, fbi_h, fbi_l, t);
                }
#pragma unroll
                for (int u = 0; u < TPW; ++u) {
                    const int tx = tx0 + u;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int k = 16 * kk + lk + t;
                        d_h[t] = Dh[k * N + 16 * tx + li];
                        d_l[t] = Dl[k * N + 16 * tx + li];
                    }
                    ar[u] = mfma3(far_h, far_l, d_h, d_l, ar[u]);
                    ai[u] = mfma3(fai_h, fai_l, d_h, d_l, ai[u]);
                    br[u] = mfma3(fbr_h, fbr_l, d_h, d_l, br[u]);
                    bi[u] = mfma3(fbi_h, fbi_l, d_h, d_l, bi[u]);
                }
                // y product: C[y][x] += sum_k T[y][k] F[k][x]; the T fragment is shared
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 16 * kk + lk + t;
                    d_h[t] = Dh[(16 * ty + li) * N + k];
                    d_l[t] = Dl[(16 * ty + li) * N + k];
                }
#pragma unroll
                for (int u = 0; u < TPW; ++u) {
                    const int tx = tx0 + u;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int k = 16 * kk + lk + t;
                        const cpx<float> uu = Fa[k * LD + 16 * tx + li];
                        const cpx<float> vv = Fb[k * LD + 16 * tx + li];
                        split_bf16(uu.re, far_h, far_l, t);
                        split_bf16(uu.im, fai_h, fai_l, t);
                        split_bf16(vv.re, fbr_h, fbr_l, t);
                        split_bf16(vv.im, fbi_h, fbi_l, t);
                    }
                    ar[u] = mfma3(d_h, d_l, far_h, far_l, ar[u]);
                    ai[u] = mfma3(d_h, d_l, fai_h, fai_l, ai[u]);
                    br[u] = mfma3(d_h, d_l, fbr_h, fbr_l, br[u]);
                    bi[u] = mfma3(d_h, d_l, fbi_h, fbi_l, bi[u]);
                }
            }
            const long long lofa = (((long long)jl * a.C + a.ca[pr]) * a.nz + z) * nxy;
            const long long lofb = (((long long)jl * a.C + a.cb[pr]) * a.nz + z) * nxy;
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int y = 16 * ty + lk + r, x = 16 * (tx0 + u) + li;
                    const int pt = y * N + x;
                    const cpx<float> Ta = mk(ar[u][r], ai[u][r]), Tb = mk(br[u][r], bi[u][r]);
                    point_epilogue<float, MODE, true, true>(a, pr, Ta, Tb, Fa[y * LD + x], Fb[y * LD + x], offa + pt,
                                                      offb + pt, (long long)z * nxy + pt, lofa + pt, lofb + pt, coef,
                                                      cdt, ej, dn[u * 4 + r], dkr[u * 4 + r], dki[u * 4 + r], ekin);
                }
            }
            __syncthreads();
        }
    }
    if (MODE == KP_KINETIC || MODE == KP_ETA) {
        double* red = reinterpret_cast<double*>(smem_raw);
        red[tid] = ekin;
        __syncthreads();
        int st = 1;
        while (st < nth) st <<= 1;
        for (st >>= 1; st > 0; st >>= 1) {
            if (tid < st && tid + st < nth) red[tid] += red[tid + st];
            __syncthreads();
        }
        if (tid == 0) a.epart[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
        return;
    }
    if (a.dens_src) {
        double* base = a.dpart + (long long)blockIdx.y * 3 * N3 + (long long)z * nxy;
#pragma unroll
        for (int u = 0; u < TPW; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pt = (16 * ty + lk + r) * N + 16 * (tx0 + u) + li;
                const int i = u * 4 + r;
                if (a.accumulate) {
                    base[pt] += dn[i];
                    base[N3 + pt] += dkr[i];
                    base[2 * N3 + pt] += dki[i];
                } else {
                    base[pt] = dn[i];
                    base[N3 + pt] = dkr[i];
                    base[2 * N3 + pt] = dki[i];
                }
            }
    }
}

}  // namespace lise
