// Bodies of the grid-sweep kernels (Formula 5 summands and their FP64 sums),
// shared by the one-problem launches (kernels_eval.hip) and the batched
// work-list launch (kernels_batch.hip).  T is the integrand type.
#pragma once
#include <type_traits>

#include "bmd_internal.hpp"
#include "device_math.hpp"
#include "eval_core.hpp"

namespace bmd {

// What a sweep accumulates per design besides the sums of the summands: the
// second half of each slice's partials holds nothing (kSums), the sums of
// squares (kSquares) or the sums of the summands' derivatives in the first
// test's level alpha_1 (kDAlpha).
constexpr int kSums = 0, kSquares = 1, kDAlpha = 2;

template <typename T>
struct EvalArgs {
    DevProblem P;
    const double* r;
    const double* z1;
    const double* z2;
    const T* A;          // axis tables [d][K][mmax]
    DrawArrays<T> D;
    const double* gl;    // packed GL table (FP64 nodes)
    const T* glw;        // packed GL table in T (weights read from here)
    int64_t slice_len;
    double* partials;    // [n_slices][2][G]: sums, then the MODE's second sums
};

// Direct sweep, one workgroup's work: designs bx * 256 + thread (one per
// thread), draws of slice `slice`.  MODE: see kSums.
template <typename T, int D, int NMAX, int MODE>
__device__ __forceinline__ void direct_body(const EvalArgs<T>& a, int64_t bx, int slice) {
    const int64_t G = a.P.G;
    const int64_t g = bx * kEvalBlock + threadIdx.x;
    const bool valid = g < G;
    const int64_t gg = valid ? g : G - 1;   // idle lanes shadow the last design
    DesignState<T, D, NMAX> s;
    s.init(a.P, gg, a.r, a.z1, a.z2, a.gl, a.glw);
    if constexpr (MODE == kDAlpha) s.init_dalpha(a.P, a.r[gg], a.z1[gg], a.z2[gg]);
    const GlobalDraws<T> src{a.D, D};
    const int64_t M = a.D.M;
    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(M, kb + a.slice_len);
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = kb; k < ke; ++k) {
        if constexpr (MODE == kDAlpha) {
            T dv;
            s1 += static_cast<double>(summand<T, D, NMAX>(a.P, s, src, k, a.A, a.D.K, &dv));
            s2 += static_cast<double>(dv);
        } else {
            const double v = static_cast<double>(summand<T, D, NMAX>(a.P, s, src, k, a.A, a.D.K));
            s1 += v;
            if constexpr (MODE == kSquares) s2 = fma(v, v, s2);
        }
    }
    if (valid) {
        double* out = a.partials + static_cast<int64_t>(slice) * 2 * G;
        out[g] = s1;
        if constexpr (MODE != kSums) out[G + g] = s2;
    }
}

// Four values of one draw read with one LDS access.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T x, y, z, w;
};

// Bit pattern type of T, and a branch-free select of two values already read.
template <typename T>
using Bits = typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned int>::type;
__device__ __forceinline__ float bit_select(unsigned int m, float a, float b) {
    return __uint_as_float((__float_as_uint(a) & m) | (__float_as_uint(b) & ~m));
}
__device__ __forceinline__ double bit_select(unsigned long long m, double a, double b) {
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(__double_as_longlong(a)) & m) |
                                                      (static_cast<unsigned long long>(__double_as_longlong(b)) & ~m)));
}

// Copy n units of U bytes (U = 4 or 16) from global memory into LDS through
// the vector memory unit's load-to-LDS path: no registers are involved and
// completion is tracked by the wavefront's vmcnt.  Every wavefront of the
// workgroup calls it; wavefront w moves units 64 (w + 4 t) + lane.  src and dst
// are U-byte aligned; dst offsets are wave-uniform, as the instruction needs.
template <int U>
__device__ __forceinline__ void lds_dma(void* dst, const void* src, int n, int wave, int lane) {
    static_assert(U == 4 || U == 16, "unit of 4 or 16 bytes");
    char* d = static_cast<char*>(dst);
    const char* s = static_cast<const char*>(src);
    for (int r = wave * 64; r < n; r += kEvalBlock) {
        if (r + lane < n) {
            const void* g = s + static_cast<size_t>(U) * (r + lane);
            auto* l = (__attribute__((address_space(3))) void*)(d + static_cast<size_t>(U) * r);
            if constexpr (U == 16)
                __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
            else
                __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
        }
    }
}

typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mf_f4 mf_step(float a, float b, mf_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf_d4 mf_step(double a, double b, mf_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Tile geometry of the matrix-core sweep: designs g = p * Sn + l with prefix
// index p (axes < split) and suffix index l (axes >= split); a workgroup owns a
// 16 x 16 tile of (p, l) and a slice of draws.
struct MfmaGeom {
    int split;
    int64_t Pn, Sn;       // prefix and suffix counts
    int64_t tiles_l;      // tiles along the suffix index
    int chunk;            // draws staged per LDS chunk
};

// Sweep for grid designs with d >= 2, step prior, exact cutoff indicator.
// Phase A (matrix cores): for each draw of the chunk,
//   O[p][l] = sum_m Pre[p][m] Suf[l][m],
//   Pre[p][m] = prod_{j < split} v_j(p)[m],  Suf[l][m] = prod_{j >= split} v_j(l)[m],
//   v_j[m] = A_j[i_j][m] if the design's cutoff on axis j lies above the drawn one
//            (i_j >= thr_j(k)), else the draw's B_j[m]  (Gauss-Hermite weights in axis 0),
// i.e. the one-factor quadrature of P(x_j > max(c_j, t_j) all j) for all 256
// designs at once; each wavefront takes every fourth draw.
// Phase B (vector units): one design per thread, the bivariate normal part.
// One workgroup's work: tile `tile`, draws of slice `slice`; lds holds
// mfma_lds_bytes<T>(geo.chunk, D, K) bytes.  The body's first LDS copies are
// issued before its first barrier and its last phase B reads LDS after its
// last one, so a caller that runs another item on the same LDS must
// synchronise the workgroup in between.  MODE: see kSums.
template <typename T, int D, int NMAX, int MODE>
__device__ __forceinline__ void mfma_tile_body(const EvalArgs<T>& a, const MfmaGeom& geo, int64_t tile, int slice,
                                               char* lds) {
    using acc_t = typename std::conditional<sizeof(T) == 8, mf_d4, mf_f4>::type;
    const int K = a.D.K;   // a multiple of 4 (node steps of four)
    const int CH = geo.chunk;
    T* sO = reinterpret_cast<T*>(lds);                                  // [CH][256]
    T* sB = sO + static_cast<size_t>(CH) * kEvalBlock;                   // [CH][K][D]
    Quad<T>* sq0 = reinterpret_cast<Quad<T>*>(sB + static_cast<size_t>(CH) * D * K);  // 2 x [CH] (b0, b1, mu1, -)
    int* sthr = reinterpret_cast<int*>(sq0 + 2 * CH);                    // [CH][D]

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t p0 = (tile / geo.tiles_l) * 16, l0 = (tile % geo.tiles_l) * 16;
    const int64_t G = a.P.G;
    const int64_t M = a.D.M;
    const int mmax = a.P.mmax;

    // phase B design: row tid/16, column tid%16 of the tile
    const int64_t pB = p0 + tid / 16, lB = l0 + tid % 16;
    const bool validB = pB < geo.Pn && lB < geo.Sn;
    const int64_t g = validB ? pB * geo.Sn + lB : G - 1;
    DesignState<T, D, NMAX> st;
    st.init(a.P, g, a.r, a.z1, a.z2, a.gl, a.glw);
    if constexpr (MODE == kDAlpha) st.init_dalpha(a.P, a.r[g], a.z1[g], a.z2[g]);

    // phase A operands: lane supplies row (p0 + lane%16) of Pre and column
    // (l0 + lane%16) of Suf at node m0 + lane/16
    const int r16 = lane & 15, kq = lane >> 4;
    const int64_t pA = p0 + r16, lA = l0 + r16;
    const bool rowA = pA < geo.Pn, colA = lA < geo.Sn;   // else: shadow design 0's indices
    int iA[D];
    {
        int64_t rem = (rowA ? pA : 0) * geo.Sn + (colA ? lA : 0);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            iA[j] = static_cast<int>(rem / a.P.stride[j]);
            rem -= static_cast<int64_t>(iA[j]) * a.P.stride[j];
        }
    }

    // This lane's axis-table values (draw independent) for the first kHoist
    // node steps stay in registers (FP32; the FP64 kernel has none to spare);
    // the remaining steps read them from memory (cached: staging the tile's
    // values in LDS instead was measured 4% slower in FP64).
    constexpr int kHoist = sizeof(T) == 4 ? (D <= 3 ? 5 : 6) : 0;
    constexpr int kChains = sizeof(T) == 4 ? 2 : 1;   // draws per wavefront pass
    const int S = K / 4;
    T aH[kHoist > 0 ? kHoist : 1][D];
#pragma unroll
    for (int s = 0; s < kHoist; ++s) {
        const int m = 4 * s + kq;
#pragma unroll
        for (int j = 0; j < D; ++j)
            aH[s][j] = (s < S && m < K) ? a.A[(static_cast<int64_t>(j) * K + m) * mmax + iA[j]] : T(0);
    }
    // Gauss-Legendre weights of this wavefront's rule: scalar registers in FP32
    const auto wts = [&]() {
        if constexpr (sizeof(T) == 4) {
            BvnWeights<NMAX> w;
            w.load(st.w, st.n);
            return w;
        } else {
            return st.w;
        }
    }();

    const int64_t kb = static_cast<int64_t>(slice) * a.slice_len;
    const int64_t ke = min(M, kb + a.slice_len);
    // Stage draws [k0, k0 + nk): their B tables, thresholds and (b0, b1, mu1)
    // quads are contiguous in HBM and land in LDS by DMA.
    auto stage = [&](int64_t k0, int nk, Quad<T>* sq) {
        lds_dma<16>(sB, a.D.B + k0 * D * K, static_cast<int>(nk * D * K * sizeof(T) / 16), wave, lane);
        lds_dma<16>(sq, a.D.q4 + 4 * k0, static_cast<int>(nk * sizeof(Quad<T>) / 16), wave, lane);
        lds_dma<4>(sthr, a.D.thr + k0 * D, nk * D, wave, lane);
    };
    if (kb < ke) stage(kb, static_cast<int>(min<int64_t>(CH, ke - kb)), sq0);
    double s1 = 0.0, s2 = 0.0;
    int buf = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += CH, buf ^= 1) {
        const int nk = __builtin_amdgcn_readfirstlane(static_cast<int>(min<int64_t>(CH, ke - k0)));
        const Quad<T>* sq = sq0 + buf * CH;
        // this wavefront's copies of the chunk have landed; after the barrier
        // everyone's have, and phase B of the previous chunk is over (sO free)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        // phase A: overlaps of the tile; a wavefront takes kChains draws per
        // pass (draws wave + 4c + 4 kChains t), one independent MFMA chain each.
        // Rows or columns past the grid (p >= Pn, l >= Sn) feed only tile
        // entries that phase B never stores, so they need no masking.  The draw
        // indices are wave-uniform (scalar loop and addressing); a lane reads
        // node m = 4 s + kq of a staged draw at a fixed offset from its base.
        constexpr int kWaves = kEvalBlock / 64;
        auto phase_a = [&](auto split_c) {
            constexpr int SPLIT = decltype(split_c)::value;
            for (int i0 = wave; i0 < nk; i0 += kChains * kWaves) {
                int ic[kChains];
                Bits<T> msk[kChains][D];   // all ones: the design's axis-j cutoff is above the draw's
                const T* Bc[kChains];
                acc_t c[kChains];
#pragma unroll
                for (int q = 0; q < kChains; ++q) {
                    ic[q] = i0 + q * kWaves < nk ? i0 + q * kWaves : i0;
#pragma unroll
                    for (int j = 0; j < D; ++j) msk[q][j] = iA[j] >= sthr[ic[q] * D + j] ? ~Bits<T>(0) : Bits<T>(0);
                    Bc[q] = sB + (static_cast<size_t>(ic[q]) * K + kq) * D;
                    c[q] = acc_t{0, 0, 0, 0};
                }
                auto step = [&](int s, const T* av) {
#pragma unroll
                    for (int q = 0; q < kChains; ++q) {
                        T pre = T(1), suf = T(1);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            const T v = bit_select(msk[q][j], av[j], Bc[q][4 * s * D + j]);
                            if (j < SPLIT) pre *= v; else suf *= v;   // j, SPLIT: compile-time after unrolling
                        }
                        c[q] = mf_step(pre, suf, c[q]);
                    }
                };
#pragma unroll
                for (int s = 0; s < kHoist; ++s)
                    if (s < S) step(s, aH[s]);
                for (int s = kHoist; s < S; ++s) {
                    const int m = 4 * s + kq;
                    T av[D];
#pragma unroll
                    for (int j = 0; j < D; ++j) av[j] = a.A[(static_cast<int64_t>(j) * K + m) * mmax + iA[j]];
                    step(s, av);
                }
#pragma unroll
                for (int q = 0; q < kChains; ++q) {
                    if (q > 0 && i0 + q * kWaves >= nk) break;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        sO[static_cast<size_t>(ic[q]) * kEvalBlock + mfma16_row<T>(kq, v) * 16 + r16] = c[q][v];
                }
            }
        };
        switch (geo.split) {
            case 1: phase_a(std::integral_constant<int, 1>{}); break;
            case 2: if constexpr (D > 2) phase_a(std::integral_constant<int, 2>{}); break;
            case 3: if constexpr (D > 3) phase_a(std::integral_constant<int, 3>{}); break;
            case 4: if constexpr (D > 4) phase_a(std::integral_constant<int, 4>{}); break;
            default: if constexpr (D > 5) phase_a(std::integral_constant<int, 5>{}); break;
        }
        __syncthreads();
        // The next chunk's copies overlap phase B: sB and sthr are no longer
        // read, and its quads go to the other buffer.
        if (k0 + CH < ke) stage(k0 + CH, static_cast<int>(min<int64_t>(CH, ke - k0 - CH)), sq0 + (buf ^ 1) * CH);
        // phase B: bivariate normal part for this thread's design; with
        // kDAlpha also the summand's derivative in alpha_1 (dalpha_term)
        struct Val {
            T v, dv;
        };
        const auto summand = [&](int i) -> Val {
            const T O = sO[static_cast<size_t>(i) * kEvalBlock + tid];
            const Quad<T> dq = sq[i];
            if constexpr (sizeof(T) == 4) {
                // arguments times sqrt(log2(e)/2):  h = z1 - mu1,
                // k = z2 - sqrt(r I) (b0 + b1 O / r)
                const float h = fmaf(dq.z, -kPhiScale, st.z1s);
                const float kq2 = fmaf(-st.a1s, dq.y * O, fmaf(-st.a0s, dq.x, st.z2s));
                float dv = 0.0f;
                if constexpr (MODE == kDAlpha) {
                    // phi(x) = 2^(-x'^2) / sqrt(2 pi) at the prescaled x'
                    const float eh = __builtin_amdgcn_exp2f(-h * h);
                    if (a.P.zinf & 2) {
                        dv = st.da1 * eh;
                    } else {
                        const float ek = __builtin_amdgcn_exp2f(-kq2 * kq2);
                        const float ph = eh * norm_cdf_scaled(fmaf(kq2, st.is, -st.rs * h));
                        const float pk = ek * norm_cdf_scaled(fmaf(h, st.is, -st.rs * kq2));
                        dv = fmaf(st.da1, ph, st.da2 * pk);
                    }
                }
                if (a.P.zinf == 0) return {bvn_sf_scaled<NMAX>(h, kq2, st.bc, wts, st.n), dv};
                if (a.P.zinf == 1) return {1.0f - norm_cdf_scaled(kq2), dv};
                if (a.P.zinf == 2) return {1.0f - norm_cdf_scaled(h), dv};
                return {0.0f, dv};
            } else {
                const T mu2 = st.srI * (dq.x + dq.y * O * st.invr);
                const T h = st.z1 - dq.z, kq2 = st.z2 - mu2;
                T dv = T(0);
                if constexpr (MODE == kDAlpha) dv = dalpha_term<T, D, NMAX>(a.P, st, h, kq2);
                // 1 - P(both statistics below their critical values)
                if (a.P.zinf == 0) return {bvn_sf<NMAX>(h, kq2, st.bc, wts, st.n), dv};
                if (a.P.zinf == 1) return {T(1) - norm_cdf(kq2), dv};
                if (a.P.zinf == 2) return {T(1) - norm_cdf(h), dv};
                return {T(0), dv};
            }
        };
        int i = 0;
        for (; i + 1 < nk; i += 2) {
            const Val v0 = summand(i), v1 = summand(i + 1);
            if constexpr (sizeof(T) == 4 && MODE == kSums) {
                s1 += static_cast<double>(v0.v + v1.v);   // pairs of draws summed in FP32 first
            } else {
                s1 += static_cast<double>(v0.v);
                s1 += static_cast<double>(v1.v);
                if constexpr (MODE == kSquares) {
                    s2 = fma(static_cast<double>(v0.v), static_cast<double>(v0.v), s2);
                    s2 = fma(static_cast<double>(v1.v), static_cast<double>(v1.v), s2);
                } else if constexpr (MODE == kDAlpha) {
                    s2 += static_cast<double>(v0.dv);
                    s2 += static_cast<double>(v1.dv);
                }
            }
        }
        if (i < nk) {
            const Val w = summand(i);
            const double v = static_cast<double>(w.v);
            s1 += v;
            if constexpr (MODE == kSquares) s2 = fma(v, v, s2);
            if constexpr (MODE == kDAlpha) s2 += static_cast<double>(w.dv);
        }
    }
    if (validB) {
        double* out = a.partials + static_cast<int64_t>(slice) * 2 * G;
        out[g] = s1;
        if constexpr (MODE != kSums) out[G + g] = s2;
    }
}

// LDS bytes of the matrix-core body for a chunk of `chunk` draws.
template <typename T>
inline size_t mfma_lds_bytes(int chunk, int d, int K) {
    return sizeof(T) * static_cast<size_t>(chunk) * (kEvalBlock + static_cast<size_t>(d) * K + 8) +
           sizeof(int) * static_cast<size_t>(chunk) * d;
}

}  // namespace bmd
