// Thin-plate spline smoothing of a grid surface (Sec. 2.3: the Monte Carlo
// estimates are fitted by a thin-plate spline, whose maximum is then refined).
// The spline of order 2 in d = 1..3 dimensions,
//   f(u) = sum_i c_i phi(|u - u_i|) + a_0 + a^T u,
//   phi(r) = r^3 (d = 1), r^2 log r (d = 2), -r (d = 3),
// on the designs with a value, their coordinates in the grid's unit box
// (u_j = i_j / (m_j - 1)), with the coefficients of the smoothing system
//   (Phi + lam I) c + P a = y,   P^T c = 0,   P = [1, u].
// The polynomial block is eliminated with the QR factors of P: d + 1
// Householder reflectors give Q^T P = [R; 0]; with c = Q [0; w] the reduced
// matrix M22 of M = Q^T (Phi + lam I) Q is positive definite when the designs
// determine a plane, so w solves M22 w = z2 (z = Q^T y) by a blocked Cholesky
// factorisation, and R a = z1 - M12 w.  FP64 throughout.
#include <cmath>

#include "bmd_internal.hpp"

namespace bmd {

struct TpsFit {
    int64_t n = 0;              // centres
    int d = 0;
    double* mem = nullptr;      // device: U [n d], c [n], a [d + 1]
};

namespace {

constexpr int kNB = 32;          // Cholesky and triangular-solve block
constexpr int kUT = 64;          // trailing-update tile (kUT x kUT outputs per workgroup)

// The radial function for D dimensions, fixed at compile time: with the
// dimension chosen at run time inside one function, the gfx950 code of an
// earlier build skipped the -r branch for D = 3 and stored the unnegated
// square root (NaN at r = 0), so every kernel that evaluates phi is a
// template on D.
template <int D>
__device__ __forceinline__ double tps_phi(double r) {
    if constexpr (D == 1) return r * r * r;
    else if constexpr (D == 2) return r > 0.0 ? r * r * log(r) : 0.0;
    else return -r;
}

// Unit-box coordinates of grid design g.
__device__ __forceinline__ void unit_coords(const DevProblem& P, int64_t g, double* u) {
    int64_t rem = g;
    for (int j = 0; j < P.d; ++j) {
        const int64_t i = rem / P.stride[j];
        rem -= i * P.stride[j];
        u[j] = static_cast<double>(i) / static_cast<double>(P.m[j] - 1);
    }
}

// Lane src's value of v on every lane (src wave-uniform): two reads into
// scalar registers, no round trip through LDS as a shuffle takes.
__device__ __forceinline__ double lane_value(double v, int src) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffu), src));
    const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(u >> 32), src));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ double block_sum(double v, double* red) {
    const int t = threadIdx.x, nt = blockDim.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nt / 64; ++w) s += red[w];   // same order on every thread
    return s;
}

// Designs with a value, in index order (one workgroup of 1024: a scan per
// tile); their count goes to *n_out.
__global__ __launch_bounds__(1024) void k_tps_compact(int64_t G, const double* __restrict__ f,
                                                      int64_t* __restrict__ idx, int64_t* __restrict__ n_out) {
    __shared__ int scan[1024];
    const int t = threadIdx.x;
    int64_t base = 0;
    for (int64_t g0 = 0; g0 < G; g0 += 1024) {
        const int64_t g = g0 + t;
        const int ok = g < G && f[g] == f[g];
        scan[t] = ok;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int v = t >= off ? scan[t - off] : 0;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        if (ok) idx[base + scan[t] - 1] = g;
        base += scan[1023];
        __syncthreads();
    }
    if (t == 0) *n_out = base;
}

// Centres U [n d], values y [n] and the polynomial block P [n][d + 1].
__global__ void k_tps_points(DevProblem P, int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ f,
                             double* __restrict__ U, double* __restrict__ y, double* __restrict__ Pm) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double u[kMaxDim];
    unit_coords(P, idx[i], u);
    const int d = P.d;
    Pm[i * (d + 1)] = 1.0;
    for (int j = 0; j < d; ++j) {
        U[i * d + j] = u[j];
        Pm[i * (d + 1) + 1 + j] = u[j];
    }
    y[i] = f[idx[i]];
}

// A = Phi + lam I (n x n, row-major).
template <int D>
__global__ void k_tps_matrix(int64_t n, const double* __restrict__ U, double lam, double* __restrict__ A) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (k >= n) return;
    double r2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double s = U[i * D + j] - U[k * D + j];
        r2 = fma(s, s, r2);
    }
    A[i * n + k] = tps_phi<D>(sqrt(r2)) + (i == k ? lam : 0.0);
}

// Householder QR of P [n][d + 1] (one workgroup): reflector k is
// I - tau_k v_k v_k^T with v_k zero above row k; R [(d+1)^2] upper
// triangular.  A column whose remaining norm is below 1e-12 of its first
// norm raises *bad (the designs do not determine a plane).
__global__ __launch_bounds__(1024) void k_tps_qr(int64_t n, int d, double* __restrict__ Pm, double* __restrict__ V,
                                                 double* __restrict__ tau, double* __restrict__ R,
                                                 int* __restrict__ bad) {
    __shared__ double red[16];
    const int t = threadIdx.x;
    const int np = d + 1;
    for (int k = 0; k < np; ++k) {
        double s = 0.0, s0 = 0.0;
        for (int64_t i = t; i < n; i += blockDim.x) {
            const double x = Pm[i * np + k];
            s0 = fma(x, x, s0);
            if (i >= k) s = fma(x, x, s);
        }
        const double sigma2 = block_sum(s, red);
        const double full2 = block_sum(s0, red);
        const double xk = Pm[k * np + k];
        const double sigma = sqrt(sigma2);
        const double alpha = xk >= 0.0 ? -sigma : sigma;
        if (!(sigma > 1e-12 * sqrt(full2)) && t == 0) *bad = 1;
        const double vk = xk - alpha;
        const double vnorm2 = sigma2 - xk * xk + vk * vk;
        const double tk = vnorm2 > 0.0 ? 2.0 / vnorm2 : 0.0;
        for (int64_t i = t; i < n; i += blockDim.x) V[i * np + k] = i < k ? 0.0 : i == k ? vk : Pm[i * np + k];
        if (t == 0) {
            tau[k] = tk;
            R[k * np + k] = alpha;
        }
        __syncthreads();
        for (int j = k + 1; j < np; ++j) {
            double dj = 0.0;
            for (int64_t i = t + k; i < n; i += blockDim.x) dj = fma(V[i * np + k], Pm[i * np + j], dj);
            const double sj = block_sum(dj, red) * tk;
            for (int64_t i = t + k; i < n; i += blockDim.x) Pm[i * np + j] -= sj * V[i * np + k];
            __syncthreads();
            if (t == 0) R[k * np + j] = Pm[k * np + j];
        }
        if (t < k && t < np) R[k * np + t] = 0.0;
        __syncthreads();
    }
}

// p = tau_k A v_k, one workgroup per row.
__global__ __launch_bounds__(256) void k_tps_gemv(int64_t n, int np, int k, const double* __restrict__ A,
                                                  const double* __restrict__ V, const double* __restrict__ tau,
                                                  double* __restrict__ p) {
    __shared__ double red[4];
    const int64_t i = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x + k; j < n; j += blockDim.x) s = fma(A[i * n + j], V[j * np + k], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) p[i] = tau[k] * s;
}

// K = tau_k / 2 v_k^T p (one workgroup).
__global__ __launch_bounds__(1024) void k_tps_kappa(int64_t n, int np, int k, const double* __restrict__ V,
                                                    const double* __restrict__ tau, const double* __restrict__ p,
                                                    double* __restrict__ kappa) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x + k; i < n; i += blockDim.x) s = fma(V[i * np + k], p[i], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) *kappa = 0.5 * tau[k] * s;
}

// A <- H A H = A - v w^T - w v^T with w = p - K v.
__global__ void k_tps_rank2(int64_t n, int np, int k, const double* __restrict__ V, const double* __restrict__ p,
                            const double* __restrict__ kappa, double* __restrict__ A) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    const double K = *kappa;
    const double vi = V[i * np + k], vj = V[j * np + k];
    const double wi = p[i] - K * vi, wj = p[j] - K * vj;
    A[i * n + j] -= vi * wj + wi * vj;
}

// Panel slices are kPanelRows rows: thread t of a slice owns its row t.
constexpr int kPanelRows = 128;

// The bs x bs block at blk (row stride n) into L by NT threads: thread t
// takes column t % kNB of rows t / kNB + (NT / kNB) i, all loads in flight
// before the first LDS write.
template <int NT>
__device__ __forceinline__ void stage_block(const double* __restrict__ blk, int64_t n, int bs, double (*L)[kNB + 1]) {
    constexpr int kStep = NT / kNB, kIt = kNB / kStep;
    const int t = threadIdx.x, c = t % kNB, r = t / kNB;
    double v[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) v[i] = (r + kStep * i < bs && c < bs) ? blk[(r + kStep * i) * n + c] : 0.0;
#pragma unroll
    for (int i = 0; i < kIt; ++i) L[r + kStep * i][c] = v[i];
}

// Rows [0, nr) x columns [0, bs) of the slice at base (row stride n) into X:
// thread t takes column t % kNB of rows t / kNB + 4 i, every load issued
// before the first LDS write so the loads' latencies overlap.
__device__ __forceinline__ void stage_rows(const double* __restrict__ base, int64_t n, int nr, int bs,
                                           double (*X)[kNB + 1]) {
    static_assert(kPanelRows == 4 * kNB, "four rows per pass");
    const int t = threadIdx.x, c = t % kNB, r = t / kNB;
    double v[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i) v[i] = (r + 4 * i < nr && c < bs) ? base[(r + 4 * i) * n + c] : 0.0;
#pragma unroll
    for (int i = 0; i < kNB; ++i) X[r + 4 * i][c] = v[i];
}

// One step of the blocked Cholesky M22 = L L^T at block column kb: the kNB x
// kNB diagonal block, then the panel below it, L21 = A21 L11^-T.  Every
// workgroup factors the diagonal block itself in its first wavefront (lane r
// holds row r in registers; per column j every lane reads the pivot from lane
// j, lanes below scale their element of column j and update their rows with
// the other lanes' column-j elements, read from their lanes), so the step is
// one launch; A's diagonal block is only read, and workgroup 0 stores the
// factor in Ld (row stride kNB, zeros above the diagonal) for the triangular
// solves.  The panel's row segments go through LDS with consecutive lanes on
// consecutive columns (a thread walking its own row in memory would touch a
// different cache line per lane on every load).  A pivot <= 0 raises *bad.
__global__ __launch_bounds__(kPanelRows) void k_chol_step(int64_t n, int64_t o, int64_t kb, int bs, int64_t n2,
                                                          double* __restrict__ A, double* __restrict__ Ld,
                                                          int* __restrict__ bad) {
    __shared__ double L[kNB][kNB + 1];
    __shared__ double X[kPanelRows][kNB + 1];
    const int t = threadIdx.x;
    const int64_t r0 = kb + bs + static_cast<int64_t>(blockIdx.x) * kPanelRows;
    const int nr = static_cast<int>(max<int64_t>(0, min<int64_t>(kPanelRows, n2 - r0)));
    double* base = A + (o + r0) * n + o + kb;
    if (nr > 0) stage_rows(base, n, nr, bs, X);
    if (t < 64) {   // the first wavefront
        double row[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) row[c] = (t < bs && c <= t) ? A[(o + kb + t) * n + o + kb + c] : 0.0;
        bool neg = false;
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            if (j < bs) {   // wave-uniform
                const double pv = lane_value(row[j], j);
                neg |= !(pv > 0.0);
                const double dj = pv > 0.0 ? sqrt(pv) : 1.0;
                const double lrj = (t > j) ? row[j] / dj : (t == j ? dj : row[j]);
                row[j] = lrj;
#pragma unroll
                for (int c = j + 1; c < kNB; ++c) {
                    const double lcj = lane_value(lrj, c);   // column j of row c
                    if (t >= c) row[c] -= lrj * lcj;
                }
            }
        }
        if (t < kNB) {
#pragma unroll
            for (int c = 0; c < kNB; ++c) L[t][c] = c <= t ? row[c] : 0.0;
        }
        if (blockIdx.x == 0 && t == 0 && neg) *bad = 1;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        double* ld = Ld + kb * kNB;
        for (int e = t; e < kNB * kNB; e += kPanelRows) ld[e] = L[e / kNB][e % kNB];
    }
    if (nr == 0) return;   // workgroup-uniform
    if (t < nr) {
        double x[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) {
            if (c < bs) {
                double s = X[t][c];
#pragma unroll
                for (int e = 0; e < kNB; ++e)
                    if (e < c) s -= x[e] * L[c][e];
                x[c] = s / L[c][c];
            }
        }
#pragma unroll
        for (int c = 0; c < kNB; ++c)
            if (c < bs) X[t][c] = x[c];
    }
    __syncthreads();
    const int c = t % kNB, r = t / kNB;
#pragma unroll
    for (int i = 0; i < kNB; ++i)
        if (r + 4 * i < nr && c < bs) base[(r + 4 * i) * n + c] = X[r + 4 * i][c];
}

// Trailing update A22 -= L21 L21^T on the lower triangle, kUT x kUT output
// tiles on the matrix cores (FP64 16x16x4): four wavefronts, each a 32 x 32
// quarter as 2 x 2 blocks of 16 x 16; the tile's rows of L21 (both factors)
// staged in LDS; one workgroup per tile on or below the diagonal.  Operand layout of the
// instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its
// result element v is row l / 16 + 4 v, column l % 16.
typedef double tps_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_chol_update(int64_t n, int64_t o, int64_t kb, int bs, int64_t n2,
                                                     double* __restrict__ A) {
    const int64_t t0 = kb + bs;
    // workgroup b -> lower-triangle tile (ti, tk), tk <= ti, b = ti (ti + 1) / 2 + tk
    const int64_t b = blockIdx.x;
    int64_t ti = static_cast<int64_t>((sqrt(8.0 * static_cast<double>(b) + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > b) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    const int64_t tk = b - ti * (ti + 1) / 2;
    __shared__ double Li[kUT][kNB + 1], Lk[kUT][kNB + 1];
    const int t = threadIdx.x;
    const int64_t i0 = t0 + ti * kUT, k0 = t0 + tk * kUT;
    {   // thread t takes column t % kNB of rows t / kNB + 8 q; every load issued before the first LDS write
        constexpr int kIt = kUT * kNB / 256;
        const int c = t % kNB, r = t / kNB;
        double vi[kIt], vk[kIt];
#pragma unroll
        for (int q = 0; q < kIt; ++q) {
            const int rr = r + 8 * q;
            vi[q] = (i0 + rr < n2 && c < bs) ? A[(o + i0 + rr) * n + o + kb + c] : 0.0;
            vk[q] = (k0 + rr < n2 && c < bs) ? A[(o + k0 + rr) * n + o + kb + c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kIt; ++q) {
            Li[r + 8 * q][c] = vi[q];
            Lk[r + 8 * q][c] = vk[q];
        }
    }
    __syncthreads();
    const int wave = t >> 6, lane = t & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int rb = (wave >> 1) * 32, cb = (wave & 1) * 32;
    tps_d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = tps_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c0 = 0; c0 < kNB; c0 += 4) {
        const double x0 = Li[rb + r16][c0 + kq], x1 = Li[rb + 16 + r16][c0 + kq];
        const double y0 = Lk[cb + r16][c0 + kq], y1 = Lk[cb + 16 + r16][c0 + kq];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + rb + 16 * a + kq + 4 * v, k = k0 + cb + 16 * b + r16;
                if (i < n2 && k <= i) A[(o + i) * n + o + k] -= acc[a][b][v];
            }
}

// z = Q^T y = H_d ... H_0 y (one workgroup).
__global__ __launch_bounds__(1024) void k_tps_qty(int64_t n, int np, const double* __restrict__ V,
                                                  const double* __restrict__ tau, const double* __restrict__ y,
                                                  double* __restrict__ z) {
    __shared__ double red[16];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) z[i] = y[i];
    __syncthreads();
    for (int k = 0; k < np; ++k) {
        double s = 0.0;
        for (int64_t i = threadIdx.x + k; i < n; i += blockDim.x) s = fma(V[i * np + k], z[i], s);
        s = block_sum(s, red) * tau[k];
        for (int64_t i = threadIdx.x + k; i < n; i += blockDim.x) z[i] -= s * V[i * np + k];
        __syncthreads();
    }
}

// One block of kNB rows of M22 w = z2 with M22 = L L^T, forward (L t = z2)
// or backward (L^T w = t): every workgroup solves the block's own rows in its
// first wavefront from the factor in Ld (lane l holds element l; per row r
// the solved value is read from lane r and subtracted from the lanes below
// it, or above it for L^T), workgroup 0 stores them in out, and each
// workgroup updates its slice of the remaining rows of in: forward the rows
// below, b[r] -= L[r][kb..] x (row segments through LDS as in the Cholesky
// step), backward the rows above, b[r] -= L[kb..][r]^T x (consecutive
// threads on consecutive elements).  The block's own elements of in are only
// read, so no workgroup sees another's results within a launch.
__global__ __launch_bounds__(kPanelRows) void k_trsv_step(int64_t n, int64_t o, int64_t kb, int bs, int64_t n2,
                                                          bool upper, const double* __restrict__ A,
                                                          const double* __restrict__ Ld, double* __restrict__ in,
                                                          double* __restrict__ out) {
    __shared__ double Lb[kNB][kNB + 1];
    __shared__ double X[kPanelRows][kNB + 1];
    __shared__ double xb[kNB];
    const int t = threadIdx.x;
    stage_block<kPanelRows>(Ld + kb * kNB, kNB, bs, Lb);
    int64_t r0 = 0;
    int nr = 0;
    if (!upper) {
        r0 = kb + bs + static_cast<int64_t>(blockIdx.x) * kPanelRows;
        nr = static_cast<int>(max<int64_t>(0, min<int64_t>(kPanelRows, n2 - r0)));
        if (nr > 0) stage_rows(A + (o + r0) * n + o + kb, n, nr, bs, X);
    }
    __syncthreads();
    if (t < 64) {   // the first wavefront
        double x = t < bs ? in[kb + t] : 0.0;
        if (!upper) {
            for (int r = 0; r < bs; ++r) {
                const double xr = lane_value(x, r) / Lb[r][r];
                if (t == r) x = xr;
                if (t > r && t < bs) x -= Lb[t][r] * xr;
            }
        } else {
            for (int r = bs - 1; r >= 0; --r) {
                const double xr = lane_value(x, r) / Lb[r][r];
                if (t == r) x = xr;
                if (t < r) x -= Lb[r][t] * xr;
            }
        }
        if (t < bs) {
            xb[t] = x;
            if (blockIdx.x == 0) out[kb + t] = x;
        }
    }
    __syncthreads();
    double s = 0.0;
    if (!upper) {
        if (t < nr) {
            for (int c = 0; c < bs; ++c) s = fma(X[t][c], xb[c], s);
            in[r0 + t] -= s;
        }
    } else {
        const int64_t r = static_cast<int64_t>(blockIdx.x) * kPanelRows + t;
        if (r < kb) {
            for (int c = 0; c < bs; ++c) s = fma(A[(o + kb + c) * n + o + r], xb[c], s);
            in[r] -= s;
        }
    }
}

// c = Q [0; w] = H_0 ... H_d [0; w] and R a = z1 - M12 w; writes c and a into
// the fit (one workgroup).
__global__ __launch_bounds__(1024) void k_tps_coeffs(int64_t n, int np, const double* __restrict__ A,
                                                     const double* __restrict__ V, const double* __restrict__ tau,
                                                     const double* __restrict__ R, const double* __restrict__ z,
                                                     double* __restrict__ c, double* __restrict__ a) {
    __shared__ double red[16];
    __shared__ double rhs[kMaxDim + 1];
    const int t = threadIdx.x;
    for (int k = 0; k < np; ++k) {   // z1_k - sum_j M[k][np + j] w_j
        double s = 0.0;
        for (int64_t j = np + t; j < n; j += blockDim.x) s = fma(A[k * n + j], z[j], s);
        s = block_sum(s, red);
        if (t == 0) rhs[k] = z[k] - s;
    }
    for (int64_t i = t; i < n; i += blockDim.x) c[i] = i < np ? 0.0 : z[i];
    __syncthreads();
    for (int k = np - 1; k >= 0; --k) {
        double s = 0.0;
        for (int64_t i = t + k; i < n; i += blockDim.x) s = fma(V[i * np + k], c[i], s);
        s = block_sum(s, red) * tau[k];
        for (int64_t i = t + k; i < n; i += blockDim.x) c[i] -= s * V[i * np + k];
        __syncthreads();
    }
    if (t == 0) {
        for (int k = np - 1; k >= 0; --k) {
            double s = rhs[k];
            for (int j = k + 1; j < np; ++j) s -= R[k * np + j] * a[j];
            a[k] = s / R[k * np + k];
        }
    }
}

// The fitted surface at every grid design (NaN where f has no value), one
// wavefront per design: the lanes take every 64th centre, a butterfly sums.
template <int D>
__global__ __launch_bounds__(256) void k_tps_eval_grid(DevProblem P, int64_t n, const double* __restrict__ U,
                                                       const double* __restrict__ c, const double* __restrict__ a,
                                                       const double* __restrict__ f, double* __restrict__ out) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= P.G) return;   // wave-uniform
    if (f[g] != f[g]) {
        if (lane == 0) out[g] = f[g];
        return;
    }
    double u[kMaxDim];
    unit_coords(P, g, u);
    double v = 0.0;
    for (int64_t i = lane; i < n; i += 64) {
        double r2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double s = u[j] - U[i * D + j];
            r2 = fma(s, s, r2);
        }
        v = fma(c[i], tps_phi<D>(sqrt(r2)), v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) {
        double poly = a[0];
#pragma unroll
        for (int j = 0; j < D; ++j) poly = fma(a[1 + j], u[j], poly);
        out[g] = poly + v;
    }
}

// Value, gradient and Hessian in unit coordinates at u (one workgroup):
// out = [value, grad (d), Hessian rows j <= l (d (d + 1) / 2)].  At a centre
// its own term adds no derivative (r^2 log r's Hessian diverges there, -r has
// a kink).
template <int D>
__global__ __launch_bounds__(1024) void k_tps_at(int64_t n, const double* __restrict__ U, const double* __restrict__ c,
                                                 const double* __restrict__ a, double u0, double u1, double u2,
                                                 double* __restrict__ out) {
    constexpr int NA = 1 + D + D * (D + 1) / 2;
    __shared__ double red[16];
    const double u[3] = {u0, u1, u2};
    double acc[NA] = {};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double s[D], r2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            s[j] = u[j] - U[i * D + j];
            r2 = fma(s[j], s[j], r2);
        }
        const double r = sqrt(r2);
        acc[0] = fma(c[i], tps_phi<D>(r), acc[0]);
        if (r == 0.0) continue;
        double p1, p2;   // phi'(r), phi''(r)
        if constexpr (D == 1) {
            p1 = 3.0 * r * r;
            p2 = 6.0 * r;
        } else if constexpr (D == 2) {
            p1 = r * (2.0 * log(r) + 1.0);
            p2 = 2.0 * log(r) + 3.0;
        } else {
            p1 = -1.0;
            p2 = 0.0;
        }
        const double g1 = c[i] * p1 / r, g2 = c[i] * (p2 - p1 / r) / r2;
        int k = 1 + D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            acc[1 + j] = fma(g1, s[j], acc[1 + j]);
#pragma unroll
            for (int l = j; l < D; ++l, ++k) acc[k] += g2 * s[j] * s[l] + (j == l ? g1 : 0.0);
        }
    }
    double poly = a[0];
#pragma unroll
    for (int j = 0; j < D; ++j) poly = fma(a[1 + j], u[j], poly);
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const double v = block_sum(acc[q], red);
        if (threadIdx.x == 0) out[q] = v + (q == 0 ? poly : q <= D ? a[q] : 0.0);
        __syncthreads();
    }
}

}  // namespace

void tps_release(bmd_problem* p) {
    if (!p || !p->tps) return;
    if (p->tps->mem) (void)hipFree(p->tps->mem);
    delete p->tps;
    p->tps = nullptr;
}

#define TPS_TRY(expr)                \
    do {                             \
        res.err = (expr);            \
        if (res.err != hipSuccess) { \
            res.code = kTpsHip;      \
            goto done;               \
        }                            \
    } while (0)

TpsFitResult tps_fit_grid(bmd_problem* p, const double* d_in, double lam, double* d_out, hipStream_t s) {
    const DevProblem& P = p->P;
    const int d = P.d, np = d + 1;
    const int64_t G = P.G;
    TpsFitResult res{kTpsOk, 0, hipSuccess};
    int64_t n = 0, n2 = 0, o = 0;
    int bad = 0;
    char* small = nullptr;   // idx [G], n, bad flag; tau, R, kappa
    double* big = nullptr;   // A [n n], V and P [n (d + 1)], y, z, p [n]
    double* fitmem = nullptr;
    int64_t* d_idx = nullptr;
    int64_t* d_n = nullptr;
    int* d_bad = nullptr;
    double *d_tau = nullptr, *d_R = nullptr, *d_kappa = nullptr;
    double *A = nullptr, *V = nullptr, *Pm = nullptr, *y = nullptr, *z = nullptr, *pv = nullptr;
    double *Ld = nullptr, *T = nullptr;   // diagonal blocks of the factor; the forward solve's result
    double *U = nullptr, *c = nullptr, *a = nullptr;
    const size_t small_bytes = sizeof(int64_t) * (G + 2) + 64 + sizeof(double) * (2 * np + np * np + 8);
    if (hipMalloc(&small, small_bytes) != hipSuccess) {
        (void)hipGetLastError();
        res.code = kTpsNoMem;
        return res;
    }
    d_idx = reinterpret_cast<int64_t*>(small);
    d_n = d_idx + G;
    d_bad = reinterpret_cast<int*>(d_n + 1);
    d_tau = reinterpret_cast<double*>(small + sizeof(int64_t) * (G + 2) + 64);
    d_R = d_tau + np;
    d_kappa = d_R + np * np;
    TPS_TRY(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_tps_compact, dim3(1), dim3(1024), 0, s, G, d_in, d_idx, d_n);
    TPS_TRY(hipGetLastError());
    TPS_TRY(hipMemcpyAsync(&n, d_n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    TPS_TRY(hipStreamSynchronize(s));
    res.n = n;
    if (n < d + 2 || n > kTpsMaxPoints) {
        res.code = kTpsCount;
        goto done;
    }
    {
        const size_t nn = static_cast<size_t>(n);
        const size_t big_count = nn * nn + 2 * nn * np + 4 * nn + kNB * (nn + kNB);
        if (hipMalloc(&big, sizeof(double) * big_count) != hipSuccess ||
            hipMalloc(&fitmem, sizeof(double) * (nn * d + nn + np)) != hipSuccess) {
            (void)hipGetLastError();
            res.code = kTpsNoMem;
            goto done;
        }
        A = big;
        V = A + nn * nn;
        Pm = V + nn * np;
        y = Pm + nn * np;
        z = y + nn;
        pv = z + nn;
        Ld = pv + nn;
        T = Ld + kNB * (nn + kNB);
        U = fitmem;
        c = U + nn * d;
        a = c + nn;
    }
    hipLaunchKernelGGL(k_tps_points, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, P, n, d_idx, d_in,
                       U, y, Pm);
    TPS_TRY(hipGetLastError());
    {
        const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n));
        if (d == 1) hipLaunchKernelGGL(k_tps_matrix<1>, grid, dim3(256), 0, s, n, U, lam, A);
        else if (d == 2) hipLaunchKernelGGL(k_tps_matrix<2>, grid, dim3(256), 0, s, n, U, lam, A);
        else hipLaunchKernelGGL(k_tps_matrix<3>, grid, dim3(256), 0, s, n, U, lam, A);
    }
    TPS_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_tps_qr, dim3(1), dim3(1024), 0, s, n, d, Pm, V, d_tau, d_R, d_bad);
    TPS_TRY(hipGetLastError());
    for (int k = 0; k < np; ++k) {   // M = Q^T A Q, one reflector at a time from both sides
        hipLaunchKernelGGL(k_tps_gemv, dim3(static_cast<unsigned>(n)), dim3(256), 0, s, n, np, k, A, V, d_tau, pv);
        hipLaunchKernelGGL(k_tps_kappa, dim3(1), dim3(1024), 0, s, n, np, k, V, d_tau, pv, d_kappa);
        hipLaunchKernelGGL(k_tps_rank2, dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n)),
                           dim3(256), 0, s, n, np, k, V, pv, d_kappa, A);
        TPS_TRY(hipGetLastError());
    }
    o = np;
    n2 = n - np;
    for (int64_t kb = 0; kb < n2; kb += kNB) {   // M22 = L L^T
        const int bs = static_cast<int>(std::min<int64_t>(kNB, n2 - kb));
        const int64_t rest = n2 - kb - bs;
        hipLaunchKernelGGL(k_chol_step, dim3(static_cast<unsigned>(std::max<int64_t>(1, (rest + kPanelRows - 1) / kPanelRows))),
                           dim3(kPanelRows), 0, s, n, o, kb, bs, n2, A, Ld, d_bad);
        if (rest > 0) {
            const int64_t tiles = (rest + kUT - 1) / kUT;
            hipLaunchKernelGGL(k_chol_update, dim3(static_cast<unsigned>(tiles * (tiles + 1) / 2)), dim3(256), 0, s, n,
                               o, kb, bs, n2, A);
        }
        TPS_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_tps_qty, dim3(1), dim3(1024), 0, s, n, np, V, d_tau, y, z);
    for (int64_t kb = 0; kb < n2; kb += kNB) {   // L t = z2: z2 = z [o, n) in, t out
        const int bs = static_cast<int>(std::min<int64_t>(kNB, n2 - kb));
        const int64_t rest = n2 - kb - bs;
        hipLaunchKernelGGL(k_trsv_step, dim3(static_cast<unsigned>(std::max<int64_t>(1, (rest + kPanelRows - 1) / kPanelRows))),
                           dim3(kPanelRows), 0, s, n, o, kb, bs, n2, false, A, Ld, z + o, T);
    }
    for (int64_t kb = ((n2 - 1) / kNB) * kNB; kb >= 0; kb -= kNB) {   // L^T w = t: t in, w out to z [o, n)
        const int bs = static_cast<int>(std::min<int64_t>(kNB, n2 - kb));
        hipLaunchKernelGGL(k_trsv_step, dim3(static_cast<unsigned>(std::max<int64_t>(1, (kb + kPanelRows - 1) / kPanelRows))),
                           dim3(kPanelRows), 0, s, n, o, kb, bs, n2, true, A, Ld, T, z + o);
    }
    hipLaunchKernelGGL(k_tps_coeffs, dim3(1), dim3(1024), 0, s, n, np, A, V, d_tau, d_R, z, c, a);
    TPS_TRY(hipGetLastError());
    TPS_TRY(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    TPS_TRY(hipStreamSynchronize(s));
    if (bad) {
        res.code = kTpsSingular;
        goto done;
    }
    if (d_out) {
        const dim3 grid(static_cast<unsigned>((G + 3) / 4));
        if (d == 1) hipLaunchKernelGGL(k_tps_eval_grid<1>, grid, dim3(256), 0, s, P, n, U, c, a, d_in, d_out);
        else if (d == 2) hipLaunchKernelGGL(k_tps_eval_grid<2>, grid, dim3(256), 0, s, P, n, U, c, a, d_in, d_out);
        else hipLaunchKernelGGL(k_tps_eval_grid<3>, grid, dim3(256), 0, s, P, n, U, c, a, d_in, d_out);
        TPS_TRY(hipGetLastError());
    }
    TPS_TRY(hipStreamSynchronize(s));
    tps_release(p);
    p->tps = new TpsFit;
    p->tps->n = n;
    p->tps->d = d;
    p->tps->mem = fitmem;
    fitmem = nullptr;
done:
    (void)hipStreamSynchronize(s);
    if (fitmem) (void)hipFree(fitmem);
    if (big) (void)hipFree(big);
    (void)hipFree(small);
    return res;
}

hipError_t tps_at_unit(const bmd_problem* p, const double* u, double* d_scratch, double* h_out, hipStream_t s) {
    const TpsFit& F = *p->tps;
    const int d = F.d;
    const double* U = F.mem;
    const double* c = U + F.n * d;
    const double* a = c + F.n;
    const double u1 = d > 1 ? u[1] : 0.0, u2 = d > 2 ? u[2] : 0.0;
    if (d == 1) hipLaunchKernelGGL(k_tps_at<1>, dim3(1), dim3(1024), 0, s, F.n, U, c, a, u[0], u1, u2, d_scratch);
    else if (d == 2) hipLaunchKernelGGL(k_tps_at<2>, dim3(1), dim3(1024), 0, s, F.n, U, c, a, u[0], u1, u2, d_scratch);
    else hipLaunchKernelGGL(k_tps_at<3>, dim3(1), dim3(1024), 0, s, F.n, U, c, a, u[0], u1, u2, d_scratch);
    hipError_t e = hipGetLastError();
    const int na = 1 + d + d * (d + 1) / 2;
    if (e == hipSuccess) e = hipMemcpyAsync(h_out, d_scratch, sizeof(double) * na, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

int tps_dims(const bmd_problem* p) { return p->tps ? p->tps->d : 0; }

}  // namespace bmd
