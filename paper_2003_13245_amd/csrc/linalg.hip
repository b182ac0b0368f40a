// Dense factorizations on the device, float64 complex, split planes.
//
//  * qr_chol / lq_chol: shifted CholeskyQR in three passes for the gauge
//    moves of the sweep (full-rank tall/wide blocks).  Every pass is a Gram
//    GEMM, a one-workgroup Cholesky and triangular inverse (held in
//    registers for n <= 128) and an update GEMM; the R factors multiply to an
//    upper factor with a real positive diagonal, i.e. the unique QR of a
//    full-rank matrix.
//  * qr_householder: blocked Householder QR (compact WY) for matrices of any
//    rank; used by the compressions, where MPO x MPS products are rank
//    deficient.  Column-major working copy; panel columns are reflected with
//    small reduction kernels, trailing columns with GEMMs.
//  * svd_jacobi: one-sided (Hestenes) Jacobi with a round-robin pairing, one
//    cooperative launch per sweep with a grid barrier between rounds, every
//    column pair on its own wavefront.
#include <hip/hip_cooperative_groups.h>

#include "common.h"

#include <algorithm>
#include <cfloat>
#include <numeric>

namespace ftd {

static dim3 grid1(int64_t n, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65535 * 4) b = 65535 * 4;
    return dim3((unsigned)b);
}

__device__ __forceinline__ double bsum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------- small dense
// Upper Cholesky of a Hermitian n x n matrix (row-major planar, in place):
// G = U^H U.  Optionally adds shift*I first.  flag[0] = 1 on breakdown.
__global__ __launch_bounds__(1024) void chol_kernel(double* G, int n, int64_t plane,
                                                    const double* shift, int* flag) {
    __shared__ double piv;
    const double s = shift ? shift[0] : 0.0;
    if (s != 0.0)
        for (int i = threadIdx.x; i < n; i += blockDim.x) G[(int64_t)i * n + i] += s;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) {
            const double dk = G[(int64_t)k * n + k];
            if (!(dk > 0.0) || !isfinite(dk)) {
                flag[0] = 1;
                piv = 1.0;
            } else {
                piv = sqrt(dk);
            }
        }
        __syncthreads();
        const double p = piv;
        // row k: U[k][j] = G[k][j] / p for j > k
        for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) {
            G[(int64_t)k * n + j] /= p;
            G[(int64_t)k * n + j + plane] /= p;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            G[(int64_t)k * n + k] = p;
            G[(int64_t)k * n + k + plane] = 0.0;
        }
        // trailing: G[i][j] -= conj(U[k][i]) U[k][j], i > k, j >= i
        const int m = n - k - 1;
        const int64_t tot = (int64_t)m * m;
        for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
            const int i = k + 1 + (int)(e / m), j = k + 1 + (int)(e % m);
            if (j < i) continue;
            const double ar = G[(int64_t)k * n + i], ai = -G[(int64_t)k * n + i + plane];
            const double br = G[(int64_t)k * n + j], bi = G[(int64_t)k * n + j + plane];
            G[(int64_t)i * n + j] -= ar * br - ai * bi;
            G[(int64_t)i * n + j + plane] -= ar * bi + ai * br;
        }
        __syncthreads();
    }
    // clear the strictly lower part
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        if (j < i) {
            G[e] = 0.0;
            G[e + plane] = 0.0;
        }
    }
}

// Inverse of an upper-triangular U (row-major planar) into X; each thread
// owns one column of X and back-substitutes.
__global__ void set_int_kernel(int* p, int v) { *p = v; }

// Cholesky factor and its inverse for small n, in LDS (one workgroup).  The
// upper triangle of the Hermitian G (row-major n x n, planar) is packed into
// LDS (row i starts at i*n - i*(i-1)/2); the kernel adds the optional shift
// to the diagonal, factors G = R^H R in place (R upper, real positive
// diagonal), writes R over G (zeros below the diagonal), inverts R in place
// and writes R^{-1} to X.  A non-positive pivot sets *flag (sticky).
constexpr int kCholThreads = 256;
__device__ __forceinline__ int pk(int i, int j, int n) { return i * n - (i * (i - 1)) / 2 + (j - i); }

// G = I + E (the later CholeskyQR passes): the factor R = I + S, S = strict
// upper part of E plus half its diagonal, and R^{-1} = I - S are exact up to
// S^H S and S^2, whose entries are below n max|E|^2; taken when that bound is
// under 1e-17 (below rounding).  Returns true when it wrote G and X.  Any
// block size up to 1024; red holds one double per wavefront.
__device__ bool chol_near_identity(double* G, double* X, int n, int64_t plane, int* converged,
                                   double* red) {
    const int tid = threadIdx.x, nt = blockDim.x, nn = n * n;
    double mx = 0.0;
    for (int base = 0; base < nn; base += 4 * nt) {
        double vr[4], vi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + u * nt + tid;
            vr[u] = e < nn ? G[e] : 0.0;
            vi[u] = e < nn ? G[e + plane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + u * nt + tid;
            if (e < nn) {
                const int i = e / n, j = e - i * n;
                mx = fmax(mx, fmax(fabs(vr[u] - ((i == j) ? 1.0 : 0.0)), fabs(vi[u])));
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < nt / 64; ++w) m = fmax(m, red[w]);
    if ((double)n * m * m > 1e-17) return false;
    // Q was already orthonormal to 1e-9: the next pass could only move it at
    // the rounding level
    if (converged && tid == 0 && m <= 1e-9) converged[0] = 1;
    for (int e = tid; e < nn; e += nt) {
        const int i = e / n, j = e - i * n;
        double sr = 0.0, si = 0.0;
        if (j > i) {
            sr = G[e];
            si = G[e + plane];
        } else if (j == i) {
            sr = 0.5 * (G[e] - 1.0);
        }
        G[e] = ((i == j) ? 1.0 : 0.0) + sr;
        G[e + plane] = si;
        X[e] = ((i == j) ? 1.0 : 0.0) - sr;
        X[e + plane] = -si;
    }
    return true;
}

// upper triangle of G (+ shift on the diagonal, real diagonal) into packed
// LDS; four elements per thread in flight
__device__ void chol_pack(const double* G, int n, int64_t plane, double s, double* Pr, double* Pi) {
    const int tid = threadIdx.x, nt = blockDim.x, nn = n * n;
    for (int base = 0; base < nn; base += 4 * nt) {
        double vr[4], vi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + u * nt + tid;
            vr[u] = e < nn ? G[e] : 0.0;
            vi[u] = e < nn ? G[e + plane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = base + u * nt + tid;
            if (e < nn) {
                const int i = e / n, j = e - i * n;
                if (j >= i) {
                    Pr[pk(i, j, n)] = vr[u] + ((i == j) ? s : 0.0);
                    Pi[pk(i, j, n)] = (i == j) ? 0.0 : vi[u];
                }
            }
        }
    }
}

__global__ __launch_bounds__(kCholThreads) void chol_inv_lds_kernel(double* G, double* X, int n,
                                                                    int64_t plane,
                                                                    const double* shift,
                                                                    int* flag, const int* stop,
                                                                    int* converged) {
    if (stop && *stop) return;
    extern __shared__ double lds[];
    const int T = n * (n + 1) / 2;
    double* Pr = lds;
    double* Pi = lds + T;
    __shared__ double piv;
    __shared__ double red[kCholThreads / 64];
    const int tid = threadIdx.x;
    const double s = shift ? shift[0] : 0.0;
    if (!shift && chol_near_identity(G, X, n, plane, converged, red)) return;
    chol_pack(G, n, plane, s, Pr, Pi);
    __syncthreads();
    // 256 threads as 8 rows x 32 columns for the trailing updates
    const int ty = tid >> 5, tx = tid & 31;
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            const double dk = Pr[pk(k, k, n)];
            if (!(dk > 0.0) || !isfinite(dk)) {
                flag[0] = 1;
                piv = 1.0;
            } else {
                piv = sqrt(dk);
            }
            Pr[pk(k, k, n)] = piv;
            // the trailing updates leave a rounding-level imaginary part here
            Pi[pk(k, k, n)] = 0.0;
        }
        __syncthreads();
        const double inv = 1.0 / piv;
        const int rk = pk(k, k, n);
        for (int j = k + 1 + tid; j < n; j += kCholThreads) {
            Pr[rk + (j - k)] *= inv;
            Pi[rk + (j - k)] *= inv;
        }
        __syncthreads();
        // G[i][j] -= conj(R[k][i]) R[k][j] for k < i <= j
        for (int i = k + 1 + ty; i < n; i += 8) {
            const double ar = Pr[rk + (i - k)], ai = -Pi[rk + (i - k)];
            const int ri = pk(i, i, n);
            for (int j = i + tx; j < n; j += 32) {
                const double br = Pr[rk + (j - k)], bi = Pi[rk + (j - k)];
                Pr[ri + (j - i)] -= ar * br - ai * bi;
                Pi[ri + (j - i)] -= ar * bi + ai * br;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += kCholThreads) {
        const int i = e / n, j = e - i * n;
        G[e] = (j >= i) ? Pr[pk(i, j, n)] : 0.0;
        G[e + plane] = (j >= i) ? Pi[pk(i, j, n)] : 0.0;
    }
    __syncthreads();
    // in-place inverse, column by column: X[j][j] = 1/R[j][j],
    // X[i][j] = -(sum_{k=i}^{j-1} X[i][k] R[k][j]) / R[j][j] for i < j, where
    // columns < j already hold X and column j still holds R
    for (int j = 0; j < n; ++j) {
        const double rjj = Pr[pk(j, j, n)];
        // one row per thread group of 4 lanes
        const int g = tid >> 2, l = tid & 3;
        double tr[1], ti[1];
        for (int i0 = 0; i0 < j; i0 += kCholThreads / 4) {
            const int i = i0 + g;
            double sr = 0.0, si = 0.0;
            if (i < j) {
                for (int k = i + l; k < j; k += 4) {
                    const double xr = Pr[pk(i, k, n)], xi = Pi[pk(i, k, n)];
                    const double rr = Pr[pk(k, j, n)], ri = Pi[pk(k, j, n)];
                    sr += xr * rr - xi * ri;
                    si += xr * ri + xi * rr;
                }
            }
            sr += __shfl_xor(sr, 1, 64);
            si += __shfl_xor(si, 1, 64);
            sr += __shfl_xor(sr, 2, 64);
            si += __shfl_xor(si, 2, 64);
            tr[0] = sr;
            ti[0] = si;
            __syncthreads();   // all reads of column j done before it is overwritten
            if (i < j && l == 0) {
                Pr[pk(i, j, n)] = -tr[0] / rjj;
                Pi[pk(i, j, n)] = -ti[0] / rjj;
            }
            __syncthreads();
        }
        if (tid == 0) Pr[pk(j, j, n)] = 1.0 / rjj;
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += kCholThreads) {
        const int i = e / n, j = e - i * n;
        X[e] = (j >= i) ? Pr[pk(i, j, n)] : 0.0;
        X[e + plane] = (j >= i) ? Pi[pk(i, j, n)] : 0.0;
    }
}

// Register-resident variant of chol_inv_lds_kernel for n <= 128, same
// contract, one workgroup of 1024 threads.  Factor and inverse come out of
// one elimination on the augmented matrix [G | I]: step k scales row k by
// 1/sqrt(pivot) and subtracts conj(R[k][i]) times it from every row i > k.
// The elimination operator E is then lower triangular with E G = R, so
// E = R^{-H}: the left block ends as R and the right block as R^{-H}.  Row i
// of the two blocks shares one n-wide register row: columns j >= i hold the
// left block's upper triangle and columns j < i the right block's strictly
// lower part; the right block's diagonal entry of row k is 1/R[k][k].
// Step k must leave columns k < j < i of row i alone (the right block is
// still zero there); the update is applied to every column anyway and the
// rubbish it leaves in those columns is discarded when column k' = j is
// reached (row i's entry in column k is zeroed before step k adds to it), so
// the inner update carries no per-lane predicate.
// Rows go to the 16 wavefronts cyclically (row i -> wave i mod 16, a
// wave-uniform index), lane l holds columns l and l + 64 (NS = 2 column
// slots; NS = 1 for n <= 64), and the multiplier conj(R[k][i]) of row i is
// read from the lane that holds column i of the published row.  The
// wavefront that owns row k+1 updates it first, takes its pivot, scales it
// and publishes it through a double-buffered LDS row at raised priority while
// the others apply step k to their rows: one workgroup barrier per step.
constexpr int kRegThreads = 1024;
constexpr int kRegWaves = kRegThreads / 64;
constexpr int kRegChunk = 32;   // rows of X per LDS transpose pass
// 1/sqrt(d) for a positive normal d: the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (quadratic convergence from its
// ~2^-23 relative error), within an ulp or two of the correctly rounded value
// at a quarter of the latency of sqrt followed by a division
__device__ __forceinline__ double rsqrt_newton(double d) {
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
template <int NS>
__global__ __launch_bounds__(kRegThreads) void chol_inv_reg_kernel(double* G, double* X, int n,
                                                                   int64_t plane,
                                                                   const double* shift,
                                                                   int* flag, const int* stop,
                                                                   int* converged) {
    constexpr int ROWS = NS * 64 / kRegWaves;   // rows per wavefront
    if (stop && *stop) return;
    __shared__ double red[kRegWaves];
    __shared__ double2 pub[2][64 * NS];
    __shared__ double dinv[64 * NS];   // 1 / R[i][i]
    // X staging: kRegChunk rows of X (columns of E), padded rows
    __shared__ double2 stage[kRegChunk][64 * NS + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double s = shift ? shift[0] : 0.0;
    if (!shift && chol_near_identity(G, X, n, plane, converged, red)) return;
    double wr[ROWS][NS], wi[ROWS][NS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i = wave + kRegWaves * r;
#pragma unroll
        for (int h = 0; h < NS; ++h) {
            const int j = lane + 64 * h;
            const bool in = i < n && j < n;
            const double vr = in ? G[(int64_t)i * n + j] : 0.0;
            const double vi = in ? G[(int64_t)i * n + j + plane] : 0.0;
            const bool up = in && j >= i;
            wr[r][h] = up ? vr + ((j == i) ? s : 0.0) : 0.0;
            wi[r][h] = (up && j != i) ? vi : 0.0;
        }
    }
    // step k on row i (slot r); column k sits in column slot KH
#define FTD_CHOL_UPDATE(r, i, KH)                                               \
    do {                                                                        \
        const bool hi_ = (r) * kRegWaves >= 64;                                 \
        const double mr_ = lane_read(hi_ ? bjr[NS - 1] : bjr[0], (i) & 63);     \
        const double mi_ = -lane_read(hi_ ? bji[NS - 1] : bji[0], (i) & 63);    \
        wr[r][KH] *= keep;                                                      \
        wi[r][KH] *= keep;                                                      \
        _Pragma("unroll") for (int h = 0; h < NS; ++h) {                        \
            wr[r][h] = fma(mi_, bji[h], fma(-mr_, bjr[h], wr[r][h]));           \
            wi[r][h] = fma(-mi_, bjr[h], fma(-mr_, bji[h], wi[r][h]));          \
        }                                                                       \
    } while (0)
    // row i (slot r of this wavefront) is final: pivot, scale, publish
#define FTD_CHOL_PUBLISH(r, i, b)                                               \
    do {                                                                        \
        const bool hi_ = (r) * kRegWaves >= 64;                                 \
        const double d_ = lane_read(hi_ ? wr[r][NS - 1] : wr[r][0], (i) & 63);  \
        double p_ = 1.0, inv_ = 1.0;                                            \
        if (!(d_ > 0.0) || !isfinite(d_)) {                                     \
            if (lane == 0) flag[0] = 1;                                         \
        } else {                                                                \
            inv_ = rsqrt_newton(d_);                                            \
            p_ = d_ * inv_;                                                     \
        }                                                                       \
        if (lane == 0) dinv[i] = inv_;                                          \
        _Pragma("unroll") for (int h = 0; h < NS; ++h) {                        \
            const int j = lane + 64 * h;                                        \
            if (j == (i)) {                                                     \
                wr[r][h] = p_;                                                  \
                wi[r][h] = 0.0;                                                 \
            } else {                                                            \
                wr[r][h] *= inv_;                                               \
                wi[r][h] *= inv_;                                               \
            }                                                                   \
            if (j < n)                                                          \
                pub[b][j] = make_double2(j == (i) ? inv_ : wr[r][h],            \
                                         j == (i) ? 0.0 : wi[r][h]);            \
        }                                                                       \
    } while (0)
    // one elimination step; KH is the column slot of column k
#define FTD_CHOL_STEP(KH)                                                       \
    do {                                                                        \
        const double2* row = pub[k & 1];                                        \
        _Pragma("unroll") for (int h = 0; h < NS; ++h) {                        \
            const int j = lane + 64 * h;                                        \
            const double2 v = (j < n) ? row[j] : make_double2(0.0, 0.0);        \
            bjr[h] = v.x;                                                       \
            bji[h] = v.y;                                                       \
        }                                                                       \
        const double keep = (lane == (k & 63)) ? 0.0 : 1.0;                     \
        const int nx = k + 1;                                                   \
        const bool piv = nx < n && wave == nx % kRegWaves;                      \
        const int rs = nx / kRegWaves;                                          \
        if (piv) {                                                              \
            __builtin_amdgcn_s_setprio(2);                                      \
            _Pragma("unroll") for (int r = 0; r < ROWS; ++r) {                  \
                if (r == rs) {                                                  \
                    FTD_CHOL_UPDATE(r, nx, KH);                                 \
                    FTD_CHOL_PUBLISH(r, nx, nx & 1);                            \
                }                                                               \
            }                                                                   \
            __builtin_amdgcn_s_setprio(0);                                      \
        }                                                                       \
        _Pragma("unroll") for (int r = 0; r < ROWS; ++r) {                      \
            const int i = wave + kRegWaves * r;                                 \
            if (i > k && i < n && !(piv && r == rs)) FTD_CHOL_UPDATE(r, i, KH); \
        }                                                                       \
        __syncthreads();                                                        \
    } while (0)
    double bjr[NS], bji[NS];
    if (wave == 0) FTD_CHOL_PUBLISH(0, 0, 0);
    __syncthreads();
    const int k64 = min(n, 64);
    for (int k = 0; k < k64; ++k) FTD_CHOL_STEP(0);
    for (int k = 64; k < n; ++k) FTD_CHOL_STEP(NS - 1);
#undef FTD_CHOL_STEP
#undef FTD_CHOL_UPDATE
#undef FTD_CHOL_PUBLISH
    // R into G (zeros below the diagonal)
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i = wave + kRegWaves * r;
#pragma unroll
        for (int h = 0; h < NS; ++h) {
            const int j = lane + 64 * h;
            if (i < n && j < n) {
                const bool up = j >= i;
                G[(int64_t)i * n + j] = up ? wr[r][h] : 0.0;
                G[(int64_t)i * n + j + plane] = up ? wi[r][h] : 0.0;
            }
        }
    }
    // X = R^{-1} = E^H: X[j][i] is conj(E[i][j]) for j < i, 1/R[i][i] for
    // j = i and zero for j > i; transposed through LDS, kRegChunk rows of X
    // (columns j of E) per pass, then written row by row
    for (int c0 = 0; c0 < n; c0 += kRegChunk) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int i = wave + kRegWaves * r;
#pragma unroll
            for (int h = 0; h < NS; ++h) {
                const int j = lane + 64 * h;
                if (i < n && j >= c0 && j < c0 + kRegChunk && j < n) {
                    const double xr = (j < i) ? wr[r][h] : (j == i ? dinv[i] : 0.0);
                    const double xi = (j < i) ? -wi[r][h] : 0.0;
                    stage[j - c0][i] = make_double2(xr, xi);
                }
            }
        }
        __syncthreads();
        const int rows = min(kRegChunk, n - c0);
        for (int e = tid; e < rows * n; e += kRegThreads) {
            const int jr = e / n, i = e - jr * n;
            const double2 v = stage[jr][i];
            X[(int64_t)(c0 + jr) * n + i] = v.x;
            X[(int64_t)(c0 + jr) * n + i + plane] = v.y;
        }
        __syncthreads();
    }
}

__global__ void triinv_kernel(const double* __restrict__ U, double* __restrict__ X, int n,
                              int64_t plane) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int i = 0; i < n; ++i) {
        X[(int64_t)i * n + j] = 0.0;
        X[(int64_t)i * n + j + plane] = 0.0;
    }
    const double djr = U[(int64_t)j * n + j];
    X[(int64_t)j * n + j] = 1.0 / djr;
    for (int i = j - 1; i >= 0; --i) {
        double sr = 0.0, si = 0.0;
        for (int k = i + 1; k <= j; ++k) {
            const double ur = U[(int64_t)i * n + k], ui = U[(int64_t)i * n + k + plane];
            const double xr = X[(int64_t)k * n + j], xi = X[(int64_t)k * n + j + plane];
            sr += ur * xr - ui * xi;
            si += ur * xi + ui * xr;
        }
        const double dii = U[(int64_t)i * n + i];   // real positive
        X[(int64_t)i * n + j] = -sr / dii;
        X[(int64_t)i * n + j + plane] = -si / dii;
    }
}

// trace of a Hermitian matrix -> shift = c * eps * trace
__global__ void shift_kernel(const double* G, int n, double c, double* out) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += G[(int64_t)i * n + i];
    s = bsum(s, sh);
    if (threadIdx.x == 0) out[0] = c * DBL_EPSILON * s;
}

__global__ void eye_kernel(double* X, int n, int64_t plane) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        X[e] = (e / n == e % n) ? 1.0 : 0.0;
        X[e + plane] = 0.0;
    }
}

static GemmParams gp(int M, int N, int K) {
    GemmParams p{};
    p.M = M;
    p.N = N;
    p.K = K;
    p.nprob = 1;
    p.prob[0].offC = 0;
    p.prob[0].t0 = 0;
    p.prob[0].t1 = 1;
    p.term[0].offA = 0;
    p.term[0].offB = 0;
    return p;
}

// Shifted CholeskyQR3.  wide == false: M is m x n (row-major), M = Q R.
// wide == true: M is n x m (row-major), M = L Q with L = R^H.
// Factor-and-invert of the n x n Gram matrix: the register kernel up to
// n = 128, the LDS kernel while the packed triangle fits the per-workgroup
// LDS, else the global-memory kernels.
static bool chol_lds_fits(Ctx* ctx, int64_t n) {
    int lim = 0;
    FTD_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    return sizeof(double) * (size_t)(n * (n + 1)) + 64 <= (size_t)lim;
}
static void chol_inv(Ctx* ctx, double* G, double* Xi, int64_t n, const double* shift, int* flag,
                     int* converged) {
    const int64_t nn = n * n;
    if (n <= 0) return;
    if (n <= 64) {
        chol_inv_reg_kernel<1><<<1, kRegThreads, 0, ctx->stream>>>(G, Xi, (int)n, nn, shift, flag,
                                                                    ctx->kstop, converged);
        FTD_HIP(hipGetLastError());
        return;
    }
    if (n <= 128) {
        chol_inv_reg_kernel<2><<<1, kRegThreads, 0, ctx->stream>>>(G, Xi, (int)n, nn, shift, flag,
                                                                    ctx->kstop, converged);
        FTD_HIP(hipGetLastError());
        return;
    }
    const size_t bytes = sizeof(double) * (size_t)(n * (n + 1));
    bool lds = chol_lds_fits(ctx, n);
    if (lds && bytes > 48 * 1024)
        lds = hipFuncSetAttribute((const void*)chol_inv_lds_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
              hipSuccess;
    if (lds) {
        chol_inv_lds_kernel<<<1, kCholThreads, bytes, ctx->stream>>>(G, Xi, (int)n, nn, shift, flag,
                                                                     ctx->kstop, converged);
    } else {
        FTD_CHECK(ctx->kstop == nullptr, FTD_EINVAL, "chol_inv: predication needs the LDS path");
        chol_kernel<<<1, 1024, 0, ctx->stream>>>(G, (int)n, nn, shift, flag);
        triinv_kernel<<<(unsigned)((n + 63) / 64), 64, 0, ctx->stream>>>(G, Xi, (int)n, nn);
    }
    FTD_HIP(hipGetLastError());
}

void chol_flag_check(Ctx* ctx) {
    int* flag = ctx->iscal + 8;
    FTD_HIP(hipMemcpyAsync(ctx->h_pinned_i, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FTD_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->h_pinned_i[0] != 0) {
        set_int_kernel<<<1, 1, 0, ctx->stream>>>(flag, 0);
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        throw Error{FTD_ENOCONV, "CholeskyQR breakdown: the block is numerically rank deficient"};
    }
}

void chol_flag_clear(Ctx* ctx) {
    set_int_kernel<<<1, 1, 0, ctx->stream>>>(ctx->iscal + 8, 0);
    FTD_HIP(hipGetLastError());
}

// The breakdown flag is sticky: kernels only set it; chol_flag_check reads
// and clears it (at once when `check`, else left to the caller).
static void chol_qr_impl(Ctx* ctx, double* M, int64_t m, int64_t n, double* Rout, bool wide,
                         bool check) {
    const int64_t nn = n * n, mn = m * n;
    ctx->ws_qr.ensure(ctx, sizeof(double) * 2 * (3 * nn + mn));
    double* G = ctx->ws_qr.as<double>();
    double* Xi = G + 2 * nn;
    double* Rt = Xi + 2 * nn;
    double* Q2 = Rt + 2 * nn;
    double* shift = ctx->scal + 32;
    int* flag = ctx->iscal + 8;
    // set by the second pass when the third would change Q only at rounding
    int* converged = ctx->iscal + 10;
    const bool lds_path = chol_lds_fits(ctx, n);
    set_int_kernel<<<1, 1, 0, ctx->stream>>>(converged, 0);
    // the passes alternate between M and Q2; after three the result is in Q2
    double* in = M;
    double* out = Q2;
    for (int pass = 0; pass < 3; ++pass) {
        // the third pass is predicated on the second pass's verdict
        const int* saved_stop = ctx->kstop;
        if (pass == 2 && lds_path) ctx->kstop = converged;
        // Gram matrix
        GemmParams p = gp((int)n, (int)n, (int)m);
        if (!wide) {
            // G[i][j] = sum_r conj(M[r][i]) M[r][j]
            p.sAm = 1; p.sAk = n; p.planeA = mn; p.conjA = 1; p.a_kcontig = 0;
            p.sBk = n; p.sBn = 1; p.planeB = mn; p.b_kcontig = 0;
        } else {
            // G[i][j] = sum_k M[i][k] conj(M[j][k])
            p.sAm = m; p.sAk = 1; p.planeA = mn; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = m; p.planeB = mn; p.conjB = 1; p.b_kcontig = 1;
        }
        p.sCm = n; p.sCn = 1; p.planeC = nn;
        gemm(ctx, Prec::F64, true, in, in, G, p, TAG_NONE);
        if (pass == 0) {
            const double c = 11.0 * ((double)m * n + (double)n * (n + 1));
            shift_kernel<<<1, 256, 0, ctx->stream>>>(G, (int)n, c, shift);
        }
        chol_inv(ctx, G, Xi, n, pass == 0 ? shift : nullptr, flag,
                 pass == 1 && lds_path ? converged : nullptr);
        // out <- in Xi (tall) or out <- Xi^H in (wide)
        GemmParams q = gp(wide ? (int)n : (int)m, wide ? (int)m : (int)n, (int)n);
        if (!wide) {
            q.sAm = n; q.sAk = 1; q.planeA = mn; q.a_kcontig = 1;
            q.sBk = n; q.sBn = 1; q.planeB = nn; q.b_kcontig = 0;
            q.sCm = n; q.sCn = 1; q.planeC = mn;
            gemm(ctx, Prec::F64, true, in, Xi, out, q, TAG_NONE);
        } else {
            // out[i][k] = sum_j conj(Xi[j][i]) in[j][k]
            q.sAm = 1; q.sAk = n; q.planeA = nn; q.conjA = 1; q.a_kcontig = 0;
            q.sBk = m; q.sBn = 1; q.planeB = mn; q.b_kcontig = 0;
            q.sCm = m; q.sCn = 1; q.planeC = mn;
            gemm(ctx, Prec::F64, true, Xi, in, out, q, TAG_NONE);
        }
        // R <- U_pass R (the first pass's factor is R itself)
        if (pass == 0) {
            k_copy_f64(ctx, G, Rout, 2 * nn);
        } else {
            GemmParams r = gp((int)n, (int)n, (int)n);
            r.sAm = n; r.sAk = 1; r.planeA = nn; r.a_kcontig = 1;
            r.sBk = n; r.sBn = 1; r.planeB = nn; r.b_kcontig = 0;
            r.sCm = n; r.sCn = 1; r.planeC = nn;
            gemm(ctx, Prec::F64, true, G, Rout, Rt, r, TAG_NONE);
            k_copy_f64(ctx, Rt, Rout, 2 * nn);
        }
        // a skipped third pass leaves the second pass's result in M
        if (pass == 2) k_copy_f64(ctx, out, M, 2 * mn);
        std::swap(in, out);
        ctx->kstop = saved_stop;
    }
    FTD_HIP(hipGetLastError());
    if (check) chol_flag_check(ctx);
    if (wide) {
        // L = R^H
        k_transpose(ctx, Rout, n, n, nn, Rt, nn, 1);
        k_copy_f64(ctx, Rt, Rout, 2 * nn);
    }
}

void qr_chol(Ctx* ctx, double* M, int64_t m, int64_t n, double* R, bool check) {
    FTD_CHECK(m >= n, FTD_EINVAL, "qr_chol: needs m >= n");
    chol_qr_impl(ctx, M, m, n, R, false, check);
}
void lq_chol(Ctx* ctx, double* M, int64_t n, int64_t m, double* L, bool check) {
    FTD_CHECK(m >= n, FTD_EINVAL, "lq_chol: needs m >= n");
    chol_qr_impl(ctx, M, m, n, L, true, check);
}

// -------------------------------------------------------------- Householder
// Working matrix W is column-major m x n: W[i + j*m], planar (plane = m*n).
__global__ void hh_colnorm_partial(const double* W, int64_t m, int64_t plane, int j,
                                   double* part) {
    __shared__ double sh[16];
    const double* col = W + (int64_t)j * m;
    double s = 0.0;
    for (int64_t i = j + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = col[i], b = col[i + plane];
        s += a * a + b * b;
    }
    s = bsum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// reflector of column j: beta, tau, scale; W[j][j] = beta.  hs: per-column
// record [tau_r, tau_i, scale_r, scale_i, beta]
__global__ void hh_make(double* W, int64_t m, int64_t plane, int j, const double* part, int nb,
                        double* hs) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    s = bsum(s, sh);
    if (threadIdx.x == 0) {
        const int64_t dj = (int64_t)j * m + j;
        const double ar = W[dj], ai = W[dj + plane];
        double* h = hs + 5 * j;
        if (s == 0.0 && ai == 0.0) {
            h[0] = 0.0; h[1] = 0.0; h[2] = 0.0; h[3] = 0.0; h[4] = ar;
        } else {
            const double nrm = sqrt(ar * ar + ai * ai + s);
            const double beta = ar >= 0.0 ? -nrm : nrm;
            h[0] = (beta - ar) / beta;
            h[1] = -ai / beta;
            // scale = 1 / (alpha - beta)
            const double xr = ar - beta, xi = ai;
            const double den = xr * xr + xi * xi;
            h[2] = xr / den;
            h[3] = -xi / den;
            h[4] = beta;
            W[dj] = beta;
            W[dj + plane] = 0.0;
        }
    }
}
__global__ void hh_scale(double* W, int64_t m, int64_t plane, int j, const double* hs) {
    const double* h = hs + 5 * j;
    if (h[0] == 0.0 && h[1] == 0.0) return;
    const double sr = h[2], si = h[3];
    double* col = W + (int64_t)j * m;
    for (int64_t i = j + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = col[i], b = col[i + plane];
        col[i] = a * sr - b * si;
        col[i + plane] = a * si + b * sr;
    }
}
// partial w_c = sum_{i>=j} conj(v_i) W[i][c], for c in (j, c1): grid (nb, c1-j-1)
__global__ void hh_pdot_partial(const double* W, int64_t m, int64_t plane, int j, double* part) {
    __shared__ double sh[16];
    const int c = j + 1 + blockIdx.y;
    const double* v = W + (int64_t)j * m;
    const double* x = W + (int64_t)c * m;
    double sr = 0.0, si = 0.0;
    for (int64_t i = j + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        double vr, vi;
        if (i == j) {
            vr = 1.0;
            vi = 0.0;
        } else {
            vr = v[i];
            vi = v[i + plane];
        }
        const double xr = x[i], xi = x[i + plane];
        sr += vr * xr + vi * xi;
        si += vr * xi - vi * xr;
    }
    sr = bsum(sr, sh);
    si = bsum(si, sh);
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        part[o] = sr;
        part[o + 1] = si;
    }
}
// reduce partials (one block per column) then W[i][c] -= conj(tau) v_i w_c
__global__ void hh_pdot_reduce(const double* part, int nb, double* wv) {
    __shared__ double sh[16];
    const int c = blockIdx.x;
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        sr += part[((int64_t)c * nb + i) * 2];
        si += part[((int64_t)c * nb + i) * 2 + 1];
    }
    sr = bsum(sr, sh);
    si = bsum(si, sh);
    if (threadIdx.x == 0) {
        wv[2 * c] = sr;
        wv[2 * c + 1] = si;
    }
}
__global__ void hh_pupdate(double* W, int64_t m, int64_t plane, int j, int ncols,
                           const double* wv, const double* hs) {
    const double* h = hs + 5 * j;
    const double tr = h[0], ti = -h[1];   // conj(tau)
    if (h[0] == 0.0 && h[1] == 0.0) return;
    const double* v = W + (int64_t)j * m;
    const int64_t rows = m - j;
    const int64_t tot = rows * ncols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int cc = (int)(e / rows);
        const int64_t i = j + e % rows;
        const int c = j + 1 + cc;
        double vr, vi;
        if (i == j) {
            vr = 1.0;
            vi = 0.0;
        } else {
            vr = v[i];
            vi = v[i + plane];
        }
        const double wr = wv[2 * cc], wi = wv[2 * cc + 1];
        // f = conj(tau) * w_c ; W -= v * f
        const double fr = tr * wr - ti * wi, fi = tr * wi + ti * wr;
        double* x = W + (int64_t)c * m;
        x[i] -= vr * fr - vi * fi;
        x[i + plane] -= vr * fi + vi * fr;
    }
}
// V panel (m x pn, column-major) from W columns p0..p0+pn-1 (unit lower trapezoid)
__global__ void hh_extract_v(const double* W, int64_t m, int64_t plane, int p0, int pn, double* V,
                             int64_t vplane) {
    const int64_t tot = m * pn;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / m);
        const int64_t i = e % m;
        const int jc = p0 + c;
        double r = 0.0, im = 0.0;
        if (i == jc) {
            r = 1.0;
        } else if (i > jc) {
            r = W[(int64_t)jc * m + i];
            im = W[(int64_t)jc * m + i + plane];
        }
        V[e] = r;
        V[e + vplane] = im;
    }
}
// T (pn x pn, row-major planar) of the compact WY form from S = V^H V:
// T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j].  Writes both
// T and Tn = -T^H (row-major).  Single thread: pn <= 64.
__global__ void hh_make_t(const double* S, int pn, const double* hs, int p0, double* T,
                          double* Tn) {
    if (threadIdx.x != 0) return;
    const int64_t pl = (int64_t)pn * pn;
    for (int e = 0; e < pn * pn; ++e) {
        T[e] = 0.0;
        T[e + pl] = 0.0;
    }
    for (int j = 0; j < pn; ++j) {
        const double tr = hs[5 * (p0 + j)], ti = hs[5 * (p0 + j) + 1];
        for (int i = 0; i < j; ++i) {
            double sr = 0.0, si = 0.0;
            for (int k = i; k < j; ++k) {
                const double ar = T[i * pn + k], ai = T[i * pn + k + pl];
                const double br = S[k * pn + j], bi = S[k * pn + j + pl];
                sr += ar * br - ai * bi;
                si += ar * bi + ai * br;
            }
            T[i * pn + j] = -(tr * sr - ti * si);
            T[i * pn + j + pl] = -(tr * si + ti * sr);
        }
        T[j * pn + j] = tr;
        T[j * pn + j + pl] = ti;
    }
    for (int i = 0; i < pn; ++i)
        for (int j = 0; j < pn; ++j) {
            Tn[i * pn + j] = -T[j * pn + i];
            Tn[i * pn + j + pl] = T[j * pn + i + pl];
        }
}
// Q0 = [I; 0] column-major m x r
__global__ void hh_q_init(double* Q, int64_t m, int r, int64_t plane) {
    const int64_t tot = m * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / m);
        const int64_t i = e % m;
        Q[e] = (i == c) ? 1.0 : 0.0;
        Q[e + plane] = 0.0;
    }
}
// Output: R (r x n row-major) from W's upper part with sign fix, and
// column signs of Q recorded in sg[j].
__global__ void hh_extract_r(const double* W, int64_t m, int64_t plane, int r, int n,
                             const double* hs, double* R, int64_t rplane) {
    const int64_t tot = (int64_t)r * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        const double sg = hs[5 * i + 4] < 0.0 ? -1.0 : 1.0;
        double a = 0.0, b = 0.0;
        if (j >= i) {
            a = sg * W[(int64_t)j * m + i];
            b = sg * W[(int64_t)j * m + i + plane];
        }
        R[e] = a;
        R[e + rplane] = b;
    }
}
// Q column-major (m x r) -> row-major output with column sign fix
__global__ void hh_store_q(const double* Qc, int64_t m, int r, int64_t plane, const double* hs,
                           double* Q, int64_t qplane) {
    const int64_t tot = m * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / r;
        const int c = (int)(e % r);
        const double sg = hs[5 * c + 4] < 0.0 ? -1.0 : 1.0;
        Q[e] = sg * Qc[(int64_t)c * m + i];
        Q[e + qplane] = sg * Qc[(int64_t)c * m + i + plane];
    }
}

__global__ void conj_copy_kernel(const double* __restrict__ s, double* __restrict__ d, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        d[i] = s[i];
        d[i + n] = -s[i + n];
    }
}

void qr_householder(Ctx* ctx, const double* M, int64_t m, int64_t n, double* Q, double* R,
                    bool adjoint) {
    FTD_CHECK(m >= 1 && n >= 1, FTD_EINVAL, "qr_householder: empty matrix");
    const int r = (int)std::min(m, n);
    const int NBP = 16;
    const int64_t mn = m * n, mr = m * r;
    // workspace: W (m x n), Qc (m x r), Vp (m x NBP), S/T/Tn (NBP^2 x 3), Y/Z (NBP x max(n,r)) x2
    const int64_t wmax = std::max<int64_t>(n, r);
    const size_t need = sizeof(double) * 2 *
                        (mn + mr + m * NBP + 3 * NBP * NBP + 2 * NBP * wmax) +
                        sizeof(double) * 5 * (size_t)r;
    ctx->ws_svd3.ensure(ctx, need);
    double* W = ctx->ws_svd3.as<double>();
    double* Qc = W + 2 * mn;
    double* Vp = Qc + 2 * mr;
    double* S = Vp + 2 * m * NBP;
    double* T = S + 2 * NBP * NBP;
    double* Tn = T + 2 * NBP * NBP;
    double* Y = Tn + 2 * NBP * NBP;
    double* Z = Y + 2 * NBP * wmax;
    double* hs = Z + 2 * NBP * wmax;
    ctx->ws_red.ensure(ctx, sizeof(double) * 2 * 512 * (kMaxKrylov + 1));
    double* part = ctx->ws_red.as<double>();
    double* wv = ctx->scal + 64;   // up to NBP complex
    // column-major working copy of the m x n matrix being factored: for a
    // row-major M that is a transpose; for the adjoint of a row-major n x m M
    // it is the element-wise conjugate of M's storage.
    if (adjoint)
        conj_copy_kernel<<<grid1(mn), 256, 0, ctx->stream>>>(M, W, mn);
    else
        k_transpose(ctx, M, m, n, mn, W, mn, 0);
    const int nbr = (int)std::min<int64_t>(256, std::max<int64_t>(1, (m + 2047) / 2048));
    std::vector<int> panels;
    for (int p0 = 0; p0 < r; p0 += NBP) panels.push_back(p0);
    for (int p0 : panels) {
        const int pn = std::min(NBP, r - p0);
        for (int j = p0; j < p0 + pn; ++j) {
            hh_colnorm_partial<<<nbr, 256, 0, ctx->stream>>>(W, m, mn, j, part);
            hh_make<<<1, 256, 0, ctx->stream>>>(W, m, mn, j, part, nbr, hs);
            hh_scale<<<grid1(m - j), 256, 0, ctx->stream>>>(W, m, mn, j, hs);
            const int nc = p0 + pn - j - 1;
            if (nc > 0) {
                hh_pdot_partial<<<dim3(nbr, nc), 256, 0, ctx->stream>>>(W, m, mn, j, part);
                hh_pdot_reduce<<<nc, 256, 0, ctx->stream>>>(part, nbr, wv);
                hh_pupdate<<<grid1((m - j) * nc), 256, 0, ctx->stream>>>(W, m, mn, j, nc, wv, hs);
            }
        }
        // compact WY
        const int64_t vpl = m * pn;
        hh_extract_v<<<grid1(m * pn), 256, 0, ctx->stream>>>(W, m, mn, p0, pn, Vp, vpl);
        {
            GemmParams p = gp(pn, pn, (int)m);
            p.sAm = m; p.sAk = 1; p.planeA = vpl; p.conjA = 1; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = m; p.planeB = vpl; p.b_kcontig = 1;
            p.sCm = pn; p.sCn = 1; p.planeC = (int64_t)pn * pn;
            gemm(ctx, Prec::F64, true, Vp, Vp, S, p, TAG_NONE);
        }
        hh_make_t<<<1, 64, 0, ctx->stream>>>(S, pn, hs, p0, T, Tn);
        const int c0 = p0 + pn, nt = (int)n - c0;
        if (nt > 0) {
            // Y = V^H W[:, c0:]  (pn x nt)
            GemmParams p = gp(pn, nt, (int)m);
            p.sAm = m; p.sAk = 1; p.planeA = vpl; p.conjA = 1; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = m; p.planeB = mn; p.b_kcontig = 1;
            p.term[0].offB = (int64_t)c0 * m;
            p.sCm = nt; p.sCn = 1; p.planeC = (int64_t)pn * nt;
            gemm(ctx, Prec::F64, true, Vp, W, Y, p, TAG_NONE);
            // Z = -T^H Y
            GemmParams q = gp(pn, nt, pn);
            q.sAm = pn; q.sAk = 1; q.planeA = (int64_t)pn * pn; q.a_kcontig = 1;
            q.sBk = nt; q.sBn = 1; q.planeB = (int64_t)pn * nt; q.b_kcontig = 0;
            q.sCm = nt; q.sCn = 1; q.planeC = (int64_t)pn * nt;
            gemm(ctx, Prec::F64, true, Tn, Y, Z, q, TAG_NONE);
            // W[:, c0:] += V Z
            GemmParams u = gp((int)m, nt, pn);
            u.sAm = 1; u.sAk = m; u.planeA = vpl; u.a_kcontig = 0;
            u.sBk = nt; u.sBn = 1; u.planeB = (int64_t)pn * nt; u.b_kcontig = 0;
            u.sCm = 1; u.sCn = m; u.planeC = mn; u.accumulate = 1;
            u.prob[0].offC = (int64_t)c0 * m;
            gemm(ctx, Prec::F64, true, Vp, Z, W, u, TAG_NONE);
        }
    }
    // R
    hh_extract_r<<<grid1((int64_t)r * n), 256, 0, ctx->stream>>>(W, m, mn, r, (int)n, hs, R,
                                                                 (int64_t)r * n);
    if (!Q) {
        FTD_HIP(hipGetLastError());
        return;
    }
    // Q = H_1 ... H_r [I; 0], applying panels last to first
    hh_q_init<<<grid1(mr), 256, 0, ctx->stream>>>(Qc, m, r, mr);
    for (int pi = (int)panels.size() - 1; pi >= 0; --pi) {
        const int p0 = panels[pi];
        const int pn = std::min(NBP, r - p0);
        const int64_t vpl = m * pn;
        hh_extract_v<<<grid1(m * pn), 256, 0, ctx->stream>>>(W, m, mn, p0, pn, Vp, vpl);
        {
            GemmParams p = gp(pn, pn, (int)m);
            p.sAm = m; p.sAk = 1; p.planeA = vpl; p.conjA = 1; p.a_kcontig = 1;
            p.sBk = 1; p.sBn = m; p.planeB = vpl; p.b_kcontig = 1;
            p.sCm = pn; p.sCn = 1; p.planeC = (int64_t)pn * pn;
            gemm(ctx, Prec::F64, true, Vp, Vp, S, p, TAG_NONE);
        }
        hh_make_t<<<1, 64, 0, ctx->stream>>>(S, pn, hs, p0, T, Tn);
        // Y = V^H Q  (pn x r)
        GemmParams p = gp(pn, r, (int)m);
        p.sAm = m; p.sAk = 1; p.planeA = vpl; p.conjA = 1; p.a_kcontig = 1;
        p.sBk = 1; p.sBn = m; p.planeB = mr; p.b_kcontig = 1;
        p.sCm = r; p.sCn = 1; p.planeC = (int64_t)pn * r;
        gemm(ctx, Prec::F64, true, Vp, Qc, Y, p, TAG_NONE);
        // Z = -T Y : use Tn^H = -T
        GemmParams q = gp(pn, r, pn);
        q.sAm = 1; q.sAk = pn; q.planeA = (int64_t)pn * pn; q.conjA = 1; q.a_kcontig = 0;
        q.sBk = r; q.sBn = 1; q.planeB = (int64_t)pn * r; q.b_kcontig = 0;
        q.sCm = r; q.sCn = 1; q.planeC = (int64_t)pn * r;
        gemm(ctx, Prec::F64, true, Tn, Y, Z, q, TAG_NONE);
        // Q += V Z
        GemmParams u = gp((int)m, r, pn);
        u.sAm = 1; u.sAk = m; u.planeA = vpl; u.a_kcontig = 0;
        u.sBk = r; u.sBn = 1; u.planeB = (int64_t)pn * r; u.b_kcontig = 0;
        u.sCm = 1; u.sCn = m; u.planeC = mr; u.accumulate = 1;
        gemm(ctx, Prec::F64, true, Vp, Z, Qc, u, TAG_NONE);
    }
    hh_store_q<<<grid1(mr), 256, 0, ctx->stream>>>(Qc, m, r, mr, hs, Q, mr);
    FTD_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Jacobi
// Sum over the 64 lanes of a wavefront; every lane receives the total (xor
// butterfly), so all lanes derive the same rotation without a broadcast.
__device__ __forceinline__ double wave_allsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kJacobiWaves = 4;   // wavefronts per 256-thread block

// Rotation of column pair (p, q) of one-sided Jacobi; returns 1 if rotated.
// One wavefront; U column-major m x n, V column-major n x n.
__device__ __forceinline__ int jacobi_pair(double* U, int64_t m, int64_t uplane, double* V, int n,
                                           int64_t vplane, int p, int q, double tol,
                                           double noise, int lane) {
    double* x = U + (int64_t)p * m;
    double* y = U + (int64_t)q * m;
    double a = 0.0, b = 0.0, cr = 0.0, ci = 0.0;
    for (int64_t k = lane; k < m; k += 64) {
        const double xr = x[k], xi = x[k + uplane], yr = y[k], yi = y[k + uplane];
        a += xr * xr + xi * xi;
        b += yr * yr + yi * yi;
        cr += xr * yr + xi * yi;
        ci += xr * yi - xi * yr;
    }
    a = wave_allsum(a);
    b = wave_allsum(b);
    cr = wave_allsum(cr);
    ci = wave_allsum(ci);
    const double ac = sqrt(cr * cr + ci * ci);
    // columns at rounding level of the whole matrix count as zero
    if (ac == 0.0 || ac <= tol * sqrt(a * b) || a <= noise || b <= noise) return 0;
    const double zeta = (b - a) / (2.0 * ac);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t);
    const double sn = t * cs;
    const double er = cr / ac, ei = -ci / ac;   // e^{-i phi}
    for (int64_t k = lane; k < m; k += 64) {
        const double xr = x[k], xi = x[k + uplane];
        const double y0r = y[k], y0i = y[k + uplane];
        const double yr = y0r * er - y0i * ei, yi = y0r * ei + y0i * er;   // y e^{-i phi}
        x[k] = cs * xr - sn * yr;
        x[k + uplane] = cs * xi - sn * yi;
        y[k] = sn * xr + cs * yr;
        y[k + uplane] = sn * xi + cs * yi;
    }
    double* vx = V + (int64_t)p * n;
    double* vy = V + (int64_t)q * n;
    for (int k = lane; k < n; k += 64) {
        const double xr = vx[k], xi = vx[k + vplane];
        const double y0r = vy[k], y0i = vy[k + vplane];
        const double yr = y0r * er - y0i * ei, yi = y0r * ei + y0i * er;
        vx[k] = cs * xr - sn * yr;
        vx[k + vplane] = cs * xi - sn * yi;
        vy[k] = sn * xr + cs * yr;
        vy[k + vplane] = sn * xi + cs * yi;
    }
    return 1;
}

// Pair i of round rd in the circle method over n2 players (player n2-1 fixed);
// the lower index first.
__device__ __forceinline__ void round_pair(int i, int rd, int n2, int& p, int& q) {
    if (i == 0) {
        p = rd % (n2 - 1);
        q = n2 - 1;
    } else {
        p = (rd + i) % (n2 - 1);
        q = (rd - i + (n2 - 1)) % (n2 - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

// One full sweep (all n2-1 rounds) in one cooperative launch: the rounds are
// separated by grid-wide barriers; each wavefront takes pairs i = its global
// wave index + k * (total waves).  Adds the number of rotations to *count.
__global__ __launch_bounds__(64 * kJacobiWaves) void jacobi_sweep(
    double* U, int64_t m, int64_t uplane, double* V, int n, int64_t vplane, int n2, double tol,
    const double* fro2, int* count) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kJacobiWaves + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * kJacobiWaves;
    const int npair = n2 / 2;
    const double noise = DBL_EPSILON * DBL_EPSILON * fro2[0];
    int rotated = 0;
    for (int rd = 0; rd < n2 - 1; ++rd) {
        for (int i = wave; i < npair; i += nwaves) {
            int p, q;
            round_pair(i, rd, n2, p, q);
            if (q < n) rotated += jacobi_pair(U, m, uplane, V, n, vplane, p, q, tol, noise, lane);
        }
        grid.sync();
    }
    if (lane == 0 && rotated) atomicAdd(count, rotated);
}
__global__ void count_kernel(const int* f, int n, int* out) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += f[i];
    s = bsum(s, sh);
    if (threadIdx.x == 0) out[0] = (int)s;
}
__global__ void fro2_kernel(const double* U, int64_t n, int64_t plane, double* out) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) s += U[k] * U[k] + U[k + plane] * U[k + plane];
    s = bsum(s, sh);
    if (threadIdx.x == 0) out[0] = s;
}
__global__ void colnorm_kernel(const double* U, int64_t m, int64_t plane, double* S) {
    __shared__ double sh[16];
    const double* x = U + (int64_t)blockIdx.x * m;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < m; k += blockDim.x) s += x[k] * x[k] + x[k + plane] * x[k + plane];
    s = bsum(s, sh);
    if (threadIdx.x == 0) S[blockIdx.x] = sqrt(s);
}

// X row-major m x n (m >= n), or with adjoint_input a row-major n x n R
// whose adjoint is diagonalised (U starts as R^H).  Outputs (column-major):
// U m x n with columns u_j * s_j (unnormalised), S[n] (unsorted), V n x n,
// so that (X or R^H) V = U.
void svd_jacobi(Ctx* ctx, const double* X, int64_t m, int64_t n, double* U, double* S,
                double* V, bool adjoint_input) {
    FTD_CHECK(m >= n && n >= 1, FTD_EINVAL, "svd_jacobi: needs m >= n >= 1");
    FTD_CHECK(!adjoint_input || m == n, FTD_EINVAL, "svd_jacobi: adjoint input must be square");
    const int64_t mn = m * n, nn = n * n;
    if (adjoint_input)
        conj_copy_kernel<<<grid1(mn), 256, 0, ctx->stream>>>(X, U, mn);
    else
        k_transpose(ctx, X, m, n, mn, U, mn, 0);
    eye_kernel<<<grid1(nn), 256, 0, ctx->stream>>>(V, (int)n, nn);
    if (n == 1) {
        colnorm_kernel<<<1, 256, 0, ctx->stream>>>(U, m, mn, S);
        FTD_HIP(hipGetLastError());
        return;
    }
    const int n2 = (int)(n + (n & 1));
    const int npair = n2 / 2;
    const double tol = 8.0 * DBL_EPSILON * sqrt((double)m);
    double* fro2 = ctx->scal + 40;
    fro2_kernel<<<1, 256, 0, ctx->stream>>>(U, mn, mn, fro2);
    // co-resident grid for the cooperative sweep
    int per_cu = 0, cus = 0;
    FTD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, jacobi_sweep, 64 * kJacobiWaves,
                                                         0));
    FTD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int max_blocks = std::max(1, per_cu * cus);
    const int nblk = std::max(1, std::min((npair + kJacobiWaves - 1) / kJacobiWaves, max_blocks));
    int* cnt = ctx->iscal + 12;
    for (int sweep = 0; sweep < 60; ++sweep) {
        set_int_kernel<<<1, 1, 0, ctx->stream>>>(cnt, 0);
        int nn_ = (int)n;
        int64_t m_ = m, mn_ = mn, nn2 = nn;
        double tol_ = tol;
        void* args[] = {&U, &m_, &mn_, &V, &nn_, &nn2, (void*)&n2, &tol_, &fro2, &cnt};
        FTD_HIP(hipLaunchCooperativeKernel((const void*)jacobi_sweep, dim3(nblk),
                                           dim3(64 * kJacobiWaves), args, 0, ctx->stream));
        FTD_HIP(hipMemcpyAsync(ctx->h_pinned_i + 1, cnt, sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
        FTD_HIP(hipStreamSynchronize(ctx->stream));
        if (ctx->h_pinned_i[1] == 0) break;
        FTD_CHECK(sweep < 59, FTD_ENOCONV, "Jacobi SVD did not converge");
    }
    colnorm_kernel<<<(unsigned)n, 256, 0, ctx->stream>>>(U, m, mn, S);
    FTD_HIP(hipGetLastError());
}

}  // namespace ftd
