// Vector kernels for the Krylov exponential, the channel mixing of the MPO
// local operators, the exact MPO x MPS product and the device-side
// exponential of the Lanczos tridiagonal matrix.
//
// All reductions are deterministic: a fixed grid-stride partition, fixed
// in-block trees, and a second pass that sums block partials in order.
#include "common.h"

#include <cfloat>

namespace ftd {

constexpr int RB = 256;      // threads per reduction block
constexpr int RMAXB = 512;   // partial sums per reduction

static int red_blocks(int64_t n) {
    int64_t b = (n + RB * 8 - 1) / (RB * 8);
    if (b < 1) b = 1;
    if (b > RMAXB) b = RMAXB;
    return (int)b;
}

static dim3 grid_for(int64_t n, int threads = 256, int64_t cap = 65535 * 4) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return dim3((unsigned)b);
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // wave reduction then across waves (fixed order)
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- basic ops
__global__ void copy_kernel(const double* __restrict__ s, double* __restrict__ d, int64_t n,
                            const int* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}
__global__ void convert_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n,
                               const int* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}
__global__ void scale_kernel(double* x, int64_t n, int64_t plane, double re, double im) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = x[i], b = x[i + plane];
        x[i] = re * a - im * b;
        x[i + plane] = re * b + im * a;
    }
}
// mode 0: x *= 1/sqrt(s[0]) (0 if s[0] == 0); mode 1: x *= s[0] (real)
__global__ void scale_dev_kernel(double* x, int64_t n, int64_t plane, const double* s, int mode) {
    double f;
    if (mode == 0) {
        const double q = s[0];
        f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    } else {
        f = s[0];
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] *= f;
        x[i + plane] *= f;
    }
}

void k_copy_f64(Ctx* ctx, const double* src, double* dst, int64_t n) {
    if (n <= 0) return;
    copy_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(src, dst, n, ctx->kstop);
    FTD_HIP(hipGetLastError());
}
void k_convert_f64_f32(Ctx* ctx, const double* src, float* dst, int64_t n) {
    if (n <= 0) return;
    convert_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(src, dst, n, ctx->kstop);
    FTD_HIP(hipGetLastError());
}
void k_scale_cplx(Ctx* ctx, double* x, int64_t n, int64_t plane, double re, double im) {
    if (n <= 0) return;
    scale_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(x, n, plane, re, im);
    FTD_HIP(hipGetLastError());
}
void k_scale_by_dev(Ctx* ctx, double* x, int64_t n, int64_t plane, const double* s, int mode) {
    if (n <= 0) return;
    scale_dev_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(x, n, plane, s, mode);
    FTD_HIP(hipGetLastError());
}
__global__ void zero_kernel(uint32_t* p, int64_t n, const int* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
// a fill kernel rather than a memset, so it can be predicated and captured
void k_zero(Ctx* ctx, void* p, size_t bytes) {
    if (bytes == 0) return;
    FTD_CHECK(bytes % 4 == 0, FTD_EINVAL, "k_zero: size not a multiple of 4 bytes");
    const int64_t n = (int64_t)(bytes / 4);
    zero_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(static_cast<uint32_t*>(p), n, ctx->kstop);
    FTD_HIP(hipGetLastError());
}

// --------------------------------------------------------------- reductions
__global__ void nrm2_partial(const double* __restrict__ x, int64_t n, int64_t plane,
                             double* __restrict__ part, const int* stop) {
    if (stop && *stop) return;
    __shared__ double sh[16];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = x[i], b = x[i + plane];
        s += a * a + b * b;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// sum `cnt` groups of `nb` partials, each group `width` wide (interleaved)
// out[g][c] = sum_i part[g][i][c]; with `alpha`, group `ga`'s first component
// is also stored to *alpha (the Lanczos diagonal element).
__global__ void sum_partials(const double* __restrict__ part, int nb, int width, double* out,
                             const int* stop, double* alpha = nullptr, int ga = -1) {
    if (stop && *stop) return;
    __shared__ double sh[16];
    const int g = blockIdx.x;
    for (int c = 0; c < width; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[((int64_t)g * nb + i) * width + c];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) {
            out[g * width + c] = s;
            if (alpha && g == ga && c == 0) alpha[0] = s;
        }
    }
}

void k_nrm2(Ctx* ctx, const double* x, int64_t n, int64_t plane, double* out) {
    const int nb = red_blocks(n);
    ctx->ws_red.ensure(ctx, sizeof(double) * 2 * RMAXB * (kMaxKrylov + 1));
    double* part = ctx->ws_red.as<double>();
    nrm2_partial<<<nb, RB, 0, ctx->stream>>>(x, n, plane, part, ctx->kstop);
    sum_partials<<<1, RB, 0, ctx->stream>>>(part, nb, 1, out, ctx->kstop);
    FTD_HIP(hipGetLastError());
}

// Several complex dot products per thread with one read of w: vectors
// V_j0 .. V_j0+kc-1 (kc <= KC), block partials into part[(j * nb + b) * 2].
template <int KC>
__device__ __forceinline__ void block_sums_out(double (&sr)[KC], double (&si)[KC], int kc, int j0,
                                               double* __restrict__ part, double* sh) {
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        if (j >= kc) break;
        const double a = block_sum(sr[j], sh), b = block_sum(si[j], sh);
        if (threadIdx.x == 0) {
            const int64_t o = ((int64_t)(j0 + j) * gridDim.x + blockIdx.x) * 2;
            part[o] = a;
            part[o + 1] = b;
        }
    }
}

// KC is the exact vector count: every load of an element is unconditional,
// so all 2 KC + 2 of them are in flight together
template <int KC>
__global__ __launch_bounds__(RB) void multidot_w1_partial(const double* __restrict__ V,
                                                         int64_t vstride, int j0,
                                                         const double* __restrict__ w, int64_t n,
                                                         int64_t plane, double* __restrict__ part,
                                                         const int* stop) {
    if (stop && *stop) return;
    __shared__ double sh[16];
    double sr[KC], si[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) sr[j] = si[j] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double wr = w[i], wi = w[i + plane];
        double vr[KC], vi[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const double* v = V + (int64_t)(j0 + j) * vstride;
            vr[j] = v[i];
            vi[j] = v[i + plane];
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            sr[j] += vr[j] * wr + vi[j] * wi;
            si[j] += vr[j] * wi - vi[j] * wr;
        }
    }
    block_sums_out<KC>(sr, si, KC, j0, part, sh);
}
// launch multidot_w1_partial<kc> (1 <= kc <= KC)
template <int KC>
static void launch_multidot_w1(int kc, int nb, hipStream_t st, const double* V, int64_t vstride,
                               int j0, const double* w, int64_t n, int64_t plane, double* part,
                               const int* stop) {
    if constexpr (KC > 1) {
        if (kc < KC) {
            launch_multidot_w1<KC - 1>(kc, nb, st, V, vstride, j0, w, n, plane, part, stop);
            return;
        }
    }
    multidot_w1_partial<KC><<<nb, RB, 0, st>>>(V, vstride, j0, w, n, plane, part, stop);
}

// One pass of w -= sum_j V_j h[j] (j < KC, the exact vector count) that
// also forms the block partials of the next projections <V_j, w> of the
// updated w (the second Gram-Schmidt pass needs exactly these),
// part[(j * nb + b) * 2], and in group KC the partials of |w|^2 after and
// before the update.
template <int KC>
__global__ __launch_bounds__(RB) void multiaxpy_dot_partial(const double* __restrict__ V,
                                                           int64_t vstride,
                                                           const double* __restrict__ h,
                                                           double* __restrict__ w, int64_t n,
                                                           int64_t plane,
                                                           double* __restrict__ part,
                                                           const int* stop) {
    constexpr int k = KC;
    if (stop && *stop) return;
    __shared__ double sh[16];
    double hr[KC], hi[KC], sr[KC], si[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        hr[j] = h[2 * j];
        hi[j] = h[2 * j + 1];
        sr[j] = si[j] = 0.0;
    }
    double s_before = 0.0, s_after = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double vr[KC], vi[KC];
        double ar = w[i], ai = w[i + plane];
        s_before += ar * ar + ai * ai;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            vr[j] = V[(int64_t)j * vstride + i];
            vi[j] = V[(int64_t)j * vstride + i + plane];
            ar -= vr[j] * hr[j] - vi[j] * hi[j];
            ai -= vr[j] * hi[j] + vi[j] * hr[j];
        }
        w[i] = ar;
        w[i + plane] = ai;
        s_after += ar * ar + ai * ai;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            sr[j] += vr[j] * ar + vi[j] * ai;
            si[j] += vr[j] * ai - vi[j] * ar;
        }
    }
    block_sums_out<KC>(sr, si, k, 0, part, sh);
    const double a = block_sum(s_after, sh), b = block_sum(s_before, sh);
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)k * gridDim.x + blockIdx.x) * 2;
        part[o] = a;
        part[o + 1] = b;
    }
}

// launch multiaxpy_dot_partial<k> (1 <= k <= KC)
template <int KC>
static void launch_multiaxpy_dot(int k, int nb, hipStream_t st, const double* V, int64_t vstride,
                                 const double* h, double* w, int64_t n, int64_t plane,
                                 double* part, const int* stop) {
    if constexpr (KC > 1) {
        if (k < KC) {
            launch_multiaxpy_dot<KC - 1>(k, nb, st, V, vstride, h, w, n, plane, part, stop);
            return;
        }
    }
    multiaxpy_dot_partial<KC><<<nb, RB, 0, st>>>(V, vstride, h, w, n, plane, part, stop);
}

// h[j] = <V_j, w>: grid (nb, k)
__global__ void multidot_partial(const double* __restrict__ V, int64_t vstride,
                                 const double* __restrict__ w, int64_t n, int64_t plane,
                                 double* __restrict__ part, const int* stop) {
    if (stop && *stop) return;
    __shared__ double sh[16];
    const int j = blockIdx.y;
    const double* v = V + (int64_t)j * vstride;
    double sr = 0.0, si = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double vr = v[i], vi = v[i + plane], wr = w[i], wi = w[i + plane];
        sr += vr * wr + vi * wi;
        si += vr * wi - vi * wr;
    }
    sr = block_sum(sr, sh);
    si = block_sum(si, sh);
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)j * gridDim.x + blockIdx.x) * 2;
        part[o] = sr;
        part[o + 1] = si;
    }
}
void k_multidot(Ctx* ctx, const double* V, int64_t vstride, int k, const double* w, int64_t n,
                int64_t plane, double* h, double* alpha) {
    if (k <= 0) return;
    ctx->ws_red.ensure(ctx, sizeof(double) * 2 * RMAXB * (kMaxKrylov + 1));
    double* part = ctx->ws_red.as<double>();
    int nb = red_blocks(n);
    if (n >= (int64_t)RB * 64) {
        // long vectors: w read once per chunk of eight Krylov vectors
        for (int j0 = 0; j0 < k; j0 += 8)
            launch_multidot_w1<8>(std::min(8, k - j0), nb, ctx->stream, V, vstride, j0, w, n,
                                  plane, part, ctx->kstop);
    } else {
        nb = std::min(nb, 128);
        multidot_partial<<<dim3(nb, k), RB, 0, ctx->stream>>>(V, vstride, w, n, plane, part,
                                                              ctx->kstop);
    }
    sum_partials<<<k, RB, 0, ctx->stream>>>(part, nb, 2, h, ctx->kstop, alpha, k - 1);
    FTD_HIP(hipGetLastError());
}

bool k_multiaxpy_dot(Ctx* ctx, const double* V, int64_t vstride, int k, double* h, double* w,
                     int64_t n, int64_t plane) {
    if (k <= 0 || k > 16 || n < (int64_t)RB * 64) return false;
    ctx->ws_red.ensure(ctx, sizeof(double) * 2 * RMAXB * (kMaxKrylov + 1));
    double* part = ctx->ws_red.as<double>();
    const int nb = red_blocks(n);
    launch_multiaxpy_dot<16>(k, nb, ctx->stream, V, vstride, h, w, n, plane, part, ctx->kstop);
    sum_partials<<<k + 1, RB, 0, ctx->stream>>>(part, nb, 2, h, ctx->kstop);
    FTD_HIP(hipGetLastError());
    return true;
}

// w -= sum_j V_j h[j], then block partials of |w|^2 (one pass over w); not
// at all when the first pass kept enough of w (skip[0] > thr2 * skip[1]).
// KC > 0: exactly KC vectors (the loop unrolls and every load is issued
// up front); KC = 0: k vectors.
template <int KC>
__global__ void multiaxpy_nrm_partial(const double* __restrict__ V, int64_t vstride, int k,
                                      const double* __restrict__ h, double* __restrict__ w,
                                      int64_t n, int64_t plane, double* __restrict__ part,
                                      const int* stop, const double* skip, double thr2) {
    if (stop && *stop) return;
    if (skip && skip[0] > thr2 * skip[1]) return;
    const int kk = KC > 0 ? KC : k;
    __shared__ double sh[16];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ar = w[i], ai = w[i + plane];
#pragma unroll
        for (int j = 0; j < kk; ++j) {
            const double hr = h[2 * j], hi = h[2 * j + 1];
            const double vr = V[(int64_t)j * vstride + i], vi = V[(int64_t)j * vstride + i + plane];
            ar -= vr * hr - vi * hi;
            ai -= vr * hi + vi * hr;
        }
        w[i] = ar;
        w[i + plane] = ai;
        s += ar * ar + ai * ai;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// launch multiaxpy_nrm_partial<k> for 1 <= k <= KC, the generic <0> above
template <int KC>
static void launch_multiaxpy_nrm(int k, int nb, hipStream_t st, const double* V, int64_t vstride,
                                 const double* h, double* w, int64_t n, int64_t plane,
                                 double* part, const int* stop, const double* skip,
                                 double thr2) {
    if (k > KC || k < 1) {
        multiaxpy_nrm_partial<0><<<nb, RB, 0, st>>>(V, vstride, k, h, w, n, plane, part, stop,
                                                    skip, thr2);
        return;
    }
    if constexpr (KC > 1) {
        if (k < KC) {
            launch_multiaxpy_nrm<KC - 1>(k, nb, st, V, vstride, h, w, n, plane, part, stop, skip,
                                         thr2);
            return;
        }
    }
    multiaxpy_nrm_partial<KC><<<nb, RB, 0, st>>>(V, vstride, k, h, w, n, plane, part, stop, skip,
                                                 thr2);
}
int k_multiaxpy_nrm2_part(Ctx* ctx, const double* V, int64_t vstride, int k, const double* h,
                          double* w, int64_t n, int64_t plane, const double* skip, double thr2) {
    const int nb = red_blocks(n);
    ctx->ws_red.ensure(ctx, sizeof(double) * 2 * RMAXB * (kMaxKrylov + 1));
    double* part = ctx->ws_red.as<double>();
    launch_multiaxpy_nrm<16>(k, nb, ctx->stream, V, vstride, h, w, n, plane, part, ctx->kstop,
                             skip, thr2);
    FTD_HIP(hipGetLastError());
    return nb;
}

__global__ void multiaxpy_kernel(const double* __restrict__ V, int64_t vstride, int k,
                                 const double* __restrict__ h, double* __restrict__ w, int64_t n,
                                 int64_t plane, const int* stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ar = w[i], ai = w[i + plane];
        for (int j = 0; j < k; ++j) {
            const double hr = h[2 * j], hi = h[2 * j + 1];
            const double vr = V[(int64_t)j * vstride + i], vi = V[(int64_t)j * vstride + i + plane];
            ar -= vr * hr - vi * hi;
            ai -= vr * hi + vi * hr;
        }
        w[i] = ar;
        w[i + plane] = ai;
    }
}
void k_multiaxpy(Ctx* ctx, const double* V, int64_t vstride, int k, const double* h, double* w,
                 int64_t n, int64_t plane) {
    if (k <= 0 || n <= 0) return;
    multiaxpy_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(V, vstride, k, h, w, n, plane,
                                                           ctx->kstop);
    FTD_HIP(hipGetLastError());
}

__global__ void lincomb_kernel(const double* __restrict__ V, int64_t vstride, int k,
                               const double* __restrict__ u, const double* __restrict__ sc,
                               double* __restrict__ y, int64_t n, int64_t plane) {
    const double s = sqrt(sc[0]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int j = 0; j < k; ++j) {
            const double ur = u[2 * j], ui = u[2 * j + 1];
            const double vr = V[(int64_t)j * vstride + i], vi = V[(int64_t)j * vstride + i + plane];
            ar += vr * ur - vi * ui;
            ai += vr * ui + vi * ur;
        }
        y[i] = s * ar;
        y[i + plane] = s * ai;
    }
}
// y = sqrt(scale_dev[0]) * sum_j V_j u_j   (scale_dev holds a squared norm)
void k_lincomb(Ctx* ctx, const double* V, int64_t vstride, int k, const double* u,
               const double* scale_dev, double* y, int64_t n, int64_t plane) {
    if (n <= 0) return;
    lincomb_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(V, vstride, k, u, scale_dev, y, n, plane);
    FTD_HIP(hipGetLastError());
}

// ------------------------------------------------------------ channel mixing
// y[a][o][q][b] (+)= sum_entries sum_p op[o][p] x[a][p][q][b] for every job
// (output channel).  Grid: x over b (the contiguous index), y over the row
// (a, q), z over jobs.  DN > 0 is the exact local dimension (unrolled); DN = 0
// handles any d <= 32.
template <typename Tin, typename Tout, int DN>
__global__ __launch_bounds__(256) void chanmix_kernel(const Tin* __restrict__ in,
                                                      const Tin* __restrict__ ops,
                                                      Tout* __restrict__ out, const MixParams p) {
    if (p.stop && *p.stop) return;
    constexpr int MAXD = DN > 0 ? DN : 32;
    const int d = DN > 0 ? DN : p.d;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.Db) return;
    const int row = blockIdx.y;            // a * d + q
    const int a = row / d, q = row - a * d;
    const int job = blockIdx.z;
    const int64_t ldi = p.ldIn ? p.ldIn : p.Db;
    const int64_t ldo = p.ldOut ? p.ldOut : p.Db;
    Tin accr[MAXD], acci[MAXD];
#pragma unroll
    for (int o = 0; o < MAXD; ++o) {
        accr[o] = 0;
        acci[o] = 0;
    }
    for (int en = p.job[job].e0; en < p.job[job].e1; ++en) {
        const Tin* x = in + p.ent[en].offIn + ((int64_t)a * d * d + q) * ldi + b;
        const Tin* opr = ops + (int64_t)p.ent[en].op * p.opStride;
        const Tin* opi = opr + (int64_t)d * d;
        for (int pp = 0; pp < d; ++pp) {
            const Tin xr = x[(int64_t)pp * d * ldi], xi = x[(int64_t)pp * d * ldi + p.planeIn];
#pragma unroll
            for (int o = 0; o < MAXD; ++o) {
                if (DN > 0 || o < d) {
                    const Tin orr = opr[o * d + pp], oi = opi[o * d + pp];
                    accr[o] += orr * xr - oi * xi;
                    acci[o] += orr * xi + oi * xr;
                }
            }
        }
    }
    Tout* y = out + p.job[job].offOut + ((int64_t)a * d * d + q) * ldo + b;
#pragma unroll
    for (int o = 0; o < MAXD; ++o) {
        if (DN == 0 && o >= d) continue;
        if (p.accumulate) {
            y[(int64_t)o * d * ldo] += (Tout)accr[o];
            y[(int64_t)o * d * ldo + p.planeOut] += (Tout)acci[o];
        } else {
            y[(int64_t)o * d * ldo] = (Tout)accr[o];
            y[(int64_t)o * d * ldo + p.planeOut] = (Tout)acci[o];
        }
    }
}

template <typename Tin, typename Tout>
static void chanmix_t(Ctx* ctx, const void* in, const void* ops, void* out, const MixParams& p) {
    if ((int64_t)p.Da * p.d * p.Db * p.njobs <= 0) return;
    const int tb = p.Db >= 256 ? 256 : (p.Db >= 128 ? 128 : 64);
    dim3 g((p.Db + tb - 1) / tb, (unsigned)(p.Da * p.d), (unsigned)p.njobs);
    const Tin* a = static_cast<const Tin*>(in);
    const Tin* o = static_cast<const Tin*>(ops);
    Tout* y = static_cast<Tout*>(out);
    switch (p.d) {
        case 2: chanmix_kernel<Tin, Tout, 2><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        case 4: chanmix_kernel<Tin, Tout, 4><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        case 6: chanmix_kernel<Tin, Tout, 6><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        case 8: chanmix_kernel<Tin, Tout, 8><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        case 10: chanmix_kernel<Tin, Tout, 10><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        case 12: chanmix_kernel<Tin, Tout, 12><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
        default: chanmix_kernel<Tin, Tout, 0><<<g, tb, 0, ctx->stream>>>(a, o, y, p); break;
    }
    FTD_HIP(hipGetLastError());
}

void chanmix(Ctx* ctx, Prec prec, bool out_f64, const void* in, const void* ops, void* out,
             const MixParams& p) {
    FTD_CHECK(p.d <= 32, FTD_EINVAL, "local dimension above 32 is not supported");
    FTD_CHECK((int64_t)p.Da * p.d < 65536, FTD_EINVAL, "channel mixer: Da * d too large");
    if (p.njobs == 0) return;
    MixParams q = p;
    q.stop = ctx->kstop;
    if (prec == Prec::F64)
        chanmix_t<double, double>(ctx, in, ops, out, q);
    else if (out_f64)
        chanmix_t<float, double>(ctx, in, ops, out, q);
    else
        chanmix_t<float, float>(ctx, in, ops, out, q);
}

// ------------------------------------------------------ MPO x MPS, embedding
__global__ void mpo_apply_kernel(const double* __restrict__ A, int Da, int d, int Db,
                                 const double* __restrict__ ops, int64_t opStride, int wl, int wr,
                                 const ApplyEnt* __restrict__ ents, int nents,
                                 double* __restrict__ B) {
    const int64_t per = (int64_t)Da * d * Db;   // (a, q, b)
    const int64_t tot = per * nents;
    const int64_t nA = (int64_t)Da * d * d * Db;
    const int64_t DA = (int64_t)Da * wl, DB = (int64_t)Db * wr;
    const int64_t nB = DA * d * d * DB;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int en = (int)(e / per);
        const int64_t r = e % per;
        const int a = (int)(r / ((int64_t)d * Db));
        const int q = (int)((r / Db) % d);
        const int b = (int)(r % Db);
        const ApplyEnt E = ents[en];
        const double* opr = ops + (int64_t)E.op * opStride;
        const double* opi = opr + (int64_t)d * d;
        const int64_t ar = (int64_t)a * wl + E.cl, bc = (int64_t)b * wr + E.cr;
        for (int P = 0; P < d; ++P) {
            double sr = 0.0, si = 0.0;
            for (int pp = 0; pp < d; ++pp) {
                const int64_t ia = (((int64_t)a * d + pp) * d + q) * Db + b;
                const double xr = A[ia], xi = A[ia + nA];
                const double orr = opr[P * d + pp], oi = opi[P * d + pp];
                sr += orr * xr - oi * xi;
                si += orr * xi + oi * xr;
            }
            const int64_t ib = ((ar * d + P) * d + q) * DB + bc;
            B[ib] = sr;
            B[ib + nB] = si;
        }
    }
}
void k_mpo_apply(Ctx* ctx, const double* A, int Da, int d, int Db, const double* ops,
                 int64_t opStride, int wl, int wr, const ApplyEnt* ents_dev, int nents,
                 double* B) {
    const int64_t nB = (int64_t)Da * wl * d * d * Db * wr;
    k_zero(ctx, B, sizeof(double) * 2 * nB);
    const int64_t tot = (int64_t)Da * d * Db * nents;
    if (tot <= 0) return;
    mpo_apply_kernel<<<grid_for(tot), 256, 0, ctx->stream>>>(A, Da, d, Db, ops, opStride, wl, wr,
                                                              ents_dev, nents, B);
    FTD_HIP(hipGetLastError());
}

__global__ void embed_kernel(const double* __restrict__ src, int Da, int dd, int Db,
                             double* __restrict__ dst, int DA, int DB, int a0, int b0, double re,
                             double im, int acc) {
    const int64_t n = (int64_t)Da * dd * Db;
    const int64_t N = (int64_t)DA * dd * DB;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(e / ((int64_t)dd * Db));
        const int s = (int)((e / Db) % dd);
        const int b = (int)(e % Db);
        const double xr = src[e], xi = src[e + n];
        const int64_t o = (((int64_t)(a + a0)) * dd + s) * DB + (b + b0);
        if (acc) {
            dst[o] += re * xr - im * xi;
            dst[o + N] += re * xi + im * xr;
        } else {
            dst[o] = re * xr - im * xi;
            dst[o + N] = re * xi + im * xr;
        }
    }
}
void k_embed(Ctx* ctx, const double* src, int Da, int dd, int Db, double* dst, int DA, int DB,
             int a0, int b0, double re, double im, int accumulate) {
    const int64_t n = (int64_t)Da * dd * Db;
    if (n <= 0) return;
    embed_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(src, Da, dd, Db, dst, DA, DB, a0, b0, re,
                                                        im, accumulate);
    FTD_HIP(hipGetLastError());
}

__global__ void transpose_kernel(const double* __restrict__ s, int64_t rows, int64_t cols,
                                 int64_t splane, double* __restrict__ d, int64_t dplane, int conj) {
    __shared__ double tr[32][33], ti[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) {
            tr[k][tx] = s[r * cols + c];
            ti[k][tx] = s[r * cols + c + splane];
        }
    }
    __syncthreads();
    const double sg = conj ? -1.0 : 1.0;
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;   // dst row = c, dst col = r
        if (r < rows && c < cols) {
            d[c * rows + r] = tr[tx][k];
            d[c * rows + r + dplane] = sg * ti[tx][k];
        }
    }
}
void k_transpose(Ctx* ctx, const double* src, int64_t rows, int64_t cols, int64_t splane,
                 double* dst, int64_t dplane, int conj) {
    if (rows <= 0 || cols <= 0) return;
    dim3 g((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    transpose_kernel<<<g, 256, 0, ctx->stream>>>(src, rows, cols, splane, dst, dplane, conj);
    FTD_HIP(hipGetLastError());
}

// ------------------------------------------------------ Krylov: tridiagonal
// Exponential of the n x n Lanczos matrix T (diag alpha, off-diagonal beta)
// applied to e_1, by the implicit QL algorithm with Wilkinson shifts (one
// wavefront: lane j owns row j of the eigenvector matrix; the scalar
// recurrences are evaluated identically in every lane and exchanged by
// lane reads).  Also records beta_{n-1} = |w| and the convergence decision.
// Value of v in lane i, for a wavefront-uniform i: two v_readlane into scalar
// registers (much cheaper than a cross-lane permute through LDS).
__device__ __forceinline__ double lane_get(double v, int i) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

// The squared norm of the new Lanczos residual arrives as `nb` block
// partials (summed here in a fixed order, and stored to kd.nrm[0]), or as
// skip[0] when the second Gram-Schmidt pass was skipped (the same test as in
// multiaxpy_nrm_partial).
__global__ __launch_bounds__(64) void tridiag_expm_kernel(KrylovDev kd, int n, double zr,
                                                          double zi, double tol, int exhausted,
                                                          int mmax, const double* nrm_part,
                                                          int nb, const double* skip,
                                                          double thr2) {
    __shared__ double Z[kMaxKrylov][kMaxKrylov + 1];
    if (kd.flag[3]) return;   // an earlier iteration converged or failed
    const int j = threadIdx.x;
    double nsq = 0.0;
    if (skip && skip[0] > thr2 * skip[1]) {
        nsq = skip[0];
    } else {
        for (int b = j; b < nb; b += 64) nsq += nrm_part[b];
        for (int o = 32; o > 0; o >>= 1) nsq += __shfl_xor(nsq, o, 64);
    }
    if (j == 0) kd.nrm[0] = nsq;
    const double bnew = sqrt(fmax(nsq, 0.0));
    double dj = (j < n) ? kd.alpha[j] : 0.0;
    double ej = (j < n - 1) ? kd.beta[j] : 0.0;
    for (int i = 0; i < n; ++i) Z[j][i] = (i == j) ? 1.0 : 0.0;
    int fail = 0;
    for (int l = 0; l < n && !fail; ++l) {
        int iter = 0;
        while (true) {
            int m;
            for (m = l; m < n - 1; ++m) {
                const double dd = fabs(lane_get(dj, m)) + fabs(lane_get(dj, m + 1));
                if (fabs(lane_get(ej, m)) <= DBL_EPSILON * dd) break;
            }
            if (m == l) break;
            if (iter++ == 60) {
                fail = 1;
                break;
            }
            const double dl = lane_get(dj, l), el = lane_get(ej, l);
            double g = (lane_get(dj, l + 1) - dl) / (2.0 * el);
            double r = sqrt(fma(g, g, 1.0));
            g = lane_get(dj, m) - dl + el / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = m - 1; i >= l; --i) {
                const double ei = lane_get(ej, i);
                const double f = s * ei, b = c * ei;
                r = sqrt(fma(f, f, g * g));
                if (j == i + 1) ej = r;
                if (r == 0.0) {
                    const double v = lane_get(dj, i + 1) - p;
                    if (j == i + 1) dj = v;
                    if (j == m) ej = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = lane_get(dj, i + 1) - p;
                r = (lane_get(dj, i) - g) * s + 2.0 * c * b;
                p = s * r;
                if (j == i + 1) dj = g + p;
                g = c * r - b;
                const double zf = Z[j][i + 1], zi0 = Z[j][i];
                Z[j][i + 1] = s * zi0 + c * zf;
                Z[j][i] = c * zi0 - s * zf;
            }
            if (early) continue;
            const double v = lane_get(dj, l) - p;
            if (j == l) {
                dj = v;
                ej = g;
            }
            if (j == m) ej = 0.0;
        }
    }
    __syncthreads();
    // u_j = sum_i Z[j][i] exp(z lambda_i) Z[0][i]; the factors
    // exp(z lambda_i) Z[0][i] are formed one eigenvalue per lane
    double cr = 0.0, ci = 0.0;
    if (j < n) {
        const double mag = exp(zr * dj);
        double sn, cs;
        sincos(zi * dj, &sn, &cs);
        cr = mag * cs * Z[0][j];
        ci = mag * sn * Z[0][j];
    }
    double ur = 0.0, ui = 0.0;
    for (int i = 0; i < n; ++i) {
        const double zz = (j < n) ? Z[j][i] : 0.0;
        ur += zz * lane_get(cr, i);
        ui += zz * lane_get(ci, i);
    }
    double nn = (j < n) ? ur * ur + ui * ui : 0.0;
    for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
    const double ulr = lane_get(ur, n - 1), uli = lane_get(ui, n - 1);
    const double err = bnew * sqrt(ulr * ulr + uli * uli);
    if (j < n) {
        kd.u[2 * j] = ur;
        kd.u[2 * j + 1] = ui;
    }
    if (j == 0) {
        kd.beta[n - 1] = bnew;
        const bool finite = isfinite(nn) && isfinite(bnew);
        const int conv = (exhausted || err <= tol * sqrt(nn) || bnew == 0.0) ? 1 : 0;
        const int ok = (finite && !fail) ? conv : 0;
        const int bad = (!finite || fail || (!conv && n >= mmax)) ? 1 : 0;
        kd.flag[0] = ok;
        kd.flag[1] = n;
        kd.flag[2] = bad;
        kd.flag[3] = (ok || bad) ? 1 : 0;
    }
}

// w /= beta_{n-1} unless converged (the next Lanczos vector); with out32,
// also its float copy
__global__ void lanczos_post_kernel(KrylovDev kd, int n, double* w, int64_t len, int64_t plane,
                                    float* out32) {
    if (kd.flag[3]) return;
    const double b = kd.beta[n - 1];
    const double f = 1.0 / b;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = w[i] * f, c = w[i + plane] * f;
        w[i] = a;
        w[i + plane] = c;
        if (out32) {
            out32[i] = (float)a;
            out32[i + plane] = (float)c;
        }
    }
}
__global__ void krylov_reset_kernel(KrylovDev kd) {
    kd.flag[0] = 0;
    kd.flag[1] = 0;
    kd.flag[2] = 0;
    kd.flag[3] = 0;
}
void k_krylov_reset(Ctx* ctx, KrylovDev kd) {
    krylov_reset_kernel<<<1, 1, 0, ctx->stream>>>(kd);
    FTD_HIP(hipGetLastError());
}

void k_tridiag_expm(Ctx* ctx, KrylovDev kd, int k, double zr, double zi, double tol,
                    int exhausted, const double* nrm_part, int nb, const double* skip,
                    double thr2) {
    tridiag_expm_kernel<<<1, 64, 0, ctx->stream>>>(kd, k, zr, zi, tol, exhausted, kMaxKrylov,
                                                   nrm_part, nb, skip, thr2);
    FTD_HIP(hipGetLastError());
}
void k_lanczos_post(Ctx* ctx, KrylovDev kd, int k, double* w, int64_t n, int64_t plane,
                    float* out32) {
    lanczos_post_kernel<<<grid_for(n), 256, 0, ctx->stream>>>(kd, k, w, n, plane, out32);
    FTD_HIP(hipGetLastError());
}

}  // namespace ftd
