// Complex split-plane GEMM on CDNA4 matrix cores.
//
// One workgroup (4 wavefronts) computes a 64x64 tile of C.  The k loop is
// software-pipelined: the next 16-deep tile is loaded into registers while
// the current one (in one of two LDS buffers) feeds the MFMAs.  Each wavefront
// owns a 32x32 quadrant as 2x2 blocks of 16x16 MFMA outputs.  Complex
// products: float64 issues four real products per block and k-step (re*re,
// im*im, re*im, im*re) into three accumulators, Re C = RR - II and
// Im C = RI + IR; float32 uses the three-multiplication form (Gauss):
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), Re C = P1 - P2,
// Im C = P3 - P1 - P2, with the sums formed when staging (a third LDS plane
// per operand), which takes a quarter of the matrix-core work away at a
// rounding cost of order eps |A| |B|.  Operands are staged through LDS as
// [plane][k][m] / [plane][k][n] so that the 16 lanes sharing a k row read 16
// consecutive elements.  Conjugation is applied while staging.  Problems (independent outputs) and summed terms (products added
// into the same output) are described by offset tables passed by value, which
// is how the channel sums of the effective Hamiltonian map onto one launch.
#include "common.h"

namespace ftd {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Output row of accumulator register r in lane `lane` within a 16x16 block.
// f64 16x16x4 spreads rows as 4*r + lane/16, f32 16x16x4 as 4*(lane/16) + r
// (checked by a lane-layout probe on gfx950).  Columns are lane % 16 and the
// operand layouts are A[i][k] in lane i + 16k, B[k][j] in lane j + 16k.
template <typename T>
struct AccT;
template <>
struct AccT<double> {
    typedef d4 type;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct AccT<float> {
    typedef f4 type;
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int GBM = 64, GBN = 64, GBK = 16, GNT = 256, GPAD = 1;

template <typename Tin, typename Tout, bool AK, bool BKC>
__global__ __launch_bounds__(GNT) void gemm_kernel(const Tin* __restrict__ A,
                                                   const Tin* __restrict__ B,
                                                   Tout* __restrict__ C,
                                                   Tin* __restrict__ partial, const GemmParams p) {
    typedef typename AccT<Tin>::type acc_t;
    // three-multiplication complex product in float32 (see the file comment)
    constexpr bool G3 = sizeof(Tin) == 4;
    constexpr int NPL = G3 ? 3 : 2;
    if (p.stop && *p.stop) return;
    if (p.tstamp && threadIdx.x == 0) atomicMin(p.tstamp, (unsigned long long)wall_clock64());
    // two LDS buffers (double buffering), each [plane][k][m] / [plane][k][n];
    // plane 2 (float32 only) holds re + im
    __shared__ Tin As[2][NPL][GBK][GBM + GPAD];
    __shared__ Tin Bs[2][NPL][GBK][GBN + GPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int prob = blockIdx.z % p.nprob;
    const int split = blockIdx.z / p.nprob;

    acc_t RR[2][2], II[2][2], IM[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            RR[i][j] = acc_t{0, 0, 0, 0};
            II[i][j] = acc_t{0, 0, 0, 0};
            IM[i][j] = acc_t{0, 0, 0, 0};
        }

    const int ktiles = (p.K + GBK - 1) / GBK;
    const int t0 = p.prob[prob].t0, t1 = p.prob[prob].t1;
    const int total = (t1 - t0) * ktiles;
    const int per = (total + p.ksplit - 1) / p.ksplit;
    const int g0 = split * per;
    const int g1 = min(total, g0 + per);
    const Tin sa = p.conjA ? Tin(-1) : Tin(1);
    const Tin sb = p.conjB ? Tin(-1) : Tin(1);

    // this thread's share of one k-tile: 4 (re, im) pairs of A and of B.
    // Loads are unconditional from clamped (always valid) addresses, so the
    // next tile's loads stay in flight during the MFMAs; out-of-range
    // elements are zeroed, and the conjugation sign applied, when staging.
    Tin ra[4], ia[4], rb[4], ib[4];
    unsigned inA = 0, inB = 0;   // bit i: element i lies inside the matrix
    auto fetch = [&](int g) {
        const int t = t0 + g / ktiles;
        const int k0 = (g % ktiles) * GBK;
        const Tin* Ab = A + p.term[t].offA;
        const Tin* Bb = B + p.term[t].offB;
        inA = 0;
        inB = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int mm = AK ? (tid >> 4) + 16 * i : (tid & 63);
            const int kk = AK ? (tid & 15) : (tid >> 6) + 4 * i;
            const int gm = m0 + mm, gk = k0 + kk;
            inA |= (unsigned)(gm < p.M && gk < p.K) << i;
            const int64_t idx = (int64_t)min(gm, p.M - 1) * p.sAm + (int64_t)min(gk, p.K - 1) * p.sAk;
            ra[i] = Ab[idx];
            ia[i] = Ab[idx + p.planeA];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int nn = BKC ? (tid >> 4) + 16 * i : (tid & 63);
            const int kk = BKC ? (tid & 15) : (tid >> 6) + 4 * i;
            const int gn = n0 + nn, gk = k0 + kk;
            inB |= (unsigned)(gn < p.N && gk < p.K) << i;
            const int64_t idx = (int64_t)min(gk, p.K - 1) * p.sBk + (int64_t)min(gn, p.N - 1) * p.sBn;
            rb[i] = Bb[idx];
            ib[i] = Bb[idx + p.planeB];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int mm = AK ? (tid >> 4) + 16 * i : (tid & 63);
            const int kk = AK ? (tid & 15) : (tid >> 6) + 4 * i;
            const bool in = (inA >> i) & 1u;
            const Tin xr = in ? ra[i] : Tin(0), xi = in ? sa * ia[i] : Tin(0);
            As[buf][0][kk][mm] = xr;
            As[buf][1][kk][mm] = xi;
            if constexpr (G3) As[buf][NPL - 1][kk][mm] = xr + xi;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int nn = BKC ? (tid >> 4) + 16 * i : (tid & 63);
            const int kk = BKC ? (tid & 15) : (tid >> 6) + 4 * i;
            const bool in = (inB >> i) & 1u;
            const Tin xr = in ? rb[i] : Tin(0), xi = in ? sb * ib[i] : Tin(0);
            Bs[buf][0][kk][nn] = xr;
            Bs[buf][1][kk][nn] = xi;
            if constexpr (G3) Bs[buf][NPL - 1][kk][nn] = xr + xi;
        }
    };

    if (g0 < g1) {
        fetch(g0);
        stash(0);
        __syncthreads();
    }
    for (int g = g0; g < g1; ++g) {
        const int cur = (g - g0) & 1;
        // the next tile's global loads are in flight during the MFMAs below
        if (g + 1 < g1) fetch(g + 1);
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 4) {
            const int kr = kk + (lane >> 4);
            const int c = lane & 15;
            Tin ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                ar[i] = As[cur][0][kr][wm * 32 + i * 16 + c];
                ai[i] = As[cur][1][kr][wm * 32 + i * 16 + c];
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                br[j] = Bs[cur][0][kr][wn * 32 + j * 16 + c];
                bi[j] = Bs[cur][1][kr][wn * 32 + j * 16 + c];
            }
            if constexpr (G3) {
                // RR = Ar Br, II = Ai Bi, IM = (Ar + Ai)(Br + Bi)
                Tin as[2], bs[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) as[i] = As[cur][NPL - 1][kr][wm * 32 + i * 16 + c];
#pragma unroll
                for (int j = 0; j < 2; ++j) bs[j] = Bs[cur][NPL - 1][kr][wn * 32 + j * 16 + c];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        RR[i][j] = mfma4(ar[i], br[j], RR[i][j]);
                        II[i][j] = mfma4(ai[i], bi[j], II[i][j]);
                        IM[i][j] = mfma4(as[i], bs[j], IM[i][j]);
                    }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        RR[i][j] = mfma4(ar[i], br[j], RR[i][j]);
                        II[i][j] = mfma4(ai[i], bi[j], II[i][j]);
                        IM[i][j] = mfma4(ar[i], bi[j], IM[i][j]);
                        IM[i][j] = mfma4(ai[i], br[j], IM[i][j]);
                    }
            }
        }
        // the other buffer was last read in the previous iteration, which
        // ended with a barrier
        if (g + 1 < g1) stash(cur ^ 1);
        __syncthreads();
    }

    const int64_t MN = (int64_t)p.M * p.N;
    const int64_t pplane = (int64_t)p.ksplit * p.nprob * MN;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + AccT<Tin>::row(lane, r);
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < p.M && col < p.N) {
                    const Tin cr = RR[i][j][r] - II[i][j][r];
                    const Tin ci = G3 ? IM[i][j][r] - RR[i][j][r] - II[i][j][r] : IM[i][j][r];
                    if (p.ksplit > 1) {
                        const int64_t idx = ((int64_t)split * p.nprob + prob) * MN + (int64_t)row * p.N + col;
                        partial[idx] = cr;
                        partial[idx + pplane] = ci;
                    } else {
                        const int64_t idx = p.prob[prob].offC + (int64_t)row * p.sCm + (int64_t)col * p.sCn;
                        if (p.accumulate) {
                            C[idx] += (Tout)cr;
                            C[idx + p.planeC] += (Tout)ci;
                        } else {
                            C[idx] = (Tout)cr;
                            C[idx + p.planeC] = (Tout)ci;
                        }
                    }
                }
            }
    if (p.tstamp) {
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(p.tstamp + 1, (unsigned long long)wall_clock64());
    }
}

// ------------------------------------------------------------ BF16x3 path
// Complex GEMM on float32 data with bf16 matrix cores: every float32
// operand x is split when staging into x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (round to nearest even), and each real product a b
// is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi with float32 accumulation
// (the dropped a_lo b_lo and the split leave a relative error of order
// 2^-17 per product).  v_mfma_f32_16x16x32_bf16: lane l holds rows/columns
// l % 16 and the eight k values 8 (l / 16) .. 8 (l / 16) + 7 of its operand;
// the 16x16 float32 result uses the float32 16x16x4 layout.  One workgroup
// (4 wavefronts, each a 32x32 quadrant as 2x2 blocks) per 64x64 tile; k
// advances 32 at a time.  The operands sit in LDS as [plane][row][k] with k
// contiguous (planes re_hi, re_lo, im_hi, im_lo), so each lane fetches its
// eight values with one 16-byte read; the next k-tile's global loads are in
// flight during the current tile's MFMAs (one LDS buffer, register staging).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits_rn(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite x)
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}

constexpr int XBK = 32, XPAD = 8;

template <typename Tout, bool AK, bool BKC>
__global__ __launch_bounds__(GNT) void gemm_bx3_kernel(const float* __restrict__ A,
                                                       const float* __restrict__ B,
                                                       Tout* __restrict__ C,
                                                       float* __restrict__ partial,
                                                       const GemmParams p) {
    if (p.stop && *p.stop) return;
    if (p.tstamp && threadIdx.x == 0) atomicMin(p.tstamp, (unsigned long long)wall_clock64());
    // [plane: re_hi, re_lo, im_hi, im_lo][row][k]
    __shared__ __align__(16) unsigned short As[4][GBM][XBK + XPAD];
    __shared__ __align__(16) unsigned short Bs[4][GBN][XBK + XPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int prob = blockIdx.z % p.nprob;
    const int split = blockIdx.z / p.nprob;

    f4 RR[2][2], II[2][2], IM[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            RR[i][j] = f4{0, 0, 0, 0};
            II[i][j] = f4{0, 0, 0, 0};
            IM[i][j] = f4{0, 0, 0, 0};
        }

    const int ktiles = (p.K + XBK - 1) / XBK;
    const int t0 = p.prob[prob].t0, t1 = p.prob[prob].t1;
    const int total = (t1 - t0) * ktiles;
    const int per = (total + p.ksplit - 1) / p.ksplit;
    const int g0 = split * per;
    const int g1 = min(total, g0 + per);
    const float sa = p.conjA ? -1.f : 1.f;
    const float sb = p.conjB ? -1.f : 1.f;

    // a 64 x 32 tile of A and a 32 x 64 tile of B: 8 (re, im) pairs each per
    // thread; element e = tid + 256 i, k fastest when the operand is
    // k-contiguous, else the row index fastest.  Clamped addresses keep every
    // load valid; out-of-range elements are zeroed at staging.
    float ra[8], ia[8], rb[8], ib[8];
    unsigned inA = 0, inB = 0;
    auto a_rc = [&](int e, int& r, int& k) {
        if (AK) { r = e / XBK; k = e % XBK; } else { r = e % GBM; k = e / GBM; }
    };
    auto b_rc = [&](int e, int& r, int& k) {
        if (BKC) { r = e / XBK; k = e % XBK; } else { r = e % GBN; k = e / GBN; }
    };
    auto fetch = [&](int g) {
        const int t = t0 + g / ktiles;
        const int k0 = (g % ktiles) * XBK;
        const float* Ab = A + p.term[t].offA;
        const float* Bb = B + p.term[t].offB;
        inA = 0;
        inB = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int mm, kk;
            a_rc(tid + 256 * i, mm, kk);
            const int gm = m0 + mm, gk = k0 + kk;
            inA |= (unsigned)(gm < p.M && gk < p.K) << i;
            const int64_t idx = (int64_t)min(gm, p.M - 1) * p.sAm + (int64_t)min(gk, p.K - 1) * p.sAk;
            ra[i] = Ab[idx];
            ia[i] = Ab[idx + p.planeA];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int nn, kk;
            b_rc(tid + 256 * i, nn, kk);
            const int gn = n0 + nn, gk = k0 + kk;
            inB |= (unsigned)(gn < p.N && gk < p.K) << i;
            const int64_t idx = (int64_t)min(gk, p.K - 1) * p.sBk + (int64_t)min(gn, p.N - 1) * p.sBn;
            rb[i] = Bb[idx];
            ib[i] = Bb[idx + p.planeB];
        }
    };
    auto split_store = [](unsigned short (*P)[XBK + XPAD], unsigned short (*Q)[XBK + XPAD], int r,
                          int k, float x) {
        const unsigned short h = bf16_bits_rn(x);
        P[r][k] = h;
        Q[r][k] = bf16_bits_rn(x - bf16_bits_to_float(h));
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int mm, kk;
            a_rc(tid + 256 * i, mm, kk);
            const bool in = (inA >> i) & 1u;
            split_store(As[0], As[1], mm, kk, in ? ra[i] : 0.f);
            split_store(As[2], As[3], mm, kk, in ? sa * ia[i] : 0.f);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int nn, kk;
            b_rc(tid + 256 * i, nn, kk);
            const bool in = (inB >> i) & 1u;
            split_store(Bs[0], Bs[1], nn, kk, in ? rb[i] : 0.f);
            split_store(Bs[2], Bs[3], nn, kk, in ? sb * ib[i] : 0.f);
        }
    };
    auto frag = [](const unsigned short* row, int kq) {
        return *reinterpret_cast<const bf16x8*>(row + 8 * kq);
    };

    if (g0 < g1) fetch(g0);
    for (int g = g0; g < g1; ++g) {
        // the previous tile's MFMAs are done reading LDS
        __syncthreads();
        stash();
        __syncthreads();
        if (g + 1 < g1) fetch(g + 1);
        const int c = lane & 15, kq = lane >> 4;
        bf16x8 a[2][4], b[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[i][q] = frag(As[q][wm * 32 + i * 16 + c], kq);
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) b[j][q] = frag(Bs[q][wn * 32 + j * 16 + c], kq);
        // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                RR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][0], RR[i][j], 0, 0, 0);
                RR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][1], RR[i][j], 0, 0, 0);
                RR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], RR[i][j], 0, 0, 0);
                II[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], b[j][2], II[i][j], 0, 0, 0);
                II[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][3], II[i][j], 0, 0, 0);
                II[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][2], II[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][1], b[j][2], IM[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][3], IM[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][3], b[j][0], IM[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][1], IM[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][2], IM[i][j], 0, 0, 0);
                IM[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][2], b[j][0], IM[i][j], 0, 0, 0);
            }
    }

    const int64_t MN = (int64_t)p.M * p.N;
    const int64_t pplane = (int64_t)p.ksplit * p.nprob * MN;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + AccT<float>::row(lane, r);
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < p.M && col < p.N) {
                    const float cr = RR[i][j][r] - II[i][j][r];
                    const float ci = IM[i][j][r];
                    if (p.ksplit > 1) {
                        const int64_t idx = ((int64_t)split * p.nprob + prob) * MN + (int64_t)row * p.N + col;
                        partial[idx] = cr;
                        partial[idx + pplane] = ci;
                    } else {
                        const int64_t idx = p.prob[prob].offC + (int64_t)row * p.sCm + (int64_t)col * p.sCn;
                        if (p.accumulate) {
                            C[idx] += (Tout)cr;
                            C[idx + p.planeC] += (Tout)ci;
                        } else {
                            C[idx] = (Tout)cr;
                            C[idx + p.planeC] = (Tout)ci;
                        }
                    }
                }
            }
    if (p.tstamp) {
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(p.tstamp + 1, (unsigned long long)wall_clock64());
    }
}

template <typename Tin, typename Tout>
__global__ void gemm_reduce_kernel(const Tin* __restrict__ partial, Tout* __restrict__ C,
                                   const GemmParams p) {
    if (p.stop && *p.stop) return;
    const int64_t MN = (int64_t)p.M * p.N;
    const int64_t pplane = (int64_t)p.ksplit * p.nprob * MN;
    const int64_t tot = MN * p.nprob;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int prob = (int)(e / MN);
        const int64_t rc = e % MN;
        const int row = (int)(rc / p.N), col = (int)(rc % p.N);
        Tout sr = 0, si = 0;
        for (int s = 0; s < p.ksplit; ++s) {
            const int64_t idx = ((int64_t)s * p.nprob + prob) * MN + rc;
            sr += (Tout)partial[idx];
            si += (Tout)partial[idx + pplane];
        }
        const int64_t idx = p.prob[prob].offC + (int64_t)row * p.sCm + (int64_t)col * p.sCn;
        if (p.accumulate) {
            C[idx] += sr;
            C[idx + p.planeC] += si;
        } else {
            C[idx] = sr;
            C[idx + p.planeC] = si;
        }
    }
}

template <typename Tout>
static void launch_bx3(Ctx* ctx, const void* A, const void* B, void* C, const GemmParams& p,
                       dim3 grid, float* partial, hipEvent_t mid) {
    const float* a = static_cast<const float*>(A);
    const float* b = static_cast<const float*>(B);
    Tout* c = static_cast<Tout*>(C);
    if (p.a_kcontig && p.b_kcontig)
        gemm_bx3_kernel<Tout, true, true><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else if (p.a_kcontig && !p.b_kcontig)
        gemm_bx3_kernel<Tout, true, false><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else if (!p.a_kcontig && p.b_kcontig)
        gemm_bx3_kernel<Tout, false, true><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else
        gemm_bx3_kernel<Tout, false, false><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    if (mid) FTD_HIP(hipEventRecord(mid, ctx->stream));
    if (p.ksplit > 1) {
        const int64_t tot = (int64_t)p.M * p.N * p.nprob;
        int nb = (int)std::min<int64_t>((tot + 255) / 256, 4096);
        gemm_reduce_kernel<float, Tout><<<nb, 256, 0, ctx->stream>>>(partial, c, p);
    }
}

template <typename Tin, typename Tout>
static void launch(Ctx* ctx, const void* A, const void* B, void* C, const GemmParams& p,
                   dim3 grid, Tin* partial, hipEvent_t mid) {
    const Tin* a = static_cast<const Tin*>(A);
    const Tin* b = static_cast<const Tin*>(B);
    Tout* c = static_cast<Tout*>(C);
    if (p.a_kcontig && p.b_kcontig)
        gemm_kernel<Tin, Tout, true, true><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else if (p.a_kcontig && !p.b_kcontig)
        gemm_kernel<Tin, Tout, true, false><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else if (!p.a_kcontig && p.b_kcontig)
        gemm_kernel<Tin, Tout, false, true><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    else
        gemm_kernel<Tin, Tout, false, false><<<grid, GNT, 0, ctx->stream>>>(a, b, c, partial, p);
    if (mid) FTD_HIP(hipEventRecord(mid, ctx->stream));
    if (p.ksplit > 1) {
        const int64_t tot = (int64_t)p.M * p.N * p.nprob;
        int nb = (int)std::min<int64_t>((tot + 255) / 256, 4096);
        gemm_reduce_kernel<Tin, Tout><<<nb, 256, 0, ctx->stream>>>(partial, c, p);
    }
}

// Number of k-splits of a launch: when the output tiles alone give fewer
// workgroups than there are compute units and there is enough depth, the
// summed k range is split so that about 1024 workgroups run, each over at
// least 4 k-tiles (at most 64 splits); a grid that already covers every
// compute unit is not split (the partial planes and their reduction would
// cost more than the imbalance of the last round of workgroups).  Returns 0
// for a launch with nothing to compute.
static int split_count(const GemmParams& p) {
    int nterms = 0;
    for (int i = 0; i < p.nprob; ++i) nterms = std::max(nterms, p.prob[i].t1 - p.prob[i].t0);
    if (p.K <= 0 || nterms == 0) return 0;
    const int tm = (p.M + GBM - 1) / GBM, tn = (p.N + GBN - 1) / GBN;
    const int ktiles = nterms * ((p.K + GBK - 1) / GBK);
    const int blocks = tm * tn * p.nprob;
    int ks = 1;
    if (blocks < 256 && ktiles >= 8) {
        ks = (1024 + blocks - 1) / blocks;
        ks = std::min(ks, ktiles / 4);
        ks = std::min(ks, 64);
        ks = std::max(ks, 1);
    }
    return ks;
}

static size_t partial_bytes(const GemmParams& p, int ks, size_t esz) {
    return ks > 1 ? 2 * (size_t)ks * p.nprob * (size_t)p.M * p.N * esz : 0;
}

void gemm_in(Ctx* ctx, Prec prec, bool out_f64, const void* A, const void* B, void* C,
             GemmParams p, void* partial, size_t partial_cap) {
    FTD_CHECK(p.nprob >= 1 && p.nprob <= kMaxProbs, FTD_EINVAL, "gemm: bad problem count");
    FTD_CHECK(prec != Prec::F64 || out_f64, FTD_EINVAL, "gemm: f64 inputs need f64 output");
    if (p.M <= 0 || p.N <= 0) return;
    int ks = split_count(p);
    if (ks == 0) {
        FTD_CHECK(p.accumulate, FTD_EINVAL, "gemm: empty contraction without accumulate");
        return;
    }
    const size_t esz = (prec == Prec::F64) ? sizeof(double) : sizeof(float);
    while (ks > 1 && partial_bytes(p, ks, esz) > partial_cap) --ks;
    p.ksplit = ks;
    p.stop = nullptr;
    p.tstamp = nullptr;
    const int tm = (p.M + GBM - 1) / GBM, tn = (p.N + GBN - 1) / GBN;
    dim3 grid(tn, tm, p.nprob * ks);
    if (prec == Prec::F64)
        launch<double, double>(ctx, A, B, C, p, grid, static_cast<double*>(partial), nullptr);
    else if (prec == Prec::BF16X3 && out_f64)
        launch_bx3<double>(ctx, A, B, C, p, grid, static_cast<float*>(partial), nullptr);
    else if (prec == Prec::BF16X3)
        launch_bx3<float>(ctx, A, B, C, p, grid, static_cast<float*>(partial), nullptr);
    else if (out_f64)
        launch<float, double>(ctx, A, B, C, p, grid, static_cast<float*>(partial), nullptr);
    else
        launch<float, float>(ctx, A, B, C, p, grid, static_cast<float*>(partial), nullptr);
    FTD_HIP(hipGetLastError());
}

void gemm(Ctx* ctx, Prec prec, bool out_f64, const void* A, const void* B, void* C,
          GemmParams p, int tag) {
    FTD_CHECK(p.nprob >= 1 && p.nprob <= kMaxProbs, FTD_EINVAL, "gemm: bad problem count");
    if (p.M <= 0 || p.N <= 0) return;
    const int ks = split_count(p);
    if (ks == 0) {
        FTD_CHECK(p.accumulate, FTD_EINVAL, "gemm: empty contraction without accumulate");
        return;
    }
    const int tm = (p.M + GBM - 1) / GBM, tn = (p.N + GBN - 1) / GBN;
    {
        double terms = 0;
        for (int i = 0; i < p.nprob; ++i) terms += p.prob[i].t1 - p.prob[i].t0;
        ctx->stats.all_flops += 8.0 * p.M * (double)p.N * p.K * terms;
    }
    p.ksplit = ks;
    p.stop = ctx->kstop;
    size_t esz = (prec == Prec::F64) ? sizeof(double) : sizeof(float);
    void* partial = nullptr;
    if (ks > 1) {
        ctx->ws_gemm_partial.ensure(ctx, partial_bytes(p, ks, esz));
        partial = ctx->ws_gemm_partial.p;
    }
    dim3 grid(tn, tm, p.nprob * ks);
    hipEvent_t e0 = nullptr, e1 = nullptr, em = nullptr;
    int slot = -1;
    p.tstamp = nullptr;
    if (ctx->timing && tag != TAG_NONE) {
        e0 = timing_event(ctx);
        em = timing_event(ctx);
        p.tstamp = timing_slot(ctx, &slot);
        FTD_HIP(hipEventRecord(e0, ctx->stream));
    }
    if (prec == Prec::F64) {
        FTD_CHECK(out_f64, FTD_EINVAL, "gemm: f64 inputs need f64 output");
        launch<double, double>(ctx, A, B, C, p, grid, static_cast<double*>(partial), em);
    } else if (prec == Prec::BF16X3 && out_f64) {
        launch_bx3<double>(ctx, A, B, C, p, grid, static_cast<float*>(partial), em);
    } else if (prec == Prec::BF16X3) {
        launch_bx3<float>(ctx, A, B, C, p, grid, static_cast<float*>(partial), em);
    } else if (out_f64) {
        launch<float, double>(ctx, A, B, C, p, grid, static_cast<float*>(partial), em);
    } else {
        launch<float, float>(ctx, A, B, C, p, grid, static_cast<float*>(partial), em);
    }
    FTD_HIP(hipGetLastError());
    if (e0) {
        double tot_terms = 0;
        e1 = timing_event(ctx);
        FTD_HIP(hipEventRecord(e1, ctx->stream));
        for (int i = 0; i < p.nprob; ++i) tot_terms += p.prob[i].t1 - p.prob[i].t0;
        const double flops = 8.0 * p.M * (double)p.N * p.K * tot_terms;
        const double cs = 2.0 * (double)esz;
        const double osz = 2.0 * (out_f64 ? 8.0 : (double)esz);
        const double bytes = tot_terms * ((double)p.M * p.K + (double)p.K * p.N) * cs +
                             (double)p.nprob * p.M * p.N * osz * (p.accumulate ? 2.0 : 1.0);
        // kernel identity: precision x operand layout
        const int kind = (int)prec * 8 + (out_f64 ? 4 : 0) + p.a_kcontig * 2 + p.b_kcontig;
        record_kernel(ctx, e0, e1, flops, bytes, tag, kind, em, slot);
    }
}

}  // namespace ftd
