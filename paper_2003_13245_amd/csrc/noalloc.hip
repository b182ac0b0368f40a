// The entry point that allocates nothing: the complex GEMM of ftd_gemm on
// device buffers, with its split-K partial sums in a fixed device array.
//
// The array `scratch` lives in this file, one copy per GPU, for the life of
// the process.  Host code never uses its name as an address (on the host it
// is a stand-in symbol): its device address is looked up once per device with
// hipGetSymbolAddress when the first context on that device is created, and
// only that address is handed to the kernels.
#include <mutex>

#include "common.h"

namespace ftd {

// 32 MiB: at most 2^20 output elements, so at least a two-way k split of the
// largest accepted float64 product fits (2 planes x 2 splits x 2^20 x 8 B).
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int64_t kNoAllocMaxOut = int64_t(1) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

void scratch_init(int device) {
    FTD_CHECK(device >= 0 && device < kMaxDevices, FTD_EINVAL, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return;
    int cur = -1;
    FTD_HIP(hipGetDevice(&cur));
    FTD_CHECK(cur == device, FTD_EDEVICE, "scratch_init: device is not current");
    void* ptr = nullptr;
    FTD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    FTD_CHECK(ptr != nullptr, FTD_EDEVICE, "scratch array has no device address");
    g_scratch_dev[device] = ptr;
}

static void* scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}

}  // namespace ftd

using namespace ftd;

extern "C" ftd_status ftd_gemm_noalloc(ftd_ctx* ctx, int32_t precision, int32_t M, int32_t N,
                                       int32_t K, int32_t transA, int32_t transB, const void* A,
                                       const void* B, double* C) {
    try {
        FTD_CHECK(ctx && A && B && C, FTD_EINVAL, "null argument");
        FTD_CHECK(M >= 1 && N >= 1 && K >= 1, FTD_EINVAL, "empty GEMM");
        FTD_CHECK((int64_t)M * N <= kNoAllocMaxOut, FTD_EINVAL,
                  "ftd_gemm_noalloc: M*N above 2^20 output elements (the scratch maximum)");
        FTD_CHECK(transA >= 0 && transA <= 2 && transB >= 0 && transB <= 2, FTD_EINVAL, "bad trans");
        FTD_CHECK(precision == FTD_C128 || precision == FTD_C64, FTD_EINVAL,
                  "ftd_gemm_noalloc: c128 or c64 only");
        Ctx* c = &ctx->c;
        void* part = scratch_of(c->device);
        FTD_CHECK(part != nullptr, FTD_EDEVICE, "scratch array not set up on this device");
        const int64_t na = (int64_t)M * K, nb = (int64_t)K * N, nc = (int64_t)M * N;
        GemmParams p{};
        p.M = M; p.N = N; p.K = K;
        if (transA == 0) { p.sAm = K; p.sAk = 1; p.a_kcontig = 1; }
        else { p.sAm = 1; p.sAk = M; p.a_kcontig = 0; p.conjA = transA == 2; }
        if (transB == 0) { p.sBk = N; p.sBn = 1; p.b_kcontig = 0; }
        else { p.sBk = 1; p.sBn = K; p.b_kcontig = 1; p.conjB = transB == 2; }
        p.planeA = na; p.planeB = nb;
        p.sCm = N; p.sCn = 1; p.planeC = nc;
        p.nprob = 1; p.prob[0].t1 = 1;
        gemm_in(c, static_cast<Prec>(precision), true, A, B, C, p, part, kScratchBytes);
        return FTD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return FTD_EDEVICE;
    } catch (...) {
        set_error("unknown error");
        return FTD_EDEVICE;
    }
}
