// Issue-rate measurement of gfx950 vector ALU instructions, for the ALU
// ceiling of the pair kernels.  Each workgroup runs independent dependency
// chains of one instruction form (12 chains per lane, 32 waves per SIMD over
// the launch) so that latency is hidden and only issue throughput counts.
// Reported per form: lanes per clock per SIMD at the nominal 2.4 GHz, the
// nominal cycles per 64-lane instruction, and for FMA the FLOP rate.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define VR_CHECK(x)                                                                     \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

namespace {
constexpr int kChains = 12;
constexpr int kThreads = 256;

enum Form { FMA_VVV, MUL_VV, ADD_VV, ADD_VS, RSQ_V, FMA64_VVV, MUL64_VV, ADD64_VV, RSQ64_V, FMA64_RSQ64 };

template <typename T, int F>
__global__ __launch_bounds__(kThreads) void chains(T* out, int iters, T a, T b)
{
    T v[kChains], w[kChains];
    const T la = a + (T)1e-9 * (T)threadIdx.x;  // per-lane values live in VGPRs
    const T lb = b + (T)1e-9 * (T)threadIdx.x;
#pragma unroll
    for (int u = 0; u < kChains; ++u) {
        v[u] = (T)1 + (T)1e-3 * (T)(threadIdx.x + u);
        w[u] = (T)0.5 + (T)1e-3 * (T)(threadIdx.x + u);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kChains; ++u) {
            if (F == FMA_VVV || F == FMA64_VVV) v[u] = v[u] * la + lb;
            else if (F == MUL_VV || F == MUL64_VV) v[u] = v[u] * la;
            else if (F == ADD_VV || F == ADD64_VV) v[u] = v[u] + w[u];
            else if (F == RSQ64_V) v[u] = __builtin_amdgcn_rsq(v[u]);
            else if (F == FMA64_RSQ64) v[u] = (u % 4 == 0) ? __builtin_amdgcn_rsq(v[u]) : v[u] * la + lb;
            else if (F == ADD_VS) v[u] = v[u] + b;  // b is uniform: an SGPR operand
            else if (F == RSQ_V) v[u] = __builtin_amdgcn_rsqf(v[u]);
        }
    }
    T s = 0;
#pragma unroll
    for (int u = 0; u < kChains; ++u) s += v[u] + w[u];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}
// 24 v_fmac_f32 per iteration, sources of mixed register parity
__global__ __launch_bounds__(kThreads) void asm_fmac_mixed_parity(float* out, int iters)
{
    float r;
    asm volatile(
        "v_mov_b32 v16, 1.0\n"
        "v_mov_b32 v18, 1.0\n"
        "v_mov_b32 v20, 1.0\n"
        "v_mov_b32 v22, 1.0\n"
        "v_mov_b32 v24, 1.0\n"
        "v_mov_b32 v26, 1.0\n"
        "v_mov_b32 v28, 1.0\n"
        "v_mov_b32 v30, 1.0\n"
        "v_mov_b32 v32, 1.0\n"
        "v_mov_b32 v34, 1.0\n"
        "v_mov_b32 v36, 1.0\n"
        "v_mov_b32 v38, 1.0\n"
        "v_mov_b32 v1, 0x3f800001\n"
        "v_mov_b32 v3, 0x3f800001\n"
        "s_mov_b32 s40, %1\n"
        "1:\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "s_sub_u32 s40, s40, 1\n"
        "s_cmp_lg_u32 s40, 0\n"
        "s_cbranch_scc1 1b\n"
        "v_mov_b32 %0, v16\n"
        : "=v"(r) : "s"(iters) : "v1", "v3", "v16", "v18", "v20", "v22", "v24", "v26", "v28", "v30", "v32", "v34", "v36", "v38", "s40", "scc");
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// 24 v_fmac_f32 per iteration, all three sources even-numbered
__global__ __launch_bounds__(kThreads) void asm_fmac_same_parity(float* out, int iters)
{
    float r;
    asm volatile(
        "v_mov_b32 v16, 1.0\n"
        "v_mov_b32 v18, 1.0\n"
        "v_mov_b32 v20, 1.0\n"
        "v_mov_b32 v22, 1.0\n"
        "v_mov_b32 v24, 1.0\n"
        "v_mov_b32 v26, 1.0\n"
        "v_mov_b32 v28, 1.0\n"
        "v_mov_b32 v30, 1.0\n"
        "v_mov_b32 v32, 1.0\n"
        "v_mov_b32 v34, 1.0\n"
        "v_mov_b32 v36, 1.0\n"
        "v_mov_b32 v38, 1.0\n"
        "v_mov_b32 v4, 0x3f800001\n"
        "v_mov_b32 v6, 0x3f800001\n"
        "s_mov_b32 s40, %1\n"
        "1:\n"
        "v_fmac_f32 v16, v4, v6\n"
        "v_fmac_f32 v18, v4, v6\n"
        "v_fmac_f32 v20, v4, v6\n"
        "v_fmac_f32 v22, v4, v6\n"
        "v_fmac_f32 v24, v4, v6\n"
        "v_fmac_f32 v26, v4, v6\n"
        "v_fmac_f32 v28, v4, v6\n"
        "v_fmac_f32 v30, v4, v6\n"
        "v_fmac_f32 v32, v4, v6\n"
        "v_fmac_f32 v34, v4, v6\n"
        "v_fmac_f32 v36, v4, v6\n"
        "v_fmac_f32 v38, v4, v6\n"
        "v_fmac_f32 v16, v4, v6\n"
        "v_fmac_f32 v18, v4, v6\n"
        "v_fmac_f32 v20, v4, v6\n"
        "v_fmac_f32 v22, v4, v6\n"
        "v_fmac_f32 v24, v4, v6\n"
        "v_fmac_f32 v26, v4, v6\n"
        "v_fmac_f32 v28, v4, v6\n"
        "v_fmac_f32 v30, v4, v6\n"
        "v_fmac_f32 v32, v4, v6\n"
        "v_fmac_f32 v34, v4, v6\n"
        "v_fmac_f32 v36, v4, v6\n"
        "v_fmac_f32 v38, v4, v6\n"
        "s_sub_u32 s40, s40, 1\n"
        "s_cmp_lg_u32 s40, 0\n"
        "s_cbranch_scc1 1b\n"
        "v_mov_b32 %0, v16\n"
        : "=v"(r) : "s"(iters) : "v4", "v6", "v16", "v18", "v20", "v22", "v24", "v26", "v28", "v30", "v32", "v34", "v36", "v38", "s40", "scc");
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// 24 v_rsq_f32 per iteration
__global__ __launch_bounds__(kThreads) void asm_rsq_only(float* out, int iters)
{
    float r;
    asm volatile(
        "v_mov_b32 v60, 1.0\n"
        "v_mov_b32 v62, 1.0\n"
        "v_mov_b32 v64, 1.0\n"
        "v_mov_b32 v66, 1.0\n"
        "v_mov_b32 v68, 1.0\n"
        "v_mov_b32 v70, 1.0\n"
        "v_mov_b32 v61, 0x3f800001\n"
        "v_mov_b32 v63, 0x3f800001\n"
        "v_mov_b32 v65, 0x3f800001\n"
        "v_mov_b32 v67, 0x3f800001\n"
        "v_mov_b32 v69, 0x3f800001\n"
        "v_mov_b32 v71, 0x3f800001\n"
        "s_mov_b32 s40, %1\n"
        "1:\n"
        "v_rsq_f32 v60, v61\n"
        "v_rsq_f32 v62, v63\n"
        "v_rsq_f32 v64, v65\n"
        "v_rsq_f32 v66, v67\n"
        "v_rsq_f32 v68, v69\n"
        "v_rsq_f32 v70, v71\n"
        "v_rsq_f32 v60, v61\n"
        "v_rsq_f32 v62, v63\n"
        "v_rsq_f32 v64, v65\n"
        "v_rsq_f32 v66, v67\n"
        "v_rsq_f32 v68, v69\n"
        "v_rsq_f32 v70, v71\n"
        "v_rsq_f32 v60, v61\n"
        "v_rsq_f32 v62, v63\n"
        "v_rsq_f32 v64, v65\n"
        "v_rsq_f32 v66, v67\n"
        "v_rsq_f32 v68, v69\n"
        "v_rsq_f32 v70, v71\n"
        "v_rsq_f32 v60, v61\n"
        "v_rsq_f32 v62, v63\n"
        "v_rsq_f32 v64, v65\n"
        "v_rsq_f32 v66, v67\n"
        "v_rsq_f32 v68, v69\n"
        "v_rsq_f32 v70, v71\n"
        "s_sub_u32 s40, s40, 1\n"
        "s_cmp_lg_u32 s40, 0\n"
        "s_cbranch_scc1 1b\n"
        "v_mov_b32 %0, v60\n"
        : "=v"(r) : "s"(iters) : "v60", "v61", "v62", "v63", "v64", "v65", "v66", "v67", "v68", "v69", "v70", "v71", "s40", "scc");
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// 96 v_fmac_f32 and 24 v_rsq_f32 per iteration, one rsq after every four FMAs
__global__ __launch_bounds__(kThreads) void asm_fmac_rsq_mixed(float* out, int iters)
{
    float r;
    asm volatile(
        "v_mov_b32 v16, 1.0\n"
        "v_mov_b32 v18, 1.0\n"
        "v_mov_b32 v20, 1.0\n"
        "v_mov_b32 v22, 1.0\n"
        "v_mov_b32 v24, 1.0\n"
        "v_mov_b32 v26, 1.0\n"
        "v_mov_b32 v28, 1.0\n"
        "v_mov_b32 v30, 1.0\n"
        "v_mov_b32 v32, 1.0\n"
        "v_mov_b32 v34, 1.0\n"
        "v_mov_b32 v36, 1.0\n"
        "v_mov_b32 v38, 1.0\n"
        "v_mov_b32 v60, 1.0\n"
        "v_mov_b32 v62, 1.0\n"
        "v_mov_b32 v64, 1.0\n"
        "v_mov_b32 v66, 1.0\n"
        "v_mov_b32 v68, 1.0\n"
        "v_mov_b32 v70, 1.0\n"
        "v_mov_b32 v1, 0x3f800001\n"
        "v_mov_b32 v3, 0x3f800001\n"
        "v_mov_b32 v61, 0x3f800001\n"
        "v_mov_b32 v63, 0x3f800001\n"
        "v_mov_b32 v65, 0x3f800001\n"
        "v_mov_b32 v67, 0x3f800001\n"
        "v_mov_b32 v69, 0x3f800001\n"
        "v_mov_b32 v71, 0x3f800001\n"
        "s_mov_b32 s40, %1\n"
        "1:\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v60, v61\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v62, v63\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v64, v65\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v66, v67\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v68, v69\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v70, v71\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v60, v61\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v62, v63\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v64, v65\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v66, v67\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v68, v69\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v70, v71\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v60, v61\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v62, v63\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v64, v65\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v66, v67\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v68, v69\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v70, v71\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v60, v61\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v62, v63\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v64, v65\n"
        "v_fmac_f32 v16, v1, v3\n"
        "v_fmac_f32 v18, v1, v3\n"
        "v_fmac_f32 v20, v1, v3\n"
        "v_fmac_f32 v22, v1, v3\n"
        "v_rsq_f32 v66, v67\n"
        "v_fmac_f32 v24, v1, v3\n"
        "v_fmac_f32 v26, v1, v3\n"
        "v_fmac_f32 v28, v1, v3\n"
        "v_fmac_f32 v30, v1, v3\n"
        "v_rsq_f32 v68, v69\n"
        "v_fmac_f32 v32, v1, v3\n"
        "v_fmac_f32 v34, v1, v3\n"
        "v_fmac_f32 v36, v1, v3\n"
        "v_fmac_f32 v38, v1, v3\n"
        "v_rsq_f32 v70, v71\n"
        "s_sub_u32 s40, s40, 1\n"
        "s_cmp_lg_u32 s40, 0\n"
        "s_cbranch_scc1 1b\n"
        "v_mov_b32 %0, v16\n"
        : "=v"(r) : "s"(iters) : "v1", "v3", "v16", "v18", "v20", "v22", "v24", "v26", "v28", "v30", "v32", "v34", "v36", "v38", "v60", "v61", "v62", "v63", "v64", "v65", "v66", "v67", "v68", "v69", "v70", "v71", "s40", "scc");
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}
}  // namespace

int main()
{
    hipDeviceProp_t pr;
    VR_CHECK(hipGetDeviceProperties(&pr, 0));
    const int cus = pr.multiProcessorCount;
    std::printf("device %s, %d CUs, nominal clock %.2f GHz\n", pr.gcnArchName, cus, pr.clockRate * 1e-6);
    const int blocks = cus * 32, iters = 4096;
    void* buf = nullptr;
    VR_CHECK(hipMalloc(&buf, (size_t)blocks * kThreads * sizeof(double)));
    hipEvent_t e0, e1;
    VR_CHECK(hipEventCreate(&e0));
    VR_CHECK(hipEventCreate(&e1));
    const double clk = 2.4e9, simds = 4.0 * cus;
    auto run = [&](const char* name, int flop_per_op, auto launch) {
        launch();
        VR_CHECK(hipDeviceSynchronize());
        VR_CHECK(hipEventRecord(e0));
        for (int r = 0; r < 5; ++r) launch();
        VR_CHECK(hipEventRecord(e1));
        VR_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        VR_CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= 5.f;
        const double lane_ops = (double)blocks * kThreads * iters * kChains;
        const double rate = lane_ops / (ms * 1e-3);
        const double lanes = rate / (simds * clk);
        std::printf("%-28s %8.3f ms  %6.2f lanes/clk/SIMD  %5.2f cycles/instr", name, ms, lanes, 64.0 / lanes);
        if (flop_per_op) std::printf("  %6.1f TFLOP/s", rate * flop_per_op * 1e-12);
        std::printf("\n");
        std::fflush(stdout);
    };
    float* f = static_cast<float*>(buf);
    double* d = static_cast<double*>(buf);
    run("v_fma_f32  (VGPR operands)", 2, [&] { chains<float, FMA_VVV><<<blocks, kThreads>>>(f, iters, 1.0000001f, 1e-7f); });
    run("v_mul_f32  (VGPR operands)", 1, [&] { chains<float, MUL_VV><<<blocks, kThreads>>>(f, iters, 1.0000001f, 1e-7f); });
    run("v_add_f32  (VGPR operands)", 1, [&] { chains<float, ADD_VV><<<blocks, kThreads>>>(f, iters, 1e-7f, 1e-7f); });
    run("v_add_f32  (an SGPR operand)", 1, [&] { chains<float, ADD_VS><<<blocks, kThreads>>>(f, iters, 1e-7f, 1e-7f); });
    run("v_rsq_f32", 0, [&] { chains<float, RSQ_V><<<blocks, kThreads>>>(f, iters, 1.f, 0.f); });
    run("v_fma_f64  (VGPR operands)", 2, [&] { chains<double, FMA64_VVV><<<blocks, kThreads>>>(d, iters, 1.0000001, 1e-7); });
    run("v_mul_f64  (VGPR operands)", 1, [&] { chains<double, MUL64_VV><<<blocks, kThreads>>>(d, iters, 1.0000001, 1e-7); });
    run("v_add_f64  (VGPR operands)", 1, [&] { chains<double, ADD64_VV><<<blocks, kThreads>>>(d, iters, 1e-7, 1e-7); });
    run("v_rsq_f64", 0, [&] { chains<double, RSQ64_V><<<blocks, kThreads>>>(d, iters, 1.0, 0.0); });
    run("v_fma_f64 x3 + v_rsq_f64 (mean)", 0,
        [&] { chains<double, FMA64_RSQ64><<<blocks, kThreads>>>(d, iters, 1.0000001, 1e-7); });

    // instruction streams with fixed registers: nominal cycles per loop iteration and SIMD
    auto run_asm = [&](const char* name, int ninstr, int nblocks, auto launch) {
        launch();
        VR_CHECK(hipDeviceSynchronize());
        VR_CHECK(hipEventRecord(e0));
        for (int r = 0; r < 5; ++r) launch();
        VR_CHECK(hipEventRecord(e1));
        VR_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        VR_CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= 5.f;
        const double iters_per_simd = (double)nblocks * (kThreads / 64) * iters / simds;
        const double cyc = ms * 1e-3 * clk / iters_per_simd;
        std::printf("%-44s %8.3f ms  %7.1f cycles/iteration  %5.2f cycles/instr\n", name, ms, cyc, cyc / ninstr);
        std::fflush(stdout);
    };
    run_asm("v_fmac_f32 x24, mixed-parity sources", 24, blocks,
            [&] { asm_fmac_mixed_parity<<<blocks, kThreads>>>(f, iters); });
    run_asm("v_fmac_f32 x24, same-parity sources", 24, blocks,
            [&] { asm_fmac_same_parity<<<blocks, kThreads>>>(f, iters); });
    run_asm("v_rsq_f32 x24", 24, blocks, [&] { asm_rsq_only<<<blocks, kThreads>>>(f, iters); });
    run_asm("v_fmac_f32 x96 + v_rsq_f32 x24, interleaved", 120, blocks,
            [&] { asm_fmac_rsq_mixed<<<blocks, kThreads>>>(f, iters); });
    // one workgroup (one wave per SIMD) per CU at a time: the LDS request keeps others off the CU
    VR_CHECK(hipFuncSetAttribute((const void*)asm_fmac_mixed_parity, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
    run_asm("v_fmac_f32 x24, one wave per SIMD", 24, cus * 4,
            [&] { asm_fmac_mixed_parity<<<cus * 4, kThreads, 96 * 1024>>>(f, iters); });
    VR_CHECK(hipFree(buf));
    return 0;
}
