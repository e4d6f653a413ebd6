// Issue-rate probes for the vector ALU of gfx950, used by the benchmark to
// check the peak rates that the pair kernels are compared against. Not part
// of the search library: built as its own shared object (libtds_probe.so).
//
// Each probe kernel runs dependence chains of one instruction kind (eight
// independent chains per lane, so a wave always has an instruction ready)
// on every SIMD of the chip; every wave stamps its start and end with the
// shader clock (s_memtime) and the constant 100 MHz reference clock
// (s_memrealtime), so the clock under load is measured alongside the rate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

constexpr int kChains = 8;
constexpr int kBlock = 256;

// Per-wave record: shader clock and reference clock at start and end.
struct Stamp {
    unsigned long long c0, c1, r0, r1;
};

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_probe(int iters, float seed, float *sink, Stamp *st) {
    const int lane = threadIdx.x & 63;
    const int wave = (int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    unsigned long long c0 = __builtin_amdgcn_s_memtime();
    unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    float acc = 0.0f;
    // The chain steps are written as inline assembly (register operands
    // only, no memory access) so that exactly the named instruction is timed.
    if constexpr (KIND <= 2 || (KIND >= 4 && KIND <= 9) || (KIND >= 11 && KIND <= 20)) {
        float a[kChains];
        float b = seed * 1e-7f + lane * 1e-9f, c = seed * 3e-7f;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = seed + k + lane;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (KIND == 0) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 1)
                    asm volatile("v_max3_f32 %0, |%0|, |%1|, |%2|" : "+v"(a[k]) : "v"(b), "v"(c));
                if constexpr (KIND == 2)
                    asm volatile("v_min3_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
                if constexpr (KIND == 4) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 5) asm volatile("v_pk_sub_u16 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 6) asm volatile("v_pk_max_u16 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 7)
                    asm volatile("v_max_f32_e64 %0, |%0|, |%1|" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 8) asm volatile("v_pk_add_f16 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 9) asm volatile("v_min_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 11)
                    asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
                if constexpr (KIND == 12) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
                if constexpr (KIND == 13) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 14) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 15) asm volatile("v_or_b32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 16)
                    asm volatile("v_or3_b32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
                if constexpr (KIND == 17) asm volatile("v_max_f32 %0, %0, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 18)
                    asm volatile("v_sub_f32_e64 %0, |%0|, %1" : "+v"(a[k]) : "v"(b));
                if constexpr (KIND == 19)  // the multiplicand in a scalar register (the argument)
                    asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[k]) : "s"(seed), "v"(c));
                if constexpr (KIND == 20)
                    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a[k]) : "s"(seed), "v"(c));
            }
        }
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc += a[k];
    } else if constexpr (KIND == 10) {  // v_cmp_le_f32 into a lane mask, masks combined
        float a[kChains];
        float b = seed * 1e-7f + lane * 1e-9f;
        unsigned long long m = 0;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = seed + k + lane;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                unsigned long long r;
                asm volatile("v_cmp_le_f32_e64 %0, %1, %2" : "=s"(r) : "v"(a[k]), "v"(b));
                m ^= r;
            }
        }
        acc = (float)(m & 1);
    } else if constexpr (KIND == 21 || KIND == 22) {
        // v_fma_f32 on fixed registers, eight chains in v40, v44, ..., v68
        // (all in register bank 0 of 4, bank = number mod 4): 21 with the
        // other two sources in banks 1 and 2, 22 with the second multiplicand
        // in bank 0 as well (the two multiplicands in one bank)
        asm volatile(
            "v_mov_b32 v40, 1.0\n v_mov_b32 v44, 1.0\n v_mov_b32 v48, 1.0\n v_mov_b32 v52, 1.0\n"
            "v_mov_b32 v56, 1.0\n v_mov_b32 v60, 1.0\n v_mov_b32 v64, 1.0\n v_mov_b32 v68, 1.0\n"
            "v_mov_b32 v72, 1.0\n v_mov_b32 v73, 1.0\n v_mov_b32 v74, 0\n" ::
                : "v40", "v44", "v48", "v52", "v56", "v60", "v64", "v68", "v72", "v73", "v74");
        for (int i = 0; i < iters; ++i) {
            if constexpr (KIND == 21)
                asm volatile(
                    "v_fma_f32 v40, v40, v73, v74\n v_fma_f32 v44, v44, v73, v74\n"
                    "v_fma_f32 v48, v48, v73, v74\n v_fma_f32 v52, v52, v73, v74\n"
                    "v_fma_f32 v56, v56, v73, v74\n v_fma_f32 v60, v60, v73, v74\n"
                    "v_fma_f32 v64, v64, v73, v74\n v_fma_f32 v68, v68, v73, v74\n" ::
                        : "v40", "v44", "v48", "v52", "v56", "v60", "v64", "v68");
            else
                asm volatile(
                    "v_fma_f32 v40, v40, v72, v74\n v_fma_f32 v44, v44, v72, v74\n"
                    "v_fma_f32 v48, v48, v72, v74\n v_fma_f32 v52, v52, v72, v74\n"
                    "v_fma_f32 v56, v56, v72, v74\n v_fma_f32 v60, v60, v72, v74\n"
                    "v_fma_f32 v64, v64, v72, v74\n v_fma_f32 v68, v68, v72, v74\n" ::
                        : "v40", "v44", "v48", "v52", "v56", "v60", "v64", "v68");
        }
        acc = seed;
    } else if constexpr (KIND == 23 || KIND == 24) {
        // binary32 matrix-core products: 23 v_mfma_f32_16x16x4_f32, 24
        // v_mfma_f32_32x32x2_f32, eight independent accumulations
        typedef float v4f __attribute__((ext_vector_type(4)));
        typedef float v16f __attribute__((ext_vector_type(16)));
        const float a = seed * 1e-7f + lane * 1e-9f, b = seed * 3e-7f;
        using Acc = typename std::conditional<KIND == 23, v4f, v16f>::type;
        Acc d[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) d[k] = Acc{} + (float)k;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) {
                if constexpr (KIND == 23)
                    d[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d[k], 0, 0, 0);
                else
                    d[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, d[k], 0, 0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc += d[k][0] + d[k][3];
    } else if constexpr (KIND == 3) {
        double a[kChains], b = 1.0 + seed * 1e-9, c = seed * 1e-12 + lane * 1e-15;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = seed + k + lane;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a[k]) : "v"(b), "v"(c));
        }
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kChains; ++k) s += a[k];
        acc = (float)s;
    }
    // keep the result live; the store is taken only for an impossible value
    if (acc == -1.2345e-30f) sink[blockIdx.x * kBlock + threadIdx.x] = acc;
    unsigned long long c1 = __builtin_amdgcn_s_memtime();
    unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    if (lane == 0) st[wave] = Stamp{c0, c1, r0, r1};
}

template <int KIND>
hipError_t run_kind(int blocks, int iters, float seed, float *sink, Stamp *st, hipStream_t s) {
    hipLaunchKernelGGL(k_probe<KIND>, dim3(blocks), dim3(kBlock), 0, s, iters, seed, sink, st);
    return hipGetLastError();
}

}  // namespace

extern "C" {

/*
 * Runs probe `kind` (0 v_sub_f32, 1 v_max3_f32 with absolute-value operands,
 * 2 v_min3_f32, 3 v_fma_f64, 4 v_add_u32, 5 v_pk_sub_u16, 6 v_pk_max_u16,
 * 7 v_max_f32 with absolute-value operands (VOP3 form), 8 v_pk_add_f16,
 * 9 v_min_f32, 10 v_cmp_le_f32 into a lane mask, 11 v_fma_f32, 12 v_fmac_f32,
 * 13 v_mul_f32, 14 v_add_f32, 15 v_or_b32, 16 v_or3_b32, 17 v_max_f32,
 * 18 v_sub_f32 with an absolute-value operand (VOP3 form), 19 v_fma_f32 and
 * 20 v_fmac_f32 with the multiplicand in a scalar register, 21 v_fma_f32 with
 * its three sources in three register banks, 22 v_fma_f32 with its two
 * multiplicands in one bank, 23 v_mfma_f32_16x16x4_f32, 24
 * v_mfma_f32_32x32x2_f32) with `blocks` workgroups of 256
 * threads, each lane running `iters` iterations of 8 independent chain
 * steps, on `stream`, and waits for it.
 * Writes: *ms the kernel's duration (HIP events), *wave_instr the vector
 * instructions of the measured kind issued (waves x iters x 8), *clock_hz
 * the shader clock over the run (shader-clock ticks / reference ticks x 1e8,
 * averaged over the waves). Device memory is allocated and freed inside.
 * Returns 0, or -3 when a HIP call fails, -1 for a bad argument.
 */
int tds_probe_valu(int kind, int blocks, int iters, void *stream, double *ms, double *wave_instr,
                   double *clock_hz) {
    if (kind < 0 || kind > 24 || blocks < 1 || iters < 1 || !ms || !wave_instr || !clock_hz) return -1;
    hipStream_t s = (hipStream_t)stream;
    const int waves = blocks * (kBlock / 64);
    float *sink = nullptr;
    Stamp *st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -3;
    if (hipMalloc(&sink, sizeof(float) * (size_t)blocks * kBlock) != hipSuccess) return -3;
    if (hipMalloc(&st, sizeof(Stamp) * (size_t)waves) != hipSuccess) goto done;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
    {
        const float seed = 1.5f;
        hipError_t err = hipEventRecord(e0, s);
        if (err == hipSuccess) {
            switch (kind) {
            case 0: err = run_kind<0>(blocks, iters, seed, sink, st, s); break;
            case 1: err = run_kind<1>(blocks, iters, seed, sink, st, s); break;
            case 2: err = run_kind<2>(blocks, iters, seed, sink, st, s); break;
            case 3: err = run_kind<3>(blocks, iters, seed, sink, st, s); break;
            case 4: err = run_kind<4>(blocks, iters, seed, sink, st, s); break;
            case 5: err = run_kind<5>(blocks, iters, seed, sink, st, s); break;
            case 6: err = run_kind<6>(blocks, iters, seed, sink, st, s); break;
            case 7: err = run_kind<7>(blocks, iters, seed, sink, st, s); break;
            case 8: err = run_kind<8>(blocks, iters, seed, sink, st, s); break;
            case 9: err = run_kind<9>(blocks, iters, seed, sink, st, s); break;
            case 10: err = run_kind<10>(blocks, iters, seed, sink, st, s); break;
            case 11: err = run_kind<11>(blocks, iters, seed, sink, st, s); break;
            case 12: err = run_kind<12>(blocks, iters, seed, sink, st, s); break;
            case 13: err = run_kind<13>(blocks, iters, seed, sink, st, s); break;
            case 14: err = run_kind<14>(blocks, iters, seed, sink, st, s); break;
            case 15: err = run_kind<15>(blocks, iters, seed, sink, st, s); break;
            case 16: err = run_kind<16>(blocks, iters, seed, sink, st, s); break;
            case 17: err = run_kind<17>(blocks, iters, seed, sink, st, s); break;
            case 18: err = run_kind<18>(blocks, iters, seed, sink, st, s); break;
            case 19: err = run_kind<19>(blocks, iters, seed, sink, st, s); break;
            case 20: err = run_kind<20>(blocks, iters, seed, sink, st, s); break;
            case 21: err = run_kind<21>(blocks, iters, seed, sink, st, s); break;
            case 22: err = run_kind<22>(blocks, iters, seed, sink, st, s); break;
            case 23: err = run_kind<23>(blocks, iters, seed, sink, st, s); break;
            default: err = run_kind<24>(blocks, iters, seed, sink, st, s); break;
            }
        }
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) goto done;
        Stamp *h = new Stamp[waves];
        if (hipMemcpy(h, st, sizeof(Stamp) * (size_t)waves, hipMemcpyDeviceToHost) != hipSuccess) {
            delete[] h;
            goto done;
        }
        double f = 0.0;
        int nf = 0;
        for (int w = 0; w < waves; ++w) {
            const double dr = (double)(h[w].r1 - h[w].r0);
            if (dr > 0) {
                f += (double)(h[w].c1 - h[w].c0) / dr * 1e8;
                ++nf;
            }
        }
        delete[] h;
        *ms = t;
        *wave_instr = (double)waves * iters * kChains;
        *clock_hz = nf ? f / nf : 0.0;
        rc = 0;
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipFree(st);
    (void)hipFree(sink);
    return rc;
}

}  // extern "C"
