// Bandwidth reference for the stencil kernels: what plain streaming code achieves on this part for
// the stencil's access mix (three arrays read, one written, per element), for a copy (one read, one
// write) and for three reads alone, over arrays of 512^3 floats (the 512^3 step's field size).
//
//   triad        out = a + b c, float4 per thread, grid-stride; b, c and out with streaming
//                (non-temporal) hints, a cached, as the stencil treats u^{n-1}, kappa, u^{n+1} and u^n
//   triad_range  the same, each workgroup over one contiguous range (a column march without the halo)
//   copy         out = a
//   read3        a + b + c reduced in registers (the loads are kept by a data-dependent store)
//
// Each kernel runs at several grid sizes (workgroups of 256 threads); the program prints the
// event-timed average of 20 launches per case.  Its kernel trace under rocprofv3 is what the profile
// summary reads.  Not part of the library: a stand-alone program built beside it.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v ld_stream(const f4v *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(f4v *p, f4v v) { __builtin_nontemporal_store(v, p); }

__global__ __launch_bounds__(256) void triad(f4v *out, const f4v *a, const f4v *b, const f4v *c, long long n)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        st_stream(out + i, a[i] + ld_stream(b + i) * ld_stream(c + i));
}

__global__ __launch_bounds__(256) void triad_range(f4v *out, const f4v *a, const f4v *b, const f4v *c, long long n)
{
    const long long per = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * per;
    const long long hi = lo + per < n ? lo + per : n;
    for (long long i = lo + threadIdx.x; i < hi; i += 256)
        st_stream(out + i, a[i] + ld_stream(b + i) * ld_stream(c + i));
}

__global__ __launch_bounds__(256) void copy(f4v *out, const f4v *a, long long n)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        out[i] = a[i];
}

__global__ __launch_bounds__(256) void read3(float *flag, const f4v *a, const f4v *b, const f4v *c, long long n)
{
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        acc += a[i] + b[i] + c[i];
    if (acc.x + acc.y + acc.z + acc.w == 12345.0f) flag[0] = 1.0f;
}

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);    \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

int main()
{
    const long long nf = 512ll * 512 * 512, n4 = nf / 4;
    f4v *a = nullptr, *b = nullptr, *c = nullptr, *o = nullptr;
    CHECK(hipMalloc(&a, nf * 4));
    CHECK(hipMalloc(&b, nf * 4));
    CHECK(hipMalloc(&c, nf * 4));
    CHECK(hipMalloc(&o, nf * 4));
    CHECK(hipMemset(a, 0, nf * 4));
    CHECK(hipMemset(b, 0, nf * 4));
    CHECK(hipMemset(c, 0, nf * 4));
    CHECK(hipMemset(o, 0, nf * 4));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char *names[4] = {"triad", "triad_range", "copy", "read3"};
    const double arrays[4] = {4.0, 4.0, 2.0, 3.0};      // arrays moved per element
    const int grids[4] = {256, 512, 1024, 2048};
    for (int gi = 0; gi < 4; ++gi) {
        const int g = grids[gi];
        for (int kind = 0; kind < 4; ++kind) {
            auto launch = [&]() {
                if (kind == 0) hipLaunchKernelGGL(triad, dim3(g), dim3(256), 0, 0, o, a, b, c, n4);
                else if (kind == 1) hipLaunchKernelGGL(triad_range, dim3(g), dim3(256), 0, 0, o, a, b, c, n4);
                else if (kind == 2) hipLaunchKernelGGL(copy, dim3(g), dim3(256), 0, 0, o, a, n4);
                else hipLaunchKernelGGL(read3, dim3(g), dim3(256), 0, 0, (float *)o, a, b, c, n4);
            };
            launch();
            CHECK(hipDeviceSynchronize());
            CHECK(hipEventRecord(e0, 0));
            for (int r = 0; r < 20; ++r) launch();
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double s = ms / 20 * 1e-3;
            std::printf("%-12s workgroups %5d  %8.1f us  %5.2f TB/s\n", names[kind], g, s * 1e6,
                        arrays[kind] * nf * 4 / s / 1e12);
            std::fflush(stdout);
        }
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(c));
    CHECK(hipFree(o));
    return 0;
}
