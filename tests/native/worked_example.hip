// The program of the paper's usage example (Sec. 4, Listing 2), in HIP: the
// result vector c is allocated for 1,000,000 floats but copied back as
// 1,000,000 doubles.  The kernel here writes only the elements that fit, so
// the program itself never touches memory outside its allocations; the copy
// back is what the checker must catch.  "correct" allocates c properly.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

__global__ void vecsum(double *c, const double *a, const double *b, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += blockDim.x * gridDim.x) c[i] = a[i] + b[i];
}

// A pitched copy whose rows are wider than the destination pitch: the last
// row runs past the allocation.  And an asynchronous copy of the example's
// size into the float-sized buffer.
static int pitched_and_async()
{
    const size_t rows = 100, pitch = 256, width = 300;
    uint8_t *d = nullptr, *big = nullptr;
    uint8_t *h = (uint8_t *)calloc(rows * width, 1);
    if (hipMalloc((void **)&d, rows * pitch) != hipSuccess || hipMalloc((void **)&big, 4000000) != hipSuccess) return 2;
    hipError_t e = hipMemcpy2D(d, pitch, h, width, pitch, rows, hipMemcpyHostToDevice);   // fits
    printf("hipMemcpy2D fitting returned %d\n", (int)e);
    e = hipMemcpy2D(d, pitch, h, width, width, rows, hipMemcpyHostToDevice);              // last row overruns
    printf("hipMemcpy2D overrun returned %d\n", (int)e);
    double *hd = (double *)calloc(1000000, sizeof(double));
    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess) return 2;
    e = hipMemcpyAsync(big, hd, 1000000 * sizeof(double), hipMemcpyHostToDevice, s);
    printf("hipMemcpyAsync returned %d\n", (int)e);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    hipFree(d);
    hipFree(big);
    free(h);
    free(hd);
    return 0;
}

// Copies on two streams with no synchronisation between them: two uploads
// into overlapping device bytes, then an upload and a download sharing 2 KiB;
// then orderings that must stay quiet (one stream, a synchronisation between,
// disjoint bytes, two reads of the same bytes).
static int streams()
{
    const size_t MB = 1 << 20;
    uint8_t *d = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr;
    if (hipMalloc((void **)&d, 2 * MB) != hipSuccess) return 2;
    if (hipHostMalloc((void **)&h1, MB) != hipSuccess || hipHostMalloc((void **)&h2, MB) != hipSuccess ||
        hipHostMalloc((void **)&h3, MB) != hipSuccess)
        return 2;
    hipMemset(d, 0, 2 * MB);
    hipStream_t s1, s2;
    if (hipStreamCreate(&s1) != hipSuccess || hipStreamCreate(&s2) != hipSuccess) return 2;
    // racing: overlapping uploads
    hipMemcpyAsync(d, h1, MB, hipMemcpyHostToDevice, s1);
    hipMemcpyAsync(d + MB / 2, h2, MB, hipMemcpyHostToDevice, s2);
    (void)hipDeviceSynchronize();
    // racing: an upload and a download sharing 2 KiB
    hipMemcpyAsync(d, h1, 4096, hipMemcpyHostToDevice, s1);
    hipMemcpyAsync(h3, d + 2048, 4096, hipMemcpyDeviceToHost, s2);
    (void)hipStreamSynchronize(s1);
    // ordered: one stream
    hipMemcpyAsync(d, h1, MB, hipMemcpyHostToDevice, s1);
    hipMemcpyAsync(h3, d, MB, hipMemcpyDeviceToHost, s1);
    (void)hipDeviceSynchronize();
    // ordered: a synchronisation between
    hipMemcpyAsync(d, h1, MB, hipMemcpyHostToDevice, s1);
    (void)hipStreamSynchronize(s1);
    hipMemcpyAsync(h3, d, MB, hipMemcpyDeviceToHost, s2);
    (void)hipDeviceSynchronize();
    // disjoint bytes
    hipMemcpyAsync(d, h1, MB, hipMemcpyHostToDevice, s1);
    hipMemcpyAsync(d + MB, h2, MB, hipMemcpyHostToDevice, s2);
    (void)hipDeviceSynchronize();
    // two reads of the same device bytes
    hipMemcpyAsync(h1, d, 1024, hipMemcpyDeviceToHost, s1);
    hipMemcpyAsync(h2, d, 1024, hipMemcpyDeviceToHost, s2);
    (void)hipDeviceSynchronize();
    (void)hipStreamDestroy(s1);
    (void)hipStreamDestroy(s2);
    hipFree(d);
    (void)hipHostFree(h1);
    (void)hipHostFree(h2);
    (void)hipHostFree(h3);
    printf("streams done\n");
    return 0;
}

// The null stream (stream 0): its work waits for earlier work on blocking
// streams, and later work on them waits for it, so copies on two blocking
// streams on either side of a fill or a copy on stream 0 are ordered; copies
// on non-blocking streams are not ordered by it.  Exactly two pairs race: an
// upload and a download on two non-blocking streams around a fill on stream 0,
// and an upload on a non-blocking stream with a download on stream 0.
static int null_stream()
{
    const size_t KB = 1 << 10;
    uint8_t *d = nullptr, *h1 = nullptr, *h2 = nullptr;
    if (hipMalloc((void **)&d, 64 * KB) != hipSuccess) return 2;
    if (hipHostMalloc((void **)&h1, 64 * KB) != hipSuccess || hipHostMalloc((void **)&h2, 64 * KB) != hipSuccess) return 2;
    hipMemset(d, 0, 64 * KB);
    hipStream_t b1, b2, n1, n2;
    if (hipStreamCreate(&b1) != hipSuccess || hipStreamCreate(&b2) != hipSuccess ||
        hipStreamCreateWithFlags(&n1, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&n2, hipStreamNonBlocking) != hipSuccess)
        return 2;
    // quiet: blocking streams on either side of a fill on stream 0
    hipMemcpyAsync(d, h1, 4 * KB, hipMemcpyHostToDevice, b1);
    hipMemsetAsync(d + 32 * KB, 0, 16, 0);
    hipMemcpyAsync(h2, d, 4 * KB, hipMemcpyDeviceToHost, b2);
    (void)hipDeviceSynchronize();
    // quiet: an upload on a blocking stream, then a download of its bytes on stream 0
    hipMemcpyAsync(d + 8 * KB, h1, 4 * KB, hipMemcpyHostToDevice, b1);
    hipMemcpyAsync(h2, d + 8 * KB, 4 * KB, hipMemcpyDeviceToHost, 0);
    (void)hipDeviceSynchronize();
    // racing: non-blocking streams on either side of a fill on stream 0
    hipMemcpyAsync(d + 16 * KB, h1, 4 * KB, hipMemcpyHostToDevice, n1);
    hipMemsetAsync(d + 32 * KB, 0, 16, 0);
    hipMemcpyAsync(h2, d + 16 * KB, 4 * KB, hipMemcpyDeviceToHost, n2);
    (void)hipDeviceSynchronize();
    // racing: an upload on a non-blocking stream, a download of its bytes on stream 0
    hipMemcpyAsync(d + 24 * KB, h1, 4 * KB, hipMemcpyHostToDevice, n1);
    hipMemcpyAsync(h2 + 8 * KB, d + 24 * KB, 4 * KB, hipMemcpyDeviceToHost, 0);
    (void)hipDeviceSynchronize();
    (void)hipStreamDestroy(b1);
    (void)hipStreamDestroy(b2);
    (void)hipStreamDestroy(n1);
    (void)hipStreamDestroy(n2);
    hipFree(d);
    (void)hipHostFree(h1);
    (void)hipHostFree(h2);
    printf("null stream done\n");
    return 0;
}

// Fills and the typed asynchronous copies: a fill racing with a download of
// bytes it writes, a typed upload and download sharing 512 bytes; fills of
// disjoint bytes and copies ordered on one stream stay quiet; a fill and
// copies past the end of the allocation are refused.
static int fills()
{
    const size_t MB = 1 << 20;
    uint8_t *d = nullptr, *h1 = nullptr, *h2 = nullptr;
    if (hipMalloc((void **)&d, 2 * MB) != hipSuccess) return 2;
    if (hipHostMalloc((void **)&h1, MB + 64) != hipSuccess || hipHostMalloc((void **)&h2, MB) != hipSuccess) return 2;
    hipStream_t s1, s2;
    if (hipStreamCreate(&s1) != hipSuccess || hipStreamCreate(&s2) != hipSuccess) return 2;
    // racing: a fill and a download of bytes it writes
    hipMemsetAsync(d, 1, 4096, s1);
    hipMemcpyDtoHAsync(h1, (hipDeviceptr_t)(d + 1024), 1024, s2);
    (void)hipDeviceSynchronize();
    // racing: typed upload and download sharing 512 bytes
    hipMemcpyHtoDAsync((hipDeviceptr_t)(d + MB), h1, 4096, s1);
    hipMemcpyDtoHAsync(h2, (hipDeviceptr_t)(d + MB + 3584), 4096, s2);
    (void)hipStreamSynchronize(s2);
    // quiet: fills of disjoint bytes on two streams, a copy ordered after a fill on one stream
    hipMemsetD32Async((hipDeviceptr_t)d, 7, 1024, s1);            // bytes [0, 4096)
    hipMemsetD8Async((hipDeviceptr_t)(d + 4096), 3, 4096, s2);     // bytes [4096, 8192)
    hipMemsetD16Async((hipDeviceptr_t)(d + 8192), 5, 2048, s2);    // bytes [8192, 12288)
    hipMemcpyDtoDAsync((hipDeviceptr_t)(d + MB), (hipDeviceptr_t)d, 4096, s1);
    (void)hipDeviceSynchronize();
    // refused: a fill and copies past the end of the allocation
    const hipError_t e1 = hipMemsetD32((hipDeviceptr_t)(d + 2 * MB - 8), 0, 4);
    const hipError_t e2 = hipMemcpyDtoDAsync((hipDeviceptr_t)(d + MB), (hipDeviceptr_t)d, MB + 1, s1);
    const hipError_t e3 = hipMemcpyWithStream(h1, d + MB, MB + 16, hipMemcpyDeviceToHost, s1);
    const hipError_t e4 = hipMemcpyWithStream(h1, d, MB, hipMemcpyDeviceToHost, s1);
    (void)hipDeviceSynchronize();
    printf("fill past the end %d, DtoD past the end %d, copy with stream past the end %d, fitting copy %d\n",
           (int)e1, (int)e2, (int)e3, (int)e4);
    (void)hipStreamDestroy(s1);
    (void)hipStreamDestroy(s2);
    hipFree(d);
    (void)hipHostFree(h1);
    (void)hipHostFree(h2);
    printf("fills done\n");
    return 0;
}

// Kernel arguments: launches with valid pointers (inside an allocation, one
// past its end, null, pinned host memory), then with a freed pointer and with
// a pointer to ordinary host memory.  The refused launches pass n = 0, so the
// kernel would touch nothing even if it ran.
static int kernel_args()
{
    const int n = 1 << 16;
    double *a = nullptr, *b = nullptr, *c = nullptr, *gone = nullptr, *pinned = nullptr;
    if (hipMalloc((void **)&a, n * sizeof(double)) != hipSuccess || hipMalloc((void **)&b, n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&c, n * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&gone, n * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&pinned, n * sizeof(double)) != hipSuccess)
        return 2;
    hipMemset(a, 0, n * sizeof(double));
    hipMemset(b, 0, n * sizeof(double));
    hipFree(gone);
    double *plain = (double *)malloc(n * sizeof(double));
    hipLaunchKernelGGL(vecsum, dim3(64), dim3(256), 0, 0, c, a, b, n);
    printf("valid launch returned %d\n", (int)hipGetLastError());
    hipLaunchKernelGGL(vecsum, dim3(64), dim3(256), 0, 0, c, a, b + n, 0);
    printf("one-past-the-end launch returned %d\n", (int)hipGetLastError());
    hipLaunchKernelGGL(vecsum, dim3(64), dim3(256), 0, 0, pinned, (const double *)nullptr, (const double *)nullptr, 0);
    printf("null and pinned launch returned %d\n", (int)hipGetLastError());
    // 16 elements into the freed block: its first byte may equal c's one-past-the-end pointer
    hipLaunchKernelGGL(vecsum, dim3(64), dim3(256), 0, 0, c, gone + 16, b, 0);
    printf("freed argument launch returned %d\n", (int)hipGetLastError());
    hipLaunchKernelGGL(vecsum, dim3(64), dim3(256), 0, 0, c, a, plain, 0);
    printf("host pointer launch returned %d\n", (int)hipGetLastError());
    (void)hipDeviceSynchronize();
    hipFree(a);
    hipFree(b);
    hipFree(c);
    (void)hipHostFree(pinned);
    free(plain);
    return 0;
}

// Pitched allocations: hipMallocPitch with a 2D copy that fits and one whose
// last row finds 100 of its 300 bytes; hipMalloc3D with a 3D copy that fits
// and one whose last row of the last slice finds 32 of its 64 bytes; an
// asynchronous 2D copy that overruns.
static int pitched_3d()
{
    const size_t w = 300, h = 50;
    uint8_t *pp = nullptr;
    size_t pitch = 0;
    if (hipMallocPitch((void **)&pp, &pitch, w, h) != hipSuccess) return 2;
    uint8_t *host = (uint8_t *)calloc(64 * 1024, 1);
    hipError_t e = hipMemcpy2D(pp, pitch, host, w, w, h, hipMemcpyHostToDevice);
    printf("pitched 2D fitting returned %d\n", (int)e);
    e = hipMemcpy2D(pp + (pitch - 100), pitch, host, w, w, h, hipMemcpyHostToDevice);
    printf("pitched 2D overrun returned %d\n", (int)e);
    hipPitchedPtr p3;
    const hipExtent ext = make_hipExtent(64, 8, 4);
    if (hipMalloc3D(&p3, ext) != hipSuccess) return 2;
    hipMemcpy3DParms q = {};
    q.srcPtr = make_hipPitchedPtr(host, 64, 64, 8);
    q.dstPtr = p3;
    q.extent = ext;
    q.kind = hipMemcpyHostToDevice;
    e = hipMemcpy3D(&q);
    printf("3D fitting returned %d\n", (int)e);
    q.dstPos = make_hipPos(p3.pitch - 32, 0, 0);
    e = hipMemcpy3D(&q);
    printf("3D overrun returned %d\n", (int)e);
    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess) return 2;
    e = hipMemcpy2DAsync(pp + (pitch - 100), pitch, host, w, w, h, hipMemcpyHostToDevice, s);
    printf("2D async overrun returned %d\n", (int)e);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    hipFree(pp);
    hipFree(p3.ptr);
    free(host);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc > 1 && strcmp(argv[1], "pitched3d") == 0) return pitched_3d();
    if (argc > 1 && strcmp(argv[1], "kernelargs") == 0) return kernel_args();
    if (argc > 1 && strcmp(argv[1], "pitched") == 0) return pitched_and_async();
    if (argc > 1 && strcmp(argv[1], "streams") == 0) return streams();
    if (argc > 1 && strcmp(argv[1], "fills") == 0) return fills();
    if (argc > 1 && strcmp(argv[1], "nullstream") == 0) return null_stream();
    const bool correct = argc > 1 && strcmp(argv[1], "correct") == 0;
    const int size = 1000000;
    double *c, *a, *b;
    double *c_host = (double *)malloc(size * sizeof(double));
    const size_t c_bytes = correct ? size * sizeof(double) : size * sizeof(float);
    if (hipMalloc((void **)&c, c_bytes) != hipSuccess || hipMalloc((void **)&a, size * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&b, size * sizeof(double)) != hipSuccess)
        return 2;
    hipMemset(a, 0, size * sizeof(double));
    hipMemset(b, 0, size * sizeof(double));
    const int fits = (int)(c_bytes / sizeof(double));
    hipLaunchKernelGGL(vecsum, dim3(256), dim3(256), 0, 0, c, a, b, fits);
    if (hipDeviceSynchronize() != hipSuccess) return 3;
    hipMemset(c, 0, c_bytes);   // stands for the kernel's writes, which the checker does not see
    const hipError_t e = hipMemcpy(c_host, c, size * sizeof(double), hipMemcpyDeviceToHost);
    printf("hipMemcpy returned %d (%s)\n", (int)e, hipGetErrorString(e));
    hipFree(c);
    hipFree(a);
    hipFree(b);
    free(c_host);
    return 0;
}
