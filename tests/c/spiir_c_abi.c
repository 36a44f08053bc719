/*
 * A consumer of the SPIIR C ABI that uses no Python and no torch: it reads a
 * bank description and an input stream from a binary file, creates the bank
 * with spiir_create on a HIP stream of its own, filters the stream block by
 * block from hipMalloc buffers with spiir_process_block, checks spiir_status,
 * writes z to an output file and destroys the bank.
 *
 * Input (little-endian): int32 T, H, base_rate, n_taps_down, n_taps_up,
 * max_block, n_blocks, block, precision; int32 n_filters[T*H]; float64
 * a1[2*total], b0[2*total]; int32 delay[total]; float64 h_down[n_taps_down],
 * h_up[n_taps_up]; float32 x[n_blocks*block].  Output: complex64
 * z[T][n_blocks*block].  Exit status 0 on success; otherwise it prints the
 * failing call.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "spiir.h"

static void* read_n(FILE* f, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

#define HIPCHECK(call)                                                   \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) {                                          \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_)); \
            return 3;                                                    \
        }                                                                \
    } while (0)

#define SPIIRCHECK(call)                                                \
    do {                                                                \
        int r_ = (call);                                                \
        if (r_ != SPIIR_OK) {                                           \
            fprintf(stderr, "%s: %s\n", #call, spiir_strerror(r_));    \
            return 4;                                                   \
        }                                                               \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 1;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t* hd = (int32_t*)read_n(f, 9 * sizeof(int32_t));
    const int T = hd[0], H = hd[1], rate = hd[2], td = hd[3], tu = hd[4], max_block = hd[5];
    const int n_blocks = hd[6], block = hd[7], precision = hd[8];
    int32_t* nf = (int32_t*)read_n(f, sizeof(int32_t) * (size_t)T * H);
    int64_t total = 0;
    for (int i = 0; i < T * H; ++i) total += nf[i];
    double* a1 = (double*)read_n(f, sizeof(double) * 2 * (size_t)total);
    double* b0 = (double*)read_n(f, sizeof(double) * 2 * (size_t)total);
    int32_t* delay = (int32_t*)read_n(f, sizeof(int32_t) * (size_t)total);
    double* h_down = (double*)read_n(f, sizeof(double) * (size_t)td);
    double* h_up = (double*)read_n(f, sizeof(double) * (size_t)tu);
    const size_t n = (size_t)n_blocks * block;
    float* x = (float*)read_n(f, sizeof(float) * n);
    fclose(f);

    spiir_bank_desc d = {0};
    d.n_templates = T;
    d.n_bands = H;
    d.base_rate_hz = rate;
    d.n_filters = nf;
    d.a1 = a1;
    d.b0 = b0;
    d.delay = delay;
    d.n_taps_down = td;
    d.h_down = h_down;
    d.n_taps_up = tu;
    d.h_up = h_up;
    d.max_block = max_block;
    d.precision = precision;

    hipStream_t s;
    HIPCHECK(hipStreamCreate(&s));
    spiir_bank* bank = NULL;
    SPIIRCHECK(spiir_create(&d, s, &bank));
    /* the HIP runtime(s) this process mapped */
    FILE* m = fopen("/proc/self/maps", "r");
    if (m) {
        char line[4096];
        while (fgets(line, sizeof line, m))
            if (strstr(line, "libamdhip64")) printf("runtime: %s", strchr(line, '/'));
        fclose(m);
    }
    float* xd = NULL;
    spiir_c32* zd = NULL;
    HIPCHECK(hipMalloc((void**)&xd, sizeof(float) * n));
    HIPCHECK(hipMalloc((void**)&zd, sizeof(spiir_c32) * (size_t)T * n));
    HIPCHECK(hipMemcpyAsync(xd, x, sizeof(float) * n, hipMemcpyHostToDevice, s));
    for (int b = 0; b < n_blocks; ++b)
        SPIIRCHECK(spiir_process_block(bank, xd + (size_t)b * block, block, zd + (size_t)b * block, (int64_t)n, s));
    HIPCHECK(hipStreamSynchronize(s));
    SPIIRCHECK(spiir_status(bank, NULL));
    int64_t done = 0;
    SPIIRCHECK(spiir_samples_done(bank, &done));
    if (done != (int64_t)n) {
        fprintf(stderr, "samples_done %lld, expected %zu\n", (long long)done, n);
        return 5;
    }
    spiir_c32* z = (spiir_c32*)malloc(sizeof(spiir_c32) * (size_t)T * n);
    HIPCHECK(hipMemcpy(z, zd, sizeof(spiir_c32) * (size_t)T * n, hipMemcpyDeviceToHost));
    SPIIRCHECK(spiir_destroy(bank));
    HIPCHECK(hipFree(xd));
    HIPCHECK(hipFree(zd));
    HIPCHECK(hipStreamDestroy(s));
    FILE* o = fopen(argv[2], "wb");
    if (!o || fwrite(z, sizeof(spiir_c32), (size_t)T * n, o) != (size_t)T * n) return 6;
    fclose(o);
    printf("ok: %d templates x %d bands, %d blocks of %d\n", T, H, n_blocks, block);
    return 0;
}
