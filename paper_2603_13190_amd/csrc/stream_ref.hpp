// Reference streaming kernels: the HBM bandwidth that plain, perfectly
// coalesced traffic reaches on this GPU, the practical ceiling against which
// the step's kernels are read beside the nominal peak.  One 16-byte element
// per lane, one pass (no grid-stride loop), loads and stores nontemporal:
// the fastest simple form measured on gfx950.
#pragma once

typedef double stream_d2 __attribute__((ext_vector_type(2)));

constexpr int STREAM_THREADS = 256;

__global__ __launch_bounds__(STREAM_THREADS) void k_stream_copy(const stream_d2* __restrict__ a,
                                                                stream_d2* __restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// each block writes the sum of its elements to out[block]
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_read(const stream_d2* __restrict__ a,
                                                                double* __restrict__ out, int64_t n)
{
    __shared__ double s[STREAM_THREADS / 64];
    const int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const stream_d2 x = __builtin_nontemporal_load(a + i);
        v = x.x + x.y;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < STREAM_THREADS / 64; w++) t += s[w];
        out[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(STREAM_THREADS) void k_stream_fill(stream_d2* __restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x;
    const stream_d2 z = {1.0, -1.0};
    if (i < n) __builtin_nontemporal_store(z, b + i);
}

// three reads and two writes per element (a[0..3n) -> b[0..2n)): about the
// read/write mix of the explicit step's kernels
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_mix(const stream_d2* __restrict__ a,
                                                               stream_d2* __restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * STREAM_THREADS + threadIdx.x;
    if (i < n) {
        const stream_d2 x = __builtin_nontemporal_load(a + i);
        const stream_d2 y = __builtin_nontemporal_load(a + n + i);
        const stream_d2 z = __builtin_nontemporal_load(a + 2 * n + i);
        __builtin_nontemporal_store(x + y, b + i);
        __builtin_nontemporal_store(y + z, b + n + i);
    }
}
