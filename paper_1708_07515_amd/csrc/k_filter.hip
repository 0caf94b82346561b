// Ramp filtering of the projections, the "initial convolution" that the paper
// leaves out of its timings (Sec. 3): textbook FDK pre-weight and Ram-Lak.
//
//   p~[u] = p[u] * R / sqrt(R^2 + a^2 + b^2)
//   q[u]  = sum_{u'=0}^{N-1} h[u - u'] p~[u'],   h = spatial Ram-Lak kernel
//
// FP32 accuracy: a smooth projection row is hundreds of times larger than its
// ramp-filtered output, and FFT rounding scales with the input.  The kernel
// therefore filters the first difference d[u] = p~[u] - p~[u-1] (p~[-1] = 0)
// with the running sum g[n] = sum_{k<=n} h[k]:
//
//   q[u] = sum_{u'=0}^{N-1} g[u - u'] d[u'] - p~[N-1] g[u - N]
//
// (summation by parts; the last term is the difference at u' = N, applied
// directly so that lags stay within +-(N-1)).  The convolution is circular of
// length M >= 2N - 1 on the zero-padded row, by an FP32 Stockham FFT held in
// LDS.  Two real rows travel in one complex transform (row0 + i row1); g is
// real, so its transform G is Hermitian and multiplying by it keeps the rows
// apart.  The inverse transform is conj(FFT(conj(.))); 1/M is folded into G.
#include "internal.h"
#include "dtype.h"

namespace fdkod {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place forward DFT of length M (natural order in and out) by Stockham
// radix-4 stages (one radix-2 stage last when log2 M is odd).  TP threads
// cooperate on one transform; every thread of the workgroup calls this the
// same number of times because it contains barriers.
template <int LOGM, int TP>
__device__ __forceinline__ void fft_lds(float2* z, int t, const float2* __restrict__ tw) {
    constexpr int M = 1 << LOGM;
    constexpr int Q = M / 4;           // radix-4 butterflies per stage
    constexpr int BPT = (Q + TP - 1) / TP;
#pragma unroll 1
    for (int ns = 1; ns * 4 <= M; ns *= 4) {
        float2 v[BPT][4];
        const int tstep = M / (4 * ns);
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TP;
            if (j < Q) {
                const int k = j & (ns - 1);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[b][r] = z[j + r * Q];
                v[b][1] = cmul(v[b][1], tw[(1 * k * tstep) & (M - 1)]);
                v[b][2] = cmul(v[b][2], tw[(2 * k * tstep) & (M - 1)]);
                v[b][3] = cmul(v[b][3], tw[(3 * k * tstep) & (M - 1)]);
                // 4-point DFT: X1 = a - i b - c + i d, X3 = a + i b - c - i d
                const float2 s02 = make_float2(v[b][0].x + v[b][2].x, v[b][0].y + v[b][2].y);
                const float2 d02 = make_float2(v[b][0].x - v[b][2].x, v[b][0].y - v[b][2].y);
                const float2 s13 = make_float2(v[b][1].x + v[b][3].x, v[b][1].y + v[b][3].y);
                const float2 d13 = make_float2(v[b][1].x - v[b][3].x, v[b][1].y - v[b][3].y);
                v[b][0] = make_float2(s02.x + s13.x, s02.y + s13.y);
                v[b][2] = make_float2(s02.x - s13.x, s02.y - s13.y);
                v[b][1] = make_float2(d02.x + d13.y, d02.y - d13.x);   // d02 - i d13
                v[b][3] = make_float2(d02.x - d13.y, d02.y + d13.x);   // d02 + i d13
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int j = t + b * TP;
            if (j < Q) {
                const int k = j & (ns - 1);
                const int dst = (j / ns) * ns * 4 + k;
#pragma unroll
                for (int r = 0; r < 4; ++r) z[dst + r * ns] = v[b][r];
            }
        }
        __syncthreads();
    }
    if (LOGM & 1) {
        // last stage, radix 2, ns = M / 2: X0 = a + w^j b, X1 = a - w^j b
        constexpr int H = M / 2;
        constexpr int B2 = (H + TP - 1) / TP;
        float2 v0[B2], v1[B2];
#pragma unroll
        for (int b = 0; b < B2; ++b) {
            const int j = t + b * TP;
            if (j < H) {
                v0[b] = z[j];
                v1[b] = cmul(z[j + H], tw[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < B2; ++b) {
            const int j = t + b * TP;
            if (j < H) {
                z[j] = make_float2(v0[b].x + v1[b].x, v0[b].y + v1[b].y);
                z[j + H] = make_float2(v0[b].x - v1[b].x, v0[b].y - v1[b].y);
            }
        }
        __syncthreads();
    }
}

template <int LOGM, int STORE>
__global__ __launch_bounds__(256) void k_filter(FilterArgs a) {
    using S = Store<STORE>;
    constexpr int M = 1 << LOGM;
    constexpr int TP = (M / 4 < 256) ? M / 4 : 256;   // threads per row pair
    constexpr int PAIRS = 256 / TP;                   // row pairs per workgroup
    __shared__ float2 buf[PAIRS * M];

    const int grp = threadIdx.x / TP;
    const int t = threadIdx.x % TP;
    const int pair = blockIdx.x * PAIRS + grp;
    const int r0 = 2 * pair, r1 = 2 * pair + 1;
    const bool has0 = r0 < a.rows, has1 = r1 < a.rows;
    float2* z = buf + grp * M;
    const int n = a.n;
    const float rr = a.r * a.r;

    // load and pre-weight (zero-padded), then take the first difference in LDS
    const float b0 = has0 ? (float)(r0 % n) - a.c : 0.0f;
    const float b1 = has1 ? (float)(r1 % n) - a.c : 0.0f;
    const float rb0 = rr + b0 * b0, rb1 = rr + b1 * b1;
    const float* p0 = a.proj + (size_t)r0 * n;
    const float* p1 = a.proj + (size_t)r1 * n;
    for (int u = t; u < M; u += TP) {
        float x0 = 0.0f, x1 = 0.0f;
        if (u < n) {
            const float au = (float)u - a.c;
            if (has0) x0 = p0[u] * (a.r * rsqrtf(rb0 + au * au));
            if (has1) x1 = p1[u] * (a.r * rsqrtf(rb1 + au * au));
        }
        z[u] = make_float2(x0, x1);
    }
    __syncthreads();
    constexpr int EPT = (M + TP - 1) / TP;
    float2 dv[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int u = t + e * TP;
        dv[e] = make_float2(0.0f, 0.0f);     // the difference at u = N is applied after the FFT
        if (u < n) {
            const float2 cur = z[u];
            const float2 prev = u > 0 ? z[u - 1] : make_float2(0.0f, 0.0f);
            dv[e] = make_float2(cur.x - prev.x, cur.y - prev.y);
        }
    }
    const float2 last = z[n - 1];
    const float last0 = last.x, last1 = last.y;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int u = t + e * TP;
        if (u < M) z[u] = dv[e];
    }
    __syncthreads();
    fft_lds<LOGM, TP>(z, t, a.twiddle);
    for (int k = t; k < M; k += TP) {
        const float2 v = cmul(z[k], a.resp[k]);
        z[k] = make_float2(v.x, -v.y);                // conj(Z G)
    }
    __syncthreads();
    fft_lds<LOGM, TP>(z, t, a.twiddle);
    typename S::T* out = (typename S::T*)a.out;
    for (int u = t; u < n; u += TP) {
        const float2 v = z[u];                        // conj of the result
        const float gt = a.gtail[u];                  // g[u - N]
        if (has0) S::put(out, (size_t)r0 * n + u, v.x - last0 * gt);
        if (has1) S::put(out, (size_t)r1 * n + u, -v.y - last1 * gt);
    }
}

template <int LOGM>
static hipError_t launch_filter_m(const FilterArgs& a, int store, hipStream_t st) {
    constexpr int M = 1 << LOGM;
    constexpr int TP = (M / 4 < 256) ? M / 4 : 256;
    constexpr int PAIRS = 256 / TP;
    const int pairs = (a.rows + 1) / 2;
    const dim3 grid((pairs + PAIRS - 1) / PAIRS);
    switch (store) {
        case 0: hipLaunchKernelGGL((k_filter<LOGM, 0>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_filter<LOGM, 1>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_filter<LOGM, 2>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_filter(const FilterArgs& a, int logm, int store, hipStream_t st) {
    switch (logm) {
        case 3: return launch_filter_m<3>(a, store, st);
        case 4: return launch_filter_m<4>(a, store, st);
        case 5: return launch_filter_m<5>(a, store, st);
        case 6: return launch_filter_m<6>(a, store, st);
        case 7: return launch_filter_m<7>(a, store, st);
        case 8: return launch_filter_m<8>(a, store, st);
        case 9: return launch_filter_m<9>(a, store, st);
        case 10: return launch_filter_m<10>(a, store, st);
        case 11: return launch_filter_m<11>(a, store, st);
        case 12: return launch_filter_m<12>(a, store, st);
        case 13: return launch_filter_m<13>(a, store, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdkod
