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
// LDS (radix-16 stages with the 16-point transforms in registers, so a
// 4096-point transform takes three passes through LDS).  Two real rows travel in one complex transform (row0 + i row1); g is
// real, so its transform G is Hermitian and multiplying by it keeps the rows
// apart.  The inverse transform is conj(FFT(conj(.))); 1/M is folded into G.
// For M = 4096 (N = 1025..2048) a four-step form with one row pair per
// wavefront replaces the Stockham stages (k_filter4096 below).
#include "internal.h"
#include "dtype.h"

namespace fdkod {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS position of transform element i: one pad slot after every 16 elements
// and another after every 256, so that the strided writes of the radix-16
// stages spread over the banks.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4) + (i >> 8); }
template <int M>
struct Padded {
    static constexpr int size = M + M / 16 + M / 256 + 1;
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// 4-point DFT in place: X1 = a - i b - c + i d, X3 = a + i b - c - i d
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
    const float2 s02 = cadd(a, c), d02 = csub(a, c);
    const float2 s13 = cadd(b, d), d13 = csub(b, d);
    a = cadd(s02, s13);
    c = csub(s02, s13);
    b = make_float2(d02.x + d13.y, d02.y - d13.x);   // d02 - i d13
    d = make_float2(d02.x - d13.y, d02.y + d13.x);   // d02 + i d13
}

// 16-point DFT in place (natural order in and out) as 4 x 4:
// X[k1 + 4 k2] = sum_n2 w16^(n2 k2 4) w16^(n2 k1) sum_n1 x[4 n1 + n2] w4^(n1 k1)
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
    // cos and sin of pi/8 and pi/4
    constexpr float C1 = 0.923879532511286756f, S1 = 0.382683432365089772f, R2 = 0.707106781186547524f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // v[n2 + 4 k1] now holds y[n2][k1]; multiply by w16^(n2 k1)
    v[5] = cmul(v[5], make_float2(C1, -S1));     // w^1
    v[9] = cmul(v[9], make_float2(R2, -R2));     // w^2
    v[13] = cmul(v[13], make_float2(S1, -C1));   // w^3
    v[6] = cmul(v[6], make_float2(R2, -R2));     // w^2
    v[10] = make_float2(v[10].y, -v[10].x);      // w^4 = -i
    v[14] = cmul(v[14], make_float2(-R2, -R2));  // w^6
    v[7] = cmul(v[7], make_float2(S1, -C1));     // w^3
    v[11] = cmul(v[11], make_float2(-R2, -R2));  // w^6
    v[15] = cmul(v[15], make_float2(-C1, S1));   // w^9
    // 4-point DFTs over n2 for each k1: inputs v[4 k1 + n2]
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
}

// Synchronisation of the TP threads of one transform.  A transform of at
// most 64 threads lives in one wavefront, whose LDS accesses complete in
// program order, so only the compiler has to be kept from moving them across
// (the other transforms of the workgroup need not wait); larger transforms
// span waves and take a workgroup barrier.
template <int TP>
__device__ __forceinline__ void transform_sync() {
    if constexpr (TP <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// One Stockham stage of radix R (16, 4 or 2) at stride NS, TP threads.  The
// first stage (NS = 1) needs no twiddles.  DIFF (first stage): the input is
// the first difference x[u] - x[u-1] of the values in LDS (x[-1] = 0) for
// u < n and zero from n on; as n <= M / 2, the upper half of every
// butterfly's inputs is zero and not read.  HALF (last stage, NS R = M):
// only outputs below M / 2 are wanted, the upper half of every butterfly's
// outputs is neither computed nor written.
template <int R, int M, int TP, int NS, bool DIFF, bool HALF>
__device__ __forceinline__ void fft_stage(float2* z, int t, const float2* __restrict__ tw, int n) {
    constexpr int NB = M / R;                       // butterflies of this stage
    constexpr int BPT = (NB + TP - 1) / TP;
    constexpr int ns = NS;
    float2 v[BPT][R];
    constexpr int tstep = M / (R * ns);
    // the twiddles (an L2-resident table) are all requested before the LDS
    // reads, so their latencies overlap instead of adding up
    float2 w[BPT][R];
    if constexpr (NS > 1) {
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            const int k = (t + b * TP) & (ns - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) w[b][r] = tw[(r * k * tstep) & (M - 1)];
        }
    }
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = t + b * TP;
        if (j < NB) {
            if constexpr (DIFF && NS == 1) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int u = j + r * NB;
                    if (r < R / 2) {
                        const float2 x1 = z[pidx(u)];
                        const float2 x0 = u > 0 ? z[pidx(u - 1)] : make_float2(0.0f, 0.0f);
                        v[b][r] = u < n ? csub(x1, x0) : make_float2(0.0f, 0.0f);
                    } else {
                        v[b][r] = make_float2(0.0f, 0.0f);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = z[pidx(j + r * NB)];
            }
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[b][r]);
            }
            if constexpr (R == 16) {
                dft16(v[b]);
            } else if constexpr (R == 4) {
                dft4(v[b][0], v[b][1], v[b][2], v[b][3]);
            } else {
                const float2 x0 = v[b][0];
                v[b][0] = cadd(x0, v[b][1]);
                v[b][1] = csub(x0, v[b][1]);
            }
        }
    }
    transform_sync<TP>();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = t + b * TP;
        if (j < NB) {
            const int k = j & (ns - 1);
            const int dst = (j / ns) * ns * R + k;
#pragma unroll
            for (int r = 0; r < (HALF && NS * R == M ? R / 2 : R); ++r) z[pidx(dst + r * ns)] = v[b][r];
        }
    }
    transform_sync<TP>();
}

// The stages from stride NS on: radix 16 while at least four bits remain,
// then 4, then 2.
template <int M, int TP, int NS, bool DIFF, bool HALF>
__device__ __forceinline__ void fft_stages(float2* z, int t, const float2* __restrict__ tw, int n) {
    if constexpr (NS * 16 <= M) {
        fft_stage<16, M, TP, NS, DIFF, HALF>(z, t, tw, n);
        fft_stages<M, TP, NS * 16, false, HALF>(z, t, tw, n);
    } else if constexpr (NS * 4 <= M) {
        fft_stage<4, M, TP, NS, DIFF, HALF>(z, t, tw, n);
        fft_stages<M, TP, NS * 4, false, HALF>(z, t, tw, n);
    } else if constexpr (NS * 2 <= M) {
        fft_stage<2, M, TP, NS, DIFF, HALF>(z, t, tw, n);
    }
}

// In-place forward DFT of length M = 2^LOGM (natural order in and out, LDS
// positions through pidx) by Stockham stages.  TP threads cooperate on one
// transform; every thread of the workgroup calls this the same number of
// times because it contains barriers.  DIFF: the transform of the first
// difference of the first n <= M / 2 values; HALF: only the lower half of
// the result is wanted (see fft_stage).
template <int LOGM, int TP, bool DIFF, bool HALF>
__device__ __forceinline__ void fft_lds(float2* z, int t, const float2* __restrict__ tw, int n) {
    fft_stages<1 << LOGM, TP, 1, DIFF, HALF>(z, t, tw, n);
}

// Threads per transform: one radix-16 butterfly per thread and stage (at
// most 256 threads, one workgroup).
// WAVES: waves per SIMD the register allocation is held to (the LDS of one
// 4096-point transform allows four workgroups per CU).
template <int LOGM>
struct FilterShape {
    static constexpr int M = 1 << LOGM;
    static constexpr int TP = filter_threads_per_pair(LOGM);
    static constexpr int WAVES = LOGM >= 13 ? 2 : (LOGM == 11 ? 3 : 4);
};

// Workgroup `block` of one volume's filter (row pairs block * PAIRS ...).
template <int LOGM, int STORE>
__device__ __forceinline__ void filter_block(const FilterArgs& a, int block) {
    using S = Store<STORE>;
    constexpr int M = 1 << LOGM;
    constexpr int TP = FilterShape<LOGM>::TP;          // threads per row pair
    constexpr int PAIRS = 256 / TP;                    // row pairs per workgroup
    constexpr int MP = Padded<M>::size;
    __shared__ float2 buf[PAIRS * MP];

    const int grp = threadIdx.x / TP;
    const int t = threadIdx.x % TP;
    // rows 2k and 2k + 1 of one projection share a transform (a projection
    // with an odd number of rows leaves its last row alone), so a band that
    // starts at an even row pairs its rows as the whole detector does
    const int hp = (a.nv + 1) >> 1;                   // row pairs per projection
    const int pair = block * PAIRS + grp;
    const int pp = pair / hp, kk = pair - pp * hp;
    const int r0 = pp * a.nv + 2 * kk, r1 = r0 + 1;
    const bool has0 = r0 < a.rows, has1 = has0 && 2 * kk + 1 < a.nv;
    float2* z = buf + grp * MP;
    const int n = a.n;
    const float rr = a.r * a.r;

    // the pre-weighted rows p~ go to LDS; the first stage of the forward
    // transform reads their first difference d[u] = p~[u] - p~[u-1]
    const float b0 = has0 ? (float)(a.v0 + r0 % a.nv) - a.c : 0.0f;
    const float b1 = has1 ? (float)(a.v0 + r1 % a.nv) - a.c : 0.0f;
    const float rb0 = rr + b0 * b0, rb1 = rr + b1 * b1;
    const float* p0 = a.proj + (size_t)r0 * n;
    const float* p1 = a.proj + (size_t)r1 * n;
    // the argument is at least R^2, a normal number, so the hardware
    // reciprocal square root needs none of the library's denormal scaling
    auto weight = [&](int u, float rb) {
        const float au = (float)u - a.c;
        return a.r * __builtin_amdgcn_rsqf(rb + au * au);
    };
    // every sample of the thread is requested before any is used: both
    // rows, all positions
    constexpr int IT = (M + TP - 1) / TP;
    float q0[IT], q1[IT];
    if constexpr (TP >= 64) {
        // one row pair per wave or more waves per pair: the rows are wave-
        // uniform, so they are read through buffer resources (32-bit offsets,
        // no per-load addresses; an absent row has an empty range and reads
        // zero, as does every sample past the row's end)
        const int u0r = __builtin_amdgcn_readfirstlane(has0 ? r0 : 0);
        const int u1r = __builtin_amdgcn_readfirstlane(has1 ? r1 : 0);
        const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(a.proj + (size_t)u0r * n), (short)0, __builtin_amdgcn_readfirstlane(has0 ? n * 4 : 0),
            0x00020000);
        const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(a.proj + (size_t)u1r * n), (short)0, __builtin_amdgcn_readfirstlane(has1 ? n * 4 : 0),
            0x00020000);
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int off = (t + i * TP) * 4;
            q0[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs0, off, 0, 0));
            q1[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs1, off, 0, 0));
        }
    } else {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int u = t + i * TP;
            const bool in = u < n;
            q0[i] = (in && has0) ? p0[u] : 0.0f;
            q1[i] = (in && has1) ? p1[u] : 0.0f;
        }
    }
    // pre-weighted rows p~[u] (zero from N on); the difference at u = N is
    // applied after the FFT
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int u = t + i * TP;
        if (u < M) {
            float d0 = 0.0f, d1 = 0.0f;
            if (u < n) {
                d0 = q0[i] * weight(u, rb0);
                d1 = q1[i] * weight(u, rb1);
            }
            z[pidx(u)] = make_float2(d0, d1);
        }
    }
    const float last0 = has0 ? p0[n - 1] * weight(n - 1, rb0) : 0.0f;
    const float last1 = has1 ? p1[n - 1] * weight(n - 1, rb1) : 0.0f;
    transform_sync<TP>();
    fft_lds<LOGM, TP, true, false>(z, t, a.twiddle, n);
    // tables (L2-resident) are requested in one batch before their first use
    float2 gr[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int k = t + i * TP;
        gr[i] = k < M ? a.resp[k] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int k = t + i * TP;
        if (k < M) {
            const float2 v = cmul(z[pidx(k)], gr[i]);
            z[pidx(k)] = make_float2(v.x, -v.y);      // conj(Z G)
        }
    }
    transform_sync<TP>();
    fft_lds<LOGM, TP, false, true>(z, t, a.twiddle, n);
    float gtl[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int u = t + i * TP;
        gtl[i] = u < n ? a.gtail[u] : 0.0f;          // g[u - N]
    }
    typename S::T* out = (typename S::T*)a.out;
    if constexpr (TP >= 64) {
        // output rows through buffer resources likewise (an absent row's
        // stores are dropped)
        constexpr int ES = (int)sizeof(typename S::T);
        const int u0r = __builtin_amdgcn_readfirstlane(has0 ? r0 : 0);
        const int u1r = __builtin_amdgcn_readfirstlane(has1 ? r1 : 0);
        const __amdgpu_buffer_rsrc_t ro0 = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(out + (size_t)u0r * n), (short)0, __builtin_amdgcn_readfirstlane(has0 ? n * ES : 0),
            0x00020000);
        const __amdgpu_buffer_rsrc_t ro1 = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(out + (size_t)u1r * n), (short)0, __builtin_amdgcn_readfirstlane(has1 ? n * ES : 0),
            0x00020000);
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int u = t + i * TP;
            if (u < n) {
                const float2 v = z[pidx(u)];          // conj of the result
                S::put_raw(ro0, u * ES, v.x - last0 * gtl[i]);
                S::put_raw(ro1, u * ES, -v.y - last1 * gtl[i]);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int u = t + i * TP;
            if (u < n) {
                const float2 v = z[pidx(u)];          // conj of the result
                if (has0) S::put(out, (size_t)r0 * n + u, v.x - last0 * gtl[i]);
                if (has1) S::put(out, (size_t)r1 * n + u, -v.y - last1 * gtl[i]);
            }
        }
    }
}

template <int LOGM, int STORE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FilterShape<LOGM>::WAVES)))
void k_filter(FilterArgs a) {
    filter_block<LOGM, STORE>(a, blockIdx.x);
}

// Many volumes of one FFT length: workgroup b is workgroup b - start[v] of
// volume v.
template <int LOGM, int STORE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FilterShape<LOGM>::WAVES)))
void k_filter_batch(FilterBatchArgs ba) {
    const int b = blockIdx.x;
    const int v = batch_volume(ba.start, ba.nvol, b);
    const FilterArgs a = const_load(ba.vols + v);
    filter_block<LOGM, STORE>(a, b - const_load(ba.start + v));
}

// ---------------------------------------------------------------------------
// M = 4096 (N = 1025..2048): four-step transform, one row pair per wavefront.
// Index u = a + 64 b (a: the lane, b: a register); the length-4096 DFT is a
// 64-point DFT over b in every lane, a twiddle w^(a c), a transpose through
// LDS, and a 64-point DFT over a in every lane: X[c + 64 d] lands in lane c,
// register d -- the same layout (lane = low six bits of the index), so the
// second transform of the filter (the forward DFT of conj(X G), section above)
// runs the same steps on it.  The 64-point DFTs are in registers (4 x 16:
// four 16-point DFTs, constant twiddles, sixteen 4-point DFTs); two passes
// through LDS per transform and no workgroup barrier (the wavefront is the
// whole workgroup).  N <= M / 2: the upper half of the first DFT's inputs
// (b >= 32) is zero and the upper half of the last DFT's outputs is unused,
// both left out.

// w64^j = exp(-2 pi i j / 64)
__device__ constexpr float kW64[64][2] = {
    {1.0f, 0.0f}, {0.9951847195625305f, -0.0980171412229538f}, {0.9807852506637573f, -0.19509032368659973f}, {0.9569403529167175f, -0.290284663438797f},
    {0.9238795042037964f, -0.3826834261417389f}, {0.8819212913513184f, -0.4713967442512512f}, {0.8314695954322815f, -0.5555702447891235f}, {0.7730104327201843f, -0.6343932747840881f},
    {0.7071067690849304f, -0.7071067690849304f}, {0.6343932747840881f, -0.7730104327201843f}, {0.5555702447891235f, -0.8314695954322815f}, {0.4713967442512512f, -0.8819212913513184f},
    {0.3826834261417389f, -0.9238795042037964f}, {0.290284663438797f, -0.9569403529167175f}, {0.19509032368659973f, -0.9807852506637573f}, {0.0980171412229538f, -0.9951847195625305f},
    {0.0f, -1.0f}, {-0.0980171412229538f, -0.9951847195625305f}, {-0.19509032368659973f, -0.9807852506637573f}, {-0.290284663438797f, -0.9569403529167175f},
    {-0.3826834261417389f, -0.9238795042037964f}, {-0.4713967442512512f, -0.8819212913513184f}, {-0.5555702447891235f, -0.8314695954322815f}, {-0.6343932747840881f, -0.7730104327201843f},
    {-0.7071067690849304f, -0.7071067690849304f}, {-0.7730104327201843f, -0.6343932747840881f}, {-0.8314695954322815f, -0.5555702447891235f}, {-0.8819212913513184f, -0.4713967442512512f},
    {-0.9238795042037964f, -0.3826834261417389f}, {-0.9569403529167175f, -0.290284663438797f}, {-0.9807852506637573f, -0.19509032368659973f}, {-0.9951847195625305f, -0.0980171412229538f},
    {-1.0f, 0.0f}, {-0.9951847195625305f, 0.0980171412229538f}, {-0.9807852506637573f, 0.19509032368659973f}, {-0.9569403529167175f, 0.290284663438797f},
    {-0.9238795042037964f, 0.3826834261417389f}, {-0.8819212913513184f, 0.4713967442512512f}, {-0.8314695954322815f, 0.5555702447891235f}, {-0.7730104327201843f, 0.6343932747840881f},
    {-0.7071067690849304f, 0.7071067690849304f}, {-0.6343932747840881f, 0.7730104327201843f}, {-0.5555702447891235f, 0.8314695954322815f}, {-0.4713967442512512f, 0.8819212913513184f},
    {-0.3826834261417389f, 0.9238795042037964f}, {-0.290284663438797f, 0.9569403529167175f}, {-0.19509032368659973f, 0.9807852506637573f}, {-0.0980171412229538f, 0.9951847195625305f},
    {0.0f, 1.0f}, {0.0980171412229538f, 0.9951847195625305f}, {0.19509032368659973f, 0.9807852506637573f}, {0.290284663438797f, 0.9569403529167175f},
    {0.3826834261417389f, 0.9238795042037964f}, {0.4713967442512512f, 0.8819212913513184f}, {0.5555702447891235f, 0.8314695954322815f}, {0.6343932747840881f, 0.7730104327201843f},
    {0.7071067690849304f, 0.7071067690849304f}, {0.7730104327201843f, 0.6343932747840881f}, {0.8314695954322815f, 0.5555702447891235f}, {0.8819212913513184f, 0.4713967442512512f},
    {0.9238795042037964f, 0.3826834261417389f}, {0.9569403529167175f, 0.290284663438797f}, {0.9807852506637573f, 0.19509032368659973f}, {0.9951847195625305f, 0.0980171412229538f}};

// 64-point forward DFT in registers, natural order in and out; HALF_IN: the
// inputs from 32 on are zero; HALF_OUT: only the outputs below 32 are used.
template <bool HALF_IN, bool HALF_OUT>
__device__ __forceinline__ void dft64(float2 (&v)[64]) {
    float2 A[4][16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1)
            A[n2][n1] = (HALF_IN && 4 * n1 + n2 >= 32) ? make_float2(0.0f, 0.0f) : v[4 * n1 + n2];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft16(A[n2]);
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) {
            const int j = n2 * k1;
            A[n2][k1] = cmul(A[n2][k1], make_float2(kW64[j][0], kW64[j][1]));
        }
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) {
        float2 a = A[0][k1], b = A[1][k1], c = A[2][k1], d = A[3][k1];
        dft4(a, b, c, d);
        v[k1] = a;
        v[k1 + 16] = b;
        if (!HALF_OUT) {
            v[k1 + 32] = c;
            v[k1 + 48] = d;
        }
    }
}

// One length-4096 forward DFT of the wavefront's data in four steps (see
// above): v[b] of lane a holds x[a + 64 b] on entry and X[a + 64 b] on exit.
template <bool HALF_IN, bool HALF_OUT>
__device__ __forceinline__ void dft4096_wave(float2 (&v)[64], float2* T, const float2* __restrict__ tw,
                                             int lane) {
    constexpr int TP = 65;                         // LDS row pitch (float2): rows spread over the banks
    dft64<HALF_IN, false>(v);
    // twiddles w^(a c), a = lane (requested together, then applied)
#pragma unroll
    for (int c0 = 0; c0 < 64; c0 += 16) {
        float2 w[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) w[c] = tw[(lane * (c0 + c)) & 4095];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c0 + c] = cmul(v[c0 + c], w[c]);
    }
    // transpose: lane a writes row a, then lane c reads column c
#pragma unroll
    for (int c = 0; c < 64; ++c) T[lane * TP + c] = v[c];
    transform_sync<64>();
#pragma unroll
    for (int a = 0; a < 64; ++a) v[a] = T[a * TP + lane];
    transform_sync<64>();
    dft64<false, HALF_OUT>(v);
}

// Row pair `pair` of one volume (a 64-thread workgroup).
template <int STORE>
__device__ __forceinline__ void filter4096_pair(const FilterArgs& a, int pair) {
    using S = Store<STORE>;
    constexpr int ES = (int)sizeof(typename S::T);
    __shared__ float2 T[64 * 65];
    const int lane = threadIdx.x;
    const int hp = (a.nv + 1) >> 1;
    const int pp = pair / hp, kk = pair - pp * hp;
    const int r0 = pp * a.nv + 2 * kk, r1 = r0 + 1;
    const bool has0 = r0 < a.rows, has1 = has0 && 2 * kk + 1 < a.nv;
    const int n = a.n;
    const float rr = a.r * a.r;
    const float b0 = has0 ? (float)(a.v0 + r0 % a.nv) - a.c : 0.0f;
    const float b1 = has1 ? (float)(a.v0 + r1 % a.nv) - a.c : 0.0f;
    const float rb0 = rr + b0 * b0, rb1 = rr + b1 * b1;
    auto weight = [&](int u, float rb) {
        const float au = (float)u - a.c;
        return a.r * __builtin_amdgcn_rsqf(rb + au * au);
    };
    const int u0r = __builtin_amdgcn_readfirstlane(has0 ? r0 : 0);
    const int u1r = __builtin_amdgcn_readfirstlane(has1 ? r1 : 0);
    const __amdgpu_buffer_rsrc_t rs0 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.proj + (size_t)u0r * n), (short)0, __builtin_amdgcn_readfirstlane(has0 ? n * 4 : 0), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.proj + (size_t)u1r * n), (short)0, __builtin_amdgcn_readfirstlane(has1 ? n * 4 : 0), 0x00020000);
    // pre-weighted rows p~[u], u = lane + 64 b < 2048 (zero from n on: past
    // the row the buffer reads zero, and the weight is finite, so no lane is
    // masked off), then their first difference: p~[u-1] is the previous
    // lane's (a DPP rotation of the wave by one lane), for lane 0 lane 63's of
    // b - 1 (the previous register's rotation, held in lane 0)
    float2 v[64];
    float q0[32], q1[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        q0[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs0, (lane + 64 * b) * 4, 0, 0));
        q1[b] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs1, (lane + 64 * b) * 4, 0, 0));
    }
    const bool lane0 = lane == 0;
    float rot0 = 0.0f, rot1 = 0.0f;                // rotation of b - 1 (p~[-1] = 0 for b = 0)
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const int u = lane + 64 * b;
        const float t0 = q0[b] * weight(u, rb0);
        const float t1 = q1[b] * weight(u, rb1);
        const float r0 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t0), 0x13C /* wave_ror:1 */, 0xf, 0xf, false));
        const float r1 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t1), 0x13C /* wave_ror:1 */, 0xf, 0xf, false));
        const float s0 = lane0 ? rot0 : r0;
        const float s1 = lane0 ? rot1 : r1;
        rot0 = r0;
        rot1 = r1;
        const bool in = u < n;
        v[b].x = in ? t0 - s0 : 0.0f;
        v[b].y = in ? t1 - s1 : 0.0f;
    }
#pragma unroll
    for (int b = 32; b < 64; ++b) v[b] = make_float2(0.0f, 0.0f);
    const float last0 = has0 ? a.proj[(size_t)u0r * n + n - 1] * weight(n - 1, rb0) : 0.0f;
    const float last1 = has1 ? a.proj[(size_t)u1r * n + n - 1] * weight(n - 1, rb1) : 0.0f;
    dft4096_wave<true, false>(v, T, a.twiddle, lane);
    // conj(X G): X[lane + 64 d] in v[d]
#pragma unroll
    for (int d0 = 0; d0 < 64; d0 += 16) {
        float2 g[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) g[d] = a.resp[lane + 64 * (d0 + d)];
#pragma unroll
        for (int d = 0; d < 16; ++d) {
            const float2 x = cmul(v[d0 + d], g[d]);
            v[d0 + d] = make_float2(x.x, -x.y);
        }
    }
    dft4096_wave<false, true>(v, T, a.twiddle, lane);
    // the result is conj(v): row 0 its real part, row 1 its imaginary part.
    // The tail table and the rows go through buffer resources of n samples:
    // from n on the table reads zero and the stores are dropped, so no lane
    // is masked off.
    const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a.gtail, (short)0, n * 4, 0x00020000);
    float gt[32];
#pragma unroll
    for (int f = 0; f < 32; ++f)
        gt[f] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, (lane + 64 * f) * 4, 0, 0));
    typename S::T* out = (typename S::T*)a.out;
    const __amdgpu_buffer_rsrc_t ro0 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(out + (size_t)u0r * n), (short)0, __builtin_amdgcn_readfirstlane(has0 ? n * ES : 0), 0x00020000);
    const __amdgpu_buffer_rsrc_t ro1 = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(out + (size_t)u1r * n), (short)0, __builtin_amdgcn_readfirstlane(has1 ? n * ES : 0), 0x00020000);
#pragma unroll
    for (int f = 0; f < 32; ++f) {
        const int u = lane + 64 * f;
        S::put_raw(ro0, u * ES, v[f].x - last0 * gt[f]);
        S::put_raw(ro1, u * ES, -v[f].y - last1 * gt[f]);
    }
}

template <int STORE>
__global__ __launch_bounds__(64) void k_filter4096(FilterArgs a) {
    filter4096_pair<STORE>(a, blockIdx.x);
}

template <int STORE>
__global__ __launch_bounds__(64) void k_filter4096_batch(FilterBatchArgs ba) {
    const int b = blockIdx.x;
    const int v = batch_volume(ba.start, ba.nvol, b);
    const FilterArgs a = const_load(ba.vols + v);
    filter4096_pair<STORE>(a, b - const_load(ba.start + v));
}

template <int LOGM>
static hipError_t launch_filter_m(const FilterArgs& a, int store, hipStream_t st) {
    constexpr int TP = FilterShape<LOGM>::TP;
    constexpr int PAIRS = 256 / TP;
    const int pairs = (a.rows / a.nv) * ((a.nv + 1) / 2);
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
        case 12: {
            // the four-step form: one row pair per 64-thread workgroup
            const dim3 grid((a.rows / a.nv) * ((a.nv + 1) / 2));
            switch (store) {
                case 0: hipLaunchKernelGGL((k_filter4096<0>), grid, dim3(64), 0, st, a); break;
                case 1: hipLaunchKernelGGL((k_filter4096<1>), grid, dim3(64), 0, st, a); break;
                default: hipLaunchKernelGGL((k_filter4096<2>), grid, dim3(64), 0, st, a); break;
            }
            return hipGetLastError();
        }
        case 13: return launch_filter_m<13>(a, store, st);
        default: return hipErrorInvalidValue;
    }
}

int filter_workgroups(const FilterArgs& a, int logm) {
    const int pairs = (a.rows / a.nv) * ((a.nv + 1) / 2);
    if (logm == 12) return pairs;
    const int per = 256 / filter_threads_per_pair(logm);
    return (pairs + per - 1) / per;
}

template <int LOGM>
static hipError_t launch_filter_batch_m(const FilterBatchArgs& a, int store, int workgroups, hipStream_t st) {
    const dim3 grid(workgroups);
    switch (store) {
        case 0: hipLaunchKernelGGL((k_filter_batch<LOGM, 0>), grid, dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_filter_batch<LOGM, 1>), grid, dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((k_filter_batch<LOGM, 2>), grid, dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_filter_batch(const FilterBatchArgs& a, int logm, int store, int workgroups, hipStream_t st) {
    if (workgroups <= 0) return hipSuccess;
    switch (logm) {
        case 3: return launch_filter_batch_m<3>(a, store, workgroups, st);
        case 4: return launch_filter_batch_m<4>(a, store, workgroups, st);
        case 5: return launch_filter_batch_m<5>(a, store, workgroups, st);
        case 6: return launch_filter_batch_m<6>(a, store, workgroups, st);
        case 7: return launch_filter_batch_m<7>(a, store, workgroups, st);
        case 8: return launch_filter_batch_m<8>(a, store, workgroups, st);
        case 9: return launch_filter_batch_m<9>(a, store, workgroups, st);
        case 10: return launch_filter_batch_m<10>(a, store, workgroups, st);
        case 11: return launch_filter_batch_m<11>(a, store, workgroups, st);
        case 12:
            switch (store) {
                case 0: hipLaunchKernelGGL((k_filter4096_batch<0>), dim3(workgroups), dim3(64), 0, st, a); break;
                case 1: hipLaunchKernelGGL((k_filter4096_batch<1>), dim3(workgroups), dim3(64), 0, st, a); break;
                default: hipLaunchKernelGGL((k_filter4096_batch<2>), dim3(workgroups), dim3(64), 0, st, a); break;
            }
            return hipGetLastError();
        case 13: return launch_filter_batch_m<13>(a, store, workgroups, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdkod
