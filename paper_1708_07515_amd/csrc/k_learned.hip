// Learned angular decimation and its training kernels (gfx950).
//
// The paper leaves the low-pass filter of the angular decimation open (Sec. 2.1:
// quality depends on the low-pass filter's implementation).  The learned filter
// adds a correction R to the plain triangle decimation T of every square q and
// detector row v:
//
//   Y_q[m][v][j] = T[m][j] + R[m][j],   R = conv2(ReLU(conv1(S)))
//   conv1: H_k(p, j) = b1_k + sum_{a,b} W1[k][a][b] S((p + (a-2) d) mod P, j + b - 2)
//   R(m, j) = b2 + sum_{k,a,b} W2[k][a][b] A_k((c(m) + (a-2) d) mod P, j + b - 2)
//
// with S the cropped, shifted full-rate sub-sinogram (Sec. 2.1), A = ReLU(H)
// on the columns [0, W) and zero outside, c(m) the original angle nearest to
// the decimated angle m, d = max(1, D / 4), 16 channels, 5 x 5 taps.
//
// Matrix cores.  conv1 is a BF16 MFMA product per 16 columns,
//   H^T[16 ch][16 col] = W1[16 ch][32 taps] x X^T[32 taps][16 col]
// (X^T gathers S at the taps), FP32 accumulation.  Its output layout (lane l
// holds channels 4(l/16)..+3 of column l%16) is exactly the B-operand layout
// of a second MFMA, which contracts the channels of conv2:
//   Q[b][col] += W2_a[16 (b, 5 used)][16 ch] x A^T[16 ch][16 col]
// over the five dilated angles a; then R[j] = b2 + sum_b Q[b][j+b-2].  The
// forward pass uses the K = 32 product (one per conv1 angle, three for conv2
// with two angles per product), the training pass the K = 16 one.  The weight
// gradient of conv1 is an MFMA reduction over positions:
//   dW1^T[32 taps][16 ch] += X[taps][16 pos] x dH[16 pos][16 ch].
// Weights are BF16 (817 values: W1 [16][5][5], b1 [16], W2 [16][5][5], b2).
//
// One workgroup per (square, row) walks the decimated angles m.  The S values
// of the nine original angles c(m) + (t - 4) d, t = 0..8, are kept in LDS as
// BF16 (the precision conv1 multiplies them in).  The next angle's S values
// and output row are loaded into registers before the current angle's matrix
// products, so the global-memory latency of one angle overlaps the
// arithmetic of the previous one; when the decimated angles fall on original
// ones the forward pass fetches only the four rows that the next angle adds.
#include "internal.h"
#include "dtype.h"
#include "geom.h"

namespace fdkod {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kSP = 16 * ((kLearnedMaxWidth + 15) / 16) + 4;  // LDS pitch of the Q rows (general forward)
constexpr int kOffW1 = 0, kOffB1 = 400, kOffW2 = 416, kOffB2 = 816;
constexpr int kThreads = 256;
static_assert(kLearnedMaxWidth + 4 <= kThreads, "one thread per staged column");

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// FP32 -> BF16, round to nearest even (hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// c(m) = floor(m P / P' + 1/2) = floor((2 m P + P') / (2 P')), walked in m
// with an integer quotient and remainder (c(m) < P for m < P').
struct CentreWalk {
    int c, rem, dq, dr, den;
    __device__ CentreWalk(int p, int pd) {
        den = 2 * pd;
        dq = (2 * p) / den;
        dr = (2 * p) % den;
        c = pd / den;      // m = 0: floor(P' / 2P') = 0
        rem = pd % den;
    }
    __device__ void next() {
        c += dq;
        rem += dr;
        if (rem >= den) {
            rem -= den;
            ++c;
        }
    }
};

// One row of S at the thread's column: the detector samples of the crop's
// interpolation -- two for the linear shift, four (offsets -1 .. 2) for Keys'
// cubic convolution -- and the fraction; value() is S.
template <bool CUBIC>
struct SRow {
    float x[CUBIC ? 4 : 2];
    float ph;
    __device__ __forceinline__ float value() const {
        if constexpr (CUBIC) {
            float c[4];
            keys_weights(ph, c);
            float s = c[0] * x[0];
            s = fmaf(c[1], x[1], s);
            s = fmaf(c[2], x[2], s);
            return fmaf(c[3], x[3], s);
        } else {
            return fmaf(ph, x[1] - x[0], x[0]);
        }
    }
};

// The detector samples of row p at the crop offset o and local column jj,
// each through its own range-checked load (zero outside the row; a column
// outside [0, W) takes offsets left of the row and reads zero).
template <int STORE, bool CUBIC>
__device__ __forceinline__ void srow_load(const LearnedArgs& a, int v, int p, float o, int jj, bool valid,
                                          SRow<CUBIC>& r) {
    using S = Store<STORE>;
    using T = typename S::T;
    constexpr int ES = (int)sizeof(T);
    const float of = floorf(o);
    r.ph = o - of;
    const __amdgpu_buffer_rsrc_t rs = row_rsrc((const T*)a.filt + ((size_t)p * a.nv + v) * a.n, a.n);
    constexpr int K = CUBIC ? 4 : 2, LO = CUBIC ? -1 : 0;
    const int off0 = valid ? ((int)of + jj + LO) * ES : -(K + 2) * ES;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        int off = off0 + i * ES;
        if (i > 0) asm volatile("" : "+v"(off));   // separately range-checked loads, never one wider load
        r.x[i] = S::raw(rs, off);
    }
}

// The nine rows of S for centre angle c at the thread's column jj: detector
// samples x0, x1 and the (row-uniform) interpolation fraction.  offr[t]: the
// row offsets (t - 4) d mod P.  Rows are read through buffer resources that
// span exactly one detector row, so samples outside the detector, and every
// sample of a column outside [0, W) (given a negative offset), read zero.
template <int STORE, bool CUBIC>
__device__ __forceinline__ void s_fetch_rows(const LearnedArgs& a, const float* acq, float u0f, int v, int c,
                                             int jj, bool valid, const int offr[9], SRow<CUBIC> (&rows)[9]) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        int p = c + offr[t];
        if (p >= a.p) p -= a.p;
        srow_load<STORE, CUBIC>(a, v, p, const_load(acq + p) + u0f, jj, valid, rows[t]);
    }
}

// The forward pass keeps the nine S rows in a pair layout: entry x of row t
// holds the BF16 values of staged columns x (low half) and x + 1 (high half),
// so one 32-bit LDS load gives a lane two of its conv1 taps.  Its K order
// groups the taps in horizontal pairs: pair pi = 3 a + e (a = 0..4, e = 0..2)
// holds taps (a, 2e) and (a, 2e + 1), where tap (a, 5) has weight zero; pair
// (0, 3) pads the K dimension (weight zero; the entries beyond the staged
// columns stay at the zeros the tile was cleared to).
constexpr int kPP = 16 * ((kLearnedMaxWidth + 15) / 16) + 8;   // pitch in pairs (index 16 ntile + 5 read)
static_assert(kPP >= kThreads + 1, "every staged column has a pair entry");

struct FwdSmem {
    int off_tab[9];
    uint32_t sp[9 * kPP];
};

// Operands of the forward pass, which runs on the K = 32 BF16 MFMA
// (16x16x32: a lane of group g = lane / 16 holds eight K slots of its row or
// column; the product pairs A's and B's slots of the same lane group and
// element, so any K order common to both is valid).
//   conv1: lane group g holds two dominoes of pairs, a horizontal one (pairs
//          (a, e) and (a, e + 1), two entries apart) and a vertical one
//          ((a, e) and (a + 1, e), one row apart), so that each is one
//          two-address LDS load into consecutive registers.  The eight
//          dominoes cover the 15 pairs and one padding pair (0, 3), i.e.
//          taps (0, 6) and (0, 7), whose weights are zero like tap (a, 5).
//          Slot (g, i): pair k = i / 2 of the group (H first, H second,
//          V first, V second), half i % 2.
//   conv2: K = two dilated angles x 16 channels, three products t = 0..2;
//          slot (g, i) is channel 4 g + i % 4 of angle 2 t + i / 4 (angle 5:
//          weight zero), which is exactly how conv1's outputs for angles 2 t
//          and 2 t + 1 sit in the lane (channels 4 g .. 4 g + 3 of its column).
typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// first pairs (a, e) of each group's horizontal and vertical domino
__device__ constexpr int kDomH[4][2] = {{0, 0}, {0, 2}, {1, 1}, {4, 1}};
__device__ constexpr int kDomV[4][2] = {{1, 0}, {2, 1}, {2, 2}, {3, 0}};

struct FwdOperands {
    bf8v w1;          // A of conv1: row = channel lr
    bf8v w2[3];       // A of conv2: row = R offset b = lr (0..4 used)
    f4v b1;           // conv1 bias of the lane's output channels 4 g .. 4 g + 3
    int hoff, voff;   // the lane's dominoes in a tile of pitch PP (column lr)
};

template <int PP>
__device__ __forceinline__ FwdOperands load_fwd_operands(const uint16_t* w) {
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    FwdOperands op;
    s8v w1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = i / 2;
        const int* dom = k < 2 ? kDomH[lg] : kDomV[lg];
        const int ta = dom[0] + (k == 3 ? 1 : 0), e = dom[1] + (k == 1 ? 1 : 0);
        const int tb = 2 * e + (i & 1);
        w1[i] = tb < 5 ? (short)w[kOffW1 + lr * 25 + ta * 5 + tb] : (short)0;
    }
    op.w1 = __builtin_bit_cast(bf8v, w1);
    op.hoff = kDomH[lg][0] * PP + 2 * kDomH[lg][1] + lr;
    op.voff = kDomV[lg][0] * PP + 2 * kDomV[lg][1] + lr;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        s8v w2;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int a2 = 2 * t + i / 4, ch = 4 * lg + i % 4;
            w2[i] = lr < 5 && a2 < 5 ? (short)w[kOffW2 + ch * 25 + a2 * 5 + lr] : (short)0;
        }
        op.w2[t] = __builtin_bit_cast(bf8v, w2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) op.b1[i] = bf2f(w[kOffB1 + 4 * lg + i]);
    return op;
}

// Stage the thread's column x of the nine rows: the low half of pair x and
// the high half of pair x - 1.
template <bool CUBIC>
__device__ __forceinline__ void s_stage_pairs(uint32_t* sp, int x, const SRow<CUBIC> (&rows)[9]) {
    uint16_t* h = reinterpret_cast<uint16_t*>(sp);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const uint16_t v = f2bf(rows[t].value());
        h[2 * (t * kPP + x)] = v;
        if (x > 0) h[2 * (t * kPP + x - 1) + 1] = v;
    }
}

// ReLU of a conv1 output (FP32, bias included) as the BF16 B operand of
// conv2.  Rounding commutes with ReLU, so the values are rounded first and
// the negative BF16 codes (sign bit set: negative as 16-bit integers) are then
// cleared by a packed integer maximum with zero.
__device__ __forceinline__ s4v relu_bf16(f4v h) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
    typedef short s2v __attribute__((ext_vector_type(2)));
    const s2v zero = {0, 0};
    const s2v lo = __builtin_elementwise_max(
        __builtin_bit_cast(s2v, __builtin_convertvector((f2v){h[0], h[1]}, bf2v)), zero);
    const s2v hi = __builtin_elementwise_max(
        __builtin_bit_cast(s2v, __builtin_convertvector((f2v){h[2], h[3]}, bf2v)), zero);
    return (s4v){lo[0], lo[1], hi[0], hi[1]};
}

// One 16-column tile of the forward pass for the nine S rows starting at sp
// (pair layout, row pitch PP): conv1 at the five dilated angles (five
// independent MFMAs, the bias as the initial accumulator), ReLU, conv2 (three
// MFMAs); Q rows 0..4 go to qt (row pitch QP, column c at index c + 2) for
// the columns inside [0, W) only: outside, A and hence Q are zero, and the Q
// tile keeps the zeros it was cleared to.
template <int PP, int QP>
__device__ __forceinline__ void fwd_tile(const uint32_t* sp, float* qt, int col0, int width,
                                         const FwdOperands& op) {
    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const uint32_t* ph = sp + col0 + op.hoff;
    const uint32_t* pv = sp + col0 + op.voff;
    f4v h[5];
#pragma unroll
    for (int a2 = 0; a2 < 5; ++a2) {
        const u4v d = {ph[a2 * PP], ph[a2 * PP + 2], pv[a2 * PP], pv[a2 * PP + PP]};
        h[a2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(op.w1, __builtin_bit_cast(bf8v, d), op.b1, 0, 0, 0);
    }
    f4v qacc = {0.0f, 0.0f, 0.0f, 0.0f};
    const s4v zero = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const s4v lo = relu_bf16(h[2 * t]);
        const s4v hi = t < 2 ? relu_bf16(h[2 * t + 1]) : zero;
        const s8v act = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        qacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(op.w2[t], __builtin_bit_cast(bf8v, act), qacc, 0, 0, 0);
    }
    if (col0 + lr < width) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int bb = 4 * lg + i;
            if (bb < 5) qt[bb * QP + col0 + lr + 2] = qacc[i];
        }
    }
}

// XCD-aware task order of the forward kernels.  Workgroups are dealt to the
// XCDs round-robin (workgroup b to XCD b mod 8), so the workgroups of XCD x
// take the detector rows v = x (mod 8), all squares of a row consecutively:
// the overlapping crops of one detector row read the same filtered rows, and
// that XCD's L2 then fetches them once.  Grid: nsq * 8 * ceil(N / 8); the
// workgroups with v >= N exit at once.
__device__ __forceinline__ bool fwd_task(const LearnedArgs& a, int& q, int& v) {
    const int x = (int)blockIdx.x % kXcds, i = (int)blockIdx.x / kXcds;
    q = i % a.nsq;
    v = (i / a.nsq) * kXcds + x;
    return v < a.nv;
}

__host__ __device__ inline unsigned fwd_grid(const LearnedArgs& a) {
    return (unsigned)a.nsq * kXcds * ((a.nv + kXcds - 1) / kXcds);
}

// Forward (inference): Y(m) += R(m) for every decimated angle of one
// (square, row).  Thread t stages column t - 2 of the tile and owns output
// column t; the waves share the 16-column tiles.  This form fetches the nine
// S rows of every angle; k_learned_fwd_ring below reuses them when the
// decimated angles fall on original ones.
template <int STORE, bool CUBIC>
__global__ __launch_bounds__(kThreads) void k_learned_fwd(LearnedArgs a) {
    using S = Store<STORE>;
    using T = typename S::T;
    __shared__ FwdSmem sm;
    __shared__ float q_tile[5 * kSP];
    int q, v;
    if (!fwd_task(a, q, v)) return;
    const int2 gd = a.grid[q];
    const int u0 = gd.x, width = gd.y;
    const int wave = threadIdx.x >> 6;
    const FwdOperands op = load_fwd_operands<kPP>(a.w);
    const float b2 = bf2f(a.w[kOffB2]);
    const int ntile = (width + 15) >> 4;
    // the crop offset of projection p is a_c(beta_p) + u0 (a_c from the
    // bounds, read through scalar loads where it is used)
    const float* acq = a.ac_p + (size_t)q * a.p;
    const float u0f = (float)u0;
    if (threadIdx.x < 9) {
        int off = ((int)threadIdx.x - 4) * a.d % a.p;
        sm.off_tab[threadIdx.x] = off < 0 ? off + a.p : off;
    }
    for (int e = threadIdx.x; e < 9 * kPP; e += kThreads) sm.sp[e] = 0u;
    for (int e = threadIdx.x; e < 5 * kSP; e += kThreads) q_tile[e] = 0.0f;
    const int col = threadIdx.x;               // staged column index (local column col - 2)
    const int jj = col - 2;
    const bool stager = col < width + 4;
    const bool valid = jj >= 0 && jj < width;
    T* ws = (T*)a.ws;
    const size_t yrow = (size_t)a.squares[q].y_off_row * a.nv + (size_t)v * width;   // + m n W + j
    const size_t yplane = (size_t)a.nv * width;
    const int j = threadIdx.x;                                           // output column
    CentreWalk cw(a.p, a.pd);
    __syncthreads();
    int offr[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) offr[t] = __builtin_amdgcn_readfirstlane(sm.off_tab[t]);

    SRow<CUBIC> rows[9];
    s_fetch_rows<STORE, CUBIC>(a, acq, u0f, v, cw.c, jj, valid, offr, rows);
    float y_cur = j < width ? S::load(ws, yrow + j) : 0.0f;
    if (stager) s_stage_pairs(sm.sp, col, rows);
    vmem_drain();
    __syncthreads();
    for (int m = 0; m < a.pd; ++m) {
        const bool more = m + 1 < a.pd;
        float y_next = 0.0f;
        if (more) {
            cw.next();
            s_fetch_rows<STORE, CUBIC>(a, acq, u0f, v, cw.c, jj, valid, offr, rows);
            if (j < width) y_next = S::load(ws, yrow + (size_t)(m + 1) * yplane + j);
        }
#pragma unroll
        for (int k = 0; k < kPP / 64; ++k) {
            const int tile = wave + 4 * k;
            if (tile < ntile) fwd_tile<kPP, kSP>(sm.sp, q_tile, tile * 16, width, op);
        }
        __syncthreads();
        if (j < width) {
            float r = b2;
#pragma unroll
            for (int bb = 0; bb < 5; ++bb) r += q_tile[bb * kSP + j + bb];
            S::put(ws, yrow + (size_t)m * yplane + j, y_cur + r);
        }
        if (more && stager) s_stage_pairs(sm.sp, col, rows);
        vmem_drain();
        y_cur = y_next;
        __syncthreads();
    }
}

// Row reuse.  When D divides P and D >= 4 (so d = D / 4), c(m) = m D and the
// nine S rows of angle m are the rows u = 4m .. 4m + 8 of the sequence
// p(u) = (u - 4) d mod P: consecutive angles share five rows.  The rows live
// in a ring of 16 LDS slots, row u in slot u mod 16; windows start at slots
// 0, 4, 8 and 12, so mirroring slots 0..4 at 16..20 makes every window of
// nine contiguous.  Each angle fetches
// its successor's four new rows and stages them while its own products run
// (their slots, and mirrors, lie outside its window), and the Q tile
// alternates between two buffers, so one barrier per angle orders the whole
// pipeline.  PW: the widest square's tiles (128, 224 or 256 columns; 224
// keeps five workgroups per compute unit within the LDS).
constexpr int kRing = 16;
constexpr int kRingMirror = 5;
constexpr int kRingSlots = kRing + kRingMirror;

template <int PW>
struct RingSmem {
    static constexpr int kPitch = PW + 8;   // pairs: a tile reads up to index 16 ntile + 5
    static constexpr int kQPitch = PW + 4;  // Q rows: columns -2 .. 16 ntile + 1
    uint32_t sp[kRingSlots * kPitch];
    float qb[2][5 * kQPitch];
};
// The ring kernel stages the crop offsets of all P projections in LDS beside
// its tile (64 KB per workgroup): up to this many projections; more take the
// general kernel, which reads each offset where it is used.
constexpr int kRingMaxP = (65536 - (int)sizeof(RingSmem<256>)) / 4;
static_assert(kRingMaxP >= 2048, "ring tile and offset table fit the LDS of a workgroup");

// Row p of S at the thread's staged column (local column jj): the two
// detector samples and the interpolation fraction (zero outside the row and
// for columns outside [0, W), as s_fetch_rows).
template <int STORE, bool CUBIC>
__device__ __forceinline__ void ring_fetch(const LearnedArgs& a, const float* o_tab, int v, int p, int jj,
                                           bool valid, SRow<CUBIC>& r) {
    srow_load<STORE, CUBIC>(a, v, p, o_tab[p], jj, valid, r);
}

// Stage the thread's column x of one row into ring slot `slot` (and its
// mirror): the low half of pair x and the high half of pair x - 1.
template <int PP, bool CUBIC>
__device__ __forceinline__ void ring_stage(uint32_t* sp, int slot, int x, const SRow<CUBIC>& r) {
    uint16_t* h = reinterpret_cast<uint16_t*>(sp);
    const uint16_t val = f2bf(r.value());
    h[2 * (slot * PP + x)] = val;
    if (x > 0) h[2 * (slot * PP + x - 1) + 1] = val;
    if (slot < kRingMirror) {
        h[2 * ((slot + kRing) * PP + x)] = val;
        if (x > 0) h[2 * ((slot + kRing) * PP + x - 1) + 1] = val;
    }
}

template <int STORE, int PW, bool CUBIC>
__global__ __launch_bounds__(kThreads) void k_learned_fwd_ring(LearnedArgs a) {
    using S = Store<STORE>;
    using T = typename S::T;
    using R = RingSmem<PW>;
    constexpr int PP = R::kPitch, QP = R::kQPitch;
    __shared__ R sm;
    extern __shared__ float o_tab[];     // [P]: a_c(beta_p) + u0
    int q, v;
    if (!fwd_task(a, q, v)) return;
    const int2 gd = a.grid[q];
    const int u0 = gd.x, width = gd.y;
    const int wave = threadIdx.x >> 6;
    const FwdOperands op = load_fwd_operands<PP>(a.w);
    const float b2 = bf2f(a.w[kOffB2]);
    const int ntile = (width + 15) >> 4;
    for (int p = threadIdx.x; p < a.p; p += kThreads) o_tab[p] = a.ac_p[(size_t)q * a.p + p] + (float)u0;
    for (int e = threadIdx.x; e < kRingSlots * PP; e += kThreads) sm.sp[e] = 0u;
    for (int e = threadIdx.x; e < 2 * 5 * QP; e += kThreads) (&sm.qb[0][0])[e] = 0.0f;
    const int x = threadIdx.x;                 // staged column index (local column x - 2)
    const int jj = x - 2;
    const bool stager = x < width + 4;
    const bool valid = jj >= 0 && jj < width;
    T* ws = (T*)a.ws;
    const size_t yrow = (size_t)a.squares[q].y_off_row * a.nv + (size_t)v * width;   // + m n W + j
    const size_t yplane = (size_t)a.nv * width;
    const int j = threadIdx.x;                                           // output column
    const int d = a.d;
    int pn = (a.p - (4 * d) % a.p) % a.p;      // p(0) = -4 d mod P
    __syncthreads();
    {
        SRow<CUBIC> rows[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            ring_fetch<STORE, CUBIC>(a, o_tab, v, pn, jj, valid, rows[u]);
            pn += d;
            if (pn >= a.p) pn -= a.p;
        }
        if (stager) {
#pragma unroll
            for (int u = 0; u < 9; ++u) ring_stage<PP, CUBIC>(sm.sp, u, x, rows[u]);
        }
        vmem_drain();
    }
    float y_cur = j < width ? S::load(ws, yrow + j) : 0.0f;
    __syncthreads();
    for (int m = 0; m < a.pd; ++m) {
        const bool more = m + 1 < a.pd;
        SRow<CUBIC> rows[4];
        float y_next = 0.0f;
        if (more) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ring_fetch<STORE, CUBIC>(a, o_tab, v, pn, jj, valid, rows[k]);
                pn += d;
                if (pn >= a.p) pn -= a.p;
            }
            if (j < width) y_next = S::load(ws, yrow + (size_t)(m + 1) * yplane + j);
        }
        const uint32_t* win = sm.sp + ((4 * m) & (kRing - 1)) * PP;
        float* qt = sm.qb[m & 1];
        // a fixed number of tile slots per wave (no inner loop: the prefetched
        // rows stay in flight across the products); PW / 16 tiles over four
        // waves, rounded up (PW = 224: 14 tiles, four slots per wave)
#pragma unroll
        for (int k = 0; k < (PW / 16 + 3) / 4; ++k) {
            const int tile = wave + 4 * k;
            if (tile < ntile) fwd_tile<PP, QP>(win, qt, tile * 16, width, op);
        }
        if (more && stager) {
#pragma unroll
            for (int k = 0; k < 4; ++k) ring_stage<PP, CUBIC>(sm.sp, (4 * m + 9 + k) & (kRing - 1), x, rows[k]);
        }
        vmem_drain();
        __syncthreads();
        if (j < width) {
            float r = b2;
#pragma unroll
            for (int bb = 0; bb < 5; ++bb) r += qt[bb * QP + j + bb];
            S::put(ws, yrow + (size_t)m * yplane + j, y_cur + r);
        }
        y_cur = y_next;
    }
}

// Backward (training): gradients of sum_{m,v,j} R[m][v][j] dY[m][v][j] with
// respect to the weights (dY = dL/dY in FP32, workspace layout), accumulated
// into grad.  A workgroup takes (square, row) tasks in the forward kernels'
// XCD-aware order with a grid stride, walks each task's decimated angles with
// the forward's staging and operands, and keeps its gradient partials in
// registers until all its tasks are done.
//
// conv1 runs in the transposed orientation, H[col][ch] = X[col][taps] x
// W1^T[taps][ch] (the forward's operands with their roles swapped), so a lane
// holds columns 4g .. 4g + 3 of channel lr.  That is the B-operand layout of a
// product over columns, so every reduction over positions is an MFMA:
//   dW2^T_a[b][ch] += G^T[b][col] x A_a[col][ch],   G[col][b] = dR[col - b + 2]
//   dA_a[col][ch]   = G[col][b] x W2_a^T[b][ch]      (b = 0..4, padded to 8)
//   dW1^T[tap][ch] += X^T[tap][col] x dH[col][ch]
// The first two take FP32 operands (16x16x4 products: A, the BF16-rounded
// activation, and dR, in FP32), the third BF16 ones (dH rounded, as S).
// db1 is a per-lane sum of dH, reduced over the lane groups at the end.
constexpr int kDrPad = 16;                          // dR row: column c at index c + 16
constexpr int kDrLen = kDrPad + 16 * ((kLearnedMaxWidth + 15) / 16) + 18;

struct BwdSmem {
    int off_tab[9];
    uint32_t sp[9 * kPP];
    float dr[kDrLen];
};

template <int STORE, bool CUBIC>
__global__ __launch_bounds__(kThreads) void k_learned_bwd(LearnedArgs a) {
    // the task state, and after the last task the waves' partial gradients
    __shared__ union {
        BwdSmem s;
        float red[4 * kLearnedParams];
    } smu;
    BwdSmem& sm = smu.s;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const FwdOperands op = load_fwd_operands<kPP>(a.w);
    const float b1l = bf2f(a.w[kOffB1 + lr]);             // bias of the lane's channel
    // B operands of dA: W2[ch = lr][a2][b = 4 t + g] (zero for b >= 5)
    float w2b[5][2];
#pragma unroll
    for (int a2 = 0; a2 < 5; ++a2)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int b = 4 * t + lg;
            w2b[a2][t] = b < 5 ? bf2f(a.w[kOffW2 + lr * 25 + a2 * 5 + b]) : 0.0f;
        }
    // the lane's dW1 rows: taps lr and lr + 16 (taps >= 25 read a valid
    // tile entry and give discarded rows)
    int xoff[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int tap = lr + 16 * mt;
        xoff[mt] = tap < 25 ? (tap / 5) * kPP + tap % 5 + 4 * lg : 4 * lg;
    }
    f4v gw1[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    f4v gw2[5];
#pragma unroll
    for (int a2 = 0; a2 < 5; ++a2) gw2[a2] = (f4v){0.0f, 0.0f, 0.0f, 0.0f};
    float gb1 = 0.0f, gb2 = 0.0f;

    const unsigned ntot = fwd_grid(a);
    for (unsigned task = blockIdx.x; task < ntot; task += gridDim.x) {
        const int x8 = (int)(task % kXcds), i8 = (int)(task / kXcds);
        const int q = i8 % a.nsq, v = (i8 / a.nsq) * kXcds + x8;
        if (v >= a.nv) continue;                           // uniform over the workgroup
        const int2 gd = a.grid[q];
        const int u0 = gd.x, width = gd.y;
        const int ntile = (width + 15) >> 4;
        __syncthreads();                                   // the previous task's reads are done
        const float* acq = a.ac_p + (size_t)q * a.p;   // crop offsets a_c(beta_p) + u0
        const float u0f = (float)u0;
        if (threadIdx.x < 9) {
            int off = ((int)threadIdx.x - 4) * a.d % a.p;
            sm.off_tab[threadIdx.x] = off < 0 ? off + a.p : off;
        }
        for (int e = threadIdx.x; e < 9 * kPP; e += kThreads) sm.sp[e] = 0u;
        for (int e = threadIdx.x; e < kDrLen; e += kThreads) sm.dr[e] = 0.0f;
        const int col = threadIdx.x;                        // staged column (local column col - 2)
        const int jj = col - 2;
        const bool stager = col < width + 4;
        const bool valid = jj >= 0 && jj < width;
        const size_t yrow = (size_t)a.squares[q].y_off_row * a.nv + (size_t)v * width;
        const size_t yplane = (size_t)a.nv * width;
        CentreWalk cw(a.p, a.pd);
        __syncthreads();
        int offr[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) offr[t] = __builtin_amdgcn_readfirstlane(sm.off_tab[t]);
        for (int m = 0; m < a.pd; ++m) {
            {
                SRow<CUBIC> rows[9];
                s_fetch_rows<STORE, CUBIC>(a, acq, u0f, v, cw.c, jj, valid, offr, rows);
                if (stager) s_stage_pairs(sm.sp, col, rows);
                cw.next();
            }
            if (col < width) {
                const float g = a.dws[yrow + (size_t)m * yplane + col];
                sm.dr[kDrPad + col] = g;
                gb2 += g;
            }
            __syncthreads();
            for (int tile = wave; tile < ntile; tile += kThreads / 64) {
                const int col0 = tile * 16;
                // dR operands of the tile (shared by the five angles):
                // G^T[b = lr][col0 + 4 g + j] and G[col0 + lr][b = 4 t + g]
                float gt[4], gc[2];
#pragma unroll
                for (int j = 0; j < 4; ++j) gt[j] = sm.dr[kDrPad + col0 + 4 * lg + j - lr + 2];
#pragma unroll
                for (int t = 0; t < 2; ++t) gc[t] = sm.dr[kDrPad + col0 + lr - (4 * t + lg) + 2];
                bool cin[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) cin[i] = col0 + 4 * lg + i < width;
                const uint32_t* ph = sm.sp + col0 + op.hoff;
                const uint32_t* pv = sm.sp + col0 + op.voff;
#pragma unroll
                for (int a2 = 0; a2 < 5; ++a2) {
                    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
                    const u4v d = {ph[a2 * kPP], ph[a2 * kPP + 2], pv[a2 * kPP], pv[a2 * kPP + kPP]};
                    const f4v b1v = {b1l, b1l, b1l, b1l};
                    // H[col0 + 4 g + i][ch = lr], bias included
                    const f4v h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, d), op.w1, b1v,
                                                                           0, 0, 0);
                    // A = ReLU(H) rounded to BF16 (the value conv2 multiplies), zero outside [0, W)
                    float av[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) av[i] = cin[i] ? bf2f(f2bf(fmaxf(h[i], 0.0f))) : 0.0f;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        gw2[a2] = __builtin_amdgcn_mfma_f32_16x16x4f32(gt[j], av[j], gw2[a2], 0, 0, 0);
                    f4v da = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        da = __builtin_amdgcn_mfma_f32_16x16x4f32(gc[t], w2b[a2][t], da, 0, 0, 0);
                    float dh[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        dh[i] = (cin[i] && h[i] > 0.0f) ? da[i] : 0.0f;
                        gb1 += dh[i];
                    }
                    // B operand of dW1: dH[col0 + 4 g + i][ch = lr] in BF16
                    const s4v dhop = {(short)f2bf(dh[0]), (short)f2bf(dh[1]), (short)f2bf(dh[2]),
                                      (short)f2bf(dh[3])};
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
                        // A operand: S of tap lr + 16 mt at columns col0 + 4 g .. + 3 (pair
                        // entries x and x + 2 hold staged columns x .. x + 3)
                        const int e = a2 * kPP + col0 + xoff[mt];
                        const uint32_t lo = sm.sp[e], hi = sm.sp[e + 2];
                        typedef uint32_t u2v __attribute__((ext_vector_type(2)));
                        const s4v xop = __builtin_bit_cast(s4v, (u2v){lo, hi});
                        gw1[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(xop, dhop, gw1[mt], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
    }
    // the wave's partials: dW1^T[tap = 4 g + i + 16 mt][ch = lr],
    // dW2^T[b = 4 g + i][ch = lr] per angle, db1 of channel lr, db2 -- each
    // parameter held by exactly one lane of the wave.  They are summed over
    // the four waves in a fixed order and written as the workgroup's partial
    // gradient; k_grad_sum adds the workgroups' partials in a fixed order, so
    // the gradient does not depend on scheduling.
    __syncthreads();                                       // the last task's reads of sm are done
    float* red = smu.red;                                  // [4][kLearnedParams]
    float* mine = red + wave * kLearnedParams;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tap = 16 * mt + 4 * lg + i;
            if (tap < 25) mine[kOffW1 + lr * 25 + tap] = gw1[mt][i];
        }
#pragma unroll
    for (int a2 = 0; a2 < 5; ++a2)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = 4 * lg + i;
            if (b < 5) mine[kOffW2 + lr * 25 + a2 * 5 + b] = gw2[a2][i];
        }
    gb1 += __shfl_xor(gb1, 16, 64);
    gb1 += __shfl_xor(gb1, 32, 64);
    if (lg == 0) mine[kOffB1 + lr] = gb1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) gb2 += __shfl_xor(gb2, off, 64);
    if (lane == 0) mine[kOffB2] = gb2;
    __syncthreads();
    for (int e = threadIdx.x; e < kLearnedParams; e += kThreads)
        a.partials[(size_t)blockIdx.x * kLearnedParams + e] =
            ((red[e] + red[kLearnedParams + e]) + red[2 * kLearnedParams + e]) + red[3 * kLearnedParams + e];
}

// grad[e] = sum over the backward pass's workgroups of their partials, in
// workgroup order.
__global__ __launch_bounds__(256) void k_grad_sum(const float* partials, int nblocks, float* grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kLearnedParams) return;
    float acc = 0.0f;
    for (int b = 0; b < nblocks; ++b) acc += partials[(size_t)b * kLearnedParams + e];
    grad[e] = acc;
}

// Transpose of the backprojection of decimated data (training): for every
// voxel and decimated angle, the residual is scattered with the bilinear
// weights and (pi / P') U^-2 into dY (workspace layout).  The sums are exact
// integer sums of the FP32 contributions rounded to multiples of 2^-e
// (fixed point in int64; e from a bound of the largest possible sum, so
// that no partial sum overflows), converted to FP32 at the end: the result
// does not depend on the order in which the atomics land.  One workgroup
// per 16 x 16 (x, y) tile of a square and slab of 32 slices (the
// backprojection's blocks).  Per angle, the block's contributions are summed
// in an LDS tile over its detector footprint, whose origin the block's
// corners bound (the column is linear-fractional in x and y, the row linear
// in z), and the tile is then added to dY with one int64 global atomic per
// non-zero entry.  A sample outside the tile (not expected) goes to dY
// directly, so the result does not depend on the bound.  The block's
// residuals sit in LDS, and in step k lane l takes slice (k + l) mod 32, so
// the lanes of one LDS atomic fall on different rows and columns of the tile
// (with one slice per step they would share a row and, several at a time, a
// column, and the atomics would serialize).  A thread sums each detector
// row of its column pair in registers and adds it once, about one row per
// slice instead of two.
constexpr int kAdjZR = 32, kAdjTW = 40, kAdjTH = 48;

// max |resid| over the voxels, as the bits of a non-negative float
__global__ __launch_bounds__(256) void k_adj_absmax(const float* resid, int64_t count, AdjScale* qs) {
    unsigned m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(resid[i]) & 0x7FFFFFFFu);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
    if ((threadIdx.x & 63) == 0 && m) atomicMax(&qs->rmax, m);
}

// clears the maximum and the sums' buffer (a fill kernel, no memset node)
__global__ void k_adj_clear(AdjScale* qs, unsigned long long* dq, int64_t count) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) qs->rmax = 0u;
    for (int64_t i = i0; i < count; i += (int64_t)gridDim.x * blockDim.x) dq[i] = 0ull;
}

// qscale = 2^e, the largest power of two with bound * max |resid| * qscale < 2^61
__global__ void k_adj_scale(AdjScale* qs, double bound) {
    const unsigned bits = qs->rmax;
    double q;
    if (bits >= 0x7F800000u) {
        q = 0.0;                                  // not finite: the result is NaN
    } else if (bits == 0u) {
        q = 1.0;                                  // all zero
    } else {
        int x;
        (void)frexp(bound * (double)__uint_as_float(bits), &x);   // the product < 2^x
        q = ldexp(1.0, 61 - x);
    }
    qs->qscale = q;
}

// dY = the int64 sums / qscale, rounded once to FP32
__global__ void k_adj_convert(const unsigned long long* dq, const AdjScale* qs, float* dws, int64_t count) {
    const double q = qs->qscale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dws[i] = q > 0.0 ? (float)((double)(long long)dq[i] / q) : __builtin_nanf("");
}

__global__ __launch_bounds__(256) void k_bp_adjoint(AdjArgs a) {
    __shared__ unsigned long long acc[kAdjTH * kAdjTW];
    __shared__ float rs[kAdjZR][256];          // residual of slice l0 + k, voxel threadIdx.x
    const int tile = (int)(blockIdx.x % (unsigned)a.ntiles), zt = (int)(blockIdx.x / (unsigned)a.ntiles);
    const BpTile tl = a.tiles[tile];
    const SquareDesc sq = a.squares[tl.sq];
    const int2 gd = a.grid[tl.sq];
    const int u0 = gd.x, width = gd.y;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int ix1 = min(tl.x0 + 15, sq.x1 - 1), iy1 = min(tl.y0 + 15, sq.y1 - 1);
    const int i = tl.x0 + tx, j = tl.y0 + ty;
    const bool own = i <= ix1 && j <= iy1;
    const int l0 = zt * kAdjZR, l1 = min(l0 + kAdjZR, a.nz) - 1;
    const float dx = (float)min(i, ix1) - a.cu - sq.xc, dy = (float)min(j, iy1) - a.cu - sq.yc;
    const float bx[2] = {(float)tl.x0 - a.cu - sq.xc, (float)ix1 - a.cu - sq.xc};
    const float by[2] = {(float)tl.y0 - a.cu - sq.yc, (float)iy1 - a.cu - sq.yc};
    const float z0 = (float)(a.zbase + l0) - a.cz, z1 = (float)(a.zbase + l1) - a.cz;
    // the block's residuals (slices l0 .. l0 + 31; zero outside the square or volume)
#pragma unroll 8
    for (int k = 0; k < kAdjZR; ++k) {
        const int l = l0 + k;
        rs[k][threadIdx.x] = own && l <= l1 ? a.resid[((size_t)l * a.n + j) * a.n + i] : 0.0f;
    }
    const int skew = threadIdx.x & 63;
    const double qscale = a.qs->qscale;
    // a contribution as an integer multiple of 1 / qscale (qscale is a power
    // of two: the product is exact, the conversion rounds to nearest)
    auto fixed = [&](float v) { return (unsigned long long)__double2ll_rn((double)v * qscale); };
    for (int m = 0; m < a.pd; ++m) {
        const float2 t = a.trig[m];
        const float dc = a.r + sq.xc * t.x + sq.yc * t.y;
        const float lc = sq.yc * t.x - sq.xc * t.y;
        const float rdc = 1.0f / dc;
        // footprint origin: the least column and row over the block's corners, less a margin
        float tlo = INFINITY, vlo = INFINITY;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float cx = bx[c & 1], cy = by[c >> 1];
            tlo = fminf(tlo, rel_column(cx, cy, t.x, t.y, a.r, dc, lc, rdc) + a.cu - (float)u0);
            const float iuc = a.r / (dc + cx * t.x + cy * t.y);
            vlo = fminf(vlo, fminf(z0 * iuc, z1 * iuc) + a.cv);
        }
        const int c0 = (int)floorf(tlo) - 1, r0 = (int)floorf(vlo) - 1;
        const size_t plane = (size_t)sq.y_off_row * a.nv + (size_t)m * a.nv * width;
        for (int e = threadIdx.x; e < kAdjTH * kAdjTW; e += 256) acc[e] = 0ull;
        __syncthreads();
        if (own) {
            const float tau = rel_column(dx, dy, t.x, t.y, a.r, dc, lc, rdc) + a.cu - (float)u0;
            const float d = dc + dx * t.x + dy * t.y;
            const float invu = a.r / d;
            const float wgt = a.scale * invu * invu;
            const float tf = floorf(tau), fu = tau - tf;
            const int iu = min(max((int)tf, 0), width - 2);
            const int cl = iu - c0;
            const bool cin = cl >= 0 && cl + 1 < kAdjTW;
            // one detector row's sum (columns iu and iu + 1 by the fixed split
            // 1 - fu, fu) into the tile, or into dY when outside it; rows
            // outside the detector are dropped
            auto flush_row = [&](int row, float val) {
                if (val == 0.0f || (unsigned)(row - a.v0) >= (unsigned)a.nv) return;
                const int rl = row - r0;
                const unsigned long long q0 = fixed(val * (1.0f - fu)), q1 = fixed(val * fu);
                if (cin && rl >= 0 && rl < kAdjTH) {
                    atomicAdd(&acc[rl * kAdjTW + cl], q0);
                    atomicAdd(&acc[rl * kAdjTW + cl + 1], q1);
                } else {
                    unsigned long long* p = a.dq + plane + (size_t)(row - a.v0) * width + iu;
                    atomicAdd(p, q0);
                    atomicAdd(p + 1, q1);
                }
            };
            // the slices in order (from the lane's skew, wrapping once) move
            // the row down monotonically: rows rc and rc + 1 are summed in
            // registers and written once the slices have passed them
            int rc = INT_MIN / 2;
            float s0 = 0.0f, s1 = 0.0f;
            for (int k = 0; k < kAdjZR; ++k) {
                const int sl = (k + skew) & (kAdjZR - 1);
                if (sl == 0 && k > 0) {              // the wrap back to slice 0
                    flush_row(rc, s0);
                    flush_row(rc + 1, s1);
                    s0 = s1 = 0.0f;
                    rc = INT_MIN / 2;
                }
                const float rv = rs[sl][threadIdx.x];
                if (rv == 0.0f) continue;
                const float vv = fmaf((float)(a.zbase + l0 + sl) - a.cz, invu, a.cv);
                const float vf = floorf(vv), fv = vv - vf;
                const int iv = (int)vf;
                if (iv != rc) {
                    flush_row(rc, s0);
                    if (iv == rc + 1) {
                        s0 = s1;
                    } else {
                        flush_row(rc + 1, s1);
                        s0 = 0.0f;
                    }
                    s1 = 0.0f;
                    rc = iv;
                }
                const float w = wgt * rv;
                s0 = fmaf(w, 1.0f - fv, s0);
                s1 = fmaf(w, fv, s1);
            }
            flush_row(rc, s0);
            flush_row(rc + 1, s1);
        }
        __syncthreads();
        // non-zero entries lie at rows in [v0, v0 + nv) and columns in
        // [0, W): only such samples were added
        for (int e = threadIdx.x; e < kAdjTH * kAdjTW; e += 256) {
            const unsigned long long val = acc[e];
            if (val != 0ull)
                atomicAdd(&a.dq[plane + (size_t)(r0 - a.v0 + e / kAdjTW) * width + (c0 + e % kAdjTW)], val);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_residual(const float* f, const float* ref, float* r, double* loss,
                                                   int64_t count, float weight) {
    __shared__ double part[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float dlt = f[i] - ref[i];
        r[i] = (2.0f * weight) * dlt;
        acc += (double)dlt * (double)dlt;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (double)weight * (part[0] + part[1] + part[2] + part[3]));
}

__global__ void k_fill_d(double* p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// AdamW on the FP32 master weights; writes their BF16 copy.
__global__ void k_adamw(AdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const float g = a.grad[i];
    float m1 = a.m1[i] = a.beta1 * a.m1[i] + (1.0f - a.beta1) * g;
    float m2 = a.m2[i] = a.beta2 * a.m2[i] + (1.0f - a.beta2) * g * g;
    const float mh = m1 / (1.0f - powf(a.beta1, (float)a.step));
    const float vh = m2 / (1.0f - powf(a.beta2, (float)a.step));
    float w = a.master[i];
    w -= a.lr * (mh / (sqrtf(vh) + a.eps) + a.weight_decay * w);
    a.master[i] = w;
    a.w_bf16[i] = (uint16_t)f2bf(w);
}

template <int STORE, bool CUBIC>
void launch_fwd_ring(const LearnedArgs& a, int max_width, hipStream_t st) {
    const size_t dyn = sizeof(float) * (size_t)a.p;
    if (max_width <= 128)
        hipLaunchKernelGGL((k_learned_fwd_ring<STORE, 128, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), dyn, st, a);
    else if (max_width <= 224)
        hipLaunchKernelGGL((k_learned_fwd_ring<STORE, 224, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), dyn, st, a);
    else
        hipLaunchKernelGGL((k_learned_fwd_ring<STORE, 256, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), dyn, st, a);
}

template <bool CUBIC>
void launch_fwd_store(const LearnedArgs& a, int max_width, bool ring, int store, hipStream_t st) {
    if (ring) {
        switch (store) {
            case 0: launch_fwd_ring<0, CUBIC>(a, max_width, st); break;
            case 1: launch_fwd_ring<1, CUBIC>(a, max_width, st); break;
            default: launch_fwd_ring<2, CUBIC>(a, max_width, st); break;
        }
        return;
    }
    switch (store) {
        case 0: hipLaunchKernelGGL((k_learned_fwd<0, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_learned_fwd<1, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), 0, st, a); break;
        default: hipLaunchKernelGGL((k_learned_fwd<2, CUBIC>), dim3(fwd_grid(a)), dim3(kThreads), 0, st, a); break;
    }
}

hipError_t launch_learned_fwd(const LearnedArgs& a, int max_width, int dfac, int store, hipStream_t st) {
    if (max_width > kLearnedMaxWidth) return hipErrorInvalidValue;
    const bool ring = dfac >= 4 && a.p % dfac == 0 && a.pd * dfac == a.p && a.d * 4 == dfac && a.p <= kRingMaxP;
    if (a.cubic) launch_fwd_store<true>(a, max_width, ring, store, st);
    else launch_fwd_store<false>(a, max_width, ring, store, st);
    return hipGetLastError();
}

// Workgroups of the backward pass: a grid stride over the tasks, a multiple of
// the XCD count (so a workgroup's tasks stay on its XCD's rows), about four
// per compute unit.
constexpr unsigned kBwdGrid = kLearnedBwdGrid;

hipError_t launch_learned_bwd(const LearnedArgs& a, int store, hipStream_t st) {
    if (!a.partials) return hipErrorInvalidValue;
    const unsigned ntot = fwd_grid(a);
    const dim3 grid(ntot < kBwdGrid ? ntot : kBwdGrid);
    switch (store) {
        case 0:
            if (a.cubic) hipLaunchKernelGGL((k_learned_bwd<0, true>), grid, dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((k_learned_bwd<0, false>), grid, dim3(kThreads), 0, st, a);
            break;
        case 1:
            if (a.cubic) hipLaunchKernelGGL((k_learned_bwd<1, true>), grid, dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((k_learned_bwd<1, false>), grid, dim3(kThreads), 0, st, a);
            break;
        default:
            if (a.cubic) hipLaunchKernelGGL((k_learned_bwd<2, true>), grid, dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((k_learned_bwd<2, false>), grid, dim3(kThreads), 0, st, a);
            break;
    }
    hipLaunchKernelGGL(k_grad_sum, dim3((kLearnedParams + 255) / 256), dim3(256), 0, st, a.partials,
                       (int)grid.x, a.grad);
    return hipGetLastError();
}

hipError_t launch_bp_adjoint(const AdjArgs& a, hipStream_t st) {
    const int64_t nblk = (int64_t)a.ntiles * ((a.nz + kAdjZR - 1) / kAdjZR);
    if (nblk <= 0 || nblk > (int64_t)1 << 31) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_clear, dim3(1024), dim3(256), 0, st, a.qs, a.dq, a.ws_elems);
    hipLaunchKernelGGL(k_adj_absmax, dim3(1024), dim3(256), 0, st, a.resid, a.nvox, a.qs);
    hipLaunchKernelGGL(k_adj_scale, dim3(1), dim3(1), 0, st, a.qs, a.bound);
    hipLaunchKernelGGL(k_bp_adjoint, dim3((unsigned)nblk), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_convert, dim3(1024), dim3(256), 0, st, (const unsigned long long*)a.dq,
                       (const AdjScale*)a.qs, a.dws, a.ws_elems);
    return hipGetLastError();
}

hipError_t launch_residual(const float* f, const float* ref, float* r, double* loss, int64_t count, float weight,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_fill_d, dim3(1), dim3(64), 0, st, loss, (int64_t)1);
    hipLaunchKernelGGL(k_residual, dim3(1024), dim3(256), 0, st, f, ref, r, loss, count, weight);
    return hipGetLastError();
}

hipError_t launch_adamw(const AdamArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_adamw, dim3((a.count + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace fdkod
