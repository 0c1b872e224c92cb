// HIP kernels of the split-explicit step for gfx950.
//
// Column kernels (3D): one 64-lane wavefront owns one vertical column of a
// cell, an edge or a vertex; lane k holds layer k (layers >= 64 live in a
// second register chunk).  Mesh indices are therefore wave-uniform (scalar
// loads) and every neighbour access is one contiguous column read; vertical
// sums and scans are cross-lane operations inside the wavefront.  Lanes past
// the last layer load a copy of the last layer; what they hold is zeroed
// before it reaches a sum or a scan over the layers.
//
// 2D kernels (barotropic loop, reconciliation): one thread per edge or cell,
// reading slot-major neighbour tables.
//
// R is double (FP64 mode) or float (mixed mode); the split between the two
// types is described in sse_kernels.h.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sse_kernels.h"

namespace sse {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8) and every XCD has its own L2.  Launches use 8 * ceil(nb / 8)
// blocks and renumber them so that XCD x processes the contiguous logical
// range [x * per, (x + 1) * per): neighbouring columns then share one L2.
// Returns -1 for the padding blocks.
__device__ __forceinline__ int xcd_block(int nb) {
    const int per = (nb + kXcd - 1) / kXcd;
    const int b = blockIdx.x;
    const int logical = (b % kXcd) * per + b / kXcd;
    return logical < nb ? logical : -1;
}

// Index of the column owned by this wavefront among n columns (n: none); a
// workgroup of w wavefronts owns w consecutive columns.
// readfirstlane tells the compiler the value is wave-uniform, so mesh-table
// reads that depend on it become scalar loads instead of 64 identical vector
// loads.
__device__ __forceinline__ int column_id(int n) {
    const int cpb = blockDim.x >> 6;
    const int lb = xcd_block((n + cpb - 1) / cpb);
    const int col = lb * cpb + (threadIdx.x >> 6);
    return __builtin_amdgcn_readfirstlane(lb < 0 ? n : col);
}

// ---------------------------------------------------------------------------
// Cross-lane operations of a column; every caller runs them with all 64
// lanes active.  Two forms, chosen by the kernel (kDpp):
//  * DPP: values move inside rows of 16 lanes, and by one lane across the
//    wavefront, as DPP operands, with no LDS round trip and no wait.  An FP32
//    step is one instruction (the move folds into the addition); an FP64
//    step takes two moves besides the addition.
//  * shuffles: lane permutes through the LDS crossbar, fewer VALU
//    instructions for FP64 values.
// The kernels of both precisions use DPP for every value type (the FP64
// edge pass, once its column loads took 32-bit scalar offsets, had the
// registers for it and became 3.7% faster than with shuffles; the assembly
// pass, 11%).  The butterfly steps that cross rows (i ^ 32, i ^ 16) are
// shuffles in both forms, and the butterfly keeps its pairwise order, so a
// column sum has the same bits in both.
// ---------------------------------------------------------------------------
template <typename R>
constexpr bool kDppFor = true;

constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowShl = 0x100;       // + n: lane j of a row reads lane j + n of the row
constexpr int kDppRowShr = 0x110;       // + n: lane j of a row reads lane j - n of the row
constexpr int kDppRowRor = 0x120;       // + n: rotation within a row
constexpr int kDppWaveShl1 = 0x130;     // lane i reads lane i + 1
constexpr int kDppWaveShr1 = 0x138;     // lane i reads lane i - 1
constexpr int kDppRowBcast15 = 0x142;   // lane 15 of a row to the lanes of the next row
constexpr int kDppRowBcast31 = 0x143;   // lane 31 to the lanes of rows 2 and 3

// Lane i receives x from the lane the control names; lanes without a source
// lane, and rows outside kRowMask, receive `old`.
template <int kCtrl, int kRowMask = 0xF, typename T>
__device__ __forceinline__ T dpp(T old, T x) {
    return __builtin_amdgcn_update_dpp(old, x, kCtrl, kRowMask, 0xF, false);
}

// The same with zero for lanes without a source lane (bound control), every
// row written: no register has to be cleared first, which matters for FP64
// values, whose moves cannot fold into the addition that consumes them.
template <int kCtrl, typename T>
__device__ __forceinline__ T dpp_z(T x) {
    return __builtin_amdgcn_update_dpp(T(0), x, kCtrl, 0xF, 0xF, true);
}

// x of lane l, as a wave-uniform value
template <typename T>
__device__ __forceinline__ T lane_value(T x, int l) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, l);
        const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
    }
}

// Sum over the 64 lanes as a butterfly: every lane adds the value of lane
// i ^ 32, then i ^ 16, i ^ 8, i ^ 4, i ^ 2, i ^ 1; the result is the pairwise
// halving sum, the same bits in both forms.  (DPP: after the i ^ 8 step the
// values repeat with period 8 inside a row, so the rotation by 4 hands every
// lane the value of lane i ^ 4.)
template <bool kDpp, typename T>
__device__ __forceinline__ T wave_sum(T x) {
    if constexpr (!kDpp) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
        return __shfl(x, 0, kWave);  // one value for the whole column
    } else {
        x += __shfl_xor(x, 32, kWave);
        x += __shfl_xor(x, 16, kWave);
        x += dpp_z<kDppRowRor + 8>(x);
        x += dpp_z<kDppRowRor + 4>(x);
        x += dpp_z<kDppQuadXor2>(x);
        x += dpp_z<kDppQuadXor1>(x);
        return lane_value(x, 0);
    }
}

// Inclusive scan over the lanes.  DPP: steps of 1, 2, 4, 8 inside each row,
// then the row totals carried into the rows after them.
template <bool kDpp, typename T>
__device__ __forceinline__ T wave_incl_prefix(T x) {
    if constexpr (!kDpp) {
        const int l = lane_id();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const T y = __shfl_up(x, d, kWave);
            if (l >= d) x += y;
        }
    } else {
        x += dpp_z<kDppRowShr + 1>(x);
        x += dpp_z<kDppRowShr + 2>(x);
        x += dpp_z<kDppRowShr + 4>(x);
        x += dpp_z<kDppRowShr + 8>(x);
        x += dpp<kDppRowBcast15, 0xA>(T(0), x);
        x += dpp<kDppRowBcast31, 0xC>(T(0), x);
    }
    return x;
}

// Inclusive suffix scan.  DPP: steps of 1, 2, 4, 8 inside each row, after
// which lane 16 r holds the total t_r of row r; row 0 then adds
// t1 + (t2 + t3), row 1 t2 + t3, row 2 t3.
template <bool kDpp, typename T>
__device__ __forceinline__ T wave_incl_suffix(T x) {
    if constexpr (!kDpp) {
        const int l = lane_id();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const T y = __shfl_down(x, d, kWave);
            if (l + d < kWave) x += y;
        }
        return x;
    } else {
        x += dpp_z<kDppRowShl + 1>(x);
        x += dpp_z<kDppRowShl + 2>(x);
        x += dpp_z<kDppRowShl + 4>(x);
        x += dpp_z<kDppRowShl + 8>(x);
        const T t3 = lane_value(x, 48);
        const T t23 = lane_value(x, 32) + t3;
        const T t123 = lane_value(x, 16) + t23;
        const int row = lane_id() >> 4;
        const T add = row == 0 ? t123 : row == 1 ? t23 : row == 2 ? t3 : T(0);
        return x + add;
    }
}

// v of lane i - 1 (lane 0: fill) and of lane i + 1 (lane 63: fill)
template <bool kDpp, typename T>
__device__ __forceinline__ T lane_prev(T fill, T v) {
    if constexpr (!kDpp) {
        const T y = __shfl_up(v, 1, kWave);
        return lane_id() == 0 ? fill : y;
    } else {
        return dpp<kDppWaveShr1>(fill, v);
    }
}
template <bool kDpp, typename T>
__device__ __forceinline__ T lane_next(T fill, T v) {
    if constexpr (!kDpp) {
        const T y = __shfl_down(v, 1, kWave);
        return lane_id() == kWave - 1 ? fill : y;
    } else {
        return dpp<kDppWaveShl1>(fill, v);
    }
}

// Sum over the layers: per-lane chunks first, then the butterfly; the result
// is the pairwise (halving) sum over the layers padded to 128.
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ T col_sum(const T (&v)[NK]) {
    T s = v[0];
#pragma unroll
    for (int c = 1; c < NK; ++c) s += v[c];
    return wave_sum<kDpp>(s);
}

// o_k = sum_{l<k} v_l
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ void col_excl_prefix(const T (&v)[NK], T (&o)[NK]) {
    T carry = T(0);
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const T inc = wave_incl_prefix<kDpp>(v[c]);
        o[c] = (kDpp ? dpp_z<kDppWaveShr1>(inc) : lane_prev<false>(T(0), inc)) + carry;
        if (c + 1 < NK) carry += __shfl(inc, kWave - 1, kWave);
    }
}

// o_k = sum_{l>k} v_l
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ void col_excl_suffix(const T (&v)[NK], T (&o)[NK]) {
    T carry = T(0);
#pragma unroll
    for (int c = NK - 1; c >= 0; --c) {
        const T inc = wave_incl_suffix<kDpp>(v[c]);
        o[c] = (kDpp ? dpp_z<kDppWaveShl1>(inc) : lane_next<false>(T(0), inc)) + carry;
        if (c > 0) carry += __shfl(inc, 0, kWave);
    }
}

// o_k = sum_{l>=k} v_l
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ void col_incl_suffix(const T (&v)[NK], T (&o)[NK]) {
    T carry = T(0);
#pragma unroll
    for (int c = NK - 1; c >= 0; --c) {
        const T inc = wave_incl_suffix<kDpp>(v[c]);
        o[c] = inc + carry;
        if (c > 0) carry += __shfl(inc, 0, kWave);
    }
}

// o_k = v_{k-1}, o_0 = 0
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ void col_up1(const T (&v)[NK], T (&o)[NK]) {
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const T prev_last = (c > 0) ? __shfl(v[c > 0 ? c - 1 : 0], kWave - 1, kWave) : T(0);
        o[c] = (kDpp && c == 0) ? dpp_z<kDppWaveShr1>(v[c]) : lane_prev<kDpp>(prev_last, v[c]);
    }
}

// o_k = v_{k+1}; zero past the last layer (lanes past L hold zeros)
template <int NK, bool kDpp = false, typename T>
__device__ __forceinline__ void col_down1(const T (&v)[NK], T (&o)[NK]) {
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const T next_first = (c < NK - 1) ? __shfl(v[c < NK - 1 ? c + 1 : c], 0, kWave) : T(0);
        o[c] = (kDpp && c == NK - 1) ? dpp_z<kDppWaveShl1>(v[c]) : lane_next<kDpp>(next_first, v[c]);
    }
}

// o_k = v_{k-s} (fill where k < s), 1 <= s <= 64, k = lane + 64 c
template <int NK, typename T>
__device__ __forceinline__ void col_shift_up(const T (&v)[NK], int s, T fill, T (&o)[NK]) {
    const int l = lane_id();
    if (s >= kWave) {
#pragma unroll
        for (int c = 0; c < NK; ++c) o[c] = c > 0 ? v[c > 0 ? c - 1 : 0] : fill;
        return;
    }
    const int src = (l - s) & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const T a = __shfl(v[c], src, kWave);
        const T b = c > 0 ? __shfl(v[c > 0 ? c - 1 : 0], src, kWave) : fill;
        o[c] = l >= s ? a : b;
    }
}

// o_k = v_{k+s} (fill past the last register chunk), 1 <= s <= 64
template <int NK, typename T>
__device__ __forceinline__ void col_shift_down(const T (&v)[NK], int s, T fill, T (&o)[NK]) {
    const int l = lane_id();
    if (s >= kWave) {
#pragma unroll
        for (int c = 0; c < NK; ++c) o[c] = c < NK - 1 ? v[c < NK - 1 ? c + 1 : c] : fill;
        return;
    }
    const int src = (l + s) & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const T a = __shfl(v[c], src, kWave);
        const T b = c < NK - 1 ? __shfl(v[c < NK - 1 ? c + 1 : c], src, kWave) : fill;
        o[c] = l + s < kWave ? a : b;
    }
}

// Solves lo_k x_{k-1} + di_k x_k + up_k x_{k+1} = d_k over the layers of a
// column, x returned in d.  Rows past the last layer must be the identity
// (lo = up = 0, di = 1, d = 0) and the first and last rows must not couple
// outwards (lo_0 = up_{L-1} = 0).  Parallel cyclic reduction (Hockney): in
// round r every row eliminates its couplings to the rows s = 2^r above and
// below with those rows' equations, so after ceil(log2 L) rounds each row
// holds one unknown.  Every lane works in every round, the cross-lane reads
// are register shuffles, and for the diagonally dominant systems of implicit
// diffusion no pivoting is needed.
template <int NK, typename T>
__device__ __forceinline__ void col_tridiag_solve(int L, T (&lo)[NK], T (&di)[NK], T (&up)[NK], T (&d)[NK]) {
    for (int s = 1; s < L; s <<= 1) {
        T rdi[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) rdi[c] = T(1) / di[c];
        T loA[NK], upA[NK], dA[NK], rA[NK], loB[NK], upB[NK], dB[NK], rB[NK];
        col_shift_up<NK>(lo, s, T(0), loA);
        col_shift_up<NK>(up, s, T(0), upA);
        col_shift_up<NK>(d, s, T(0), dA);
        col_shift_up<NK>(rdi, s, T(1), rA);
        col_shift_down<NK>(lo, s, T(0), loB);
        col_shift_down<NK>(up, s, T(0), upB);
        col_shift_down<NK>(d, s, T(0), dB);
        col_shift_down<NK>(rdi, s, T(1), rB);
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const T al = -lo[c] * rA[c];
            const T ga = -up[c] * rB[c];
            di[c] = di[c] + al * upA[c] + ga * loB[c];
            d[c] = d[c] + al * dA[c] + ga * dB[c];
            lo[c] = al * loA[c];
            up[c] = ga * upB[c];
        }
    }
#pragma unroll
    for (int c = 0; c < NK; ++c) d[c] = d[c] / di[c];
}

// a b + c rounded once
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Quotients by 3 and 6 in the bits of x / d but without the division
// sequence (about ten instructions).  With r = RN(1/d), q = RN(x r) and the
// residual x - q d (exact in one fused multiply-add), Markstein's theorem
// makes RN(q + (x - q d) r) the correctly rounded quotient whenever q lies
// within one ulp of x / d, which holds when |1 - d r| <= 2^-(p+1) for
// precision p: 1 - 3 RN(1/3) is 2^-54 in FP64 and 2^-25 in FP32 (and RN(1/6)
// is RN(1/3) / 2).  Valid while the quotient and the residual stay normal
// (|x / d| above about 2^-960 in FP64, 2^-100 in FP32); x = -0 gives +0.
// (Divisions by the run's dt and rho0 done this way, with host reciprocals,
// made the edge pass slower, so those stay divisions.)
template <typename T>
__device__ __forceinline__ T div_by_near(T x, T d, T r) {
    const T q = x * r;
    return fmadd(fmadd(-q, d, x), r, q);
}

// The 3/4 combination is one fused multiply-add with an explicit operand
// order (1/4 x is exact), so every kernel that forms it rounds alike.
template <typename T>
__device__ __forceinline__ T combine(int mode, T b, T x) {
    switch (mode) {
        case COMB_34: return fmadd(T(0.75), b, T(0.25) * x);
        case COMB_THIRD: return div_by_near(b, T(3), T(1) / T(3)) + div_by_near(T(2) * x, T(3), T(1) / T(3));
        case COMB_HALF: return T(0.5) * (b + x);
        default: return x;
    }
}

// Lane k holds layer k (chunk c: layer k + 64 c).  Lanes past the last layer
// load layer L - 1 (always in bounds), so loads are never predicated: no
// branches split the load stream and all loads of a stencil can be in flight
// together.  What those lanes loaded is zeroed where it can reach a sum or a
// scan over the layers; elsewhere it only feeds results that are not stored.
template <int NK>
__device__ __forceinline__ void lane_layers(int L, int (&kk)[NK], bool (&ok)[NK]) {
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        ok[c] = k < L;
        kk[c] = ok[c] ? k : L - 1;
    }
}

// Column access.  `col` is the first layer of a column and must be
// wave-uniform; the lane reads or writes layer k.  The address is a scalar
// base plus a 32-bit lane offset, a form the load and store instructions take
// directly, so the columns of a stencil share one offset register and need no
// 64-bit address arithmetic per lane (where scalar registers run short, the
// compiler still forms some of the addresses in vector registers).  Measured
// on the C1 edge pass: 6% faster than per-lane 64-bit addresses.
typedef __attribute__((address_space(1))) char global_char;

template <typename T>
__device__ __forceinline__ global_char *uniform_global(const T *col) {
    const unsigned long long p = reinterpret_cast<unsigned long long>(col);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)p);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(p >> 32));
    return (global_char *)(((unsigned long long)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T col_ld(const T *col, int k) {
    return *(const __attribute__((address_space(1))) T *)(uniform_global(col) + (unsigned)k * (unsigned)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void col_st(T *col, int k, T v) {
    *(__attribute__((address_space(1))) T *)(uniform_global(col) + (unsigned)k * (unsigned)sizeof(T)) = v;
}

// Layer k of the column that starts off elements into arr.  kWide: a 64-bit
// scalar base per column (col_ld).  Otherwise (arrays below 4 GiB) through
// one buffer descriptor of the whole array, with the column's byte offset in
// a single 32-bit scalar register and the layer's in the lane's: half the
// scalar registers per column and no 64-bit address arithmetic, which keeps
// the edge pass, with its ~30 columns, from spilling scalar registers.
template <bool kWide, typename T>
__device__ __forceinline__ T col_ldv(const T *arr, size_t off, int k) {
    if constexpr (kWide) {
        return col_ld(arr + off, k);
    } else {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc((void *)uniform_global(arr), (short)0, -1, 0x00020000);
        const unsigned so = __builtin_amdgcn_readfirstlane((unsigned)(off * sizeof(T)));
        if constexpr (sizeof(T) == 8)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)k * 8u, so, 0));
        else
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)k * 4u, so, 0));
    }
}

// ---------------------------------------------------------------------------
// Baroclinic forward Euler (Algorithm 1): cell pass.
// kAdd: the velocity is X + ubar_add (ubar_add non-null), else X itself.
// ---------------------------------------------------------------------------
template <int NK, typename R, bool kAdd>
__device__ __forceinline__ void fe_cell_body(const FECellArgs<R> &a, int col) {
    const DevMesh &m = a.m;
    const int i = col;
    if (i >= m.C) return;
    const int L = a.L;
    const size_t base = (size_t)i * L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    if (!m.cmask[i]) {
#pragma unroll
        for (int c = 0; c < NK; ++c)
            if (ok[c]) {
                a.B[base + kk[c]] = R(0);
                a.Wtop[base + kk[c]] = R(0);
                if (a.D1) a.D1[base + kk[c]] = R(0);
            }
        if (lane_id() == 0) a.Kbot[i] = 0.0;
        return;
    }
    double hi[NK];
    R divhu[NK], divu[NK], K[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        hi[c] = col_ld(a.h + base, kk[c]);
        divhu[c] = divu[c] = K[c] = R(0);
    }
    // Padded slots hold a valid index with zero coefficients, so the stencil
    // is unrolled to its full width.
#pragma unroll
    for (int j = 0; j < kMaxEdges; ++j) {
        const int e = m.cell_edges[i * kMaxEdges + j];
        const int nb = m.cell_nbrs[i * kMaxEdges + j];
        const R cd = (R)m.cell_div[i * kMaxEdges + j];
        const R ck = (R)m.cell_ke[i * kMaxEdges + j];
        const R add = kAdd ? (R)a.ubar_add[e] : R(0);
        const size_t eb = (size_t)e * L, nbb = (size_t)nb * L;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const R x = col_ld(a.X + eb, kk[c]);
            const double hn = col_ld(a.h + nbb, kk[c]);
            const R u = ok[c] ? x + add : R(0);
            const R he = (R)(0.5 * (hi[c] + hn));
            divhu[c] += cd * (he * u);
            divu[c] += cd * u;
            K[c] += ck * (u * u);
        }
    }
    R w[NK];
    if (a.frac) {
        // z-star: T^h_k = -frac_k sum_l div(h u)_l, and w_k - w_{k+1} = -div_k - T^h_k
        const R tot = col_sum<NK, kDppFor<R>>(divhu);
        R src[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const R th = -(R)col_ld(a.frac + base, kk[c]) * tot;
            src[c] = ok[c] ? (-divhu[c] - th) : R(0);
        }
        col_incl_suffix<NK, kDppFor<R>>(src, w);
    } else {
#pragma unroll
        for (int c = 0; c < NK; ++c) w[c] = R(0);
    }
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        if (ok[c]) {
            col_st(a.B + base, kk[c], K[c] - (R)a.nu_h * divu[c]);
            if (a.D1) col_st(a.D1 + base, kk[c], divu[c]);
            col_st(a.Wtop + base, kk[c], w[c]);
            if (kk[c] == L - 1) a.Kbot[i] = (double)K[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Baroclinic forward Euler: vertex pass (relative vorticity of X + ubar_add)
// ---------------------------------------------------------------------------
template <int NK, typename R, bool kAdd, int Q>
__device__ __forceinline__ void fe_vertex_body(const FEVertexArgs<R> &a, int first) {
    const DevMesh &m = a.m;
    if (first >= m.V) return;
    const int L = a.L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    int vi[Q];
    bool has[Q];
    R x[Q][3][NK], cr[Q][3], add[Q][3];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        has[q] = first + q < m.V;
        vi[q] = has[q] ? first + q : first;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int e = m.vert_edges[vi[q] * 3 + j];
            cr[q][j] = (R)m.vert_curl[vi[q] * 3 + j];
            add[q][j] = kAdd ? (R)a.ubar_add[e] : R(0);
            const size_t eb = (size_t)e * L;
#pragma unroll
            for (int c = 0; c < NK; ++c) x[q][j][c] = col_ld(a.X + eb, kk[c]);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!has[q]) continue;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            R z = R(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) z += cr[q][j] * (x[q][j][c] + add[q][j]);
            if (ok[c]) col_st(a.Z + (size_t)vi[q] * L, kk[c], z);
        }
    }
}

// ---------------------------------------------------------------------------
// Biharmonic viscosity: the vector Laplacian of u at edges, then the
// divergence of that field at cells (its curl at vertices is the vertex pass
// applied to it).
// ---------------------------------------------------------------------------
template <int NK, typename R, int Q>
__device__ __forceinline__ void lap_body(const LapArgs<R> &a, int first) {
    const DevMesh &m = a.m;
    if (first >= m.E) return;
    const int L = a.L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    int ei[Q];
    bool has[Q];
    R d1[Q][NK], d2[Q][NK], z1[Q][NK], z2[Q][NK];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        has[q] = first + q < m.E;
        const int e = ei[q] = has[q] ? first + q : first;
        const size_t b1 = (size_t)m.edge_cells[2 * e] * L, b2 = (size_t)m.edge_cells[2 * e + 1] * L;
        const size_t w1 = (size_t)m.edge_verts[2 * e] * L, w2 = (size_t)m.edge_verts[2 * e + 1] * L;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            d1[q][c] = col_ld(a.D + b1, kk[c]);
            d2[q][c] = col_ld(a.D + b2, kk[c]);
            z1[q][c] = col_ld(a.Z + w1, kk[c]);
            z2[q][c] = col_ld(a.Z + w2, kk[c]);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!has[q]) continue;
        const int e = ei[q];
        const bool wet = m.emask[e] != 0;
        const R idc = (R)m.inv_dc[e], idv = (R)m.inv_dv[e];
#pragma unroll
        for (int c = 0; c < NK; ++c)
            if (ok[c])
                col_st(a.out + (size_t)e * L, kk[c],
                       wet ? (d2[q][c] - d1[q][c]) * idc - (z2[q][c] - z1[q][c]) * idv : R(0));
    }
}

template <int NK, typename R, int Q>
__device__ __forceinline__ void div_body(const DivArgs<R> &a, int first) {
    const DevMesh &m = a.m;
    if (first >= m.C) return;
    const int L = a.L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    int ci[Q];
    bool has[Q];
    R x[Q][kMaxEdges][NK], cd[Q][kMaxEdges];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        has[q] = first + q < m.C;
        const int i = ci[q] = has[q] ? first + q : first;
#pragma unroll
        for (int j = 0; j < kMaxEdges; ++j) {
            const size_t eb = (size_t)m.cell_edges[i * kMaxEdges + j] * L;
            cd[q][j] = (R)m.cell_div[i * kMaxEdges + j];
#pragma unroll
            for (int c = 0; c < NK; ++c) x[q][j][c] = col_ld(a.X + eb, kk[c]);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!has[q]) continue;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            R d = R(0);
#pragma unroll
            for (int j = 0; j < kMaxEdges; ++j) d += cd[q][j] * x[q][j][c];
            if (ok[c]) col_st(a.out + (size_t)ci[q] * L, kk[c], d);
        }
    }
}

// ---------------------------------------------------------------------------
// Baroclinic forward Euler: edge pass (Algorithm 1 and the stage combination)
//
// The direct-gather and the LDS-staged kernels share everything after the
// operand loads: fe_edge_finish receives the column values of the edge, its
// cells and vertices and the accumulated reconstruction sums.
// ---------------------------------------------------------------------------
// TRiSK weight pairs (W / 4, W (f_e + f_j) / 2) of the edge pass in its real type.
template <typename R>
__device__ __forceinline__ const R *wpair_of(const DevMesh &m);
template <>
__device__ __forceinline__ const double *wpair_of<double>(const DevMesh &m) { return m.wpair; }
template <>
__device__ __forceinline__ const float *wpair_of<float>(const DevMesh &m) { return m.wpair_f; }

// The barotropic velocity at edge e as the pass computes with it: FP64 as
// stored, or (FP32 pass) the copy rounded to FP32 once per pass.
template <typename R>
__device__ __forceinline__ R ubar_at(const FEEdgeArgs<R> &a, const double *ubar, int e) {
    if constexpr (sizeof(R) == 4) return a.ubar_r[e];
    else return ubar[e];
}

template <int NK, typename R>
struct EdgeOperands {
    R u[NK], ut[NK], za[NK], zb[NK], B1[NK], B2[NK], W1[NK], W2[NK];
    double h1[NK], h2[NK], r1[NK], r2[NK];
    R cor[NK], vor[NK];
    R lap2[NK];   // lap(lap u) (biharmonic runs; zero otherwise)
};

// kMix: D^u is left out of the tendency and applied by the implicit column
// solve of Algorithm 2 (the vertical-mixing form of the stage).
template <int NK, typename R, bool kMix, bool kWide>
__device__ __forceinline__ void fe_edge_finish(const FEEdgeArgs<R> &a, int e, int c1, int c2, double idc, double idv,
                                               const EdgeOperands<NK, R> &o) {
    const int lane = lane_id();
    const DevMesh &m = a.m;
    const int L = a.L;
    const size_t base = (size_t)e * L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    // Operands of lanes past the last layer are copies of layer L - 1; the
    // edge thickness and the PGF differences, which reach the column sums and
    // scans, are zeroed there.
    R he[NK];
    double hed[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        hed[c] = ok[c] ? 0.5 * (o.h1[c] + o.h2[c]) : 0.0;
        he[c] = (R)hed[c];
    }
    // Pressure gradient in z-star layers from the column differences, in FP64
    // in both modes: its two terms cancel down to the density anomaly.
    double pgf[NK];
    {
        double drh[NK], dh[NK], sp[NK], ss[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            drh[c] = ok[c] ? o.r2[c] * o.h2[c] - o.r1[c] * o.h1[c] : 0.0;
            dh[c] = ok[c] ? o.h2[c] - o.h1[c] : 0.0;
        }
        col_excl_prefix<NK, kDppFor<R>>(drh, sp);
        col_excl_suffix<NK, kDppFor<R>>(dh, ss);
        const double dH = m.H[c2] - m.H[c1];
        const double pgf_scale = idc / a.rho0;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const double dp = a.g * (sp[c] + 0.5 * drh[c]);
            const double dz = -dH + ss[c] + 0.5 * dh[c];
            pgf[c] = -(dp + a.g * (0.5 * (o.r1[c] + o.r2[c])) * dz) * pgf_scale;
        }
    }

    // Vertical advection and vertical viscosity at interior interfaces.
    R uu[NK], hu[NK], at[NK], tau[NK], atn[NK], taun[NK];
    col_up1<NK, kDppFor<R>>(o.u, uu);
    col_up1<NK, kDppFor<R>>(he, hu);
    const R nu_v = (R)a.nu_v;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        if (k >= 1 && k < L) {
            const R dzt = (uu[c] - o.u[c]) * (R(1) / (R(0.5) * (hu[c] + he[c])));
            const R we = R(0.5) * (o.W1[c] + o.W2[c]);
            at[c] = we * dzt;
            tau[c] = nu_v * dzt;
        } else {
            at[c] = R(0);
            tau[c] = R(0);
        }
    }
    col_down1<NK, kDppFor<R>>(at, atn);
    col_down1<NK, kDppFor<R>>(tau, taun);
    const R speed = (R)sqrt(a.Kbot[c1] + a.Kbot[c2]);
    const R gz = (R)(a.g * (a.zeta[c2] - a.zeta[c1]) * idc);
    const R dt = (R)a.dt, nu_h = (R)a.nu_h, c_drag = (R)a.c_drag;
    const R ridc = (R)idc, ridv = (R)idv;

    R ut1[NK];
    double hut1[NK], hu_in[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        if (k < L) {
            if (k == L - 1) taun[c] = c_drag * speed * o.u[c];
            const R gradB = (o.B2[c] - o.B1[c]) * ridc;
            const R curlp = (o.zb[c] - o.za[c]) * ridv;
            const R vadv = R(0.5) * (at[c] + atn[c]);
            const R tu = -gradB + o.vor[c] - vadv + (R)pgf[c] - nu_h * curlp - (R)a.nu4 * o.lap2[c];
            const R du = kMix ? R(0) : (tau[c] - taun[c]) * (R(1) / he[c]);
            ut1[c] = o.ut[c] + dt * (o.cor[c] + tu + du + gz);
        } else {
            ut1[c] = R(0);
        }
        hut1[c] = hed[c] * (double)ut1[c];
        hu_in[c] = hed[c] * (double)o.u[c];
    }
    // Column sums that feed the barotropic forcing and the reconciliation are
    // formed in FP64 in both modes.
    const double Sh = col_sum<NK, kDppFor<R>>(hed);
    const double G = col_sum<NK, kDppFor<R>>(hut1) / Sh / a.dt;
    const R dtG = (R)(a.dt * G);
    R x[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) x[c] = (lane + c * kWave < L) ? ut1[c] - dtG : R(0);
    if constexpr (kMix) {
        // Algorithm 2: u1 - dt D^u(u1) = ut1 + ubar with the drag speed of the
        // input, then ut1 = u1 - ubar (ubar: the input's barotropic velocity).
        const R ubin = (R)((a.ubar_add ? a.ubar_add[e] : 0.0) + (a.ubar_sub ? a.ubar_sub[e] : 0.0));
        R Aup[NK], Adn[NK], lo[NK], di[NK], up[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int k = lane + c * kWave;
            Aup[c] = (k >= 1 && k < L) ? nu_v / (R(0.5) * (hu[c] + he[c])) : R(0);
        }
        col_down1<NK, kDppFor<R>>(Aup, Adn);
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int k = lane + c * kWave;
            if (k == L - 1) Adn[c] = c_drag * speed;
            const bool in = k < L;
            lo[c] = in ? -dt * Aup[c] / he[c] : R(0);
            up[c] = (in && k < L - 1) ? -dt * Adn[c] / he[c] : R(0);
            di[c] = in ? R(1) + dt * (Aup[c] + Adn[c]) / he[c] : R(1);
            x[c] = in ? x[c] + ubin : R(0);
        }
        col_tridiag_solve<NK, R>(L, lo, di, up, x);
#pragma unroll
        for (int c = 0; c < NK; ++c) x[c] = (lane + c * kWave < L) ? x[c] - ubin : R(0);
    }
    const double ubn = a.Un ? a.ubar_n[e] : 0.0;
    R outv[NK];
    double hp[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        R utn = R(0);
        if (a.Un) {
            const double un = (double)col_ldv<kWide>(a.Un, base, kk[c]);
            utn = k < L ? (R)(un - ubn) : R(0);
        }
        outv[c] = (k < L) ? combine<R>(a.comb, utn, x[c]) : R(0);
        if (k < L) col_st(a.out + base, k, outv[c]);
        hp[c] = hed[c] * (a.psum_a * (double)utn + a.psum_b * (double)outv[c]);
    }
    double shu = 0.0, shp = 0.0;
    if (a.sum_hu) shu = col_sum<NK, kDppFor<R>>(hu_in);
    if (a.sum_hp) shp = col_sum<NK, kDppFor<R>>(hp);
    if (lane == 0) {
        a.G[e] = G;
        a.sum_h[e] = Sh;
        if (a.sum_hu) a.sum_hu[e] = shu;
        if (a.sum_hp) a.sum_hp[e] = shp;
        if (a.Gi) {
            if (a.interp == 3)
                a.Gi[e] = div_by_near(a.Ga[e], 6.0, 1.0 / 6.0) + div_by_near(a.Gb[e], 6.0, 1.0 / 6.0) +
                          div_by_near(2.0 * G, 3.0, 1.0 / 3.0);
            else
                a.Gi[e] = 0.5 * a.Ga[e] + 0.5 * G;
        }
    }
}

template <int NK, typename R>
__device__ __forceinline__ void fe_edge_dry(const FEEdgeArgs<R> &a, int e) {
    const int lane = lane_id();
    const size_t base = (size_t)e * a.L;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        if (k < a.L) a.out[base + k] = R(0);
    }
    if (lane == 0) {
        a.G[e] = 0.0;
        a.sum_h[e] = 0.0;
        if (a.sum_hu) a.sum_hu[e] = 0.0;
        if (a.sum_hp) a.sum_hp[e] = 0.0;
        if (a.Gi) a.Gi[e] = 0.0;
    }
}

// kChain: the stencil is in canonical two-cell order (sse_mesh.cpp) and the
// edge record holds the two cells' vertex chains, so the vorticity of the 10
// distinct vertices is read once instead of at both ends of every stencil
// edge; otherwise every stencil edge carries its own two vertices.
// kVar bit 0: kChain; bit 1: kMix (see fe_edge_finish); bit 2: kDel4, the
// biharmonic operand lap(lap u) is gathered (div and curl of lap u at the
// edge's cells and vertices).
template <int NK, typename R, bool kAdd, int kVar>
__device__ __forceinline__ void fe_edge_body(const FEEdgeArgs<R> &a, int col) {
    constexpr bool kChain = (kVar & 1) != 0;
    constexpr bool kMix = (kVar & 2) != 0;
    constexpr bool kDel4 = (kVar & 4) != 0;
    constexpr bool kWide = (kVar & 8) != 0;
    const DevMesh &m = a.m;
    const int E = m.E;
    const int e = col;
    if (e >= E) return;
    const int L = a.L;
    const size_t base = (size_t)e * L;
    if (!m.emask[e]) {
        fe_edge_dry<NK, R>(a, e);
        return;
    }
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    // u = X + ubar (kAdd) or ut = X - ubar (otherwise); the other one equals X.
    const double *ubar = kAdd ? a.ubar_add : a.ubar_sub;
    const int32_t *rec = m.erec + (size_t)e * kEdgeRec;
    const int c1 = rec[30], c2 = rec[31];
    const double idc = m.inv_dc[e], idv = m.inv_dv[e];
    const R ub_e = ubar_at<R>(a, ubar, e);
    const size_t b1 = (size_t)c1 * L, b2 = (size_t)c2 * L;

    EdgeOperands<NK, R> o;
    R q[NK];
    // vertex vorticity: chain A0..A5 around c1 (A0, A5 the end points of e),
    // B0..B3 the inner vertices of the chain around c2
    R zA[6][NK], zB[4][NK];
    if constexpr (kChain) {
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const size_t zo = (size_t)rec[10 + i] * L;
#pragma unroll
            for (int c = 0; c < NK; ++c) zA[i][c] = col_ldv<kWide>(a.Z, zo, kk[c]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t zo = (size_t)rec[16 + i] * L;
#pragma unroll
            for (int c = 0; c < NK; ++c) zB[i][c] = col_ldv<kWide>(a.Z, zo, kk[c]);
        }
    }
    const bool a0_is_v1 = kChain ? rec[20] != 0 : false;
    const size_t bv1 = kChain ? 0 : (size_t)m.edge_verts[2 * e] * L;
    const size_t bv2 = kChain ? 0 : (size_t)m.edge_verts[2 * e + 1] * L;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = kk[c];
        const R x = col_ldv<kWide>(a.X, base, k);
        R za, zb;
        if constexpr (kChain) {
            za = a0_is_v1 ? zA[0][c] : zA[5][c];
            zb = a0_is_v1 ? zA[5][c] : zA[0][c];
        } else {
            za = col_ldv<kWide>(a.Z, bv1, k);
            zb = col_ldv<kWide>(a.Z, bv2, k);
        }
        o.u[c] = kAdd ? x + ub_e : x;
        o.ut[c] = kAdd ? x : x - ub_e;
        o.h1[c] = col_ldv<kWide>(a.h, b1, k);
        o.h2[c] = col_ldv<kWide>(a.h, b2, k);
        o.r1[c] = col_ldv<kWide>(a.rho, b1, k);
        o.r2[c] = col_ldv<kWide>(a.rho, b2, k);
        o.za[c] = za;
        o.zb[c] = zb;
        o.B1[c] = col_ldv<kWide>(a.B, b1, k);
        o.B2[c] = col_ldv<kWide>(a.B, b2, k);
        o.W1[c] = col_ldv<kWide>(a.Wtop, b1, k);
        o.W2[c] = col_ldv<kWide>(a.Wtop, b2, k);
        q[c] = o.za[c] + o.zb[c];  // twice the edge vorticity
        o.cor[c] = o.vor[c] = R(0);
        o.lap2[c] = R(0);
    }
    if constexpr (kDel4) {
        // lap(lap u) at the edge from div(lap u) at its cells and curl(lap u)
        // at its vertices
        const int v1 = kChain ? (a0_is_v1 ? rec[10] : rec[15]) : m.edge_verts[2 * e];
        const int v2 = kChain ? (a0_is_v1 ? rec[15] : rec[10]) : m.edge_verts[2 * e + 1];
        const size_t w1 = (size_t)v1 * L, w2 = (size_t)v2 * L;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int k = kk[c];
            const R d1 = col_ldv<kWide>(a.D2, b1, k), d2 = col_ldv<kWide>(a.D2, b2, k);
            const R z1 = col_ldv<kWide>(a.Z2, w1, k), z2 = col_ldv<kWide>(a.Z2, w2, k);
            o.lap2[c] = (d2 - d1) * (R)idc - (z2 - z1) * (R)idv;
        }
    }

    // Coriolis on the baroclinic velocity (-f ut^perp) and the vorticity flux
    // -(k.curl u) u^perp through the TRiSK tangential reconstruction.  The
    // table holds W / 4 beside W (f_e + f_j) / 2, and the vertex sums are
    // twice the edge vorticities, so W ((q_e + q_j) / 2) is (W / 4)(2 q_e +
    // 2 q_j): the same bits with two multiplications fewer per stencil term
    // (scaling by powers of two is exact).  Padded
    // stencil slots point at the edge itself with zero weights, so the loop
    // runs its full width; its column loads carry no branch between them.
    // the weight pairs in R (mixed precision: the FP32 table, the same values
    // as converting the FP64 ones, without a conversion per term)
    const R *wp = wpair_of<R>(m) + (size_t)e * 2 * kMaxEdges2;
#pragma unroll
    for (int j = 0; j < kMaxEdges2; ++j) {
        const int ep = rec[j];
        const R wj = wp[2 * j], wfj = wp[2 * j + 1];
        const R ubp = ubar_at<R>(a, ubar, ep);
        const size_t pb = (size_t)ep * L;
        const size_t pb1 = kChain ? 0 : (size_t)rec[10 + 2 * j] * L;
        const size_t pb2 = kChain ? 0 : (size_t)rec[11 + 2 * j] * L;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const R xp = col_ldv<kWide>(a.X, pb, kk[c]);
            const R up = kAdd ? xp + ubp : xp, utp = kAdd ? xp : xp - ubp;
            R qp;
            if constexpr (kChain) {
                // chain of c1: A_j, A_{j+1}; chain of c2: A5, B0, B1, B2, B3, A0
                const int s = j - 5;
                const R za_ = j < 5 ? zA[j < 5 ? j : 0][c] : (s == 0 ? zA[5][c] : zB[s > 0 ? s - 1 : 0][c]);
                const R zb_ = j < 5 ? zA[j < 5 ? j + 1 : 0][c] : (s == 4 ? zA[0][c] : zB[s < 4 && s >= 0 ? s : 0][c]);
                qp = za_ + zb_;
            } else {
                qp = col_ldv<kWide>(a.Z, pb1, kk[c]) + col_ldv<kWide>(a.Z, pb2, kk[c]);
            }
            o.cor[c] += wfj * utp;
            o.vor[c] += (wj * (q[c] + qp)) * up;
        }
    }
    fe_edge_finish<NK, R, kMix, kWide>(a, e, c1, c2, idc, idv, o);
}

// ---------------------------------------------------------------------------
// Measurement aid: the edge pass's column loads without its arithmetic.
// Each wavefront gathers the columns the direct edge pass reads for its edge
// (canonical stencils, one register chunk): u and u^n at the edge, h, rho,
// K - nu div u and w at both cells, the 10 stencil edges and the 10 chain
// vertices, and writes their sum; a launch takes the pass's gather time at
// its access pattern.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(1024, 8) edge_gather_kernel(FEEdgeArgs<R> a) {
    const DevMesh &m = a.m;
    const int e = column_id(m.E);
    if (e >= m.E) return;
    const int L = a.L;
    int kk[1];
    bool ok[1];
    lane_layers<1>(L, kk, ok);
    const int k = kk[0];
    if (!m.emask[e]) {
        if (ok[0]) col_st(a.out + (size_t)e * L, k, R(0));
        return;
    }
    const int32_t *rec = m.erec + (size_t)e * kEdgeRec;
    const size_t b1 = (size_t)rec[30] * L, b2 = (size_t)rec[31] * L;
    R v[30];
    v[0] = col_ldv<false>(a.X, (size_t)e * L, k);
    v[1] = col_ldv<false>(a.Un, (size_t)e * L, k);
    v[2] = (R)col_ldv<false>(a.h, b1, k);
    v[3] = (R)col_ldv<false>(a.h, b2, k);
    v[4] = (R)col_ldv<false>(a.rho, b1, k);
    v[5] = (R)col_ldv<false>(a.rho, b2, k);
    v[6] = col_ldv<false>(a.B, b1, k);
    v[7] = col_ldv<false>(a.B, b2, k);
    v[8] = col_ldv<false>(a.Wtop, b1, k);
    v[9] = col_ldv<false>(a.Wtop, b2, k);
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        v[10 + j] = col_ldv<false>(a.X, (size_t)rec[j] * L, k);
        v[20 + j] = col_ldv<false>(a.Z, (size_t)rec[10 + j] * L, k);
    }
    R sum = R(0);
#pragma unroll
    for (int j = 0; j < 30; ++j) sum += v[j];
    if (ok[0]) col_st(a.out + (size_t)e * L, k, sum);
}

// ---------------------------------------------------------------------------
// Baroclinic forward Euler: edge pass staged through LDS.
//
// One workgroup of T wavefronts owns a tile of T consecutive edges.  It first
// copies every column the tile reads (stencil edges, their vertices, the
// edges' cells for h, rho, K - nu div u and w) from global memory into LDS,
// each column exactly once, then each wavefront evaluates its edge from LDS.
// The copy uses 16-byte loads, so one load instruction moves two FP64 (four
// FP32) layers per lane and several columns per wavefront; the vector-memory
// address path, which bounds the direct-gather kernel, then handles about a
// quarter of the instructions.
// ---------------------------------------------------------------------------

constexpr int kTileWaves = 4;  // wavefronts per workgroup of the tiled edge pass

// One list of columns to stage: column i of the list is the global column
// src + ids[i] L and goes to dst + i L in LDS.
template <typename T>
struct StageSeg {
    const T *src;
    const int32_t *ids;
    int n;
    T *dst;
};

// Copy the columns of NS lists (L values of type T each) into LDS with
// 16-byte loads.  The lists are walked as one: every lane group takes up to
// 8 columns, loads their ids, then their data, then stores them, so one
// wavefront has 8 column loads in flight and the whole copy costs two
// memory round trips.
template <typename T, int NS>
__device__ __forceinline__ void stage_columns(const StageSeg<T> (&seg)[NS], int L) {
    constexpr int V = 16 / sizeof(T);
    constexpr int B = 8;
    int start[NS + 1];
    start[0] = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) start[q + 1] = start[q] + seg[q].n;
    const int total = start[NS];
    if (total == 0) return;
    const int lane = lane_id(), wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (L % V == 0 && L <= V * kWave) {
        const int lpc = L / V, cpw = kWave / lpc;  // lanes per column, columns per wavefront
        const int slot = lane / lpc, part = lane - slot * lpc;
        const bool lane_on = slot < cpw;
        const int step = nw * cpw;
        for (int c0 = wv * cpw + slot; c0 < total + (B - 1) * step; c0 += B * step) {
            int seg_of[B], pos[B], id[B];
            bool on[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int c = c0 + u * step;
                on[u] = lane_on && c < total;
                const int cs = c < total ? c : total - 1;
                int q = 0, p0 = cs;
#pragma unroll
                for (int r = 1; r < NS; ++r) {
                    if (cs >= start[r]) {
                        q = r;
                        p0 = cs - start[r];
                    }
                }
                seg_of[u] = q;
                pos[u] = p0;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int32_t *ids = seg[0].ids;
#pragma unroll
                for (int r = 1; r < NS; ++r) ids = seg_of[u] == r ? seg[r].ids : ids;
                id[u] = ids[pos[u]];
            }
            uint4 v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const T *src = seg[0].src;
#pragma unroll
                for (int r = 1; r < NS; ++r) src = seg_of[u] == r ? seg[r].src : src;
                v[u] = *reinterpret_cast<const uint4 *>(src + (size_t)id[u] * L + part * V);
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                T *dst = seg[0].dst;
#pragma unroll
                for (int r = 1; r < NS; ++r) dst = seg_of[u] == r ? seg[r].dst : dst;
                if (on[u]) *reinterpret_cast<uint4 *>(dst + (size_t)pos[u] * L + part * V) = v[u];
            }
        }
    } else {
        // Local arrays are indexed with compile-time indices only (select
        // chains), so that they stay in registers.
        for (int c = wv; c < total; c += nw) {
            int i = c;
            const int32_t *ids = seg[0].ids;
            const T *src = seg[0].src;
            T *dst = seg[0].dst;
#pragma unroll
            for (int r = 1; r < NS; ++r) {
                if (c >= start[r]) {
                    i = c - start[r];
                    ids = seg[r].ids;
                    src = seg[r].src;
                    dst = seg[r].dst;
                }
            }
            const T *col = src + (size_t)ids[i] * L;
            for (int k = lane; k < L; k += kWave) dst[(size_t)i * L + k] = col[k];
        }
    }
}

template <typename R>
size_t fe_edge_tiled_lds(const DevTiles &t, int L) {
    return (size_t)(t.max_ue + t.max_uv) * L * sizeof(R);   // X and Z columns
}

template <int NK, typename R, bool kAdd, bool kMix>
__global__ void __launch_bounds__(kTileWaves * kWave) fe_edge_tiled_kernel(FEEdgeArgs<R> a, DevTiles t) {
    extern __shared__ __align__(16) double lds_d[];
    const DevMesh &m = a.m;
    const int tile = xcd_block(t.nT);
    if (tile < 0) return;
    const int T = t.T, L = a.L, E = m.E;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ue0 = t.ue_off[tile], nue = t.ue_off[tile + 1] - ue0;
    const int uv0 = t.uv_off[tile], nuv = t.uv_off[tile + 1] - uv0;
    const int uc0 = t.uc_off[tile], nuc = t.uc_off[tile + 1] - uc0;
    // LDS holds the reused stencil operands only: the X columns of the tile's
    // edges and stencil edges, then the vorticity columns of their vertices.
    // The cell operands (h, rho, K - nu div u, w: two columns each, little
    // reuse across the tile) are read from global memory per edge.
    R *sX = reinterpret_cast<R *>(lds_d);
    R *sZ = sX + (size_t)nue * L;
    const double *ubar = kAdd ? a.ubar_add : a.ubar_sub;
    const int32_t *le = t.ue + ue0, *lv = t.uv + uv0;
    (void)uc0;
    (void)nuc;
    const StageSeg<R> seg[2] = {{a.X, le, nue, sX}, {a.Z, lv, nuv, sZ}};
    stage_columns<R, 2>(seg, L);
    __syncthreads();

    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    // A workgroup has at most kTileWaves wavefronts (a 256-register budget per
    // lane, no spills); with larger tiles each wavefront evaluates several edges.
    const int nw = blockDim.x >> 6;
    for (int el = wv; el < T; el += nw) {
        const int e = tile * T + el;
        if (e >= E) break;
        if (!m.emask[e]) {
            fe_edge_dry<NK, R>(a, e);
            continue;
        }
        // 8-bit positions of this edge's operands in the staged lists.
        const uint32_t *lw = reinterpret_cast<const uint32_t *>(t.loc + (size_t)e * kLocPerEdge);
        uint32_t word[kLocPerEdge / 4];
#pragma unroll
        for (int qq = 0; qq < kLocPerEdge / 4; ++qq) word[qq] = lw[qq];
        auto locb = [&](int i) -> int { return (word[i >> 2] >> (8 * (i & 3))) & 0xff; };
        const int ls = locb(0), lv1 = locb(3), lv2 = locb(4);
        const int32_t *rec = m.erec + (size_t)e * kEdgeRec;
        const R ub_e = ubar_at<R>(a, ubar, e);
        const int c1 = rec[30], c2 = rec[31];
        const double idcv = m.inv_dc[e], idvv = m.inv_dv[e];

        const size_t b1 = (size_t)c1 * L, b2 = (size_t)c2 * L;
        EdgeOperands<NK, R> o;
        R q[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const int k = kk[c];
            const double h1 = a.h[b1 + k], h2 = a.h[b2 + k], r1 = a.rho[b1 + k], r2 = a.rho[b2 + k];
            const R B1 = a.B[b1 + k], B2 = a.B[b2 + k], W1 = a.Wtop[b1 + k], W2 = a.Wtop[b2 + k];
            const R x = sX[(size_t)ls * L + k];
            o.u[c] = ok[c] ? (kAdd ? x + ub_e : x) : R(0);
            o.ut[c] = ok[c] ? (kAdd ? x : x - ub_e) : R(0);
            o.h1[c] = ok[c] ? h1 : 0.0;
            o.h2[c] = ok[c] ? h2 : 0.0;
            o.r1[c] = ok[c] ? r1 : 0.0;
            o.r2[c] = ok[c] ? r2 : 0.0;
            o.za[c] = ok[c] ? sZ[(size_t)lv1 * L + k] : R(0);
            o.zb[c] = ok[c] ? sZ[(size_t)lv2 * L + k] : R(0);
            o.B1[c] = ok[c] ? B1 : R(0);
            o.B2[c] = ok[c] ? B2 : R(0);
            o.W1[c] = ok[c] ? W1 : R(0);
            o.W2[c] = ok[c] ? W2 : R(0);
            q[c] = o.za[c] + o.zb[c];  // twice the edge vorticity
            o.cor[c] = o.vor[c] = R(0);
            o.lap2[c] = R(0);  // the tiled variants run without the biharmonic term
        }
        const R *wp = wpair_of<R>(m) + (size_t)e * 2 * kMaxEdges2;
#pragma unroll
        for (int j = 0; j < kMaxEdges2; ++j) {
            const R wj = wp[2 * j], wfj = wp[2 * j + 1];
            const int sl = locb(5 + j), sa = locb(15 + 2 * j), sb = locb(16 + 2 * j);
            const R ubp = ubar_at<R>(a, ubar, rec[j]);
#pragma unroll
            for (int c = 0; c < NK; ++c) {
                const int k = kk[c];
                const R xp = sX[(size_t)sl * L + k];
                const R up = kAdd ? xp + ubp : xp, utp = kAdd ? xp : xp - ubp;
                const R qp = sZ[(size_t)sa * L + k] + sZ[(size_t)sb * L + k];
                o.cor[c] += wfj * utp;
                o.vor[c] += (wj * (q[c] + qp)) * up;
            }
        }
        fe_edge_finish<NK, R, kMix, true>(a, e, c1, c2, idcv, idvv, o);
    }
}

// ---------------------------------------------------------------------------
// Barotropic forward-Euler evaluation (Algorithms 3 and 4, one stage)
// ---------------------------------------------------------------------------
template <typename R>
struct BTTables;
template <>
struct BTTables<double> {
    __device__ static const double *wf(const DevMesh &m) { return m.wf; }
    __device__ static const double *inv_dc(const DevMesh &m) { return m.inv_dc; }
    __device__ static const double *cdiv(const DevMesh &m) { return m.cell_div_t; }
    __device__ static const double *H(const DevMesh &m) { return m.H; }
};
template <>
struct BTTables<float> {
    __device__ static const float *wf(const DevMesh &m) { return m.wf_f; }
    __device__ static const float *inv_dc(const DevMesh &m) { return m.inv_dc_f; }
    __device__ static const float *cdiv(const DevMesh &m) { return m.cell_div_t_f; }
    __device__ static const float *H(const DevMesh &m) { return m.H_f; }
};

// One block of edges (edge_part) or of cells of one evaluation.  kD16: the
// index tables are read as 16-bit offsets (half the index bytes).
// The barotropic kernels (one evaluation / one tiled substep) spell every
// fused multiply-add out and contract nothing else, so that the two forms
// give the same bits whatever the compiler would fuse in either context.
template <typename R, bool kD16>
__device__ __forceinline__ void bt_eval_body(const BTEvalArgs<R> &a, bool edge_part, int lb) {
#pragma clang fp contract(off)
    const DevMesh &m = a.m;
    const R tau = (R)a.tau, g = (R)a.g;
    if (edge_part) {
        const int e = lb * blockDim.x + threadIdx.x;
        if (e >= m.E) return;
        if (!m.emask[e]) {
            a.uo[e] = R(0);
            if (a.F && a.zeroF) a.F[e] = 0.0;
            return;
        }
        const R *__restrict__ wf = BTTables<R>::wf(m);
        int c1, c2;
        if constexpr (kD16) {
            const int pk = m.ecells16[e], bc = delta_base(e, m.ratio_ce);
            c1 = bc + (int)(int16_t)(pk & 0xffff);
            c2 = bc + (int)(int16_t)((unsigned)pk >> 16);
        } else {
            c1 = m.edge_cells[2 * e];
            c2 = m.edge_cells[2 * e + 1];
        }
        const R ua = a.ua[e];
        const R z1 = a.za[c1], z2 = a.za[c2];
        // Padded stencil slots point at the edge itself with zero weight: the
        // loop runs its full width so that all its gathers issue together.
        R cor = R(0);
#pragma unroll
        for (int j = 0; j < kMaxEdges2; ++j) {
            const int ep = kD16 ? e + (int)m.eoe16[(size_t)j * m.E + e] : m.eoe[(size_t)j * m.E + e];
            cor = fmadd(wf[(size_t)j * m.E + e], a.ua[ep], cor);
        }
        const R ru = fmadd(-(g * (z2 - z1)), BTTables<R>::inv_dc(m)[e], cor) + (R)a.G[e];
        // the first stage of a substep combines with nothing: no base read
        const R base = a.comb != COMB_NONE ? a.ub[e] : R(0);
        a.uo[e] = combine<R>(a.comb, base, fmadd(tau, ru, ua));
        if (a.F) {
            // The transport accumulates in FP64 in both modes.
            const double flux = (double)ua * (0.5 * (((double)z1 + m.H[c1]) + ((double)z2 + m.H[c2])));
            a.F[e] = fmadd(a.wF, flux, a.zeroF ? 0.0 : a.F[e]);
        }
    } else {
        const int i = lb * blockDim.x + threadIdx.x;
        if (i >= m.C) return;
        if (!m.cmask[i]) { a.zo[i] = R(0); return; }
        const R *__restrict__ Ht = BTTables<R>::H(m);
        const R *__restrict__ cd_t = BTTables<R>::cdiv(m);
        const R zi = a.za[i] + Ht[i];
        R div = R(0);
        const int be = kD16 ? delta_base(i, m.ratio_ec) : 0;
#pragma unroll
        for (int j = 0; j < kMaxEdges; ++j) {
            const R cd = cd_t[(size_t)j * m.C + i];
            const int e = kD16 ? be + (int)m.cedges16[(size_t)j * m.C + i] : m.cell_edges_t[(size_t)j * m.C + i];
            const int nb = kD16 ? i + (int)m.cnbrs16[(size_t)j * m.C + i] : m.cell_nbrs_t[(size_t)j * m.C + i];
            const R zn = a.za[nb] + Ht[nb];
            div = fmadd(cd, a.ua[e] * (R(0.5) * (zi + zn)), div);
        }
        const R base = a.comb != COMB_NONE ? a.zb[i] : R(0);
        a.zo[i] = combine<R>(a.comb, base, fmadd(tau, -div, a.za[i]));
    }
}

// ---------------------------------------------------------------------------
// Tiled barotropic substep: one workgroup advances one cell patch (with its
// halo rings) through a whole SSPRK3 (three evaluations) or SSPRK2 (two)
// substep.  The substep input and every stage live in LDS; each thread holds
// the stencil tables of its edges (at most KS) and of its cell in registers
// for all evaluations, so the tables are read once per substep instead of
// once per evaluation.  Evaluation k computes the region level that the next
// one reads (level 2, then 1, then 0 = the patch's own cells and edges) with
// exactly the arithmetic of the one-evaluation kernel, so both paths give the
// same bits.
// ---------------------------------------------------------------------------
template <typename R>
struct BtTab;
template <>
struct BtTab<double> {
    __device__ static const double *w(const DevBtTiles &t) { return t.ew; }
    __device__ static const double *idc(const DevBtTiles &t) { return t.eidc; }
    __device__ static const double *cd(const DevBtTiles &t) { return t.ccd; }
};
template <>
struct BtTab<float> {
    __device__ static const float *w(const DevBtTiles &t) { return t.ew_f; }
    __device__ static const float *idc(const DevBtTiles &t) { return t.eidc_f; }
    __device__ static const float *cd(const DevBtTiles &t) { return t.ccd_f; }
};

// Grid-wide barrier of a cooperative launch: the writes of every workgroup
// before it are visible to every workgroup after it.  One thread per
// workgroup arrives on a counter (after the workgroup barrier and a
// device-scope release, which writes back its XCD's L2); the last of the
// k-th round (the counter reaching k * gridDim.x) publishes generation k, for
// which the others poll; a device-scope acquire then drops stale cache lines.
// The wait is bounded: if it runs out (or another workgroup's did), the
// workgroup sets *err and stops waiting, so every wavefront of the launch
// still finishes; the host reports the error and the results are not used.
__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned *gen, int *err, unsigned round,
                                             unsigned max_spins) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned target = round * gridDim.x;
        const unsigned old = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == target) {
            __hip_atomic_store(gen, round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < round) {
                if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                if (++spins > max_spins) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// The persistent form of the tiled substep (bt_substep_body below): all l.M
// substeps of the loop for patch p in one workgroup of a cooperative launch
// in which every patch has its own workgroup (p < 0: a padding workgroup that
// only takes part in the barriers).  The stencil tables, the frozen forcing
// and the F^zeta sums stay in registers for the whole loop; substep s reads
// the previous substep's output (the loop input for s = 0) and writes one of
// two stage buffers (the loop output for the last), with a grid barrier
// between substeps.  Every evaluation performs exactly the arithmetic of the
// one-evaluation kernel, so all forms give the same bits.
template <typename R, int kScheme, int KS>
__device__ __forceinline__ void bt_loop_body(const BTTileArgs<R> &a, const BtLoop<R> &l, int p) {
#pragma clang fp contract(off)
    extern __shared__ __align__(16) double lds_d[];
    const DevBtTiles &T = a.t;
    const int tid = threadIdx.x;
    const bool on_patch = p >= 0;
    const int pp = on_patch ? p : 0;
    const int32_t *rec = T.patch + (size_t)pp * kBtRec;
    const int e0 = rec[0], es0 = rec[1], c0 = rec[2], cs0 = rec[3];
    int ne[4], nc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ne[k] = on_patch ? rec[4 + k] : 0;
        nc[k] = on_patch ? rec[8 + k] : 0;
    }
    constexpr int kIn = kScheme == 3 ? 3 : 2;  // level of the substep input
    const int nEin = ne[kIn], nCin = nc[kIn];
    const int nE1 = ne[kIn - 1], nC1 = nc[kIn - 1];  // level of the first evaluation
    const int se = ne[2], sc = nc[2];                // strides of the stencil tables

    // LDS: H (double) | U0 U1 U2 | Z0 Z1 Z2 | H in R (FP32 state only)
    double *H64b = lds_d;
    R *U0b = reinterpret_cast<R *>(H64b + nc[3]);
    R *U1b = U0b + ne[3];
    R *U2b = U1b + ne[2];
    R *Z0b = U2b + ne[1];
    R *Z1b = Z0b + nc[3];
    R *Z2b = Z1b + nc[2];
    const R *Hrb;
    if constexpr (sizeof(R) == 8) {
        Hrb = reinterpret_cast<const R *>(H64b);
    } else {
        R *h = Z2b + nc[1];
        for (int lc = tid; lc < nCin; lc += kBtThreads) h[lc] = T.cH_f[c0 + lc];
        Hrb = h;
    }
    for (int lc = tid; lc < nCin; lc += kBtThreads) H64b[lc] = T.cH[c0 + lc];

    // this thread's edges (le = s kBtThreads + tid) and cell (lc = tid)
    const R *__restrict__ wt = BtTab<R>::w(T);
    R w[KS][kMaxEdges2], idc[KS], Gv[KS];
    uint32_t nbw[KS][kMaxEdges2 / 2], ecw[KS];
    double Fa[KS];
    int ge[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int le = s * kBtThreads + tid;
        const bool on = le < nE1;
        const int q = on ? le : 0;
        ecw[s] = on ? T.ec[es0 + q] : 0u;
        ge[s] = T.eid[e0 + q];
        idc[s] = BtTab<R>::idc(T)[es0 + q];
        Gv[s] = (R)a.G[ge[s]];
#pragma unroll
        for (int j = 0; j < kMaxEdges2; ++j) w[s][j] = wt[(size_t)kMaxEdges2 * es0 + (size_t)j * se + q];
#pragma unroll
        for (int i = 0; i < kMaxEdges2 / 2; ++i) nbw[s][i] = T.enb[(size_t)(kMaxEdges2 / 2) * es0 + (size_t)i * se + q];
        Fa[s] = (a.F && le < ne[0]) ? (a.zeroF ? 0.0 : a.F[ge[s]]) : 0.0;
    }
    const bool con = tid < nC1;
    const int qc = con ? tid : 0;
    const bool cwet = con && T.cwet[cs0 + qc] != 0;
    const int gc = T.cid[c0 + qc];
    R cd[kMaxEdges];
    uint32_t cen[kMaxEdges];
#pragma unroll
    for (int j = 0; j < kMaxEdges; ++j) {
        cd[j] = BtTab<R>::cd(T)[(size_t)kMaxEdges * cs0 + (size_t)j * sc + qc];
        cen[j] = T.cen[(size_t)kMaxEdges * cs0 + (size_t)j * sc + qc];
    }

    const R tau = (R)a.tau, g = (R)a.g;
    const int nsub = l.M;
#pragma unroll 1
    for (int sub = 0; sub < nsub; ++sub) {
        // LDS bases offset by an opaque zero, so that the compiler recomputes
        // the stage addresses in every substep instead of hoisting all of them
        // out of the loop (which needs more registers than the tables)
        int zoff = 0;
        {
            asm volatile("" : "+s"(zoff));
            // the packed index words likewise: decoded once per substep, not
            // kept decoded across the loop
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) {
                asm volatile("" : "+v"(ecw[s2]));
#pragma unroll
                for (int i = 0; i < kMaxEdges2 / 2; ++i) asm volatile("" : "+v"(nbw[s2][i]));
            }
#pragma unroll
            for (int j = 0; j < kMaxEdges; ++j) asm volatile("" : "+v"(cen[j]));
        }
        R *const U0 = U0b + zoff, *const U1 = U1b + zoff, *const U2 = U2b + zoff;
        R *const Z0 = Z0b + zoff, *const Z1 = Z1b + zoff, *const Z2 = Z2b + zoff;
        const double *const H64 = H64b + zoff;
        const R *const Hr = Hrb + zoff;
        const bool odd = (sub & 1) != 0;
        const R *ua = sub == 0 ? l.u_in : (odd ? l.bu0 : l.bu1);
        const R *za = sub == 0 ? l.z_in : (odd ? l.bz0 : l.bz1);
        R *uo = sub == nsub - 1 ? l.u_out : (odd ? l.bu1 : l.bu0);
        R *zo = sub == nsub - 1 ? l.z_out : (odd ? l.bz1 : l.bz0);
#pragma unroll 1
        for (int le = tid; le < nEin; le += kBtThreads) U0[le] = ua[T.eid[e0 + le]];
#pragma unroll 1
        for (int lc = tid; lc < nCin; lc += kBtThreads) Z0[lc] = za[T.cid[c0 + lc]];
        __syncthreads();

        // One evaluation producing level lvl from (Ui, Zi); the last one writes
        // the substep output to global memory.
        auto evaluate = [&](const R *Ui, const R *Zi, int lvl, int comb, double wF, R *Uo, R *Zo, bool last) {
#pragma clang fp contract(off)
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int le = s * kBtThreads + tid;
                if (le < ne[lvl]) {
                    const uint32_t c = ecw[s];
                    R out = R(0);
                    if ((c >> 30) & 1u) {
                        const int l1 = (int)(c & 0x7fffu), l2 = (int)((c >> 15) & 0x7fffu);
                        const R u = Ui[le];
                        const R z1 = Zi[l1], z2 = Zi[l2];
                        R cor = R(0);
#pragma unroll
                        for (int j = 0; j < kMaxEdges2; ++j) {
                            const int lj = (int)((nbw[s][j >> 1] >> (16 * (j & 1))) & 0xffffu);
                            cor = fmadd(w[s][j], Ui[lj], cor);
                        }
                        const R ru = fmadd(-(g * (z2 - z1)), idc[s], cor) + Gv[s];
                        const R base = comb != COMB_NONE ? U0[le] : R(0);
                        out = combine<R>(comb, base, fmadd(tau, ru, u));
                        if (a.F && le < ne[0]) {
                            const double flux = (double)u * (0.5 * (((double)z1 + H64[l1]) + ((double)z2 + H64[l2])));
                            Fa[s] = fmadd(wF, flux, Fa[s]);
                        }
                    }
                    if (last) uo[ge[s]] = out;
                    else Uo[le] = out;
                }
            }
            if (tid < nc[lvl]) {
                R out = R(0);
                if (cwet) {
                    const R zi = Zi[tid] + Hr[tid];
                    R div = R(0);
#pragma unroll
                    for (int j = 0; j < kMaxEdges; ++j) {
                        const int le = (int)(cen[j] & 0xffffu), ln = (int)(cen[j] >> 16);
                        const R zn = Zi[ln] + Hr[ln];
                        div = fmadd(cd[j], Ui[le] * (R(0.5) * (zi + zn)), div);
                    }
                    const R base = comb != COMB_NONE ? Z0[tid] : R(0);
                    out = combine<R>(comb, base, fmadd(tau, -div, Zi[tid]));
                }
                if (last) zo[gc] = out;
                else Zo[tid] = out;
            }
        };
        if constexpr (kScheme == 3) {
            evaluate(U0, Z0, 2, COMB_NONE, a.w1, U1, Z1, false);
            __syncthreads();
            evaluate(U1, Z1, 1, COMB_34, a.w1, U2, Z2, false);
            __syncthreads();
            evaluate(U2, Z2, 0, COMB_THIRD, a.w3, nullptr, nullptr, true);
        } else {
            evaluate(U0, Z0, 1, COMB_NONE, a.w1, U1, Z1, false);
            __syncthreads();
            evaluate(U1, Z1, 0, COMB_HALF, a.w1, nullptr, nullptr, true);
        }
        if (sub + 1 < nsub) grid_barrier(l.bar, l.gen, l.err, (unsigned)(sub + 1), l.spins);
    }
    if (a.F) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (s * kBtThreads + tid < ne[0]) a.F[ge[s]] = Fa[s];
    }
}

// kDry: the mesh has land or coast edges (see the table loads below).
template <typename R, int kScheme, int KS, bool kDry = false>
__device__ __forceinline__ void bt_substep_body(const BTTileArgs<R> &a, int p) {
#pragma clang fp contract(off)
    extern __shared__ __align__(16) double lds_d[];
    const DevBtTiles &T = a.t;
    const int tid = threadIdx.x;
    const int32_t *rec = T.patch + (size_t)p * kBtRec;
    const int e0 = rec[0], es0 = rec[1], c0 = rec[2], cs0 = rec[3];
    int ne[4], nc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ne[k] = rec[4 + k];
        nc[k] = rec[8 + k];
    }
    constexpr int kIn = kScheme == 3 ? 3 : 2;  // level of the substep input
    const int nEin = ne[kIn], nCin = nc[kIn];
    const int nE1 = ne[kIn - 1], nC1 = nc[kIn - 1];  // level of the first evaluation
    const int se = ne[2], sc = nc[2];                // strides of the stencil tables

    // LDS: H (double) | U0 U1 U2 | Z0 Z1 Z2 | H in R (FP32 state only)
    double *H64 = lds_d;
    R *U0 = reinterpret_cast<R *>(H64 + nc[3]);
    R *U1 = U0 + ne[3];
    R *U2 = U1 + ne[2];
    R *Z0 = U2 + ne[1];
    R *Z1 = Z0 + nc[3];
    R *Z2 = Z1 + nc[2];
    const R *Hr;
    if constexpr (sizeof(R) == 8) {
        Hr = reinterpret_cast<const R *>(H64);
    } else {
        R *h = Z2 + nc[1];
        for (int lc = tid; lc < nCin; lc += kBtThreads) h[lc] = T.cH_f[c0 + lc];
        Hr = h;
    }
    for (int le = tid; le < nEin; le += kBtThreads) U0[le] = a.ua[T.eid[e0 + le]];
    for (int lc = tid; lc < nCin; lc += kBtThreads) {
        Z0[lc] = a.za[T.cid[c0 + lc]];
        H64[lc] = T.cH[c0 + lc];
    }

    // this thread's edges (le = s kBtThreads + tid) and cell (lc = tid)
    constexpr bool kSkipDry = kDry && sizeof(R) == 8;
    const R *__restrict__ wt = BtTab<R>::w(T);
    R w[KS][kMaxEdges2], idc[KS], Gv[KS];
    uint32_t nbw[KS][kMaxEdges2 / 2], ecw[KS];
    double Fa[KS];
    int ge[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int le = s * kBtThreads + tid;
        const bool on = le < nE1;
        const int q = on ? le : 0;
        ecw[s] = on ? T.ec[es0 + q] : 0u;
        ge[s] = T.eid[e0 + q];
        // a coast or land edge keeps a zero velocity and never reads its
        // stencil: on meshes with land, in FP64, its tables are not loaded,
        // which skips their share of the table bytes (level-7 sphere with 30%
        // land: 3.01 -> 2.81 ms per step).  With the FP32 tables the
        // exec-masked loads cost more than they save (2.31 -> 2.46 ms), and on
        // a mesh without land they only add their test, so there every edge
        // loads its row
        const bool wet = !kSkipDry || ((ecw[s] >> 30) & 1u) != 0;
        idc[s] = wet ? BtTab<R>::idc(T)[es0 + q] : R(0);
        Gv[s] = wet ? (R)a.G[ge[s]] : R(0);
#pragma unroll
        for (int j = 0; j < kMaxEdges2; ++j) w[s][j] = wet ? wt[(size_t)kMaxEdges2 * es0 + (size_t)j * se + q] : R(0);
#pragma unroll
        for (int i = 0; i < kMaxEdges2 / 2; ++i)
            nbw[s][i] = wet ? T.enb[(size_t)(kMaxEdges2 / 2) * es0 + (size_t)i * se + q] : 0u;
        Fa[s] = (a.F && le < ne[0]) ? (a.zeroF ? 0.0 : a.F[ge[s]]) : 0.0;
    }
    const bool con = tid < nC1;
    const int qc = con ? tid : 0;
    const bool cwet = con && T.cwet[cs0 + qc] != 0;
    const int gc = T.cid[c0 + qc];
    R cd[kMaxEdges];
    uint32_t cen[kMaxEdges];
#pragma unroll
    for (int j = 0; j < kMaxEdges; ++j) {  // land cells keep zeta = 0 and read no stencil
        const bool ld = !kSkipDry || cwet;
        cd[j] = ld ? BtTab<R>::cd(T)[(size_t)kMaxEdges * cs0 + (size_t)j * sc + qc] : R(0);
        cen[j] = ld ? T.cen[(size_t)kMaxEdges * cs0 + (size_t)j * sc + qc] : 0u;
    }
    __syncthreads();

    const R tau = (R)a.tau, g = (R)a.g;
    // One evaluation producing level lvl from (Ui, Zi); the last one writes the
    // substep output to global memory.
    auto evaluate = [&](const R *Ui, const R *Zi, int lvl, int comb, double wF, R *Uo, R *Zo, bool last) {
#pragma clang fp contract(off)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int le = s * kBtThreads + tid;
            if (le < ne[lvl]) {
                const uint32_t c = ecw[s];
                R out = R(0);
                if ((c >> 30) & 1u) {
                    const int l1 = (int)(c & 0x7fffu), l2 = (int)((c >> 15) & 0x7fffu);
                    const R ua = Ui[le];
                    const R z1 = Zi[l1], z2 = Zi[l2];
                    R cor = R(0);
#pragma unroll
                    for (int j = 0; j < kMaxEdges2; ++j) {
                        const int lj = (int)((nbw[s][j >> 1] >> (16 * (j & 1))) & 0xffffu);
                        cor = fmadd(w[s][j], Ui[lj], cor);
                    }
                    const R ru = fmadd(-(g * (z2 - z1)), idc[s], cor) + Gv[s];
                    const R base = comb != COMB_NONE ? U0[le] : R(0);
                    out = combine<R>(comb, base, fmadd(tau, ru, ua));
                    if (a.F && le < ne[0]) {
                        const double flux = (double)ua * (0.5 * (((double)z1 + H64[l1]) + ((double)z2 + H64[l2])));
                        Fa[s] = fmadd(wF, flux, Fa[s]);
                    }
                }
                if (last) a.uo[ge[s]] = out;
                else Uo[le] = out;
            }
        }
        if (tid < nc[lvl]) {
            R out = R(0);
            if (cwet) {
                const R zi = Zi[tid] + Hr[tid];
                R div = R(0);
#pragma unroll
                for (int j = 0; j < kMaxEdges; ++j) {
                    const int le = (int)(cen[j] & 0xffffu), ln = (int)(cen[j] >> 16);
                    const R zn = Zi[ln] + Hr[ln];
                    div = fmadd(cd[j], Ui[le] * (R(0.5) * (zi + zn)), div);
                }
                const R base = comb != COMB_NONE ? Z0[tid] : R(0);
                out = combine<R>(comb, base, fmadd(tau, -div, Zi[tid]));
            }
            if (last) a.zo[gc] = out;
            else Zo[tid] = out;
        }
    };
    if constexpr (kScheme == 3) {
        evaluate(U0, Z0, 2, COMB_NONE, a.w1, U1, Z1, false);
        __syncthreads();
        evaluate(U1, Z1, 1, COMB_34, a.w1, U2, Z2, false);
        __syncthreads();
        evaluate(U2, Z2, 0, COMB_THIRD, a.w3, nullptr, nullptr, true);
    } else {
        evaluate(U0, Z0, 1, COMB_NONE, a.w1, U1, Z1, false);
        __syncthreads();
        evaluate(U1, Z1, 0, COMB_HALF, a.w1, nullptr, nullptr, true);
    }
    if (a.F) {
#pragma unroll
        for (int s = 0; s < KS; ++s)
            if (s * kBtThreads + tid < ne[0]) a.F[ge[s]] = Fa[s];
    }
}


// ---------------------------------------------------------------------------
// Thickness stage (z-star): h_out = comb(h_n, h_in + dt T^h), zeta = sum h - H
// ---------------------------------------------------------------------------
template <int NK, int Q>
__device__ __forceinline__ void thickness_body(const THArgs &a, int first) {
    const int lane = lane_id();
    const DevMesh &m = a.m;
    if (first >= m.C) return;
    const int L = a.L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    int ci[Q];
    bool has[Q], wet[Q];
    double divF[Q], fr[Q][NK], hin[Q][NK], hb[Q][NK];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        has[q] = first + q < m.C;
        const int i = ci[q] = has[q] ? first + q : first;
        const size_t base = (size_t)i * L;
        wet[q] = m.cmask[i] != 0;
        // Padded stencil slots hold a valid edge with a zero coefficient, so
        // the sum runs its full width and all its loads are in flight together.
        divF[q] = 0.0;
        if (wet[q]) {
#pragma unroll
            for (int j = 0; j < kMaxEdges; ++j)
                divF[q] += m.cell_div[i * kMaxEdges + j] * a.Ftot[m.cell_edges[i * kMaxEdges + j]];
        }
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            fr[q][c] = col_ld(a.frac + base, kk[c]);
            hin[q][c] = col_ld(a.h_in + base, kk[c]);
            hb[q][c] = (a.comb != COMB_NONE) ? col_ld(a.h_n + base, kk[c]) : 0.0;
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!has[q]) continue;
        const int i = ci[q];
        const size_t base = (size_t)i * L;
        double hv[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const double th = wet[q] ? -fr[q][c] * divF[q] : 0.0;
            const double x = hin[q][c] + a.dt * th;
            hv[c] = ok[c] ? combine<double>(a.comb, hb[q][c], x) : 0.0;
            if (ok[c]) col_st(a.h_out + base, kk[c], hv[c]);
            bad |= ok[c] && !isfinite(hv[c]);
        }
        const double sum = col_sum<NK, true>(hv);
        if (lane == 0) a.zeta_out[i] = wet[q] ? sum - m.H[i] : 0.0;
    }
    if (bad && a.nonfinite) *a.nonfinite = 1;
}

// Thickness stage fused with the temperature tracer stage (tracer runs).
template <int NK, typename R>
__device__ __forceinline__ void tracer_body(const TracerArgs<R> &a, int col) {
    const int lane = lane_id();
    const DevMesh &m = a.m;
    const int i = col;
    if (i >= m.C) return;
    const int L = a.L;
    const size_t base = (size_t)i * L;
    const bool wet = m.cmask[i] != 0;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    double hi[NK], Ti[NK], dhv[NK], dhtv[NK], dif[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const double h = a.h_in[base + kk[c]], t = a.T_in[base + kk[c]];
        hi[c] = ok[c] ? h : 0.0;
        Ti[c] = ok[c] ? t : 0.0;
        dhv[c] = dhtv[c] = dif[c] = 0.0;
    }
    if (wet) {
        // padded slots carry zero coefficients
#pragma unroll
        for (int j = 0; j < kMaxEdges; ++j) {
            const int e = m.cell_edges[i * kMaxEdges + j];
            const int nb = m.cell_nbrs[i * kMaxEdges + j];
            const double cd = m.cell_div[i * kMaxEdges + j];
            const double ae = (a.a1 ? a.ca1 * a.a1[e] : 0.0) + (a.uA ? a.uA[e] : 0.0);
            const double ew = m.emask[e] ? 1.0 : 0.0;
            // (T_c2 - T_c1) / d_e seen from this cell
            const double gs = (m.edge_cells[2 * e] == i ? 1.0 : -1.0) * m.inv_dc[e];
            const size_t eb = (size_t)e * L, nbb = (size_t)nb * L;
#pragma unroll
            for (int c = 0; c < NK; ++c) {
                const int k = kk[c];
                const double x1 = (double)a.X1[eb + k], x2 = a.X2 ? (double)a.X2[eb + k] : 0.0;
                const double hn = a.h_in[nbb + k], tn = a.T_in[nbb + k];
                // lanes past the last layer loaded layer L - 1: they carry no flux
                const double on = ok[c] ? ew : 0.0;
                const double u = on * (a.c1 * x1 + a.c2 * x2 + ae);
                const double he = 0.5 * (hi[c] + hn), te = 0.5 * (Ti[c] + tn);
                dhv[c] += cd * (he * u);
                dhtv[c] += cd * (he * te * u);
                dif[c] += cd * (on * (he * a.kappa_h * ((tn - Ti[c]) * gs)));
            }
        }
    }
    // thickness tendency and w at the top of every layer
    double th[NK], w[NK];
    if (a.frac) {
        const double tot = col_sum<NK, kDppFor<R>>(dhv);
        double src[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            th[c] = ok[c] ? -a.frac[base + kk[c]] * tot : 0.0;
            src[c] = ok[c] ? (-dhv[c] - th[c]) : 0.0;
        }
        col_incl_suffix<NK, kDppFor<R>>(src, w);
    } else {
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            th[c] = -dhv[c];
            w[c] = 0.0;
        }
    }
    // vertical fluxes at the interfaces: advective Tbar^t w and diffusive
    // kappa_v (T_{k-1} - T_k) / hbar^t, zero at the surface and the bottom
    double Tu[NK], hu[NK], fa[NK], fd[NK], fan[NK], fdn[NK];
    col_up1<NK, kDppFor<R>>(Ti, Tu);
    col_up1<NK, kDppFor<R>>(hi, hu);
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        const bool inner = k >= 1 && k < L;
        fa[c] = inner ? 0.5 * (Tu[c] + Ti[c]) * w[c] : 0.0;
        fd[c] = inner ? a.kappa_v * ((Tu[c] - Ti[c]) / (0.5 * (hu[c] + hi[c]))) : 0.0;
    }
    col_down1<NK, kDppFor<R>>(fa, fan);
    col_down1<NK, kDppFor<R>>(fd, fdn);
    double hv[NK];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k = lane + c * kWave;
        hv[c] = 0.0;
        if (k < L) {
            const double tend = wet ? (-dhtv[c] - (fa[c] - fan[c]) + dif[c] + (fd[c] - fdn[c])) : 0.0;
            const double x = hi[c] + a.dt * (wet ? th[c] : 0.0);
            const double xt = hi[c] * Ti[c] + a.dt * tend;
            const double hb = a.comb != COMB_NONE ? a.h_n[base + k] : 0.0;
            const double tb = a.comb != COMB_NONE ? a.h_n[base + k] * a.T_n[base + k] : 0.0;
            hv[c] = combine<double>(a.comb, hb, x);
            const double ht = combine<double>(a.comb, tb, xt);
            const double T = wet ? ht / hv[c] : 0.0;
            a.h_out[base + k] = hv[c];
            a.T_out[base + k] = T;
            a.rho_out[base + k] = a.rho0 * (1.0 - a.alpha * (T - a.tref));
            bad |= !isfinite(hv[c]) || !isfinite(T);
        }
    }
    const double s = col_sum<NK, kDppFor<R>>(hv);
    if (lane == 0) a.zeta_out[i] = wet ? s - m.H[i] : 0.0;
    if (bad && a.nonfinite) *a.nonfinite = 1;
}

// Thickness stage (isopycnal): per-layer flux divergence, w = 0.
template <int NK, typename R>
__device__ __forceinline__ void thickness_iso_body(const THIsoArgs<R> &a, int col) {
    const int lane = lane_id();
    const DevMesh &m = a.m;
    const int i = col;
    if (i >= m.C) return;
    const int L = a.L;
    const size_t base = (size_t)i * L;
    const bool wet = m.cmask[i] != 0;
    double hi[NK], div[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        int k = lane + c * kWave;
        hi[c] = (k < L) ? a.h_in[base + k] : 0.0;
        div[c] = 0.0;
    }
    if (wet) {
        const int n = m.cell_nedges[i];
        for (int j = 0; j < n; ++j) {
            const int e = m.cell_edges[i * kMaxEdges + j];
            const int nb = m.cell_nbrs[i * kMaxEdges + j];
            const double cd = m.cell_div[i * kMaxEdges + j];
            const double ae = (a.a1 ? a.ca1 * a.a1[e] : 0.0) + (a.uA ? a.uA[e] : 0.0);
            const bool ew = m.emask[e] != 0;
            const size_t eb = (size_t)e * L, nbb = (size_t)nb * L;
#pragma unroll
            for (int c = 0; c < NK; ++c) {
                int k = lane + c * kWave;
                if (k < L && ew) {
                    double u = a.c1 * (double)a.X1[eb + k] + (a.X2 ? a.c2 * (double)a.X2[eb + k] : 0.0) + ae;
                    double he = 0.5 * (hi[c] + a.h_in[nbb + k]);
                    div[c] += cd * (he * u);
                }
            }
        }
    }
    double hv[NK];
    bool bad = false;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        int k = lane + c * kWave;
        hv[c] = 0.0;
        if (k < L) {
            double x = hi[c] + a.dt * (-div[c]);
            double b = (a.comb != COMB_NONE) ? a.h_n[base + k] : 0.0;
            hv[c] = combine<double>(a.comb, b, x);
            a.h_out[base + k] = hv[c];
            bad |= !isfinite(hv[c]);
        }
    }
    const double s = col_sum<NK, kDppFor<R>>(hv);
    if (lane == 0) a.zeta_out[i] = wet ? s - m.H[i] : 0.0;
    if (bad && a.nonfinite) *a.nonfinite = 1;
}

// ---------------------------------------------------------------------------
// Reconciliation deficits D^e and adjusted total fluxes (Section 3.4)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void recon_body(const ReconArgs &a, int lb) {
    const DevMesh &m = a.m;
    const int e = lb * blockDim.x + threadIdx.x;
    if (e >= m.E) return;
    if (a.ub_half) a.ub_half[e] = 0.75 * a.ub_n[e] + 0.25 * a.ub2[e];
    if (!m.emask[e]) {
        a.Ftot[e] = 0.0;
        if (a.uA) a.uA[e] = 0.0;
        return;
    }
    const double Sh = a.Sh[e];
    double Ftot, uA = 0.0;
    if (a.mode == 0) {
        const double Fh = a.Fh[e];
        if (a.rec) uA = (a.Fz[e] - Fh) / Sh;
        Ftot = Fh + uA * Sh;
    } else if (a.mode == 1) {
        const double P = a.Pp[e] + (a.ub_n[e] + a.ub_new[e]) * Sh;
        if (a.rec) {
            const double f1 = (a.rec == SSE_RECONCILE_EXACT) ? a.Fz1[e] : a.Fh1[e];
            const double f2 = (a.rec == SSE_RECONCILE_EXACT) ? a.Fz2[e] : a.Fh2[e];
            const double Fh3 = (f1 + f2 + 2.0 * P) / 6.0;
            uA = 1.5 * (a.Fz[e] - Fh3) / Sh;
        }
        Ftot = 0.5 * P + uA * Sh;
    } else {
        const double P = a.Pp[e] + a.ub_new[e] * Sh;
        if (a.rec) {
            const double f1 = (a.rec == SSE_RECONCILE_EXACT) ? a.Fz1[e] : a.Fh1[e];
            const double Fh2 = 0.5 * (f1 + P);
            uA = 2.0 * (a.Fz[e] - Fh2) / Sh;
        }
        Ftot = P + uA * Sh;
    }
    a.Ftot[e] = Ftot;
    if (a.uA) a.uA[e] = uA;
}

// ---------------------------------------------------------------------------
// u^{n+1} = ubar^{n+1} + ut^{n+1}; split (BBspl) with h^{n+1}
// ---------------------------------------------------------------------------
template <int NK, typename R, int Q>
__device__ __forceinline__ void assemble_body(const AssembleArgs<R> &a, int first) {
    const int lane = lane_id();
    const DevMesh &m = a.m;
    if (first >= m.E) return;
    const int L = a.L;
    int kk[NK];
    bool ok[NK];
    lane_layers<NK>(L, kk, ok);
    int ei[Q];
    bool has[Q], wet[Q];
    R ub[Q], x[Q][NK];
    double h1[Q][NK], h2[Q][NK];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        has[q] = first + q < m.E;
        const int e = ei[q] = has[q] ? first + q : first;
        wet[q] = m.emask[e] != 0;
        const int c1 = m.edge_cells[2 * e], c2 = m.edge_cells[2 * e + 1];
        ub[q] = (a.ubar_bt && wet[q]) ? (R)a.ubar_bt[e] : R(0);
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            x[q][c] = col_ld(a.X + (size_t)e * L, kk[c]);
            h1[q][c] = col_ld(a.h + (size_t)c1 * L, kk[c]);
            h2[q][c] = col_ld(a.h + (size_t)c2 * L, kk[c]);
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!has[q]) continue;
        const int e = ei[q];
        const size_t base = (size_t)e * L;
        double he[NK], hu[NK];
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const R u = wet[q] ? (a.ubar_bt ? ub[q] + x[q][c] : x[q][c]) : R(0);
            if (ok[c]) col_st(a.U + base, kk[c], u);
            he[c] = ok[c] ? 0.5 * (h1[q][c] + h2[q][c]) : 0.0;
            hu[c] = he[c] * (double)u;
            bad |= ok[c] && !isfinite((double)u);
        }
        const double sh = col_sum<NK, true>(he);
        const double shu = col_sum<NK, true>(hu);
        if (lane == 0) a.ubar[e] = wet[q] ? shu / sh : 0.0;
    }
    if (bad && a.nonfinite) *a.nonfinite = 1;
}

template <int NK>
__global__ void __launch_bounds__(1024) zeta_kernel(DevMesh m, int L, const double *h, double *zeta) {
    const int lane = lane_id();
    const int i = column_id(m.C);
    if (i >= m.C) return;
    double hv[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        int k = lane + c * kWave;
        hv[c] = (k < L) ? h[(size_t)i * L + k] : 0.0;
    }
    const double s = col_sum<NK, true>(hv);
    if (lane == 0) zeta[i] = m.cmask[i] ? s - m.H[i] : 0.0;
}

// F_e = sum_k h_e (X_k + uA_e)
template <int NK, typename R>
__global__ void __launch_bounds__(1024) edge_flux_sum_kernel(DevMesh m, int L, const double *h, const R *X,
                                                               const double *uA, double *F) {
    const int lane = lane_id();
    const int e = column_id(m.E);
    if (e >= m.E) return;
    const int c1 = m.edge_cells[2 * e], c2 = m.edge_cells[2 * e + 1];
    const double ua = uA ? uA[e] : 0.0;
    double f[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        int k = lane + c * kWave;
        f[c] = 0.0;
        if (k < L) {
            double he = 0.5 * (h[(size_t)c1 * L + k] + h[(size_t)c2 * L + k]);
            f[c] = he * ((double)X[(size_t)e * L + k] + ua);
        }
    }
    const double s = col_sum<NK, true>(f);
    if (lane == 0) F[e] = m.emask[e] ? s : 0.0;
}

template <typename Tin, typename Tout>
__device__ __forceinline__ void convert_body(const ConvArgs<Tin, Tout> &a, int lb) {
    const size_t i = (size_t)lb * blockDim.x + threadIdx.x;
    if (i < a.n) a.dst[i] = (Tout)a.src[i];
}

// ---------------------------------------------------------------------------
// Entry points.  Every kernel body above runs either from a single-state
// wrapper (the kernel arguments hold the state's argument block) or from a
// batched wrapper: one launch over the workgroups of several states, where
// each workgroup reads its (member, block) pair from a device table and the
// member's argument block from device memory.
// ---------------------------------------------------------------------------

// The single-state launches of the light streaming column kernels (vertex,
// thickness, assembly, Laplacian and divergence passes) give every wavefront
// several consecutive columns and issue all their loads before any
// arithmetic: the wavefront then has several times the loads in flight,
// which these kernels need to reach HBM rates.  Measured per 3 C1 steps,
// FP64 / mixed, one column against two: vertex pass 1.44 -> 1.19 / 1.23 ->
// 0.89 ms, thickness 1.35 -> 1.14 ms, assembly and reconciliation 1.06 ->
// 0.93 ms; two against four: vertex 1.19 / 1.13, assembly 0.92 / 0.81,
// thickness 1.15 / 1.24.  The cell pass, with 13 columns per cell, lost
// occupancy with two cells (65 VGPRs, 106 scalar registers) and ran 5%
// slower, so it keeps one.  (Processing the columns one after the other
// instead made these kernels slower.)  Batched launches take the same
// groups (their workgroup tables count groups of columns); the arithmetic
// per column is the same in every form.  The counts are in sse_kernels.h.

// (member, member-local block) of this workgroup in a batched launch, with
// the same XCD renumbering as the single-state launches.
__device__ __forceinline__ bool batch_entry(const int2 *table, int blocks, int2 &ent) {
    const int lb = xcd_block(blocks);
    if (lb < 0) return false;
    const int2 t = table[lb];
    ent.x = __builtin_amdgcn_readfirstlane(t.x);
    ent.y = __builtin_amdgcn_readfirstlane(t.y);
    return true;
}

__device__ __forceinline__ int batch_column(int local_block) {
    return __builtin_amdgcn_readfirstlane(local_block * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6));
}

template <int NK, typename R, bool kAdd>
__global__ void __launch_bounds__(1024) fe_cell_kernel(FECellArgs<R> a) {
    fe_cell_body<NK, R, kAdd>(a, column_id(a.m.C));
}
template <int NK, typename R, bool kAdd>
__global__ void __launch_bounds__(1024) fe_cell_batch(BatchLaunch<FECellArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) fe_cell_body<NK, R, kAdd>(b.args[t.x], batch_column(t.y));
}

template <int NK, typename R, bool kAdd>
__global__ void __launch_bounds__(1024) fe_vertex_kernel(FEVertexArgs<R> a) {
    fe_vertex_body<NK, R, kAdd, kVertexCols>(a, kVertexCols * column_id(wave_groups<kVertexCols>(a.m.V)));
}
template <int NK, typename R, bool kAdd>
__global__ void __launch_bounds__(1024) fe_vertex_batch(BatchLaunch<FEVertexArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t))
        fe_vertex_body<NK, R, kAdd, kVertexCols>(b.args[t.x], kVertexCols * batch_column(t.y));
}

// Minimum waves per SIMD requested for the one-register-chunk edge pass.
// Left alone the compiler settles at 79-81 VGPRs (5-6 waves); the
// gather-bound pass runs faster with more loads in flight.  With 64-bit
// column bases the best request was 7 (C1 edge-pass time over 3 steps, FP64:
// none 12.1, 5: 11.2, 6: 11.6, 7: 10.8, 8: 11.4 ms).  With 32-bit scalar
// column offsets and DPP lane moves the pass fits 8 waves (57-63 VGPRs, 78
// SGPRs, no scratch): FP64 9.78 -> 9.65 ms, C1 mixed 6.03 -> 5.94 ms/step.
// The variants with the implicit vertical-mixing solve (kVar bit 1) hold
// its tridiagonal operands as well and run better at 7 (C1 with mixing 8.68
// -> 8.57 ms/step; the biharmonic variant gains nothing from 7).
template <int NK, typename R, int kVar>
constexpr int edge_min_waves() { return NK != 1 ? kEdge2Waves : (kVar & 2) ? 7 : 8; }
// The two-chunk pass (L > 64) holds twice the operands per lane; with
// workgroups of at most kEdge2MaxCols wavefronts its launch bound lets the
// compiler keep them in registers instead of scratch.
template <int NK>
constexpr int edge_max_threads() { return NK == 1 ? 1024 : kEdge2MaxCols * kWave; }

template <int NK, typename R>
__global__ void __launch_bounds__(1024) tracer_kernel(TracerArgs<R> a) { tracer_body<NK, R>(a, column_id(a.m.C)); }
template <int NK, typename R>
__global__ void __launch_bounds__(1024) tracer_batch(BatchLaunch<TracerArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) tracer_body<NK, R>(b.args[t.x], batch_column(t.y));
}

template <int NK, typename R>
__global__ void __launch_bounds__(1024) lap_kernel(LapArgs<R> a) {
    lap_body<NK, R, kLapCols>(a, kLapCols * column_id(wave_groups<kLapCols>(a.m.E)));
}
template <int NK, typename R>
__global__ void __launch_bounds__(1024) lap_batch(BatchLaunch<LapArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) lap_body<NK, R, kLapCols>(b.args[t.x], kLapCols * batch_column(t.y));
}
template <int NK, typename R>
__global__ void __launch_bounds__(1024) div_kernel(DivArgs<R> a) {
    div_body<NK, R, kDivCols>(a, kDivCols * column_id(wave_groups<kDivCols>(a.m.C)));
}
template <int NK, typename R>
__global__ void __launch_bounds__(1024) div_batch(BatchLaunch<DivArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) div_body<NK, R, kDivCols>(b.args[t.x], kDivCols * batch_column(t.y));
}

template <int NK, typename R, bool kAdd, int kVar>
__global__ void __launch_bounds__(edge_max_threads<NK>(), (edge_min_waves<NK, R, kVar>())) fe_edge_kernel(FEEdgeArgs<R> a) {
    fe_edge_body<NK, R, kAdd, kVar>(a, column_id(a.m.E));
}
template <int NK, typename R, bool kAdd, int kVar>
__global__ void __launch_bounds__(edge_max_threads<NK>(), (edge_min_waves<NK, R, kVar>())) fe_edge_batch(BatchLaunch<FEEdgeArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) fe_edge_body<NK, R, kAdd, kVar>(b.args[t.x], batch_column(t.y));
}

template <int NK>
__global__ void __launch_bounds__(1024) thickness_kernel(THArgs a) {
    thickness_body<NK, kThickCols>(a, kThickCols * column_id(wave_groups<kThickCols>(a.m.C)));
}
template <int NK>
__global__ void __launch_bounds__(1024) thickness_batch(BatchLaunch<THArgs> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) thickness_body<NK, kThickCols>(b.args[t.x], kThickCols * batch_column(t.y));
}

template <int NK, typename R>
__global__ void __launch_bounds__(1024) thickness_iso_kernel(THIsoArgs<R> a) { thickness_iso_body<NK, R>(a, column_id(a.m.C)); }
template <int NK, typename R>
__global__ void __launch_bounds__(1024) thickness_iso_batch(BatchLaunch<THIsoArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) thickness_iso_body<NK, R>(b.args[t.x], batch_column(t.y));
}

template <int NK, typename R>
__global__ void __launch_bounds__(1024) assemble_kernel(AssembleArgs<R> a) {
    assemble_body<NK, R, kAssembleCols>(a, kAssembleCols * column_id(wave_groups<kAssembleCols>(a.m.E)));
}
template <int NK, typename R>
__global__ void __launch_bounds__(1024) assemble_batch(BatchLaunch<AssembleArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t))
        assemble_body<NK, R, kAssembleCols>(b.args[t.x], kAssembleCols * batch_column(t.y));
}

// Barotropic evaluation: XCD x owns edge blocks [x pe, (x + 1) pe) and cell
// blocks [x pc, (x + 1) pc), one contiguous region of the mesh per L2.
template <typename R, bool kD16>
__global__ void __launch_bounds__(1024) bt_eval_kernel(BTEvalArgs<R> a, int nEdgeBlocks, int nCellBlocks) {
    const int pe = (nEdgeBlocks + kXcd - 1) / kXcd, pc = (nCellBlocks + kXcd - 1) / kXcd;
    const int x = blockIdx.x % kXcd, local = blockIdx.x / kXcd;
    if (local < pe) {
        const int lb = x * pe + local;
        if (lb < nEdgeBlocks) bt_eval_body<R, kD16>(a, true, lb);
    } else {
        const int lb = x * pc + (local - pe);
        if (lb < nCellBlocks) bt_eval_body<R, kD16>(a, false, lb);
    }
}
template <typename R, bool kD16>
__global__ void __launch_bounds__(1024) bt_eval_batch(BatchLaunch<BTEvalArgs<R>> b) {
    int2 t;
    if (!batch_entry(b.table, b.blocks, t)) return;
    const BTEvalArgs<R> &a = b.args[t.x];
    const int nEB = (a.m.E + (int)blockDim.x - 1) / (int)blockDim.x;
    if (t.y < nEB)
        bt_eval_body<R, kD16>(a, true, t.y);
    else
        bt_eval_body<R, kD16>(a, false, t.y - nEB);
}

template <typename R, int kScheme, int KS, bool kDry = false>
__global__ void __launch_bounds__(kBtThreads, kBtWavesPerSimd) bt_substep_kernel(BTTileArgs<R> a) {
    const int p = xcd_block(a.t.nP);
    if (p >= 0) bt_substep_body<R, kScheme, KS, kDry>(a, p);
}
// Batched: one workgroup per (member, patch); the dynamic LDS is the
// largest member's.
template <typename R, int kScheme, int KS>
__global__ void __launch_bounds__(kBtThreads, kBtWavesPerSimd) bt_substep_batch(BatchLaunch<BTTileArgs<R>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) bt_substep_body<R, kScheme, KS>(b.args[t.x], t.y);
}

// The whole barotropic loop in one cooperative launch, one workgroup per
// patch (workgroups past the last patch only take part in the barriers).
template <typename R, int kScheme, int KS>
__global__ void __launch_bounds__(kBtThreads, kBtWavesPerSimd) bt_loop_kernel(BTTileArgs<R> a, BtLoop<R> l) {
    bt_loop_body<R, kScheme, KS>(a, l, xcd_block(a.t.nP));
}

__global__ void __launch_bounds__(64) bt_loop_reset_kernel(unsigned *bar, unsigned *gen) {
    if (threadIdx.x == 0) {
        *bar = 0u;
        *gen = 0u;
    }
}

__global__ void __launch_bounds__(1024) recon_kernel(ReconArgs a) { recon_body(a, blockIdx.x); }
__global__ void __launch_bounds__(1024) recon_batch(BatchLaunch<ReconArgs> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) recon_body(b.args[t.x], t.y);
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(1024) convert_kernel(ConvArgs<Tin, Tout> a) { convert_body<Tin, Tout>(a, blockIdx.x); }
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(1024) convert_batch(BatchLaunch<ConvArgs<Tin, Tout>> b) {
    int2 t;
    if (batch_entry(b.table, b.blocks, t)) convert_body<Tin, Tout>(b.args[t.x], t.y);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
bool geom_valid(const Geom &g) {
    const int c = g.cols_per_block;
    return (c == 1 || c == 2 || c == 4 || c == 8 || c == 16) && g.block_2d >= 64 && g.block_2d <= 1024 &&
           g.block_2d % 64 == 0;
}
int col_blocks(int n, const Geom &g) { return (n + g.cols_per_block - 1) / g.cols_per_block; }
Geom edge_geom(const Geom &g, int nk) {
    Geom e = g;
    if (nk == 2 && e.cols_per_block > kEdge2MaxCols) e.cols_per_block = kEdge2MaxCols;
    return e;
}
int flat_blocks(size_t n, const Geom &g) { return (int)((n + g.block_2d - 1) / g.block_2d); }
int bt_blocks(int E, int C, const Geom &g) { return flat_blocks(E, g) + flat_blocks(C, g); }

// Grids are rounded up to a multiple of the 8 XCDs; the kernels renumber the
// workgroups and the padding workgroups exit.
static inline dim3 xcd_grid(int nb) { return dim3((unsigned)(kXcd * ((nb + kXcd - 1) / kXcd))); }
static inline dim3 col_block(const Geom &g) { return dim3((unsigned)(kWave * g.cols_per_block)); }

// The column kernels are instantiated for one or two register chunks
// (L <= 64 or L <= 128) and for the two velocity forms: u = X + ubar
// (ubar_add non-null) or u = X (the edge pass then forms ut = X - ubar_sub;
// exactly one of ubar_add and ubar_sub is non-null there).
#define SSE_NK_ADD(NK2, ADD, KERNEL, GRID, BLOCK, ARG)                                  \
    do {                                                                               \
        if (!(NK2)) {                                                                  \
            if (ADD) KERNEL<1, R, true><<<GRID, BLOCK, 0, s>>>(ARG);                   \
            else KERNEL<1, R, false><<<GRID, BLOCK, 0, s>>>(ARG);                      \
        } else {                                                                       \
            if (ADD) KERNEL<2, R, true><<<GRID, BLOCK, 0, s>>>(ARG);                   \
            else KERNEL<2, R, false><<<GRID, BLOCK, 0, s>>>(ARG);                      \
        }                                                                              \
    } while (0)

template <typename R>
void launch_fe_cell(const FECellArgs<R> &a, const Geom &g, hipStream_t s) {
    SSE_NK_ADD(a.L > kWave, a.ubar_add != nullptr, fe_cell_kernel, xcd_grid(col_blocks(a.m.C, g)), col_block(g), a);
}
template <typename R>
void launch_fe_vertex(const FEVertexArgs<R> &a, const Geom &g, hipStream_t s) {
    SSE_NK_ADD(a.L > kWave, a.ubar_add != nullptr, fe_vertex_kernel, xcd_grid(col_blocks(wave_groups<kVertexCols>(a.m.V), g)), col_block(g), a);
}
// The edge pass has a fourth template parameter, the variant: bit 0 for
// canonical stencils with vertex chains (the mesh's chain flag), bit 1 for
// implicit vertical mixing (the state's vmix parameter), bit 2 for the
// biharmonic viscosity (hdiff).  Every member of a batched launch shares it.
#define SSE_NK_ADD_V(NK2, ADD, V, KERNEL, GRID, BLOCK, ARG)                             \
    do {                                                                               \
        if (!(NK2)) {                                                                  \
            if (ADD) KERNEL<1, R, true, V><<<GRID, BLOCK, 0, s>>>(ARG);                \
            else KERNEL<1, R, false, V><<<GRID, BLOCK, 0, s>>>(ARG);                   \
        } else {                                                                       \
            if (ADD) KERNEL<2, R, true, V><<<GRID, BLOCK, 0, s>>>(ARG);                \
            else KERNEL<2, R, false, V><<<GRID, BLOCK, 0, s>>>(ARG);                   \
        }                                                                              \
    } while (0)
#define SSE_NK_ADD_VAR(NK2, ADD, VAR, KERNEL, GRID, BLOCK, ARG)                         \
    do {                                                                               \
        switch (VAR) {                                                                 \
            case 0: SSE_NK_ADD_V(NK2, ADD, 0, KERNEL, GRID, BLOCK, ARG); break;        \
            case 1: SSE_NK_ADD_V(NK2, ADD, 1, KERNEL, GRID, BLOCK, ARG); break;        \
            case 2: SSE_NK_ADD_V(NK2, ADD, 2, KERNEL, GRID, BLOCK, ARG); break;        \
            case 3: SSE_NK_ADD_V(NK2, ADD, 3, KERNEL, GRID, BLOCK, ARG); break;        \
            case 4: SSE_NK_ADD_V(NK2, ADD, 4, KERNEL, GRID, BLOCK, ARG); break;        \
            case 5: SSE_NK_ADD_V(NK2, ADD, 5, KERNEL, GRID, BLOCK, ARG); break;        \
            case 6: SSE_NK_ADD_V(NK2, ADD, 6, KERNEL, GRID, BLOCK, ARG); break;        \
            case 7: SSE_NK_ADD_V(NK2, ADD, 7, KERNEL, GRID, BLOCK, ARG); break;        \
            case 8: SSE_NK_ADD_V(NK2, ADD, 8, KERNEL, GRID, BLOCK, ARG); break;        \
            case 9: SSE_NK_ADD_V(NK2, ADD, 9, KERNEL, GRID, BLOCK, ARG); break;        \
            case 10: SSE_NK_ADD_V(NK2, ADD, 10, KERNEL, GRID, BLOCK, ARG); break;      \
            case 11: SSE_NK_ADD_V(NK2, ADD, 11, KERNEL, GRID, BLOCK, ARG); break;      \
            case 12: SSE_NK_ADD_V(NK2, ADD, 12, KERNEL, GRID, BLOCK, ARG); break;      \
            case 13: SSE_NK_ADD_V(NK2, ADD, 13, KERNEL, GRID, BLOCK, ARG); break;      \
            case 14: SSE_NK_ADD_V(NK2, ADD, 14, KERNEL, GRID, BLOCK, ARG); break;      \
            default: SSE_NK_ADD_V(NK2, ADD, 15, KERNEL, GRID, BLOCK, ARG); break;      \
        }                                                                              \
    } while (0)

template <typename R>
void launch_tracer(const TracerArgs<R> &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(a.m.C, g)), block = col_block(g);
    if (a.L <= kWave) tracer_kernel<1, R><<<grid, block, 0, s>>>(a);
    else tracer_kernel<2, R><<<grid, block, 0, s>>>(a);
}
template <typename R>
void launch_tracer_batch(const BatchLaunch<TracerArgs<R>> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) tracer_batch<1, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else tracer_batch<2, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}

template <typename R>
void launch_lap(const LapArgs<R> &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(wave_groups<kLapCols>(a.m.E), g)), block = col_block(g);
    if (a.L <= kWave) lap_kernel<1, R><<<grid, block, 0, s>>>(a);
    else lap_kernel<2, R><<<grid, block, 0, s>>>(a);
}
template <typename R>
void launch_div(const DivArgs<R> &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(wave_groups<kDivCols>(a.m.C), g)), block = col_block(g);
    if (a.L <= kWave) div_kernel<1, R><<<grid, block, 0, s>>>(a);
    else div_kernel<2, R><<<grid, block, 0, s>>>(a);
}
template <typename R>
void launch_lap_batch(const BatchLaunch<LapArgs<R>> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) lap_batch<1, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else lap_batch<2, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}
template <typename R>
void launch_div_batch(const BatchLaunch<DivArgs<R>> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) div_batch<1, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else div_batch<2, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}

int fe_edge_variant(const DevMesh &m, int L, int vmix, bool del4) {
    // 32-bit column offsets cover every array the pass reads while the
    // largest (edges, vertices or cells) x L x 8 bytes stays below 4 GiB,
    // with a margin for the layer offsets
    const size_t n = (size_t)std::max(m.E, std::max(m.V, m.C));
    const bool wide = n * (size_t)L * 8 + 4096 > ((size_t)1 << 32);
    return (m.chain ? 1 : 0) | (vmix ? 2 : 0) | (del4 ? 4 : 0) | (wide ? 8 : 0);
}

template <typename R>
void launch_fe_edge(const FEEdgeArgs<R> &a, const Geom &g0, hipStream_t s, bool wide) {
    const int var = fe_edge_variant(a.m, a.L, a.vmix, a.D2 != nullptr) | (wide ? 8 : 0);
    const Geom g = edge_geom(g0, a.L > kWave ? 2 : 1);
    SSE_NK_ADD_VAR(a.L > kWave, a.ubar_add != nullptr, var, fe_edge_kernel, xcd_grid(col_blocks(a.m.E, g)), col_block(g), a);
}
template <typename R>
void launch_fe_cell_batch(const BatchLaunch<FECellArgs<R>> &b, int nk, bool add, const Geom &g, hipStream_t s) {
    SSE_NK_ADD(nk == 2, add, fe_cell_batch, xcd_grid(b.blocks), col_block(g), b);
}
template <typename R>
void launch_fe_vertex_batch(const BatchLaunch<FEVertexArgs<R>> &b, int nk, bool add, const Geom &g, hipStream_t s) {
    SSE_NK_ADD(nk == 2, add, fe_vertex_batch, xcd_grid(b.blocks), col_block(g), b);
}
template <typename R>
void launch_fe_edge_batch(const BatchLaunch<FEEdgeArgs<R>> &b, int nk, bool add, int var, const Geom &g,
                          hipStream_t s) {
    SSE_NK_ADD_VAR(nk == 2, add, var, fe_edge_batch, xcd_grid(b.blocks), col_block(edge_geom(g, nk)), b);
}

template <typename R>
void launch_edge_gathers(const FEEdgeArgs<R> &a, const Geom &g0, hipStream_t s) {
    const Geom g = edge_geom(g0, 1);
    edge_gather_kernel<R><<<xcd_grid(col_blocks(a.m.E, g)), col_block(g), 0, s>>>(a);
}

template <typename R>
void launch_fe_edge_tiled(const FEEdgeArgs<R> &a, const DevTiles &t, hipStream_t s) {
    const size_t lds = fe_edge_tiled_lds<R>(t, a.L);
    const dim3 grid(kXcd * ((t.nT + kXcd - 1) / kXcd)), block((t.T < kTileWaves ? t.T : kTileWaves) * kWave);
    const bool add = a.ubar_add != nullptr;
    const int v = a.vmix ? 1 : 0;
#define SSE_TILED(NK_, ADD_, MIX_) fe_edge_tiled_kernel<NK_, R, ADD_, MIX_><<<grid, block, lds, s>>>(a, t)
    if (a.L <= kWave) {
        if (add) { if (v) SSE_TILED(1, true, true); else SSE_TILED(1, true, false); }
        else { if (v) SSE_TILED(1, false, true); else SSE_TILED(1, false, false); }
    } else {
        if (add) { if (v) SSE_TILED(2, true, true); else SSE_TILED(2, true, false); }
        else { if (v) SSE_TILED(2, false, true); else SSE_TILED(2, false, false); }
    }
#undef SSE_TILED
}

template <typename R, int kScheme, int KS>
static const void *bt_loop_fn() {
    return reinterpret_cast<const void *>(bt_loop_kernel<R, kScheme, KS>);
}

template <typename R>
static const void *bt_loop_select(int scheme, int ks) {
    if (scheme == 3) return ks == 1 ? bt_loop_fn<R, 3, 1>() : bt_loop_fn<R, 3, 2>();
    return ks == 1 ? bt_loop_fn<R, 2, 1>() : bt_loop_fn<R, 2, 2>();
}

// Allow the tiled kernels the device's full LDS per workgroup.
void set_tiled_lds_limit(size_t bytes) {
#define SSE_TILED_FN(NK_, R_, ADD_, MIX_) reinterpret_cast<const void *>(fe_edge_tiled_kernel<NK_, R_, ADD_, MIX_>)
#define SSE_TILED_FNS(R_, MIX_)                                                                            \
    SSE_TILED_FN(1, R_, true, MIX_), SSE_TILED_FN(1, R_, false, MIX_), SSE_TILED_FN(2, R_, true, MIX_), \
        SSE_TILED_FN(2, R_, false, MIX_)
    const void *fns[] = {SSE_TILED_FNS(double, false), SSE_TILED_FNS(double, true), SSE_TILED_FNS(float, false),
                         SSE_TILED_FNS(float, true)};
#undef SSE_TILED_FNS
#undef SSE_TILED_FN
    const void *bt[] = {reinterpret_cast<const void *>(bt_substep_kernel<double, 3, 1>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 3, 2>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 2, 1>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 2, 2>),
                        reinterpret_cast<const void *>(bt_substep_kernel<float, 3, 1>),
                        reinterpret_cast<const void *>(bt_substep_kernel<float, 3, 2>),
                        reinterpret_cast<const void *>(bt_substep_kernel<float, 2, 1>),
                        reinterpret_cast<const void *>(bt_substep_kernel<float, 2, 2>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 3, 1, true>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 3, 2, true>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 2, 1, true>),
                        reinterpret_cast<const void *>(bt_substep_kernel<double, 2, 2, true>)};
    for (const void *f : bt) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    const void *btb[] = {reinterpret_cast<const void *>(bt_substep_batch<double, 3, 1>),
                         reinterpret_cast<const void *>(bt_substep_batch<double, 3, 2>),
                         reinterpret_cast<const void *>(bt_substep_batch<double, 2, 1>),
                         reinterpret_cast<const void *>(bt_substep_batch<double, 2, 2>),
                         reinterpret_cast<const void *>(bt_substep_batch<float, 3, 1>),
                         reinterpret_cast<const void *>(bt_substep_batch<float, 3, 2>),
                         reinterpret_cast<const void *>(bt_substep_batch<float, 2, 1>),
                         reinterpret_cast<const void *>(bt_substep_batch<float, 2, 2>)};
    for (const void *f : btb) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    const void *btl[] = {bt_loop_fn<double, 3, 1>(), bt_loop_fn<double, 3, 2>(), bt_loop_fn<double, 2, 1>(),
                         bt_loop_fn<double, 2, 2>(), bt_loop_fn<float, 3, 1>(),  bt_loop_fn<float, 3, 2>(),
                         bt_loop_fn<float, 2, 1>(),  bt_loop_fn<float, 2, 2>()};
    for (const void *f : btl) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    for (const void *f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R>
void launch_bt_substep(const BTTileArgs<R> &a, int scheme, hipStream_t s) {
    const dim3 grid = xcd_grid(a.t.nP), block(kBtThreads);
    const size_t lds = sizeof(R) == 8 ? a.t.lds_d : a.t.lds_f;
    if (sizeof(R) == 8 && a.t.dry) {
        if (scheme == 3) {
            if (a.t.ks == 1) bt_substep_kernel<R, 3, 1, true><<<grid, block, lds, s>>>(a);
            else bt_substep_kernel<R, 3, 2, true><<<grid, block, lds, s>>>(a);
        } else {
            if (a.t.ks == 1) bt_substep_kernel<R, 2, 1, true><<<grid, block, lds, s>>>(a);
            else bt_substep_kernel<R, 2, 2, true><<<grid, block, lds, s>>>(a);
        }
    } else if (scheme == 3) {
        if (a.t.ks == 1) bt_substep_kernel<R, 3, 1><<<grid, block, lds, s>>>(a);
        else bt_substep_kernel<R, 3, 2><<<grid, block, lds, s>>>(a);
    } else {
        if (a.t.ks == 1) bt_substep_kernel<R, 2, 1><<<grid, block, lds, s>>>(a);
        else bt_substep_kernel<R, 2, 2><<<grid, block, lds, s>>>(a);
    }
}

template <typename R>
int bt_loop_capacity(const DevBtTiles &t, int scheme) {
    if (t.nP <= 0) return 0;
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const size_t lds = sizeof(R) == 8 ? t.lds_d : t.lds_f;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bt_loop_select<R>(scheme, t.ks), kBtThreads, lds) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

template <typename R>
hipError_t launch_bt_loop(const BTTileArgs<R> &a, const BtLoop<R> &l, int scheme, hipStream_t s) {
    bt_loop_reset_kernel<<<1, 64, 0, s>>>(l.bar, l.gen);
    const size_t lds = sizeof(R) == 8 ? a.t.lds_d : a.t.lds_f;
    BTTileArgs<R> aa = a;
    BtLoop<R> ll = l;
    void *args[] = {&aa, &ll};
    return hipLaunchCooperativeKernel(bt_loop_select<R>(scheme, a.t.ks), xcd_grid(a.t.nP), dim3(kBtThreads), args,
                                      (unsigned)lds, s);
}

template <typename R>
void launch_bt_substep_batch(const BatchLaunch<BTTileArgs<R>> &b, int scheme, int ks, size_t lds, hipStream_t s) {
    const dim3 grid = xcd_grid(b.blocks), block(kBtThreads);
    if (scheme == 3) {
        if (ks == 1) bt_substep_batch<R, 3, 1><<<grid, block, lds, s>>>(b);
        else bt_substep_batch<R, 3, 2><<<grid, block, lds, s>>>(b);
    } else {
        if (ks == 1) bt_substep_batch<R, 2, 1><<<grid, block, lds, s>>>(b);
        else bt_substep_batch<R, 2, 2><<<grid, block, lds, s>>>(b);
    }
}

template <typename R>
void launch_bt_eval(const BTEvalArgs<R> &a, const Geom &g, hipStream_t s) {
    const int nEB = flat_blocks(a.m.E, g), nCB = flat_blocks(a.m.C, g);
    const int per = (nEB + kXcd - 1) / kXcd + (nCB + kXcd - 1) / kXcd;
    if (a.m.delta16)
        bt_eval_kernel<R, true><<<dim3(kXcd * per), g.block_2d, 0, s>>>(a, nEB, nCB);
    else
        bt_eval_kernel<R, false><<<dim3(kXcd * per), g.block_2d, 0, s>>>(a, nEB, nCB);
}
template <typename R>
void launch_bt_eval_batch(const BatchLaunch<BTEvalArgs<R>> &b, bool delta16, const Geom &g, hipStream_t s) {
    if (delta16)
        bt_eval_batch<R, true><<<xcd_grid(b.blocks), g.block_2d, 0, s>>>(b);
    else
        bt_eval_batch<R, false><<<xcd_grid(b.blocks), g.block_2d, 0, s>>>(b);
}

void launch_thickness(const THArgs &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(wave_groups<kThickCols>(a.m.C), g));
    if (a.L <= kWave) thickness_kernel<1><<<grid, col_block(g), 0, s>>>(a);
    else thickness_kernel<2><<<grid, col_block(g), 0, s>>>(a);
}
void launch_thickness_batch(const BatchLaunch<THArgs> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) thickness_batch<1><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else thickness_batch<2><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}
template <typename R>
void launch_thickness_iso(const THIsoArgs<R> &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(a.m.C, g));
    if (a.L <= kWave) thickness_iso_kernel<1, R><<<grid, col_block(g), 0, s>>>(a);
    else thickness_iso_kernel<2, R><<<grid, col_block(g), 0, s>>>(a);
}
template <typename R>
void launch_thickness_iso_batch(const BatchLaunch<THIsoArgs<R>> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) thickness_iso_batch<1, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else thickness_iso_batch<2, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}
template <typename R>
void launch_assemble(const AssembleArgs<R> &a, const Geom &g, hipStream_t s) {
    const dim3 grid = xcd_grid(col_blocks(wave_groups<kAssembleCols>(a.m.E), g));
    if (a.L <= kWave) assemble_kernel<1, R><<<grid, col_block(g), 0, s>>>(a);
    else assemble_kernel<2, R><<<grid, col_block(g), 0, s>>>(a);
}
template <typename R>
void launch_assemble_batch(const BatchLaunch<AssembleArgs<R>> &b, int nk, const Geom &g, hipStream_t s) {
    if (nk == 1) assemble_batch<1, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
    else assemble_batch<2, R><<<xcd_grid(b.blocks), col_block(g), 0, s>>>(b);
}
void launch_zeta_from_h(const DevMesh &m, int L, const double *h, double *zeta, hipStream_t s) {
    const dim3 grid = xcd_grid((m.C + 3) / 4);
    if (L <= kWave) zeta_kernel<1><<<grid, 256, 0, s>>>(m, L, h, zeta);
    else zeta_kernel<2><<<grid, 256, 0, s>>>(m, L, h, zeta);
}
template <typename R>
void launch_edge_flux_sum(const DevMesh &m, int L, const double *h, const R *X, const double *uA, double *F,
                          hipStream_t s) {
    const dim3 grid = xcd_grid((m.E + 3) / 4);
    if (L <= kWave) edge_flux_sum_kernel<1, R><<<grid, 256, 0, s>>>(m, L, h, X, uA, F);
    else edge_flux_sum_kernel<2, R><<<grid, 256, 0, s>>>(m, L, h, X, uA, F);
}
__global__ void permute_kernel(const double *__restrict__ src, const int32_t *__restrict__ idx,
                               double *__restrict__ dst, int n, int scatter) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = idx[i];
    if (scatter) dst[j] = src[i];
    else dst[i] = src[j];
}
void launch_permute(const double *src, const int32_t *idx, double *dst, int n, bool scatter, const Geom &g,
                    hipStream_t s) {
    if (n > 0) permute_kernel<<<flat_blocks((size_t)n, g), g.block_2d, 0, s>>>(src, idx, dst, n, scatter ? 1 : 0);
}
void launch_recon(const ReconArgs &a, const Geom &g, hipStream_t s) {
    recon_kernel<<<flat_blocks(a.m.E, g), g.block_2d, 0, s>>>(a);
}
void launch_recon_batch(const BatchLaunch<ReconArgs> &b, const Geom &g, hipStream_t s) {
    recon_batch<<<xcd_grid(b.blocks), g.block_2d, 0, s>>>(b);
}
template <typename Tin, typename Tout>
void launch_convert(const ConvArgs<Tin, Tout> &a, const Geom &g, hipStream_t s) {
    if (a.n) convert_kernel<Tin, Tout><<<flat_blocks(a.n, g), g.block_2d, 0, s>>>(a);
}
template <typename Tin, typename Tout>
void launch_convert_batch(const BatchLaunch<ConvArgs<Tin, Tout>> &b, const Geom &g, hipStream_t s) {
    convert_batch<Tin, Tout><<<xcd_grid(b.blocks), g.block_2d, 0, s>>>(b);
}

#define SSE_INSTANTIATE(R)                                                                                   \
    template void launch_fe_cell<R>(const FECellArgs<R> &, const Geom &, hipStream_t);                     \
    template void launch_fe_vertex<R>(const FEVertexArgs<R> &, const Geom &, hipStream_t);                 \
    template void launch_lap<R>(const LapArgs<R> &, const Geom &, hipStream_t);                           \
    template void launch_tracer<R>(const TracerArgs<R> &, const Geom &, hipStream_t);                     \
    template void launch_tracer_batch<R>(const BatchLaunch<TracerArgs<R>> &, int, const Geom &, hipStream_t); \
    template void launch_div<R>(const DivArgs<R> &, const Geom &, hipStream_t);                           \
    template void launch_lap_batch<R>(const BatchLaunch<LapArgs<R>> &, int, const Geom &, hipStream_t);  \
    template void launch_div_batch<R>(const BatchLaunch<DivArgs<R>> &, int, const Geom &, hipStream_t);  \
    template void launch_fe_edge<R>(const FEEdgeArgs<R> &, const Geom &, hipStream_t, bool);               \
    template void launch_fe_cell_batch<R>(const BatchLaunch<FECellArgs<R>> &, int, bool, const Geom &,     \
                                          hipStream_t);                                                    \
    template void launch_fe_vertex_batch<R>(const BatchLaunch<FEVertexArgs<R>> &, int, bool, const Geom &, \
                                            hipStream_t);                                                  \
    template void launch_fe_edge_batch<R>(const BatchLaunch<FEEdgeArgs<R>> &, int, bool, int, const Geom &, \
                                          hipStream_t);                                                    \
    template size_t fe_edge_tiled_lds<R>(const DevTiles &, int);                                           \
    template void launch_fe_edge_tiled<R>(const FEEdgeArgs<R> &, const DevTiles &, hipStream_t);           \
    template void launch_edge_gathers<R>(const FEEdgeArgs<R> &, const Geom &, hipStream_t);                \
    template void launch_bt_eval<R>(const BTEvalArgs<R> &, const Geom &, hipStream_t);                     \
    template void launch_bt_substep<R>(const BTTileArgs<R> &, int, hipStream_t);                           \
    template int bt_loop_capacity<R>(const DevBtTiles &, int);                                             \
    template hipError_t launch_bt_loop<R>(const BTTileArgs<R> &, const BtLoop<R> &, int, hipStream_t);       \
    template void launch_bt_substep_batch<R>(const BatchLaunch<BTTileArgs<R>> &, int, int, size_t, hipStream_t); \
    template void launch_bt_eval_batch<R>(const BatchLaunch<BTEvalArgs<R>> &, bool, const Geom &, hipStream_t); \
    template void launch_thickness_iso<R>(const THIsoArgs<R> &, const Geom &, hipStream_t);                \
    template void launch_thickness_iso_batch<R>(const BatchLaunch<THIsoArgs<R>> &, int, const Geom &,      \
                                                hipStream_t);                                              \
    template void launch_assemble<R>(const AssembleArgs<R> &, const Geom &, hipStream_t);                  \
    template void launch_assemble_batch<R>(const BatchLaunch<AssembleArgs<R>> &, int, const Geom &,        \
                                           hipStream_t);                                                   \
    template void launch_edge_flux_sum<R>(const DevMesh &, int, const double *, const R *, const double *, \
                                          double *, hipStream_t);
SSE_INSTANTIATE(double)
SSE_INSTANTIATE(float)
template void launch_convert<double, float>(const ConvArgs<double, float> &, const Geom &, hipStream_t);
template void launch_convert<float, double>(const ConvArgs<float, double> &, const Geom &, hipStream_t);
template void launch_convert_batch<double, float>(const BatchLaunch<ConvArgs<double, float>> &, const Geom &,
                                                  hipStream_t);
template void launch_convert_batch<float, double>(const BatchLaunch<ConvArgs<float, double>> &, const Geom &,
                                                  hipStream_t);

}  // namespace sse
