// HIP kernels of the wavelet-domain MCAO tomography solve, written for CDNA4
// (gfx950, 64-wide wavefronts).  Every stage of one operator apply is here:
//
//   W^-1  : k_idwt_coarse (whole low-pass band in LDS) + k_idwt_tile (one
//           level per launch, LDS tiles with a 2-coefficient halo)
//   P     : k_project (bilinear samples of every layer at the sensor nodes,
//           plus per-band slope sums for the tip/tilt means)
//   Gamma, C^-1, (I-T), Gamma^T : k_weights (per band of node rows) in an
//           apply; k_sensor (one block per sensor and frame) for the right
//           side and the forward model
//   P^T   : k_adjoint (separable footprint image per sensor and layer), summed
//           over sensors in the first analysis level
//   W + alpha D + <p,Ap> : k_fdwt_tile (level 1 adds up the footprint images,
//           no atomics) + k_fdwt_coarse
//   PCG vector updates with FP64 partial inner products: k_init, k_update_r,
//           k_update_p, k_replace_r
//   plan time: k_jacobi (separable closed form of the Jacobi diagonal)
//
// Three types parameterise the kernels.  T (float or double) is the storage
// of the PCG vectors (x, b, r, p, A p, J) and of the caller's slopes.  S is the
// storage of the operator's intermediates in HBM: the layer pixel fields, the
// adjoint node fields and footprint images.  C is the arithmetic of the
// wavelet and adjoint-projection stages, the type of their LDS tiles and of
// the low-pass scratch bands that carry a transform from one level to the
// next (a coarse band rounded to single precision loses the small details the
// next analysis level takes from it).  FP64 plans use S = C = double; FP32 plans use S = float
// with C chosen per stage, or S = C = double.  The projection's node fields,
// the Fried slopes and the noise weighting are FP64 in every plan (the slopes
// are differences of nearly equal node values), and every inner product is
// accumulated in FP64 and reduced in a fixed order (one partial per block,
// summed by the consumer), so a frame's result does not depend on what else
// is in the batch.
#include <algorithm>
#include <initializer_list>
#include <type_traits>

#include "wmcao_internal.hpp"

namespace wm {

using Acc = double;

// ---------------------------------------------------------------- helpers ----
template <class T>
__device__ __forceinline__ T* vptr(const JobPlan& J, int v, int frame) {
    return reinterpret_cast<T*>(J.vec[v]) + static_cast<int64_t>(frame) * J.stride[v];
}

// A device array through a global-memory pointer.  Arrays reached through two
// or more loaded pointers (plan tables, the Jacobi diagonal) are too deep for
// the compiler to infer their address space; as flat loads they would also
// count against the LDS counter, so that every wait for an LDS value would
// wait for them too.
template <class T>
using gptr = const T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
    return (gptr<T>)p;
}

// Low-pass scratch of a frame: its region holds ll_size 8-byte elements
// whatever type a stage keeps there, so that frames never overlap when stages
// of different arithmetic run side by side.
template <class C>
__device__ __forceinline__ C* ll_ptr(const JobPlan& J, int frame) {
    return reinterpret_cast<C*>(reinterpret_cast<char*>(J.vec[V_LL]) +
                                static_cast<int64_t>(frame) * J.stride[V_LL] * 8);
}

__device__ __forceinline__ double* part_ptr(const JobPlan& J, int frame, int seg) {
    const int slots = J.P->slots;
    return J.part + static_cast<int64_t>(frame) * (NPT * slots) + seg * slots;
}

// Deterministic block sum (fixed shuffle tree, then wave partials in order).
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
        red[16] = s;
    }
    __syncthreads();
    return red[16];
}

// Two deterministic block sums in the order of block_sum, for a result only
// thread 0 needs (it is valid there only, and no barrier broadcasts it); red
// holds 32 doubles.
__device__ void block_sum2_first(double& a, double& b, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[wid] = a;
        red[16 + wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, t = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
        for (int i = 0; i < nw; ++i) t += red[16 + i];
        a = s;
        b = t;
    }
}

// Four deterministic block sums at once (same tree as block_sum); red holds
// 4 * 16 + 4 doubles.
__device__ void block_sum4(double* v, double* red) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[16 * k + wid] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[16 * threadIdx.x + i];
        red[64 + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = red[64 + k];
}

__device__ double sum_slots(const double* p, int n, double* red) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return block_sum(v, red);
}

// Three slot sums in one pass (same order as sum_slots for each; loads at
// clamped addresses so that all three are in flight at once).  red: 68 doubles.
__device__ void sum_slots3(const double* a, int na, const double* b, int nb, const double* c,
                           int nc, double* out, double* red) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int n = max(na, max(nb, nc));
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double x = a[min(i, na - 1)], y = b[min(i, nb - 1)], z = c[min(i, nc - 1)];
        if (i < na) v[0] += x;
        if (i < nb) v[1] += y;
        if (i < nc) v[2] += z;
    }
    block_sum4(v, red);
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2];
}

// Sum of n <= 64 values with the shuffle tree of one wave of block_sum4 (so
// the same value as sum_slots for n <= 64), broadcast to every lane; no LDS
// and no barrier.
__device__ double wave_sum_small(const double* p, int n) {
    const int lane = threadIdx.x & 63;
    double v = p[min(lane, n - 1)];
    v = lane < n ? v : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return __shfl(v, 0, 64);
}

// Per-frame scalars of a solve: [0] the step size a of the current
// iteration, [1] the residual norm, [2 + parity] rho = <r, z> of the residual
// of that parity (written by k_update_p, read by the next k_update_r).
__device__ __forceinline__ double* frame_scal(const JobPlan& J, int f) { return J.alpha + 4 * f; }

// Scale index k (1 = finest details, levels = coarsest details and low-pass)
// of the Mallat coefficient (x, y) of an N x N layer.
__device__ __forceinline__ int level_of(int x, int y, int N, int levels) {
    const int m = x > y ? x : y;
    int k = levels;
    for (int lev = levels; lev >= 1; --lev)
        if (m >= (N >> lev)) k = lev;
    return k;
}

template <class C>
__device__ __forceinline__ void load_filters(const PlanDev& P, C* hf, C* gf) {
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        hf[n] = static_cast<C>(P.h[n]);
        gf[n] = static_cast<C>(P.g[n]);
    }
}

// One in-place periodic synthesis step on the leading M x M block of A (row
// stride ld), along y (columns within a row) or along x, staged through
// registers.  A work item is one coarse position k of one line and yields the
// output pair x[2k + par] = sum_t h[par + 2t] lo[k - t] + g[par + 2t] hi[k - t]
// (par = 0, 1; indices mod M/2), so every filter tap is a compile-time index.
template <class C>
__device__ void syn_pass(C* A, int ld, int M, int along_y, const C* hf, const C* gf) {
    const int H = M >> 1, cnt = M * H;
    C r0v[WM_QMAX / 2], r1v[WM_QMAX / 2];
#pragma unroll
    for (int r = 0; r < WM_QMAX / 2; ++r) {
        const int e = threadIdx.x + r * blockDim.x;
        if (e < cnt) {
            int line, k;
            if (along_y) { line = e / H; k = e - line * H; } else { k = e / M; line = e - k * M; }
            C x0 = 0, x1 = 0;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                int kk = k - t;
                if (kk < 0) kk += H;
                const C lo = along_y ? A[line * ld + kk] : A[kk * ld + line];
                const C hi = along_y ? A[line * ld + H + kk] : A[(H + kk) * ld + line];
                x0 += hf[2 * t] * lo + gf[2 * t] * hi;
                x1 += hf[2 * t + 1] * lo + gf[2 * t + 1] * hi;
            }
            r0v[r] = x0;
            r1v[r] = x1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WM_QMAX / 2; ++r) {
        const int e = threadIdx.x + r * blockDim.x;
        if (e < cnt) {
            int line, k;
            if (along_y) { line = e / H; k = e - line * H; } else { k = e / M; line = e - k * M; }
            if (along_y) {
                A[line * ld + 2 * k] = r0v[r];
                A[line * ld + 2 * k + 1] = r1v[r];
            } else {
                A[(2 * k) * ld + line] = r0v[r];
                A[(2 * k + 1) * ld + line] = r1v[r];
            }
        }
    }
    __syncthreads();
}

// One in-place periodic analysis step: a work item is one coarse position c
// of one line and yields a_c = sum_n h_n x[(2c+n) mod M] (low half) and
// d_c = sum_n g_n x[(2c+n) mod M] (high half).
template <class C>
__device__ void ana_pass(C* A, int ld, int M, int along_y, const C* hf, const C* gf) {
    const int H = M >> 1, cnt = M * H;
    C r0v[WM_QMAX / 2], r1v[WM_QMAX / 2];
#pragma unroll
    for (int r = 0; r < WM_QMAX / 2; ++r) {
        const int e = threadIdx.x + r * blockDim.x;
        if (e < cnt) {
            int line, c;
            if (along_y) { line = e / H; c = e - line * H; } else { c = e / M; line = e - c * M; }
            C lo = 0, hi = 0;
#pragma unroll
            for (int n = 0; n < 6; ++n) {
                int idx = 2 * c + n;
                if (idx >= M) idx -= M;
                const C v = along_y ? A[line * ld + idx] : A[idx * ld + line];
                lo += hf[n] * v;
                hi += gf[n] * v;
            }
            r0v[r] = lo;
            r1v[r] = hi;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WM_QMAX / 2; ++r) {
        const int e = threadIdx.x + r * blockDim.x;
        if (e < cnt) {
            int line, c;
            if (along_y) { line = e / H; c = e - line * H; } else { c = e / M; line = e - c * M; }
            if (along_y) {
                A[line * ld + c] = r0v[r];
                A[line * ld + H + c] = r1v[r];
            } else {
                A[c * ld + line] = r0v[r];
                A[(H + c) * ld + line] = r1v[r];
            }
        }
    }
    __syncthreads();
}

// Item of this block.  A launch deals its work-groups to the 8 XCDs in turn
// (block b to XCD b mod 8), and every XCD has its own L2.  The lists hold a
// frame's items together, so XCD x takes the x-th contiguous share of the
// list: blocks that read the same frame data (layer pixels, node rows, tile
// halos, footprint images) then meet in one L2 instead of fetching it eight
// times.  The map is a bijection on [0, gridDim.x); results do not depend on
// it, because every partial sum is stored by item, not by block.
__device__ __forceinline__ int xcd_item() {
    const int b = blockIdx.x, n = gridDim.x;
    const int x = b & 7, q = b >> 3, base = n >> 3, rem = n & 7;
    return x * base + min(x, rem) + q;
}

// Item of a block of the streaming vector sweeps (no data shared between
// blocks of one frame).  Launches of at least VEC_PLAIN_MIN blocks keep the
// plain order, which measured faster at batch 32 (5,824 blocks); smaller ones
// take the XCD shares, faster at batch 1 (182 blocks).
constexpr int VEC_PLAIN_MIN = 1024;
__device__ __forceinline__ int vec_item() {
    return static_cast<int>(gridDim.x) >= VEC_PLAIN_MIN ? static_cast<int>(blockIdx.x) : xcd_item();
}

// Bilinear sample position of node i on one axis: lower pixel i0 (clamped to
// [0, N-2]) and the weight t of pixel i0 + 1 (Sec. 2.1).  The forward and the
// adjoint projection both evaluate it, so they are exact transposes.
__device__ __forceinline__ void node_stencil(double pa, double pb, int i, int N, int& i0, Acc& t) {
    const double u = fma(pa, static_cast<double>(i), pb);   // same rounding as the plan's tables
    i0 = min(max(static_cast<int>(floor(u)), 0), N - 2);
    t = u - i0;
}

// Raw buffer resource over the `bytes` bytes at `base`.  The hardware checks
// every raw-buffer offset against the size and returns 0 for a load at or past
// it (an offset that wrapped below zero is a large unsigned value, so also
// past it) without touching memory: reads that may fall outside an image need
// no bounds branch and no select.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes),
                                             0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
constexpr uint32_t BUF_OOB = 0x80000000u;   // a byte offset past every image
constexpr int GNS = 2;                      // footprint images per gather step

// Two consecutive elements (a = x[i], b = x[i + 1]) from a raw buffer at a
// byte offset (element aligned): one 8-byte load for floats, two for doubles.
template <class S>
struct Pair {
    S a, b;
};
template <class S>
__device__ __forceinline__ Pair<S> ld_pair(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(S) == 4) {
        // the whole 8-byte value is reinterpreted (element access of the
        // builtin's vector result is not used)
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        return {v.x, v.y};
    } else {
        return {buf_ld(r, off, S()), buf_ld(r, off + 8u, S())};
    }
}

// P^T over a window of PR x PC pixels of layer l starting at (px0, py0)
// (periodic indices, px0 + PR < 2N), written into G (row stride ldg):
// the sum, in sensor order, of the footprint images of the sensors in mask
// (k_adjoint).  A thread owns one window column and every rstep-th row, so
// each G entry has one writer: no atomics and no barrier.  Rows go in chunks
// of RC held in registers, GNS sensors per step, with all GNS RC loads in
// flight before the first is added.  Loads go through raw buffers over each image, so
// a pixel outside a footprint reads 0: the byte offset of row k of a chunk is
// that of row 0 plus k rstep W (modulo 2^32, exact for rows inside the image;
// rows above or below it land past its end), and a column outside the
// footprint starts from BUF_OOB.  Windows that wrap around the layer's last
// row take the offsets row by row.
template <class S, class C, int RC>
__device__ void pt_gather_window(const PlanDev& P, const S* img, int l, int N, int px0, int py0,
                                 int PR, int PC, C* G, int ldg, unsigned mask) {
    const int tid = threadIdx.x, bd = blockDim.x;
    int c0, r0, rstep, cstep;
    if (PC <= bd) {
        c0 = tid % PC;
        r0 = tid / PC;
        rstep = bd / PC;
        cstep = PC;
        if (r0 >= rstep) return;
    } else {
        c0 = tid;
        r0 = 0;
        rstep = 1;
        cstep = bd;
    }
    const bool wrap = px0 + PR > N;   // uniform
    for (int c = c0; c < PC; c += cstep) {
        int gy = py0 + c;
        if (gy >= N) gy -= N;
        for (int rb = r0; rb < PR; rb += RC * rstep) {
            C g[RC];
#pragma unroll
            for (int k = 0; k < RC; ++k) g[k] = 0.0;
            // the mask is the same for every lane: keep it (and the sensor
            // indices drawn from it) in scalar registers, so the footprint
            // fields below are scalar loads
            unsigned mm = __builtin_amdgcn_readfirstlane(mask);
            while (mm) {
                // the next GNS sensors of the mask (a step past the last one
                // reads nothing: its buffer holds no bytes)
                S v[GNS][RC];
#pragma unroll
                for (int s = 0; s < GNS; ++s) {
                    const bool has = mm != 0;
                    const int ms = __builtin_amdgcn_readfirstlane(has ? __ffs(static_cast<int>(mm)) - 1 : 0);
                    if (has) mm &= mm - 1;
                    const int W = P.fp_w[ms][l], yc = gy - P.fp_y0[ms][l], x0 = P.fp_x0[ms][l];
                    const __amdgpu_buffer_rsrc_t rs =
                        buf_rsrc(img + P.fp_off[ms][l], has ? static_cast<uint32_t>(P.fp_h[ms][l] * W * sizeof(S)) : 0u);
                    // one unsigned compare per bound pair: negative offsets wrap high
                    const bool cok = static_cast<unsigned>(yc) < static_cast<unsigned>(W);
                    if (!wrap) {
                        const uint32_t o = cok ? static_cast<uint32_t>(((px0 + rb - x0) * W + yc) * static_cast<int>(sizeof(S))) : BUF_OOB;
                        const uint32_t st = static_cast<uint32_t>(rstep * W * static_cast<int>(sizeof(S)));
#pragma unroll
                        for (int k = 0; k < RC; ++k) v[s][k] = buf_ld(rs, o + k * st, S());
                    } else {
#pragma unroll
                        for (int k = 0; k < RC; ++k) {
                            int gx = px0 + rb + k * rstep;
                            gx -= gx >= N ? N : 0;
                            const uint32_t o = cok ? static_cast<uint32_t>(((gx - x0) * W + yc) * static_cast<int>(sizeof(S))) : BUF_OOB;
                            v[s][k] = buf_ld(rs, o, S());
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < GNS; ++s)
#pragma unroll
                    for (int k = 0; k < RC; ++k) g[k] += static_cast<C>(v[s][k]);
            }
#pragma unroll
            for (int k = 0; k < RC; ++k)
                if (rb + k * rstep < PR) G[(rb + k * rstep) * ldg + c] = g[k];
        }
    }
}

// Copy the M0 x M0 top-left block of a band with row stride ld into LDS (row
// stride M0), converting to C.  Eight elements per thread are loaded before
// any is stored, so the loads go out together (one element per loop trip
// waits for each load before the next); past the block's end a thread
// reloads its own first element of the round (distinct addresses across the
// wave, rather than every thread reading the last element).
template <class C, class T>
__device__ __forceinline__ void load_block(const T* src, int ld, int M0, C* dst) {
    constexpr int R = 8;
    const int n = M0 * M0, bd = blockDim.x;
    for (int e0 = threadIdx.x; e0 < n; e0 += R * bd) {
        T v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k * bd < n ? e0 + k * bd : e0;   // a valid element
            v[k] = src[static_cast<int64_t>(e / M0) * ld + e % M0];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k * bd;
            if (e < n) dst[e] = static_cast<C>(v[k]);
        }
    }
}

// ------------------------------------------------------------------ W^-1 ----
// Levels J..k0+1 of the synthesis of one layer, with the whole M0 x M0
// (M0 = N / 2^k0) low-pass block resident in LDS.  Coefficients in T; the
// result in C (LL_k0 scratch) or, at k0 = 0, in S (the pixels).
template <class T, class S, class C>
__global__ void __launch_bounds__(1024)
k_idwt_coarse(const JobArgs args, const Item* __restrict__ items, int in_vec, int out_vec) {
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const LayerInfo& Ly = P.layer[it.a];
    const int N = Ly.N, k0 = Ly.k0, M0 = N >> k0;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* A = reinterpret_cast<C*>(smem_raw);
    C hf[6], gf[6];
    load_filters(P, hf, gf);
    const T* src = vptr<T>(J, in_vec, it.frame) + Ly.coff;
    for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x)
        A[e] = static_cast<C>(src[static_cast<int64_t>(e / M0) * N + (e % M0)]);
    __syncthreads();
    for (int lev = P.levels; lev > k0; --lev) {
        const int M = N >> (lev - 1);
        syn_pass(A, M0, M, 0, hf, gf);   // undo the x step
        syn_pass(A, M0, M, 1, hf, gf);   // undo the y step
    }
    if (k0 > 0) {   // low-pass band of the finest coarse level: scratch (C)
        C* dst = ll_ptr<C>(J, it.frame) + Ly.ll_off[k0];
        for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x) dst[e] = A[e];
    } else {
        S* dst = vptr<S>(J, out_vec, it.frame) + Ly.coff;
        for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x) dst[e] = static_cast<S>(A[e]);
    }
}

// One synthesis level k <= k0 over a TS x TS output tile: reads the low-pass
// band LL_k (scratch) and the three level-k detail bands (Mallat regions of the
// input coefficients) on a (TS/2+2)^2 window, writes LL_{k-1} (scratch) or, at
// k = 1, the layer pixels (S).
template <class T, class S, class C, int TS>
__global__ void __launch_bounds__(TILE_NT)
k_idwt_tile(const JobArgs args, const Item* __restrict__ items, int level, int in_vec,
            int out_vec) {
    constexpr int CW = TS / 2 + 2;
    __shared__ C sLL[CW][CW + 1], sLH[CW][CW + 1], sHL[CW][CW + 1], sHH[CW][CW + 1];
    __shared__ C sAL[TS][CW + 1], sAH[TS][CW + 1];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const LayerInfo& Ly = P.layer[it.a];
    const int N = Ly.N, M = N >> (level - 1), H = M >> 1;
    const int ntx = (M + TS - 1) / TS;
    const int x0 = (it.b % ntx) * TS, y0 = (it.b / ntx) * TS;
    C hf[6], gf[6];
    load_filters(P, hf, gf);
    const T* src = vptr<T>(J, in_vec, it.frame) + Ly.coff;
    const C* llg = ll_ptr<C>(J, it.frame) + Ly.ll_off[level];
    // the window's detail coefficients (and, from scratch, its low-pass
    // values) are loaded first into registers, so that a fused tile's coarse
    // rebuild overlaps their latency; clamped, always valid addresses
    const int cx0 = (x0 >> 1) - 2, cy0 = (y0 >> 1) - 2;
    constexpr int WIT = (CW * CW + TILE_NT - 1) / TILE_NT;
    int wo[WIT];
    T rLH[WIT], rHL[WIT], rHH[WIT];
    C rLL[WIT];
    const bool fused = level == Ly.k0 && Ly.fuse;
    // a fused tile's coarse block (the Mallat top-left H x H of the input),
    // when it fits four elements per thread, is loaded before the window, so
    // that both sets of loads are in flight together
    constexpr int CR = 4;
    const bool coarse_regs = fused && H * H <= CR * TILE_NT;
    T cv[CR] = {};
    if (coarse_regs) {
#pragma unroll
        for (int k = 0; k < CR; ++k) {
            const int e = min(static_cast<int>(threadIdx.x) + k * TILE_NT, H * H - 1);
            cv[k] = src[static_cast<int64_t>(e / H) * N + e % H];
        }
    }
#pragma unroll
    for (int k = 0; k < WIT; ++k) {
        const int e = min(static_cast<int>(threadIdx.x) + k * TILE_NT, CW * CW - 1);
        const int a = e / CW, b = e % CW;
        int gx = cx0 + a, gy = cy0 + b;   // periodic wrap (|offset| < 2H)
        gx += gx < 0 ? H : 0;
        gy += gy < 0 ? H : 0;
        while (gx >= H) gx -= H;
        while (gy >= H) gy -= H;
        wo[k] = gx * H + gy;
        rLH[k] = src[static_cast<int64_t>(gx) * N + H + gy];
        rHL[k] = src[static_cast<int64_t>(H + gx) * N + gy];
        rHH[k] = src[static_cast<int64_t>(H + gx) * N + H + gy];
        rLL[k] = fused ? C(0) : llg[wo[k]];
    }
    if (fused) {
        // rebuild LL_k0 = the synthesis of levels J..k0+1 of the coarse block
        // (Mallat top-left M0 x M0) in LDS; every tile of this level repeats it
        extern __shared__ __align__(16) unsigned char smem_raw[];
        C* Ac = reinterpret_cast<C*>(smem_raw);
        const int M0 = H;
        if (coarse_regs) {
#pragma unroll
            for (int k = 0; k < CR; ++k) {
                const int e = static_cast<int>(threadIdx.x) + k * TILE_NT;
                if (e < M0 * M0) Ac[e] = static_cast<C>(cv[k]);
            }
        } else {
            load_block(src, N, M0, Ac);
        }
        __syncthreads();
        for (int lev = P.levels; lev > level; --lev) {
            const int Mc = N >> (lev - 1);
            syn_pass(Ac, M0, Mc, 0, hf, gf);
            syn_pass(Ac, M0, Mc, 1, hf, gf);
        }
#pragma unroll
        for (int k = 0; k < WIT; ++k) rLL[k] = Ac[wo[k]];
    }
#pragma unroll
    for (int k = 0; k < WIT; ++k) {
        const int e = static_cast<int>(threadIdx.x) + k * TILE_NT;
        if (e < CW * CW) {
            const int a = e / CW, b = e % CW;
            sLL[a][b] = rLL[k];
            sLH[a][b] = static_cast<C>(rLH[k]);
            sHL[a][b] = static_cast<C>(rHL[k]);
            sHH[a][b] = static_cast<C>(rHH[k]);
        }
    }
    __syncthreads();
    // along x: output rows 2p and 2p + 1 (x0 is even) from coarse rows p + 2 - t
#pragma unroll
    for (int e = threadIdx.x; e < (TS / 2) * CW; e += TILE_NT) {
        const int pr = e / CW, b = e % CW;
        C al0 = 0, al1 = 0, ah0 = 0, ah1 = 0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int k = pr + 2 - t;
            const C ll_ = sLL[k][b], hl = sHL[k][b], lh = sLH[k][b], hh = sHH[k][b];
            al0 += hf[2 * t] * ll_ + gf[2 * t] * hl;
            al1 += hf[2 * t + 1] * ll_ + gf[2 * t + 1] * hl;
            ah0 += hf[2 * t] * lh + gf[2 * t] * hh;
            ah1 += hf[2 * t + 1] * lh + gf[2 * t + 1] * hh;
        }
        sAL[2 * pr][b] = al0;
        sAL[2 * pr + 1][b] = al1;
        sAH[2 * pr][b] = ah0;
        sAH[2 * pr + 1][b] = ah1;
    }
    __syncthreads();
    // level > 1: the next finer low-pass band (scratch); level 1: pixels
    C* dll = level > 1 ? ll_ptr<C>(J, it.frame) + Ly.ll_off[level - 1] : nullptr;
    S* dst = vptr<S>(J, out_vec, it.frame) + Ly.coff;
    const int ld = level > 1 ? M : N;
    // along y: output columns 2q and 2q + 1 from coarse columns q + 2 - t
#pragma unroll
    for (int e = threadIdx.x; e < TS * (TS / 2); e += TILE_NT) {
        const int li = e / (TS / 2), q = e % (TS / 2);
        const int i = x0 + li, j = y0 + 2 * q;
        C v0 = 0, v1 = 0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int k = q + 2 - t;
            const C lo = sAL[li][k], hi = sAH[li][k];
            v0 += hf[2 * t] * lo + gf[2 * t] * hi;
            v1 += hf[2 * t + 1] * lo + gf[2 * t + 1] * hi;
        }
        if (i >= M || j >= M) continue;   // M is even, so j + 1 < M too
        const int64_t o = static_cast<int64_t>(i) * ld + j;
        if (level > 1) {
            dll[o] = v0;
            dll[o + 1] = v1;
        } else {
            dst[o] = static_cast<S>(v0);
            dst[o + 1] = static_cast<S>(v1);
        }
    }
}

// Element offsets of a thread's share of a PW x PW window at (px0, py0) of
// an M x M band stored with row stride ld, wrapped periodically (the origin
// lies in the band, so offsets are non-negative; a window wider than the band
// wraps more than once).  All offsets are formed before any load is issued,
// so that the loads go out back to back rather than one per wrap loop.
template <int PW, int WIN_IT>
__device__ __forceinline__ void window_offsets(int px0, int py0, int M, int ld, int64_t* off) {
#pragma unroll
    for (int k = 0; k < WIN_IT; ++k) {
        const int e = min(static_cast<int>(threadIdx.x) + k * TILE_NT, PW * PW - 1);
        int gx = px0 + e / PW, gy = py0 + e % PW;
        if (M >= PW) {   // one wrap at most (uniform branch)
            gx -= gx >= M ? M : 0;
            gy -= gy >= M ? M : 0;
        } else {
            gx %= M;
            gy %= M;
        }
        off[k] = static_cast<int64_t>(gx) * ld + gy;
    }
}

// --------------------------------------------------------- W (+ P^T, D) ----
// One analysis level k <= k0 over a (TS/2)^2 tile of each band.  The input
// window of (TS+4)^2 values (S in HBM) is LL_{k-1} (scratch) or, at k = 1, the layer
// pixels: read from memory (SRC_PIX) or summed from the adjoint footprint
// images (SRC_PT).  LL_k goes to scratch; the three detail bands go to the
// output (T) with, under EPI_APPLY, + alpha D_k p and an FP64 partial <p, out>.
template <class T, class S, class C, int TS>
__global__ void __launch_bounds__(TILE_NT)
k_fdwt_tile(const JobArgs args, const Item* __restrict__ items, int level, int src, int in_vec,
            int out_vec, int epi, int aux_vec) {
    constexpr int HT = TS / 2, PW = TS + 4;
    __shared__ C sA[PW][PW + 1];
    __shared__ C sL[PW][HT + 1], sH[PW][HT + 1];
    __shared__ double red[17];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const LayerInfo& Ly = P.layer[it.a];
    const int N = Ly.N, M = N >> (level - 1), H = M >> 1;
    const int ntx = (H + HT - 1) / HT;
    const int cx0 = (it.b % ntx) * HT, cy0 = (it.b / ntx) * HT;
    const int px0 = 2 * cx0, py0 = 2 * cy0;
    C hf[6], gf[6];
    load_filters(P, hf, gf);
    // p at this thread's first epilogue coefficients, loaded before the window
    // so that its latency overlaps the analysis
    // Loads below go to clamped, always valid addresses with the value
    // selected afterwards, so that none sits under a branch of its own (such
    // a load is waited for at the branch's end, serialising the loop).
    constexpr int PQ_PF = 2;
    T pp[PQ_PF][3];
    {
        const T* pv0 = vptr<T>(J, aux_vec, it.frame) + Ly.coff;   // valid for every caller
#pragma unroll
        for (int q = 0; q < PQ_PF; ++q) {
            const int e = threadIdx.x + q * TILE_NT;
            int X = cx0 + e / HT, Y = cy0 + e % HT;
            const bool ok = e < HT * HT && X < H && Y < H;
            X = ok ? X : 0;
            Y = ok ? Y : 0;
            pp[q][0] = pv0[static_cast<int64_t>(X) * N + H + Y];
            pp[q][1] = pv0[static_cast<int64_t>(H + X) * N + Y];
            pp[q][2] = pv0[static_cast<int64_t>(H + X) * N + H + Y];
        }
    }
    constexpr int WIN_IT = (PW * PW + TILE_NT - 1) / TILE_NT;
    if (level == 1 && src == SRC_PT) {
        // rows per thread of the PW x PW window, at most 8 per register chunk
        constexpr int RPT = (PW + TILE_NT / PW - 1) / (TILE_NT / PW);
        // the tile's sensor mask is one value for the whole block: a scalar
        // load (constant address space), which waits for none of the vector
        // loads issued above
        const unsigned tmask = static_cast<unsigned>(
            ((const int __attribute__((address_space(4)))*)P.tmeta)[P.tmeta_off[it.a] + it.b]);
        pt_gather_window<S, C, (RPT < 8 ? RPT : 8)>(P, vptr<S>(J, in_vec, it.frame), it.a, N, px0,
                                                    py0, PW, PW, &sA[0][0], PW + 1, tmask);
    } else if (level > 1) {
        // the low-pass band of the level below (scratch)
        const C* ind = ll_ptr<C>(J, it.frame) + Ly.ll_off[level - 1];
        int64_t off[WIN_IT];
        window_offsets<PW, WIN_IT>(px0, py0, M, M, off);
        C v[WIN_IT];
#pragma unroll
        for (int k = 0; k < WIN_IT; ++k) v[k] = ind[off[k]];
#pragma unroll
        for (int k = 0; k < WIN_IT; ++k) {
            const int e0 = threadIdx.x + k * TILE_NT;
            if (e0 < PW * PW) sA[e0 / PW][e0 % PW] = v[k];
        }
    } else {
        const S* in = vptr<S>(J, in_vec, it.frame) + Ly.coff;
        int64_t off[WIN_IT];
        window_offsets<PW, WIN_IT>(px0, py0, M, N, off);
        S v[WIN_IT];
#pragma unroll
        for (int k = 0; k < WIN_IT; ++k) v[k] = in[off[k]];
#pragma unroll
        for (int k = 0; k < WIN_IT; ++k) {
            const int e0 = threadIdx.x + k * TILE_NT;
            if (e0 < PW * PW) sA[e0 / PW][e0 % PW] = static_cast<C>(v[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = threadIdx.x; e < PW * HT; e += TILE_NT) {
        const int a = e / HT, c = e % HT;
        C lo = 0, hi = 0;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const C v = sA[a][2 * c + n];
            lo += hf[n] * v;
            hi += gf[n] * v;
        }
        sL[a][c] = lo;
        sH[a][c] = hi;
    }
    __syncthreads();
    T* out = vptr<T>(J, out_vec, it.frame) + Ly.coff;
    const T* pv = vptr<T>(J, aux_vec, it.frame) + Ly.coff;   // valid for every caller
    const C aD = static_cast<C>(P.alpha * Ly.D[level - 1]);
    C* llo = ll_ptr<C>(J, it.frame) + Ly.ll_off[level];
    double acc = 0.0;
    constexpr int EPI_IT = (HT * HT + TILE_NT - 1) / TILE_NT;
#pragma unroll
    for (int q = 0; q < EPI_IT; ++q) {
        const int e = threadIdx.x + q * TILE_NT, ec = min(e, HT * HT - 1);
        const int c1 = ec / HT, c2 = ec % HT;
        const int X = cx0 + c1, Y = cy0 + c2;
        const bool ok = e < HT * HT && X < H && Y < H;
        C ll = 0, hl = 0, lh = 0, hh = 0;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const C l = sL[2 * c1 + n][c2], h = sH[2 * c1 + n][c2];
            ll += hf[n] * l;
            hl += gf[n] * l;
            lh += hf[n] * h;
            hh += gf[n] * h;
        }
        const int Xc = ok ? X : 0, Yc = ok ? Y : 0;
        const int64_t iLH = static_cast<int64_t>(Xc) * N + H + Yc;
        const int64_t iHL = static_cast<int64_t>(H + Xc) * N + Yc;
        const int64_t iHH = static_cast<int64_t>(H + Xc) * N + H + Yc;
        const T pr1 = q < PQ_PF ? pp[q][0] : pv[iLH];
        const T pr2 = q < PQ_PF ? pp[q][1] : pv[iHL];
        const T pr3 = q < PQ_PF ? pp[q][2] : pv[iHH];
        if (ok) {
            llo[X * H + Y] = ll;
            if (epi == EPI_APPLY) {
                const T o1 = static_cast<T>(lh + aD * static_cast<C>(pr1));
                const T o2 = static_cast<T>(hl + aD * static_cast<C>(pr2));
                const T o3 = static_cast<T>(hh + aD * static_cast<C>(pr3));
                acc += static_cast<Acc>(pr1) * static_cast<Acc>(o1) + static_cast<Acc>(pr2) * static_cast<Acc>(o2) +
                       static_cast<Acc>(pr3) * static_cast<Acc>(o3);
                out[iLH] = o1;
                out[iHL] = o2;
                out[iHH] = o3;
            } else {
                out[iLH] = static_cast<T>(lh);
                out[iHL] = static_cast<T>(hl);
                out[iHH] = static_cast<T>(hh);
            }
        }
    }
    if (epi == EPI_APPLY) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) part_ptr(J, it.frame, PT_PQ)[it.slot] = s;
    }
}

// Levels k0+1..J of the analysis with the M0 x M0 block in LDS (C), then
// the epilogue over every coefficient of that block.  At k0 = 0 the block is
// the whole layer, read (SRC_PIX) or gathered through P^T (SRC_PT).  Dynamic
// LDS: the M0 x M0 block.
template <class T, class S, class C>
__global__ void __launch_bounds__(1024)
k_fdwt_coarse(const JobArgs args, const Item* __restrict__ items, int src, int in_vec,
              int out_vec, int epi, int aux_vec) {
    __shared__ double red[32];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const LayerInfo& Ly = P.layer[it.a];
    const int N = Ly.N, k0 = Ly.k0, M0 = N >> k0;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* A = reinterpret_cast<C*>(smem_raw);
    C hf[6], gf[6];
    load_filters(P, hf, gf);
    if (k0 > 0) {
        const C* ll = ll_ptr<C>(J, it.frame) + Ly.ll_off[k0];
        for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x) A[e] = ll[e];
    } else if (src == SRC_PIX) {
        const S* in = vptr<S>(J, in_vec, it.frame) + Ly.coff;
        for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x) A[e] = static_cast<C>(in[e]);
    } else {
        pt_gather_window<S, C, 4>(P, vptr<S>(J, in_vec, it.frame), it.a, N, 0, 0, N, N, A, N,
                                  static_cast<unsigned>(P.tmeta[P.tmeta_off[it.a]]));
    }
    __syncthreads();
    for (int lev = k0 + 1; lev <= P.levels; ++lev) {
        const int M = N >> (lev - 1);
        ana_pass(A, M0, M, 1, hf, gf);   // along y first
        ana_pass(A, M0, M, 0, hf, gf);   // then along x
    }
    T* out = vptr<T>(J, out_vec, it.frame) + Ly.coff;
    const T* pv = (epi == EPI_APPLY) ? vptr<T>(J, aux_vec, it.frame) + Ly.coff : nullptr;
    double acc = 0.0;
    for (int e = threadIdx.x; e < M0 * M0; e += blockDim.x) {
        const int x = e / M0, y = e % M0;
        const int64_t gi = static_cast<int64_t>(x) * N + y;
        const C v = A[e];
        if (epi == EPI_APPLY) {
            const int k = max(level_of(x, y, N, P.levels), 1);
            const T p = pv[gi];
            const T o = static_cast<T>(v + static_cast<C>(P.alpha * Ly.D[k - 1]) * static_cast<C>(p));
            acc += static_cast<Acc>(p) * static_cast<Acc>(o);
            out[gi] = o;
        } else {
            out[gi] = static_cast<T>(v);
        }
    }
    if (epi == EPI_APPLY) {
        // this layer's total: its tile partials (pad0.., pad1 of them, summed
        // in a fixed order) plus this block's own
        double* pq = part_ptr(J, it.frame, PT_PQ);
        double t = 0.0;
        for (int i = threadIdx.x; i < it.pad1; i += blockDim.x) t += pq[it.pad0 + i];
        double tiles = t, own = acc;
        block_sum2_first(tiles, own, red);
        if (threadIdx.x == 0) pq[it.slot] = tiles + own;
    }
}
// --------------------------------------------------------- projection ----
// P: sensor node field u_m = sum over layers of the bilinear samples of each
// layer at the node's projected position (Sec. 2.1, cone factor for LGS), in
// FP64.  One block per (frame, sensor, band of P.proj_rows node rows).  With
// sums set (operator applies), the block also forms the Fried slopes of the
// band's subapertures (Sec. 2.2; one extra halo node row) and writes their
// sums for the tip/tilt projection and the low-order cells (one record per
// band, reduced in a fixed order by k_weights).  u is kept in FP64 so that the
// Fried differences do not cancel single-precision digits.
// LB: layers whose samples a thread loads together.  Three, at most 64 VGPRs
// (eight waves per SIMD), for launches that fill the GPU: left free, the
// compiler keeps every layer's weights in registers and halves the
// occupancy.  Nine (one round of loads per node) for small launches, where
// occupancy does not bind and every round trip is on the critical path.
constexpr int PROJ_LB = 3;
constexpr int PROJ_LB_WIDE = 9;
constexpr int PROJ_WIDE_MAX = 256;    // most work items of a launch that loads nine at once
template <class T, class S, int LB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(LB > PROJ_LB ? 4 : 8)))
k_project(const JobArgs args, const Item* __restrict__ items, int in_vec, int sums) {
    __shared__ double red[68];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const int m = it.a;
    const WfsInfo& w = P.wfs[m];
    const int nn = w.nn, L = P.L;
    const int PR = P.proj_rows, PR1 = PR + 1;
    const int r0 = it.b * PR;
    const int rows = min(PR, nn - r0);
    const bool slopes = sums && w.kind == 0;
    const int rows_c = slopes ? min(PR1, nn - r0) : rows;
    const int K = rows_c + nn;
    // dynamic LDS (proj_lds_bytes): the u window for the slopes, then per
    // layer the bilinear stencils of every node column (weight s of the
    // second pixel column, first pixel column) and of the block's node rows
    // (weight t of the second pixel row, element offset of the first sample
    // in the frame's pixel vector)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* su = reinterpret_cast<double*>(smem_raw);
    double* cs = su + PR1 * nn;
    double* rt = cs + L * nn;
    int* cj0 = reinterpret_cast<int*>(rt + L * PR1);
    int* rbase = cj0 + L * nn;
    // e = l K + k, split with a float reciprocal: exact here, since
    // (e + 1/2) / K is at least 1 / (2 K) > 2^-9 away from an integer, while
    // the product's error is below 2^-19 (quotient under 16, relative error
    // under 2^-23)
    const float rK = 1.0f / static_cast<float>(K);
    for (int e = threadIdx.x; e < L * K; e += blockDim.x) {
        const int l = static_cast<int>((static_cast<float>(e) + 0.5f) * rK), k = e - l * K;
        const int N = P.layer[l].N;
        int i0;
        Acc t;
        if (k < rows_c) {
            node_stencil(P.pa[m][l], P.pb[0][m][l], r0 + k, N, i0, t);
            rbase[l * PR1 + k] = static_cast<int>(P.layer[l].coff) + i0 * N;
            rt[l * PR1 + k] = t;
        } else {
            const int c = k - rows_c;
            node_stencil(P.pa[m][l], P.pb[1][m][l], c, N, i0, t);
            cj0[l * nn + c] = i0;
            cs[l * nn + c] = t;
        }
    }
    __syncthreads();
    // a thread owns node column j and rows g, g + G, ... of the block (G =
    // threads per column); the two samples of a node's sample row on a layer
    // (pixels i0 and i0 + 1) are one load, through a raw buffer over the
    // frame's pixels with 32-bit offsets
    const int G = blockDim.x / nn;
    const int j = threadIdx.x % nn, g = threadIdx.x / nn;
    if (g < G) {
        const __amdgpu_buffer_rsrc_t rp =
            buf_rsrc(vptr<S>(J, in_vec, it.frame), static_cast<uint32_t>(P.n * sizeof(S)));
        double* u = vptr<double>(J, V_U, it.frame) + w.node_off;
        for (int li = g; li < rows_c; li += G) {
            Acc acc = 0;
            // LB layers per step: their samples are loaded before any is used
            for (int l0 = 0; l0 < L; l0 += LB) {
                Pair<S> v[LB][2];
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    const int l = min(l0 + k, L - 1);   // past the last layer: a valid load, unused
                    const uint32_t o = static_cast<uint32_t>((rbase[l * PR1 + li] + cj0[l * nn + j]) * static_cast<int>(sizeof(S)));
                    v[k][0] = ld_pair<S>(rp, o);
                    v[k][1] = ld_pair<S>(rp, o + static_cast<uint32_t>(P.layer[l].N * static_cast<int>(sizeof(S))));
                }
#pragma unroll
                for (int k = 0; k < LB; ++k) {
                    const int l = l0 + k;
                    if (l < L) {
                        // bilinear: lerp along y in both sample rows, then along x
                        const Acc s = cs[l * nn + j], t = rt[l * PR1 + li];
                        const Acc a0 = static_cast<Acc>(v[k][0].a), a1 = static_cast<Acc>(v[k][0].b);
                        const Acc b0 = static_cast<Acc>(v[k][1].a), b1 = static_cast<Acc>(v[k][1].b);
                        const Acc x = fma(s, a1 - a0, a0), y = fma(s, b1 - b0, b0);
                        acc += fma(t, y - x, x);
                    }
                }
            }
            if (li < rows) u[(r0 + li) * nn + j] = acc;
            if (slopes) su[li * nn + j] = acc;
        }
    }
    if (!slopes) return;
    __syncthreads();
    const int ns = w.n_sub;
    double* rec = vptr<double>(J, V_SPART, it.frame) + w.sp_off + it.b * SP_K;
    const int nsub_rows = min(PR, min(ns - r0, rows_c - 1));
    // a thread owns subaperture column js and rows gs, gs + GS, ...
    const int GS = blockDim.x / ns, js = threadIdx.x % ns;
    const int gs = threadIdx.x / ns < GS ? threadIdx.x / ns : nsub_rows;   // spare threads: no rows
    if (!w.agg) {
        Acc p0 = 0, p1 = 0, p2 = 0, p3 = 0;
        for (int li = gs; li < nsub_rows; li += GS) {
            const int j = js;
            const int q = as_global(w.maskmap)[(r0 + li) * ns + j];
            if (q < 0) continue;
            const Acc u00 = su[li * nn + j], u10 = su[(li + 1) * nn + j];
            const Acc u01 = su[li * nn + j + 1], u11 = su[(li + 1) * nn + j + 1];
            const Acc sx = 0.5 * ((u10 - u00) + (u11 - u01));
            const Acc sy = 0.5 * ((u01 - u00) + (u11 - u10));
            const gptr<double> bq = as_global(w.blocks) + 3 * q;
            p0 += sx;
            p1 += sy;
            p2 += bq[0] * sx + bq[1] * sy;
            p3 += bq[1] * sx + bq[2] * sy;
        }
        double pv[4] = {p0, p1, p2, p3};
        block_sum4(pv, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) rec[k] = pv[k];
    } else {
        // two cells per pass: x and y sums of cells c and c + 1
        for (int c = 0; c < w.S; c += 2) {
            double pv[4] = {0.0, 0.0, 0.0, 0.0};
            for (int li = gs; li < nsub_rows; li += GS) {
                const int j = js;
                const int k = as_global(w.maskmap)[(r0 + li) * ns + j] - c;
                if (k != 0 && k != 1) continue;
                const Acc u00 = su[li * nn + j], u10 = su[(li + 1) * nn + j];
                const Acc u01 = su[li * nn + j + 1], u11 = su[(li + 1) * nn + j + 1];
                pv[2 * k] += 0.5 * ((u10 - u00) + (u11 - u01));
                pv[2 * k + 1] += 0.5 * ((u01 - u00) + (u11 - u10));
            }
            block_sum4(pv, red);
            if (threadIdx.x == 0) {
                rec[2 * c] = pv[0];
                rec[2 * c + 1] = pv[1];
                if (c + 1 < w.S) {
                    rec[2 * c + 2] = pv[2];
                    rec[2 * c + 3] = pv[3];
                }
            }
        }
    }
}

// Gamma^T C^-1 (I - T) Gamma for one band of node rows of one sensor (Sec. 2.2,
// eqs. (17)-(18)): the band's slope sums of every band give the tip/tilt means
// (or the low-order cell averages); the Fried slopes of the subaperture rows
// next to the band are formed again from u, weighted by the 2x2 blocks with
// the means removed before and after, and Gamma^T maps them to the band's node
// rows.  Phase sensors scale u at their nodes.  One block per (frame, sensor,
// band), no atomics.
//   plain:  w = B (s - mu) - nu,  mu = mean s,  nu = mean B (s - mu)
//           = (sum B s - mu_x sum(a, b) - mu_y sum(b, c)) / S  (tip/tilt-removed
//           sensors; mu = nu = 0 otherwise)
//   cells:  cell slopes = cell sums / cell counts, then the same with per-cell
//           blocks, divided by the cell count for the fine subapertures.
template <class T, class SO>
__global__ void __launch_bounds__(256)
k_weights(const JobArgs args, const Item* __restrict__ items, int out_vec) {
    // su, swx, swy: dynamic LDS of weights_lds_bytes(nn, ns, rows) for this sensor
    // (the launch gives the largest over its sensors)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double cval[2 * WM_MAXCELL], cwx[WM_MAXCELL], cwy[WM_MAXCELL];
    __shared__ double srec[((WM_NSUB_MAX + 1 + PROJ_ROWS_MIN - 1) / PROJ_ROWS_MIN) * SP_K];
    __shared__ double tsum[SP_K];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const int m = it.a;
    const WfsInfo& w = P.wfs[m];
    const int nn = w.nn, ns = w.n_sub;
    const int PR = P.wgt_rows;
    const int r0 = it.b * PR;
    const int rows = min(PR, nn - r0);
    double* su = reinterpret_cast<double*>(smem_raw);
    double* swx = su + (PR + 2) * nn;
    double* swy = swx + (PR + 1) * ns;
    const gptr<double> ug = as_global(vptr<double>(J, V_U, it.frame) + w.node_off);
    SO* vout = vptr<SO>(J, out_vec, it.frame) + w.node_off;
    const gptr<int> maskmap = as_global(w.maskmap);
    if (w.kind == 1) {
        for (int e = threadIdx.x; e < rows * nn; e += blockDim.x) {
            const int node = r0 * nn + e;
            const int q = maskmap[node];
            vout[node] = static_cast<SO>(q >= 0 ? as_global(w.blocks)[3 * q] * ug[node] : 0.0);
        }
        return;
    }
    const int ua = max(r0 - 1, 0), ub = min(r0 + PR, nn - 1);
    // measurement index of this thread's first WQ subapertures of the weighted
    // rows ia..ib, loaded with the node rows (their latency then overlaps the
    // means); clamped, always valid addresses
    const int ia = ua, ib = min(r0 + PR - 1, ns - 1);
    const int nsl = (ib - ia + 1) * ns;
    constexpr int WQ = 4;
    int qpre[WQ];
#pragma unroll
    for (int k = 0; k < WQ; ++k) {
        const int e = min(static_cast<int>(threadIdx.x) + k * static_cast<int>(blockDim.x), nsl - 1);
        qpre[k] = maskmap[(ia + e / ns) * ns + e % ns];
    }
    for (int e = threadIdx.x; e < (ub - ua + 1) * nn; e += blockDim.x) su[e] = ug[ua * nn + e];
    // the band records of this sensor (one per projection band), gathered in parallel
    const int nb = (nn + P.proj_rows - 1) / P.proj_rows;
    const int K = w.agg ? 2 * w.S : 4;
    {
        const gptr<double> rec = as_global(vptr<double>(J, V_SPART, it.frame) + w.sp_off);
        for (int e = threadIdx.x; e < nb * K; e += blockDim.x)
            srec[e] = rec[(e / K) * SP_K + e % K];
    }
    __syncthreads();
    // lane k of the first wave sums record component k over the bands, in
    // band order (the same order in every block of the sensor)
    if (threadIdx.x < K) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc += srec[b * K + threadIdx.x];
        tsum[threadIdx.x] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const gptr<double> blk = as_global(w.blocks);
        const auto cell_count = as_global(w.cell_count);
        if (!w.agg) {
            const double t[4] = {tsum[0], tsum[1], tsum[2], tsum[3]};
            double mx = 0.0, my = 0.0, nx = 0.0, ny = 0.0;
            if (w.remove_tt) {
                const double S = w.S_fine;
                mx = t[0] / S;
                my = t[1] / S;
                nx = (t[2] - mx * w.bsum[0] - my * w.bsum[1]) / S;
                ny = (t[3] - mx * w.bsum[1] - my * w.bsum[2]) / S;
            }
            cval[0] = mx;
            cval[1] = my;
            cval[2] = nx;
            cval[3] = ny;
        } else {
            const int S = w.S;
            double mx = 0.0, my = 0.0;
            for (int c = 0; c < S; ++c) {
                cval[2 * c] = tsum[2 * c] / cell_count[c];
                cval[2 * c + 1] = tsum[2 * c + 1] / cell_count[c];
                mx += cval[2 * c];
                my += cval[2 * c + 1];
            }
            if (w.remove_tt) {
                mx /= S;
                my /= S;
            } else {
                mx = my = 0.0;
            }
            double nx = 0.0, ny = 0.0;
            for (int c = 0; c < S; ++c) {
                const double ax = cval[2 * c] - mx, ay = cval[2 * c + 1] - my;
                cwx[c] = blk[3 * c] * ax + blk[3 * c + 1] * ay;
                cwy[c] = blk[3 * c + 1] * ax + blk[3 * c + 2] * ay;
                nx += cwx[c];
                ny += cwy[c];
            }
            if (w.remove_tt) {
                nx /= S;
                ny /= S;
            } else {
                nx = ny = 0.0;
            }
            for (int c = 0; c < S; ++c) {
                cval[2 * c] = (cwx[c] - nx) / cell_count[c];
                cval[2 * c + 1] = (cwy[c] - ny) / cell_count[c];
            }
        }
    }
    __syncthreads();
    // weighted slopes of subaperture rows ia..ib (the rows next to the band)
    int kq = 0;
    for (int e = threadIdx.x; e < nsl; e += blockDim.x, ++kq) {
        const int li = e / ns, j = e % ns;
        const int i = ia + li;
        int q = qpre[0];
#pragma unroll
        for (int k = 1; k < WQ; ++k) q = kq == k ? qpre[k] : q;
        if (kq >= WQ) q = maskmap[i * ns + j];
        Acc wx = 0, wy = 0;
        if (q >= 0) {
            if (w.agg) {
                wx = cval[2 * q];
                wy = cval[2 * q + 1];
            } else {
                const int lu = i - ua;
                const Acc u00 = su[lu * nn + j], u10 = su[(lu + 1) * nn + j];
                const Acc u01 = su[lu * nn + j + 1], u11 = su[(lu + 1) * nn + j + 1];
                const Acc sx = 0.5 * ((u10 - u00) + (u11 - u01)) - cval[0];
                const Acc sy = 0.5 * ((u01 - u00) + (u11 - u10)) - cval[1];
                const gptr<double> bq = as_global(w.blocks) + 3 * q;
                wx = bq[0] * sx + bq[1] * sy - cval[2];
                wy = bq[1] * sx + bq[2] * sy - cval[3];
            }
        }
        swx[e] = wx;
        swy[e] = wy;
    }
    __syncthreads();
    // Gamma^T: node (a, b) takes +-1/2 of the four subapertures around it
    for (int e = threadIdx.x; e < rows * nn; e += blockDim.x) {
        const int a = r0 + e / nn, b = e % nn;
        const int up = (a - 1 - ia) * ns, dn = (a - ia) * ns;
        Acc v = 0;
        if (a >= 1 && b < ns) v += swx[up + b] - swy[up + b];
        if (a < ns && b < ns) v -= swx[dn + b] + swy[dn + b];
        if (a >= 1 && b >= 1) v += swx[up + b - 1] + swy[up + b - 1];
        if (a < ns && b >= 1) v += swy[dn + b - 1] - swx[dn + b - 1];
        vout[a * nn + b] = static_cast<SO>(0.5 * v);
    }
}

// ------------------------------------------------------- adjoint P^T ----
// Footprint image of sensor m on layer l, g = B_x^T V B_y (Sec. 2.1), over a
// band of footprint rows.  The node rows the band needs are copied to LDS in
// one coalesced sweep; then T[r][b] = sum_a wx(a, r) V[a][b] for the band's
// pixel rows and every node column (LDS, FP64), and g[r][c] = sum_b wy(b, c)
// T[r][b].  The weights are the forward bilinear ones read backwards: node a
// feeds pixel i0_a with 1 - t_a and pixel i0_a + 1 with t_a.  A pixel row or
// column is fed by at most TAPS consecutive nodes on the fast path; TAPS (2
// to 4) is the largest count the plans of the launch need (3 for node spacings
// from 2/3 of a pixel up), and any row or column fed by more takes the general
// loop.  LDS: the staged node rows and T (both C), sized by the plan.  The tap
// weights are formed in FP64 (the same stencil as the forward projection) and
// rounded to C; the images are stored in S.

__device__ __forceinline__ Acc adj_weight(double pa, double pb, int i, int N, int g) {
    int i0;
    Acc t;
    node_stencil(pa, pb, i, N, i0, t);
    return i0 == g ? 1.0 - t : (i0 + 1 == g ? t : 0.0);
}

template <class T, class S, class C, int TAPS>
__global__ void __launch_bounds__(256)
k_adjoint(const JobArgs args, const Item* __restrict__ items, int in_vec, int out_vec) {
    static_assert(TAPS <= ADJ_TAPS_MAX, "adjoint taps");
    __shared__ C wrow[TAPS][ADJ_BAND];
    __shared__ int frow[ADJ_BAND], fofs[ADJ_BAND], crow[ADJ_BAND];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const int m = it.a, l = it.b;
    const int nn = P.wfs[m].nn, N = P.layer[l].N;
    const double pa = P.pa[m][l], pbx = P.pb[0][m][l], pby = P.pb[1][m][l];
    const int x0 = P.fp_x0[m][l], y0 = P.fp_y0[m][l];
    const int Hf = P.fp_h[m][l], Wf = P.fp_w[m][l], br = P.fp_br[m][l];
    const int r0 = it.slot * br, BR = min(Hf, r0 + br) - r0;
    const gptr<int> rt = as_global(P.fp_rc) + 2 * P.fp_tab[m][l];
    const gptr<int> ct = rt + 2 * Hf;
    const int alo = ct[2 * Wf + 2 * it.slot], ahi = ct[2 * Wf + 2 * it.slot + 1];
    S* out = vptr<S>(J, out_vec, it.frame) + P.fp_off[m][l] + r0 * Wf;
    if (ahi < alo) {
        for (int e = threadIdx.x; e < BR * Wf; e += blockDim.x) out[e] = S(0);
        return;
    }
    // the staged rows are followed by TAPS - 1 rows of zeros, so the fast
    // path reads rows f .. f + TAPS - 1 without clamping
    const int NR = ahi - alo + 1, NRP = NR + TAPS - 1;
    C* Vs = reinterpret_cast<C*>(smem_raw);
    C* Tb = reinterpret_cast<C*>(smem_raw + ((static_cast<size_t>(NRP) * nn * sizeof(C) + 15) & ~size_t(15)));
    const S* V = vptr<S>(J, in_vec, it.frame) + P.wfs[m].node_off + static_cast<int64_t>(alo) * nn;
    {
        // ADJ_PF loads in flight per thread: clamped addresses, predicated stores
        constexpr int ADJ_PF = 8;
        const int tot = NR * nn, bd0 = blockDim.x;
        for (int e0 = threadIdx.x; e0 < tot; e0 += ADJ_PF * bd0) {
            S v[ADJ_PF];
#pragma unroll
            for (int j = 0; j < ADJ_PF; ++j) v[j] = V[min(e0 + j * bd0, tot - 1)];
#pragma unroll
            for (int j = 0; j < ADJ_PF; ++j)
                if (e0 + j * bd0 < tot) Vs[e0 + j * bd0] = static_cast<C>(v[j]);
        }
        for (int e = tot + threadIdx.x; e < NRP * nn; e += bd0) Vs[e] = C(0);
    }
    // row taps of the band: first staged row, count, weights
    if (threadIdx.x < BR) {
        const int r = r0 + threadIdx.x, f = rt[2 * r], cnt = rt[2 * r + 1];
        const int fr = cnt > 0 ? f - alo : 0;   // a row no node reaches reads row 0 with weight 0
        frow[threadIdx.x] = fr;
        fofs[threadIdx.x] = fr * nn;
        crow[threadIdx.x] = cnt;
#pragma unroll
        for (int q = 0; q < TAPS; ++q)
            wrow[q][threadIdx.x] = static_cast<C>(q < cnt ? adj_weight(pa, pbx, f + q, N, x0 + r) : 0.0);
    }
    __syncthreads();
    const int bd = blockDim.x;
    // stage 1: a thread owns one node column and every G1-th band row
    {
        const int G1 = nn < bd ? bd / nn : 1, g1 = threadIdx.x / (nn < bd ? nn : bd);
        const int b0 = nn < bd ? threadIdx.x % nn : threadIdx.x, bstep = nn < bd ? nn : bd;
        if (g1 < G1)
            for (int b = b0; b < nn; b += bstep)
                for (int lr = g1; lr < BR; lr += G1) {
                    const int cnt = crow[lr];
                    const C* vc = Vs + fofs[lr] + b;
                    C acc = 0;
                    if (cnt <= TAPS) {
#pragma unroll
                        for (int q = 0; q < TAPS; ++q) acc += wrow[q][lr] * vc[q * nn];
                    } else {
                        const int r = r0 + lr, f = frow[lr];
                        for (int q = 0; q < cnt; ++q)
                            acc += static_cast<C>(adj_weight(pa, pbx, alo + f + q, N, x0 + r)) * vc[q * nn];
                    }
                    Tb[lr * nn + b] = acc;
                }
    }
    __syncthreads();
    // stage 2: a thread owns one footprint column and every G2-th band row
    const int G2 = Wf < bd ? bd / Wf : 1, g2 = threadIdx.x / (Wf < bd ? Wf : bd);
    const int c0 = Wf < bd ? threadIdx.x % Wf : threadIdx.x, cstep = Wf < bd ? Wf : bd;
    if (g2 >= G2) return;
    for (int c = c0; c < Wf; c += cstep) {
        const int f = ct[2 * c], cnt = ct[2 * c + 1], gy = y0 + c;
        if (cnt <= TAPS) {
            C w[TAPS];
            int ix[TAPS];
#pragma unroll
            for (int q = 0; q < TAPS; ++q) {
                w[q] = static_cast<C>(q < cnt ? adj_weight(pa, pby, f + q, N, gy) : 0.0);
                ix[q] = min(f + q, nn - 1);
            }
            for (int lr = g2; lr < BR; lr += G2) {
                const C* tr = Tb + lr * nn;
                C acc = 0;
#pragma unroll
                for (int q = 0; q < TAPS; ++q) acc += w[q] * tr[ix[q]];
                out[lr * Wf + c] = static_cast<S>(acc);
            }
        } else {
            for (int lr = g2; lr < BR; lr += G2) {
                const C* tr = Tb + lr * nn;
                C acc = 0;
                for (int q = 0; q < cnt; ++q) acc += static_cast<C>(adj_weight(pa, pby, f + q, N, gy)) * tr[f + q];
                out[lr * Wf + c] = static_cast<S>(acc);
            }
        }
    }
}

// ----------------------------------------------------------- one sensor ----
// u of one sensor at every node (Sec. 2.1): the sum over layers of the
// bilinear samples of the layer pixels (in_vec), with the stencils and the
// order of operations of k_project, into U (FP64, nn x nn).
template <class S>
__device__ void project_sensor(const JobPlan& J, const PlanDev& P, int m, int frame, int in_vec,
                               int nn, Acc* U) {
    const gptr<S> pix = as_global(vptr<S>(J, in_vec, frame));
    for (int e = threadIdx.x; e < nn * nn; e += blockDim.x) {
        const int r = e / nn, c = e % nn;
        Acc acc = 0;
        for (int l = 0; l < P.L; ++l) {
            const int N = P.layer[l].N;
            int i0, j0;
            Acc t, sw;
            node_stencil(P.pa[m][l], P.pb[0][m][l], r, N, i0, t);
            node_stencil(P.pa[m][l], P.pb[1][m][l], c, N, j0, sw);
            const gptr<S> q = pix + P.layer[l].coff + static_cast<int64_t>(i0) * N + j0;
            const Acc a0 = static_cast<Acc>(q[0]), a1 = static_cast<Acc>(q[1]);
            const Acc b0 = static_cast<Acc>(q[N]), b1 = static_cast<Acc>(q[N + 1]);
            const Acc x = fma(sw, a1 - a0, a0), y = fma(sw, b1 - b0, b0);
            acc += fma(t, y - x, x);
        }
        U[e] = acc;
    }
}

// SM_APPLY: node field u (from k_project) -> Fried slopes (aggregated for a
//           low-order sensor) -> C^-1 with (I - T) for tip/tilt-removed
//           sensors -> Gamma^T -> node field v.
// SM_PAPPLY: the same, with u formed here from the layer pixels (in_vec):
//           the projection and the weighting of a small sensor in one launch.
// SM_RHS:   input slopes -> C^-1 (and (I - T)) -> Gamma^T -> v.
// SM_FWD:   node field u -> raw slopes to the output.
// One block of 1024 threads per (frame, sensor); the node field and the
// weighted-slope grids live in LDS in FP64; QM elements per thread.
template <class T, class SO, int QM>
__global__ void __launch_bounds__(1024)
k_sensor(const JobArgs args, const Item* __restrict__ items, int mode, int in_vec, int out_vec) {
    __shared__ double red[17];
    __shared__ double cellx[WM_MAXCELL], celly[WM_MAXCELL], cwx[WM_MAXCELL], cwy[WM_MAXCELL];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Acc* U = reinterpret_cast<Acc*>(smem_raw);
    const Item it = items[xcd_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const int m = it.a;
    const WfsInfo& w = P.wfs[m];
    const int ns = w.n_sub, nn = w.nn, Sf = w.S_fine, S = w.S;
    // the sensor's tables, read as global memory (see as_global)
    const gptr<int> act = as_global(w.act), cell_of = as_global(w.cell_of);
    const gptr<int> cell_count = as_global(w.cell_count);
    const gptr<double> blk = as_global(w.blocks);
    const int tid = threadIdx.x, bd = blockDim.x;
    Acc sx[QM], sy[QM];
#pragma unroll
    for (int r = 0; r < QM; ++r) sx[r] = sy[r] = 0;

    if (w.kind == 1) {
        // phase at the pupil nodes: measurement q is node act[q], weight a_q
        if (mode == SM_PAPPLY) {
            project_sensor<SO>(J, P, m, it.frame, in_vec, nn, U);
            __syncthreads();
        } else if (mode != SM_RHS) {
            const double* ug = vptr<double>(J, V_U, it.frame) + w.node_off;
            for (int e = tid; e < nn * nn; e += bd) U[e] = ug[e];
            __syncthreads();
        }
        const T* in = vptr<T>(J, in_vec, it.frame) + w.soff;
#pragma unroll
        for (int r = 0; r < QM; ++r) {
            const int q = tid + r * bd;
            if (q < S) sx[r] = (mode != SM_RHS) ? U[act[q]] : static_cast<Acc>(in[q]);
        }
        if (mode == SM_FWD) {
            T* out = vptr<T>(J, out_vec, it.frame) + w.soff;
#pragma unroll
            for (int r = 0; r < QM; ++r) {
                const int q = tid + r * bd;
                if (q < S) out[q] = static_cast<T>(sx[r]);
            }
            return;
        }
        __syncthreads();
        for (int e = tid; e < nn * nn; e += bd) U[e] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QM; ++r) {
            const int q = tid + r * bd;
            if (q < S) U[act[q]] = blk[3 * q] * sx[r];
        }
        __syncthreads();
        SO* vout = vptr<SO>(J, out_vec, it.frame) + w.node_off;
        for (int e = tid; e < nn * nn; e += bd) vout[e] = static_cast<SO>(U[e]);
        return;
    }

    if (mode != SM_RHS) {
        if (mode == SM_PAPPLY) {
            project_sensor<SO>(J, P, m, it.frame, in_vec, nn, U);
        } else {
            const double* ug = vptr<double>(J, V_U, it.frame) + w.node_off;
            for (int e = tid; e < nn * nn; e += bd) U[e] = ug[e];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QM; ++r) {
            const int q = tid + r * bd;
            if (q < Sf) {
                const int pk = act[q];
                const int i = pk / ns, j = pk % ns;
                const Acc u00 = U[i * nn + j], u10 = U[(i + 1) * nn + j];
                const Acc u01 = U[i * nn + j + 1], u11 = U[(i + 1) * nn + j + 1];
                sx[r] = 0.5 * ((u10 - u00) + (u11 - u01));
                sy[r] = 0.5 * ((u01 - u00) + (u11 - u10));
            }
        }
    }

    if (w.agg) {
        if (mode != SM_RHS) {
            for (int c = 0; c < S; ++c) {
                Acc px = 0.0, py = 0.0;
#pragma unroll
                for (int r = 0; r < QM; ++r) {
                    const int q = tid + r * bd;
                    if (q < Sf && cell_of[q] == c) {
                        px += sx[r];
                        py += sy[r];
                    }
                }
                px = block_sum(px, red);
                py = block_sum(py, red);
                if (tid == 0) {
                    cellx[c] = px / cell_count[c];
                    celly[c] = py / cell_count[c];
                }
            }
        } else if (tid < S) {
            const T* in = vptr<T>(J, in_vec, it.frame) + w.soff;
            cellx[tid] = static_cast<Acc>(in[tid]);
            celly[tid] = static_cast<Acc>(in[S + tid]);
        }
        __syncthreads();
        if (mode == SM_FWD) {
            if (tid < S) {
                T* out = vptr<T>(J, out_vec, it.frame) + w.soff;
                out[tid] = static_cast<T>(cellx[tid]);
                out[S + tid] = static_cast<T>(celly[tid]);
            }
            return;
        }
        if (tid == 0) {
            Acc mx = 0.0, my = 0.0;
            if (w.remove_tt) {
                for (int c = 0; c < S; ++c) { mx += cellx[c]; my += celly[c]; }
                mx /= S;
                my /= S;
            }
            Acc nx = 0.0, ny = 0.0;
            for (int c = 0; c < S; ++c) {
                const Acc ax = cellx[c] - mx, ay = celly[c] - my;
                cwx[c] = blk[3 * c] * ax + blk[3 * c + 1] * ay;
                cwy[c] = blk[3 * c + 1] * ax + blk[3 * c + 2] * ay;
                nx += cwx[c];
                ny += cwy[c];
            }
            if (w.remove_tt) { nx /= S; ny /= S; } else { nx = ny = 0.0; }
            for (int c = 0; c < S; ++c) {
                cellx[c] = (cwx[c] - nx) / cell_count[c];
                celly[c] = (cwy[c] - ny) / cell_count[c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < QM; ++r) {
            const int q = tid + r * bd;
            if (q < Sf) {
                const int c = cell_of[q];
                sx[r] = cellx[c];
                sy[r] = celly[c];
            }
        }
    } else {
        if (mode == SM_RHS) {
            const T* in = vptr<T>(J, in_vec, it.frame) + w.soff;
#pragma unroll
            for (int r = 0; r < QM; ++r) {
                const int q = tid + r * bd;
                if (q < Sf) { sx[r] = in[q]; sy[r] = in[Sf + q]; }
            }
        }
        if (mode == SM_FWD) {
            T* out = vptr<T>(J, out_vec, it.frame) + w.soff;
#pragma unroll
            for (int r = 0; r < QM; ++r) {
                const int q = tid + r * bd;
                if (q < Sf) { out[q] = static_cast<T>(sx[r]); out[Sf + q] = static_cast<T>(sy[r]); }
            }
            return;
        }
        if (w.remove_tt) {
            Acc px = 0.0, py = 0.0;
#pragma unroll
            for (int r = 0; r < QM; ++r) { px += sx[r]; py += sy[r]; }
            const Acc mx = block_sum(px, red) / Sf;
            const Acc my = block_sum(py, red) / Sf;
#pragma unroll
            for (int r = 0; r < QM; ++r)
                if (tid + r * bd < Sf) { sx[r] -= mx; sy[r] -= my; }
        }
#pragma unroll
        for (int r = 0; r < QM; ++r) {
            const int q = tid + r * bd;
            if (q < Sf) {
                const Acc a = blk[3 * q], b = blk[3 * q + 1], c = blk[3 * q + 2];
                const Acc vx = a * sx[r] + b * sy[r];
                const Acc vy = b * sx[r] + c * sy[r];
                sx[r] = vx;
                sy[r] = vy;
            }
        }
        if (w.remove_tt) {
            Acc px = 0.0, py = 0.0;
#pragma unroll
            for (int r = 0; r < QM; ++r) { px += sx[r]; py += sy[r]; }
            const Acc mx = block_sum(px, red) / Sf;
            const Acc my = block_sum(py, red) / Sf;
#pragma unroll
            for (int r = 0; r < QM; ++r)
                if (tid + r * bd < Sf) { sx[r] -= mx; sy[r] -= my; }
        }
    }

    // Gamma^T: weighted slopes -> node field, x part then y part through LDS.
    Acc vacc[QM];
    __syncthreads();
    for (int e = tid; e < ns * ns; e += bd) U[e] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QM; ++r) {
        const int q = tid + r * bd;
        if (q < Sf) U[act[q]] = sx[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QM; ++r) {
        const int e = tid + r * bd;
        Acc v = 0;
        if (e < nn * nn) {
            const int a = e / nn, b = e % nn;
            if (a >= 1 && b < ns) v += U[(a - 1) * ns + b];
            if (a < ns && b < ns) v -= U[a * ns + b];
            if (a >= 1 && b >= 1) v += U[(a - 1) * ns + b - 1];
            if (a < ns && b >= 1) v -= U[a * ns + b - 1];
        }
        vacc[r] = v;
    }
    __syncthreads();
    for (int e = tid; e < ns * ns; e += bd) U[e] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QM; ++r) {
        const int q = tid + r * bd;
        if (q < Sf) U[act[q]] = sy[r];
    }
    __syncthreads();
    SO* vout = vptr<SO>(J, out_vec, it.frame) + w.node_off;
#pragma unroll
    for (int r = 0; r < QM; ++r) {
        const int e = tid + r * bd;
        if (e < nn * nn) {
            const int a = e / nn, b = e % nn;
            Acc v = vacc[r];
            if (a < ns && b >= 1) v += U[a * ns + b - 1];
            if (a < ns && b < ns) v -= U[a * ns + b];
            if (a >= 1 && b >= 1) v += U[(a - 1) * ns + b - 1];
            if (a >= 1 && b < ns) v -= U[(a - 1) * ns + b];
            vout[e] = static_cast<SO>(0.5 * v);
        }
    }
}

// ------------------------------------------------------------- PCG steps ----
// The vector kernels move 4 consecutive elements per access (16 B for FP32,
// 2 x 16 B for FP64) when the frame length is a multiple of 4; otherwise
// element by element.  One block covers P.vec_chunk elements of one frame.
// True when the frame length is a multiple of 4 and every pointer allows
// 16-byte accesses (a caller's vector may be any element-aligned address).
__device__ __forceinline__ bool can_vec4(int64_t n, std::initializer_list<const void*> ptrs) {
    uintptr_t bits = static_cast<uintptr_t>(n & 3);
    for (const void* q : ptrs) bits |= reinterpret_cast<uintptr_t>(q) & 15;
    return bits == 0;
}

// VEC is a compile-time flag so that no load sits under a run-time branch of
// its own (a load inside a divergent branch is waited for at the branch's end,
// which serialises the loads of a loop).
template <bool VEC, class T>
__device__ __forceinline__ void ld4(const T* p, int64_t i, int64_t n, Acc* v) {
    if constexpr (VEC) {
        if constexpr (sizeof(T) == 4) {
            const float4 q = *reinterpret_cast<const float4*>(p + i);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
            const double2 q0 = *reinterpret_cast<const double2*>(p + i);
            const double2 q1 = *reinterpret_cast<const double2*>(p + i + 2);
            v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (i + j < n) ? static_cast<Acc>(p[i + j]) : 0.0;
    }
}

template <bool VEC, class T>
__device__ __forceinline__ void st4(T* p, int64_t i, int64_t n, const T* v) {
    if constexpr (VEC) {
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4*>(p + i) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            *reinterpret_cast<double2*>(p + i) = make_double2(v[0], v[1]);
            *reinterpret_cast<double2*>(p + i + 2) = make_double2(v[2], v[3]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (i + j < n) p[i + j] = v[j];
    }
}

template <bool VEC, class T>
__device__ __forceinline__ void ld4(gptr<T> p, int64_t i, int64_t n, Acc* v) {
    if constexpr (VEC) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        typedef T v4 __attribute__((ext_vector_type(4)));
        if constexpr (sizeof(T) == 4) {
            const v4 q = *(const v4 __attribute__((address_space(1)))*)(p + i);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
            const v2 q0 = *(const v2 __attribute__((address_space(1)))*)(p + i);
            const v2 q1 = *(const v2 __attribute__((address_space(1)))*)(p + i + 2);
            v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (i + j < n) ? static_cast<Acc>(p[i + j]) : 0.0;
    }
}

// z = J^-1 v with the Jacobi preconditioner (PRE), else v.  Under VEC every
// element of a group exists, so the quotient is taken unconditionally and the
// diagonal's four values are one load issued with the other operands' (behind
// a run-time test of its own, the load of the first value sank into that
// branch and waited for the other loads: two memory round trips per group).
// Elements past n (scalar groups only) keep v.
template <bool VEC, bool PRE>
__device__ __forceinline__ Acc jacobi_z(Acc v, Acc d, bool exists) {
    if constexpr (!PRE)
        return v;
    else if constexpr (VEC)
        return v / d;
    else
        return exists ? v / d : v;
}

// Run a sweep lambda taking (VEC tag, PRE tag) with both flags as constants.
template <class F>
__device__ __forceinline__ void vec_dispatch(bool vec, bool pre, F&& sweep) {
    if (vec) {
        if (pre) sweep(std::true_type{}, std::true_type{});
        else sweep(std::true_type{}, std::false_type{});
    } else {
        if (pre) sweep(std::false_type{}, std::true_type{});
        else sweep(std::false_type{}, std::false_type{});
    }
}

// r0 = b (cold: x = 0) or b - A x0 (warm, A x0 in V_Q); p0 = z0 = J^-1 r0;
// partials of <r0, z0> and <r0, r0> into the parity-0 segments.
template <class T>
__global__ void __launch_bounds__(256)
k_init(const JobArgs args, const Item* __restrict__ items, int warm) {
    __shared__ double red[32];
    const Item it = items[vec_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    T* x = vptr<T>(J, V_X, it.frame);
    const T* b = vptr<T>(J, V_B, it.frame);
    const T* q = vptr<T>(J, V_Q, it.frame);
    T* r = vptr<T>(J, V_R, it.frame);
    T* p = vptr<T>(J, V_P, it.frame);
    const T* jac = reinterpret_cast<const T*>(P.jac);
    const bool vec = can_vec4(P.n, {x, b, q, r, p, jac});
    Acc rz = 0.0, rr = 0.0;
    const int chunk = P.vec_chunk;
    const int64_t i0 = static_cast<int64_t>(it.b) * chunk;
    const int64_t n_ = P.n;            // plan fields read once: the stores below may alias them
    const bool pre_ = P.precond != 0;
    auto sweep = [&](auto vec_tag, auto pre_tag) {
        constexpr bool VEC = decltype(vec_tag)::value, PRE = decltype(pre_tag)::value;
        for (int k = 4 * threadIdx.x; k < chunk; k += 4 * blockDim.x) {
            const int64_t i = i0 + k;
            if (i >= n_) break;
            Acc bv[4], qv[4], jv[4] = {};
            T rs[4], ps[4], zero[4] = {0, 0, 0, 0};
            ld4<VEC>(b, i, n_, bv);
            if constexpr (PRE) ld4<VEC>(as_global(jac), i, n_, jv);
            if (warm) ld4<VEC>(q, i, n_, qv);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rs[j] = static_cast<T>(warm ? bv[j] - qv[j] : bv[j]);
                const Acc rv = rs[j];
                const Acc z = jacobi_z<VEC, PRE>(rv, jv[j], i + j < n_);
                ps[j] = static_cast<T>(z);
                rz += rv * z;
                rr += rv * rv;
            }
            st4<VEC>(r, i, n_, rs);
            st4<VEC>(p, i, n_, ps);
            if (!warm) st4<VEC>(x, i, n_, zero);
        }
    };
    vec_dispatch(vec, pre_, sweep);
    block_sum2_first(rz, rr, red);
    if (threadIdx.x == 0) {
        part_ptr(J, it.frame, PT_RZ0)[it.slot] = rz;
        part_ptr(J, it.frame, PT_RR0)[it.slot] = rr;
        if (it.b == 0) J.status[it.frame] = WMCAO_FRAME_OK;
    }
}

// a = rho_i / <p, q>; r -= a q; partials of <r, J^-1 r>, <r, r> (next parity).
template <class T>
__global__ void __launch_bounds__(256)
k_update_r(const JobArgs args, const Item* __restrict__ items, int iter, int fresh) {
    __shared__ double red[68];
    const Item it = items[vec_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    // <p, Ap> (one total per layer) and rho_i.  rho_i is the sum k_update_p
    // formed one iteration earlier, except on the first iteration and after a
    // residual replacement (fresh), where the residual's partials are reduced
    // here, together with <r0, r0> on the first iteration.
    double pq, rho, sums[3] = {0.0, 0.0, 0.0};
    if (fresh || iter == 0) {
        sum_slots3(part_ptr(J, it.frame, PT_PQ) + P.pq_base, P.L,
                   part_ptr(J, it.frame, PT_RZ0 + (iter & 1)), P.n_vec_slots,
                   part_ptr(J, it.frame, PT_RR0), iter == 0 ? P.n_vec_slots : 1, sums, red);
        pq = sums[0];
        rho = sums[1];
    } else {
        pq = wave_sum_small(part_ptr(J, it.frame, PT_PQ) + P.pq_base, P.L);
        rho = frame_scal(J, it.frame)[2 + (iter & 1)];
    }
    int st = J.status[it.frame];
    double a = 0.0;
    if (st == WMCAO_FRAME_OK) {
        if (rho == 0.0)
            st = WMCAO_FRAME_CONVERGED;
        else if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho))
            st = WMCAO_FRAME_BREAKDOWN;
        else
            a = rho / pq;
    }
    if (iter == 0) {
        const double rr0 = sums[2];
        if (it.b == 0 && threadIdx.x == 0) {
            frame_scal(J, it.frame)[1] = sqrt(rr0);
            if (J.resid) J.resid[static_cast<int64_t>(it.frame) * J.resid_ld] = sqrt(rr0);
        }
    }
    if (it.b == 0 && threadIdx.x == 0) {
        frame_scal(J, it.frame)[0] = a;
        J.status[it.frame] = st;
    }
    if (st != WMCAO_FRAME_OK) return;
    T* r = vptr<T>(J, V_R, it.frame);
    const T* q = vptr<T>(J, V_Q, it.frame);
    const T* jac = reinterpret_cast<const T*>(P.jac);
    const bool vec = can_vec4(P.n, {r, q, jac});
    Acc rz = 0.0, rr = 0.0;
    const int chunk = P.vec_chunk;
    const int64_t i0 = static_cast<int64_t>(it.b) * chunk;
    const int64_t n_ = P.n;            // plan fields read once: the stores below may alias them
    const bool pre_ = P.precond != 0;
    auto sweep = [&](auto vec_tag, auto pre_tag) {
        constexpr bool VEC = decltype(vec_tag)::value, PRE = decltype(pre_tag)::value;
        for (int k = 4 * threadIdx.x; k < chunk; k += 4 * blockDim.x) {
            const int64_t i = i0 + k;
            if (i >= n_) break;
            Acc rv[4], qv[4], jv[4] = {};
            T rs[4];
            ld4<VEC>(r, i, n_, rv);
            ld4<VEC>(q, i, n_, qv);
            if constexpr (PRE) ld4<VEC>(as_global(jac), i, n_, jv);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rs[j] = static_cast<T>(rv[j] - a * qv[j]);
                const Acc v = rs[j];
                const Acc z = jacobi_z<VEC, PRE>(v, jv[j], i + j < n_);
                rz += v * z;
                rr += v * v;
            }
            st4<VEC>(r, i, n_, rs);
        }
    };
    vec_dispatch(vec, pre_, sweep);
    block_sum2_first(rz, rr, red);
    if (threadIdx.x == 0) {
        part_ptr(J, it.frame, PT_RZ0 + ((iter + 1) & 1))[it.slot] = rz;
        part_ptr(J, it.frame, PT_RR0 + ((iter + 1) & 1))[it.slot] = rr;
    }
}

// beta = rho_{i+1} / rho_i; x += a p; p = J^-1 r + beta p.
template <class T>
__global__ void __launch_bounds__(256)
k_update_p(const JobArgs args, const Item* __restrict__ items, int iter) {
    __shared__ double red[68];
    const Item it = items[vec_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    const int st = J.status[it.frame];
    if (st != WMCAO_FRAME_OK) {
        if (it.b == 0 && threadIdx.x == 0 && J.resid)
            J.resid[static_cast<int64_t>(it.frame) * J.resid_ld + iter + 1] = frame_scal(J, it.frame)[1];
        return;
    }
    const double a = frame_scal(J, it.frame)[0];
    // rho_i, rho_{i+1} and <r, r>, reduced together
    double sums[3];
    sum_slots3(part_ptr(J, it.frame, PT_RZ0 + (iter & 1)), P.n_vec_slots,
               part_ptr(J, it.frame, PT_RZ0 + ((iter + 1) & 1)), P.n_vec_slots,
               part_ptr(J, it.frame, PT_RR0 + ((iter + 1) & 1)), P.n_vec_slots, sums, red);
    const double rho0 = sums[0], rho1 = sums[1];
    const double beta = rho1 / rho0;
    if (it.b == 0) {
        const double rr = sums[2];
        if (threadIdx.x == 0) {
            frame_scal(J, it.frame)[1] = sqrt(rr);
            frame_scal(J, it.frame)[2 + ((iter + 1) & 1)] = rho1;   // rho of the next iteration
            if (J.resid) J.resid[static_cast<int64_t>(it.frame) * J.resid_ld + iter + 1] = sqrt(rr);
        }
    }
    T* x = vptr<T>(J, V_X, it.frame);
    T* p = vptr<T>(J, V_P, it.frame);
    const T* r = vptr<T>(J, V_R, it.frame);
    const T* jac = reinterpret_cast<const T*>(P.jac);
    const bool vec = can_vec4(P.n, {x, p, r, jac});
    const int chunk = P.vec_chunk;
    const int64_t i0 = static_cast<int64_t>(it.b) * chunk;
    const int64_t n_ = P.n;            // plan fields read once: the stores below may alias them
    const bool pre_ = P.precond != 0;
    auto sweep = [&](auto vec_tag, auto pre_tag) {
        constexpr bool VEC = decltype(vec_tag)::value, PRE = decltype(pre_tag)::value;
        for (int k = 4 * threadIdx.x; k < chunk; k += 4 * blockDim.x) {
            const int64_t i = i0 + k;
            if (i >= n_) break;
            Acc pv[4], xv[4], rv[4], jv[4] = {};
            T xs[4], ps[4];
            ld4<VEC>(p, i, n_, pv);
            ld4<VEC>(x, i, n_, xv);
            ld4<VEC>(r, i, n_, rv);
            if constexpr (PRE) ld4<VEC>(as_global(jac), i, n_, jv);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xs[j] = static_cast<T>(xv[j] + a * pv[j]);
                const Acc z = jacobi_z<VEC, PRE>(rv[j], jv[j], i + j < n_);
                ps[j] = static_cast<T>(z + beta * pv[j]);
            }
            st4<VEC>(x, i, n_, xs);
            st4<VEC>(p, i, n_, ps);
        }
    };
    vec_dispatch(vec, pre_, sweep);
}

// Residual replacement: r = b - A x (A x in V_Q), fresh partials for rho_i.
template <class T>
__global__ void __launch_bounds__(256)
k_replace_r(const JobArgs args, const Item* __restrict__ items, int iter) {
    __shared__ double red[32];
    const Item it = items[vec_item()];
    const JobPlan& J = args.jp[it.jp];
    const PlanDev& P = *J.P;
    if (J.status[it.frame] != WMCAO_FRAME_OK) return;
    const T* b = vptr<T>(J, V_B, it.frame);
    const T* q = vptr<T>(J, V_Q, it.frame);
    T* r = vptr<T>(J, V_R, it.frame);
    const T* jac = reinterpret_cast<const T*>(P.jac);
    const bool vec = can_vec4(P.n, {b, q, r, jac});
    Acc rz = 0.0, rr = 0.0;
    const int chunk = P.vec_chunk;
    const int64_t i0 = static_cast<int64_t>(it.b) * chunk;
    const int64_t n_ = P.n;            // plan fields read once: the stores below may alias them
    const bool pre_ = P.precond != 0;
    auto sweep = [&](auto vec_tag, auto pre_tag) {
        constexpr bool VEC = decltype(vec_tag)::value, PRE = decltype(pre_tag)::value;
        for (int k = 4 * threadIdx.x; k < chunk; k += 4 * blockDim.x) {
            const int64_t i = i0 + k;
            if (i >= n_) break;
            Acc bv[4], qv[4], jv[4] = {};
            T rs[4];
            ld4<VEC>(b, i, n_, bv);
            ld4<VEC>(q, i, n_, qv);
            if constexpr (PRE) ld4<VEC>(as_global(jac), i, n_, jv);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rs[j] = static_cast<T>(bv[j] - qv[j]);
                const Acc v = rs[j];
                const Acc z = jacobi_z<VEC, PRE>(v, jv[j], i + j < n_);
                rz += v * z;
                rr += v * v;
            }
            st4<VEC>(r, i, n_, rs);
        }
    };
    vec_dispatch(vec, pre_, sweep);
    block_sum2_first(rz, rr, red);
    if (threadIdx.x == 0) {
        part_ptr(J, it.frame, PT_RZ0 + (iter & 1))[it.slot] = rz;
        part_ptr(J, it.frame, PT_RR0 + (iter & 1))[it.slot] = rr;
    }
}

// ------------------------------------------------------------ plan time ----
struct JacArgs {
    const double* protos;
    const int* proto_off;     // [l][k-1][type]
    const double* txd;
    const double* tyd;
    const double* blocksd;
};

// Jacobi diagonal in closed form, one thread per coefficient.  A level-k
// coefficient (x, y) has the basis function f_x (outer) f_y, f = a shift by
// 2^k * position of the level-k scaling or wavelet prototype; its slopes in
// sensor m are s^x_ij = dF_i sG_j and s^y_ij = sF_i dG_j with F = B_x f_x.
__global__ void __launch_bounds__(128)
k_jacobi(const PlanDev* __restrict__ Pp, JacArgs ja, int64_t n, double* __restrict__ out) {
    const int64_t lam = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lam >= n) return;
    const PlanDev& P = *Pp;
    int l = 0;
    while (l + 1 < P.L && lam >= P.layer[l + 1].coff) ++l;
    const LayerInfo& Ly = P.layer[l];
    const int N = Ly.N;
    const int64_t loc = lam - Ly.coff;
    const int x = static_cast<int>(loc / N), y = static_cast<int>(loc % N);
    // level k (0 without a wavelet transform: the basis is the unit pixel)
    const int k = level_of(x, y, N, P.levels);
    const int kk = k > 0 ? k : 1;
    const int Hk = N >> k;
    const int txy = x >= Hk, tyy = y >= Hk;
    const int ax = txy ? x - Hk : x, ay = tyy ? y - Hk : y;
    const double* fx = ja.protos + ja.proto_off[(l * WM_MAXLEV + (kk - 1)) * 2 + txy];
    const double* fy = ja.protos + ja.proto_off[(l * WM_MAXLEV + (kk - 1)) * 2 + tyy];
    const int shx = ax << k, shy = ay << k;
    double acc = P.alpha * Ly.D[kk - 1];
    for (int m = 0; m < P.W; ++m) {
        const WfsInfo& w = P.wfs[m];
        if (!w.in_precond) continue;
        const int ns = w.n_sub;
        const int no = P.node_tab_off[m][l];
        auto Fv = [&](int i) {
            const int i0 = P.ix0[no + i];
            const double t = ja.txd[no + i];
            int p0 = (i0 - shx) % N;
            if (p0 < 0) p0 += N;
            int p1 = p0 + 1;
            if (p1 == N) p1 = 0;
            return (1.0 - t) * fx[p0] + t * fx[p1];
        };
        auto Gv = [&](int j) {
            const int j0 = P.jy0[no + j];
            const double t = ja.tyd[no + j];
            int p0 = (j0 - shy) % N;
            if (p0 < 0) p0 += N;
            int p1 = p0 + 1;
            if (p1 == N) p1 = 0;
            return (1.0 - t) * fy[p0] + t * fy[p1];
        };
        if (w.kind == 1) {   // phase sensor: sum over active nodes of a (F_i G_j)^2
            const int nn = ns + 1;
            int ilo = nn, ihi = -1, jlo = nn, jhi = -1;
            for (int i = 0; i < nn; ++i)
                if (Fv(i) != 0.0) { if (i < ilo) ilo = i; ihi = i; }
            for (int j = 0; j < nn; ++j)
                if (Gv(j) != 0.0) { if (j < jlo) jlo = j; jhi = j; }
            const double* B = ja.blocksd + w.boff * 3;
            for (int i = ilo; i <= ihi; ++i) {
                const double F = Fv(i);
                for (int j = jlo; j <= jhi; ++j) {
                    const int q = w.maskmap[i * nn + j];
                    if (q < 0) continue;
                    const double v = F * Gv(j);
                    acc += B[3 * q] * v * v;
                }
            }
            continue;
        }
        int ilo = ns, ihi = -1, jlo = ns, jhi = -1;
        double prev = Fv(0);
        for (int i = 0; i < ns; ++i) {
            const double nx = Fv(i + 1);
            if (prev != 0.0 || nx != 0.0) { if (i < ilo) ilo = i; ihi = i; }
            prev = nx;
        }
        if (ihi < 0) continue;
        prev = Gv(0);
        for (int j = 0; j < ns; ++j) {
            const double nx = Gv(j + 1);
            if (prev != 0.0 || nx != 0.0) { if (j < jlo) jlo = j; jhi = j; }
            prev = nx;
        }
        if (jhi < 0) continue;
        // blocks are packed per sensor in slope order: 3 values per measurement
        const double* B = ja.blocksd + w.boff * 3;
        if (!w.agg) {
            for (int i = ilo; i <= ihi; ++i) {
                const double F0 = Fv(i), F1 = Fv(i + 1);
                const double dF = F1 - F0, sF = 0.5 * (F0 + F1);
                for (int j = jlo; j <= jhi; ++j) {
                    const int q = w.maskmap[i * ns + j];
                    if (q < 0) continue;
                    const double G0 = Gv(j), G1 = Gv(j + 1);
                    const double dG = G1 - G0, sG = 0.5 * (G0 + G1);
                    const double sxv = dF * sG, syv = sF * dG;
                    acc += B[3 * q] * sxv * sxv + 2.0 * B[3 * q + 1] * sxv * syv +
                           B[3 * q + 2] * syv * syv;
                }
            }
        } else {
            double cx[WM_MAXCELL], cy[WM_MAXCELL];
            for (int c = 0; c < WM_MAXCELL; ++c) cx[c] = cy[c] = 0.0;
            for (int i = ilo; i <= ihi; ++i) {
                const double F0 = Fv(i), F1 = Fv(i + 1);
                const double dF = F1 - F0, sF = 0.5 * (F0 + F1);
                for (int j = jlo; j <= jhi; ++j) {
                    const int c = w.maskmap[i * ns + j];
                    if (c < 0) continue;
                    const double G0 = Gv(j), G1 = Gv(j + 1);
                    const double dG = G1 - G0, sG = 0.5 * (G0 + G1);
                    cx[c] += dF * sG;
                    cy[c] += sF * dG;
                }
            }
            for (int c = 0; c < w.S; ++c) {
                const double vx = cx[c] / w.cell_count[c], vy = cy[c] / w.cell_count[c];
                acc += B[3 * c] * vx * vx + 2.0 * B[3 * c + 1] * vx * vy + B[3 * c + 2] * vy * vy;
            }
        }
    }
    out[lam] = acc;
}

// out = a x + b y, elementwise (out may alias x or y).
template <class T>
__global__ void __launch_bounds__(256)
k_axpby(int64_t n, double a, const T* x, double b, const T* y, T* out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = static_cast<T>(a * static_cast<Acc>(x[i]) + b * static_cast<Acc>(y[i]));
}

template <class T>
void launch_axpby(int64_t n, double a, const T* x, double b, const T* y, T* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby<T>, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                       n, a, x, b, y, out);
}

// Row i copies len[i] 4-byte words from src[i] to dst[i] (blockIdx.y = row),
// 16 bytes per access where the row allows it: the staging copies of a
// served launch, in one launch before and one after the solve.
__global__ void __launch_bounds__(256)
k_copy_rows(const CopyRows c) {
    const int i = blockIdx.y;
    const int64_t n = c.len[i];
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const uintptr_t al = reinterpret_cast<uintptr_t>(c.src[i]) | reinterpret_cast<uintptr_t>(c.dst[i]);
    if ((al & 15) == 0 && (n & 3) == 0) {
        const uint4* s4 = static_cast<const uint4*>(c.src[i]);
        uint4* d4 = static_cast<uint4*>(c.dst[i]);
        for (int64_t e = t0; e < n / 4; e += step) d4[e] = s4[e];
    } else {
        const uint32_t* s1 = static_cast<const uint32_t*>(c.src[i]);
        uint32_t* d1 = static_cast<uint32_t*>(c.dst[i]);
        for (int64_t e = t0; e < n; e += step) d1[e] = s1[e];
    }
}

void launch_copy_rows(const CopyRows& c, int rows, int64_t max_len, hipStream_t s) {
    if (rows <= 0 || max_len <= 0) return;
    const unsigned bx = static_cast<unsigned>(std::min<int64_t>((max_len / 4 + 255) / 256 + 1, 256));
    hipLaunchKernelGGL(k_copy_rows, dim3(bx, static_cast<unsigned>(rows)), dim3(256), 0, s, c);
}

template <class S, class D>
__global__ void k_cast(const S* in, D* out, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = static_cast<D>(in[i]);
}

// -------------------------------------------------------------- launchers ----
template <class T, class S, class C>
void launch_idwt_coarse(const JobArgs& a, const Item* items, int n, int in_vec, int out_vec,
                        int lds_bytes, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_idwt_coarse<T, S, C>), dim3(n), dim3(1024), lds_bytes, s, a, items, in_vec,
                       out_vec);
}

template <class T, class S, class C>
void launch_idwt_tile(const JobArgs& a, const Item* items, int n, int level, int in_vec,
                      int out_vec, int tile, int lds_bytes, hipStream_t s) {
    if (n <= 0) return;
    if (tile == 16)
        hipLaunchKernelGGL((k_idwt_tile<T, S, C, 16>), dim3(n), dim3(TILE_NT), lds_bytes, s, a, items, level, in_vec, out_vec);
    else if (tile == 64)
        hipLaunchKernelGGL((k_idwt_tile<T, S, C, 64>), dim3(n), dim3(TILE_NT), lds_bytes, s, a, items, level, in_vec, out_vec);
    else
        hipLaunchKernelGGL((k_idwt_tile<T, S, C, 32>), dim3(n), dim3(TILE_NT), lds_bytes, s, a, items, level, in_vec, out_vec);
}

template <class T, class S, class C>
void launch_fdwt_tile(const JobArgs& a, const Item* items, int n, int level, int src, int in_vec,
                      int out_vec, int epi, int aux_vec, int tile, hipStream_t s) {
    if (n <= 0) return;
    if (tile == 16)
        hipLaunchKernelGGL((k_fdwt_tile<T, S, C, 16>), dim3(n), dim3(TILE_NT), 0, s, a, items, level, src, in_vec, out_vec, epi, aux_vec);
    else if (tile == 64)
        hipLaunchKernelGGL((k_fdwt_tile<T, S, C, 64>), dim3(n), dim3(TILE_NT), 0, s, a, items, level, src, in_vec, out_vec, epi, aux_vec);
    else
        hipLaunchKernelGGL((k_fdwt_tile<T, S, C, 32>), dim3(n), dim3(TILE_NT), 0, s, a, items, level, src, in_vec, out_vec, epi, aux_vec);
}

template <class T, class S, class C>
void launch_fdwt_coarse(const JobArgs& a, const Item* items, int n, int src, int in_vec,
                        int out_vec, int epi, int aux_vec, int lds_bytes, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_fdwt_coarse<T, S, C>), dim3(n), dim3(1024), lds_bytes, s, a, items, src, in_vec,
                       out_vec, epi, aux_vec);
}

template <class T, class S>
void launch_project(const JobArgs& a, const Item* items, int n, int in_vec, int sums, int lds_bytes,
                    int max_layers, hipStream_t s) {
    if (n <= 0) return;
    if (n <= PROJ_WIDE_MAX && max_layers > PROJ_LB)
        hipLaunchKernelGGL((k_project<T, S, PROJ_LB_WIDE>), dim3(n), dim3(512), lds_bytes, s, a, items, in_vec, sums);
    else
        hipLaunchKernelGGL((k_project<T, S, PROJ_LB>), dim3(n), dim3(512), lds_bytes, s, a, items, in_vec, sums);
}

template <class T, class S>
void launch_weights(const JobArgs& a, const Item* items, int n, int out_vec, int lds_bytes,
                    hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_weights<T, S>), dim3(n), dim3(256), lds_bytes, s, a, items, out_vec);
}

template <class T, class S, class C>
void launch_adjoint(const JobArgs& a, const Item* items, int n, int in_vec, int out_vec,
                    int lds_bytes, int taps, hipStream_t s) {
    if (n <= 0) return;
    if (taps <= 2)
        hipLaunchKernelGGL((k_adjoint<T, S, C, 2>), dim3(n), dim3(256), lds_bytes, s, a, items, in_vec, out_vec);
    else if (taps == 3)
        hipLaunchKernelGGL((k_adjoint<T, S, C, 3>), dim3(n), dim3(256), lds_bytes, s, a, items, in_vec, out_vec);
    else
        hipLaunchKernelGGL((k_adjoint<T, S, C, 4>), dim3(n), dim3(256), lds_bytes, s, a, items, in_vec, out_vec);
}

template <class T, class S>
void launch_sensor(const JobArgs& a, const Item* items, int n, int mode, int in_vec, int out_vec,
                   int lds_bytes, hipStream_t s) {
    if (n <= 0) return;
    // lds_bytes carries the node-field size; elements per thread follow from it
    const int elems = lds_bytes / static_cast<int>(sizeof(Acc));
    if (elems <= 8 * 1024)
        hipLaunchKernelGGL((k_sensor<T, S, 8>), dim3(n), dim3(1024), lds_bytes, s, a, items, mode, in_vec, out_vec);
    else
        hipLaunchKernelGGL((k_sensor<T, S, 16>), dim3(n), dim3(1024), lds_bytes, s, a, items, mode, in_vec, out_vec);
}

template <class T>
void launch_init(const JobArgs& a, const Item* items, int n, int warm, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_init<T>, dim3(n), dim3(256), 0, s, a, items, warm);
}

template <class T>
void launch_update_r(const JobArgs& a, const Item* items, int n, int iter, int fresh, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update_r<T>, dim3(n), dim3(256), 0, s, a, items, iter, fresh);
}

template <class T>
void launch_update_p(const JobArgs& a, const Item* items, int n, int iter, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update_p<T>, dim3(n), dim3(256), 0, s, a, items, iter);
}

template <class T>
void launch_replace_r(const JobArgs& a, const Item* items, int n, int iter, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_replace_r<T>, dim3(n), dim3(256), 0, s, a, items, iter);
}

void launch_jacobi(const PlanDev* P, const double* protos, const int* proto_off,
                   const double* txd, const double* tyd, const double* blocksd, int64_t n,
                   double* out, hipStream_t s) {
    JacArgs ja{protos, proto_off, txd, tyd, blocksd};
    const int nb = static_cast<int>((n + 127) / 128);
    hipLaunchKernelGGL(k_jacobi, dim3(nb), dim3(128), 0, s, P, ja, n, out);
}

template <class S, class D>
void launch_cast(const S* in, D* out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int nb = static_cast<int>((n + 255) / 256);
    hipLaunchKernelGGL((k_cast<S, D>), dim3(nb), dim3(256), 0, s, in, out, n);
}

// Let the whole-band kernels use up to the 160 KB of LDS of a CDNA4 compute
// unit (static shared memory included); clear any error this leaves behind.
template <class K>
static void allow_full_lds(K* k) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void*>(k)) == hipSuccess) {
        const int dyn = 160 * 1024 - static_cast<int>(at.sharedSizeBytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    }
    (void)hipGetLastError();
}

template <class T, class S, class C>
static void allow_full_lds_ops() {
    allow_full_lds(&k_idwt_coarse<T, S, C>);
    allow_full_lds(&k_idwt_tile<T, S, C, 16>);
    allow_full_lds(&k_idwt_tile<T, S, C, 32>);
    allow_full_lds(&k_idwt_tile<T, S, C, 64>);
    allow_full_lds(&k_fdwt_coarse<T, S, C>);
    allow_full_lds(&k_adjoint<T, S, C, 2>);
    allow_full_lds(&k_adjoint<T, S, C, 3>);
    allow_full_lds(&k_adjoint<T, S, C, 4>);
}

void configure_kernels() {
    allow_full_lds_ops<float, float, float>();
    allow_full_lds_ops<float, float, double>();
    allow_full_lds_ops<float, double, double>();
    allow_full_lds_ops<double, double, double>();
    allow_full_lds(&k_sensor<float, float, 8>);
    allow_full_lds(&k_sensor<float, float, 16>);
    allow_full_lds(&k_sensor<float, double, 8>);
    allow_full_lds(&k_sensor<float, double, 16>);
    allow_full_lds(&k_sensor<double, double, 8>);
    allow_full_lds(&k_sensor<double, double, 16>);
}

// Wavelet and adjoint-projection stages: vector storage T, operator storage S,
// arithmetic C.
#define WM_INSTANTIATE_STAGES(T, S, C)                                                             \
    template void launch_idwt_coarse<T, S, C>(const JobArgs&, const Item*, int, int, int, int, hipStream_t); \
    template void launch_idwt_tile<T, S, C>(const JobArgs&, const Item*, int, int, int, int, int, int, hipStream_t); \
    template void launch_fdwt_tile<T, S, C>(const JobArgs&, const Item*, int, int, int, int, int, int, int, int, hipStream_t); \
    template void launch_fdwt_coarse<T, S, C>(const JobArgs&, const Item*, int, int, int, int, int, int, int, hipStream_t); \
    template void launch_adjoint<T, S, C>(const JobArgs&, const Item*, int, int, int, int, int, hipStream_t);

// Projection and sensor stages (FP64 arithmetic): vector storage T, operator storage S.
#define WM_INSTANTIATE_SENSORS(T, S)                                                               \
    template void launch_sensor<T, S>(const JobArgs&, const Item*, int, int, int, int, int, hipStream_t); \
    template void launch_project<T, S>(const JobArgs&, const Item*, int, int, int, int, int, hipStream_t); \
    template void launch_weights<T, S>(const JobArgs&, const Item*, int, int, int, hipStream_t);

// The PCG vector steps: storage T.
#define WM_INSTANTIATE_VEC(T)                                                                      \
    template void launch_init<T>(const JobArgs&, const Item*, int, int, hipStream_t);             \
    template void launch_update_r<T>(const JobArgs&, const Item*, int, int, int, hipStream_t);    \
    template void launch_update_p<T>(const JobArgs&, const Item*, int, int, hipStream_t);         \
    template void launch_replace_r<T>(const JobArgs&, const Item*, int, int, hipStream_t);        \
    template void launch_axpby<T>(int64_t, double, const T*, double, const T*, T*, hipStream_t);

WM_INSTANTIATE_STAGES(float, float, float)
WM_INSTANTIATE_STAGES(float, float, double)
WM_INSTANTIATE_STAGES(float, double, double)
WM_INSTANTIATE_STAGES(double, double, double)
WM_INSTANTIATE_SENSORS(float, float)
WM_INSTANTIATE_SENSORS(float, double)
WM_INSTANTIATE_SENSORS(double, double)
WM_INSTANTIATE_VEC(float)
WM_INSTANTIATE_VEC(double)
template void launch_cast<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_cast<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_cast<float, float>(const float*, float*, int64_t, hipStream_t);
template void launch_cast<double, double>(const double*, double*, int64_t, hipStream_t);

}  // namespace wm
