// Internal structures shared by the plan builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wmcao.h"

#define WM_MAXL 16        // layers per plan
#define WM_MAXW 32        // sensors per plan
#define WM_MAXLEV 8       // wavelet levels
#define WM_MAXCELL 16     // cells of a low-order sensor (k <= 4)
#define WM_MAXJP 8        // plans packed into one launch
#define WM_QMAX 16        // elements per thread of the 1024-thread kernels
#define WM_NSUB_MAX 127   // nodes per sensor <= 128^2

namespace wm {

// Kinds of per-frame vectors a kernel can read or write.
enum Vec : int {
    V_X = 0,      // caller's coefficients (x0 in, x out)
    V_B,          // right side
    V_R,          // residual
    V_P,          // search direction
    V_Q,          // A p
    V_PHI,        // layer pixel fields (scratch, operator type)
    V_LL,         // intermediate low-pass bands (scratch, operator type)
    V_NODE,       // adjoint sensor node fields (scratch, operator type)
    V_SLOPES,     // caller's slopes (in)
    V_IN,         // caller's generic input
    V_OUT,        // caller's generic output
    V_U,          // sensor node fields of the projection, FP64 (scratch)
    V_FP,         // per (sensor, layer) adjoint-projection footprint images (scratch, operator type)
    V_SPART,      // per (sensor, node band) slope sums for tip/tilt and cells, FP64 (scratch)
    NV
};

// Per-frame partial-sum segments (deterministic reductions, one slot per block).
enum Part : int { PT_PQ = 0, PT_RZ0, PT_RZ1, PT_RR0, PT_RR1, NPT };

struct LayerInfo {
    int N;                          // pixels per side
    int k0;                         // levels done by tiled kernels (0..levels-1)
    int fuse;                       // 1: the level-k0 synthesis tiles rebuild LL_k0 themselves
    int64_t coff;                   // offset in a coefficient / pixel frame vector
    int64_t ll_off[WM_MAXLEV + 1];  // offset of LL_k (k = 1..k0) in a frame's LL scratch
    double D[WM_MAXLEV];            // prior at scale index k (entry k-1), alpha not applied
};

struct WfsInfo {
    int n_sub, nn;          // subapertures across, nodes across (n_sub + 1)
    int S_fine;             // active fine subapertures
    int S;                  // measurements (S_fine, or active cells)
    int agg;                // 0 or k of a k x k low-order sensor
    int remove_tt;
    int in_precond;
    int kind;               // 0: Fried Shack-Hartmann; 1: phase at the pupil nodes
    int64_t soff;           // slope offset in a frame
    int64_t node_off;       // node-field offset in a frame's node scratch
    int64_t boff;           // index of the sensor's first noise block
    const int* act;         // [S_fine] packed i * n_sub + j (row-major); phase: node i * nn + j
    const int* cell_of;     // [S_fine] measurement (cell) index of each fine subaperture
    const int* cell_count;  // [S] fine subapertures per cell
    const double* blocks;   // [S][3] (a, b, c) of the symmetric 2x2 block of C~^-1
    const int* maskmap;     // [n_sub^2] measurement of a fine subaperture or -1 (phase: [nn^2] per node)
    int sp_off;             // first slope-sum record of the sensor in a V_SPART frame
    int pad_;
    double bsum[3];         // sums over the measurements of the noise-block entries a, b, c
};

struct PlanDev {
    int L, W, levels, dtype;
    int op64;               // 1: operator storage S = double, 0: S = float
    int proj_rows;          // sensor node rows per work item of the projection (one slope record each)
    int wgt_rows;           // sensor node rows per work item of the noise weighting
    int vec_chunk;          // elements per work item of the vector kernels
    int precond;
    int n_fdwt_slots;       // partial slots written by one wavelet-analysis pass per frame
    int pq_base;            // first of the L per-layer <p, Ap> totals
    int n_vec_slots;        // partial slots written by one vector pass per frame
    int slots;              // stride of one partial segment
    int64_t n, n_slopes, n_nodes, ll_size;
    double alpha;
    double h[6], g[6];      // db3 analysis filters
    LayerInfo layer[WM_MAXL];
    WfsInfo wfs[WM_MAXW];
    // projection tables, per (sensor, layer): node_tab_off -> [nn] entries,
    // pix_tab_off -> [N_l] entries.
    const int* ix0;
    const int* jy0;
    const double* tx;       // bilinear weight of the right/upper pixel per node
    const double* ty;
    // node i of sensor m sits at grid coordinate u = pa * i + pb[axis] on layer l
    // (Sec. 2.1 with the cone factor): the forward and adjoint projections
    // evaluate their bilinear weights from it.
    double pa[WM_MAXW][WM_MAXL];
    double pia[WM_MAXW][WM_MAXL];       // 1 / pa
    double pb[2][WM_MAXW][WM_MAXL];
    const int* tmeta;       // per (layer, level-1 tile), one per layer if k0 = 0: bit m set
                            // if sensor m reaches the tile's pixel window
    // adjoint-projection footprint of sensor m on layer l: pixel rows
    // fp_x0 .. fp_x0 + fp_h - 1, columns fp_y0 .. fp_y0 + fp_w - 1; its image
    // starts at fp_off in a V_FP frame; fp_rc + 2 * fp_tab holds (first node,
    // node count) per footprint row, then per footprint column, then (first,
    // last) node row per band of fp_br rows (one work item each).
    int fp_x0[WM_MAXW][WM_MAXL], fp_y0[WM_MAXW][WM_MAXL];
    int fp_h[WM_MAXW][WM_MAXL], fp_w[WM_MAXW][WM_MAXL];
    int fp_off[WM_MAXW][WM_MAXL], fp_tab[WM_MAXW][WM_MAXL], fp_br[WM_MAXW][WM_MAXL];
    const int* fp_rc;
    int tmeta_off[WM_MAXL];
    int node_tab_off[WM_MAXW][WM_MAXL];
    const void* jac;        // [n] Jacobi diagonal, plan dtype
};

struct JobPlan {
    const PlanDev* P;       // device copy of the plan constants
    void* vec[NV];          // frame-0 base pointer of each vector kind
    int64_t stride[NV];     // frame stride (elements)
    double* part;           // [frames][NPT * slots]
    double* alpha;          // [frames] step size of the current iteration
    int* status;            // [frames] WMCAO_FRAME_*
    double* resid;          // optional [frames][resid_ld]
    int resid_ld;
    int nframes;
};

struct JobArgs {
    int njp;
    int pad_;
    JobPlan jp[WM_MAXJP];
};

// One block's work: plan slot, frame, layer or sensor, tile or chunk, partial slot.
struct Item {
    int jp, frame, a, b, slot, pad0, pad1, pad2;
};

enum SrcMode : int { SRC_LL = 0, SRC_PIX = 1, SRC_PT = 2 };
enum EpiMode : int { EPI_NONE = 0, EPI_APPLY = 1 };
enum SensorMode : int { SM_APPLY = 0, SM_RHS = 1, SM_FWD = 2, SM_PAPPLY = 3 };

// ---- launchers (defined in wmcao_kernels.hip) --------------------------------
// T: storage of the PCG vectors and of the caller's slopes; S: storage of the
// operator's intermediates (low-pass scratch, layer pixels, adjoint node fields
// and footprint images); C: arithmetic and LDS tiles of the wavelet and
// adjoint-projection stages.
template <class T, class S, class C>
void launch_idwt_coarse(const JobArgs& a, const Item* items, int n, int in_vec, int out_vec,
                        int lds_bytes, hipStream_t s);
template <class T, class S, class C>
void launch_idwt_tile(const JobArgs& a, const Item* items, int n, int level, int in_vec,
                      int out_vec, int tile, int lds_bytes, hipStream_t s);
template <class T, class S, class C>
void launch_fdwt_tile(const JobArgs& a, const Item* items, int n, int level, int src, int in_vec,
                      int out_vec, int epi, int aux_vec, int tile, hipStream_t s);
template <class T, class S, class C>
void launch_fdwt_coarse(const JobArgs& a, const Item* items, int n, int src, int in_vec,
                        int out_vec, int epi, int aux_vec, int lds_bytes, hipStream_t s);
template <class T, class S>
void launch_project(const JobArgs& a, const Item* items, int n, int in_vec, int sums, int lds_bytes,
                    int max_layers, hipStream_t s);
template <class T, class S>
void launch_weights(const JobArgs& a, const Item* items, int n, int out_vec, int lds_bytes,
                    hipStream_t s);
template <class T, class S, class C>
void launch_adjoint(const JobArgs& a, const Item* items, int n, int in_vec, int out_vec,
                    int lds_bytes, int taps, hipStream_t s);
template <class T, class S>
void launch_sensor(const JobArgs& a, const Item* items, int n, int mode, int in_vec, int out_vec,
                   int lds_bytes, hipStream_t s);
template <class T>
void launch_init(const JobArgs& a, const Item* items, int n, int warm, hipStream_t s);
template <class T>
void launch_update_r(const JobArgs& a, const Item* items, int n, int iter, int fresh, hipStream_t s);
template <class T>
void launch_update_p(const JobArgs& a, const Item* items, int n, int iter, hipStream_t s);
template <class T>
void launch_replace_r(const JobArgs& a, const Item* items, int n, int iter, hipStream_t s);
void launch_jacobi(const PlanDev* P, const double* protos, const int* proto_off,
                   const double* txd, const double* tyd, const double* blocksd,
                   int64_t n, double* out, hipStream_t s);
void configure_kernels();
template <class T>
void launch_axpby(int64_t n, double a, const T* x, double b, const T* y, T* out, hipStream_t s);
template <class S, class D>
void launch_cast(const S* in, D* out, int64_t n, hipStream_t s);

constexpr int SERVE_ROWS = 40;   // rows of one staging copy (2 x 16 frames in, or results out)
struct CopyRows {
    const void* src[SERVE_ROWS];
    void* dst[SERVE_ROWS];
    int64_t len[SERVE_ROWS];   // 4-byte words
};
void launch_copy_rows(const CopyRows& c, int rows, int64_t max_len, hipStream_t s);

constexpr size_t NOALLOC_BYTES = size_t(32) << 20;   // scratch of the allocation-free solve
constexpr int FUSE_LDS = 32 * 1024;   // largest low-pass block a synthesis tile rebuilds
constexpr int TILE_NT = 256;          // threads of a wavelet tile block
constexpr int VEC_CHUNK = 2048;   // default elements per work item of the vector kernels
constexpr int PROJ_ROWS = 8;      // default node rows per projection work item
constexpr int PROJ_ROWS_MIN = 4;  // fewest node rows per projection work item
constexpr int PROJ_ROWS_MAX = 48; // most node rows per projection work item
constexpr int WGT_ROWS_MAX = 8;   // most node rows per weighting work item
constexpr int SENSOR_FUSE_NN = 40;   // sensors of at most this many nodes per side project in k_sensor

// Dynamic LDS of k_weights for a sensor of nn nodes and ns subapertures per
// side: the band's node rows with one halo row on each side and the weighted
// x and y slopes of the subaperture rows next to the band (FP64).
constexpr int weights_lds_bytes(int nn, int ns, int rows) {
    return ((rows + 2) * nn + 2 * (rows + 1) * ns) * 8;
}
// Dynamic LDS of k_project for L layers, a sensor of nn nodes per side and
// `rows` node rows per item: the u window of rows + 1 node rows (FP64), then
// per layer an FP64 weight and an int per node column and per window row.
constexpr int proj_lds_bytes(int L, int nn, int rows) {
    return (rows + 1) * nn * 8 + L * nn * 12 + L * (rows + 1) * 12;
}
constexpr int SP_K = 2 * WM_MAXCELL;   // doubles per slope-sum record
constexpr int ADJ_BAND = 32;      // footprint rows per adjoint work item (at most)
constexpr int ADJ_TAPS_MAX = 4;   // most fast-path taps of the adjoint
constexpr int ADJ_LDS = 32 * 1024;   // default LDS of the adjoint's staged rows and row-pass buffer

}  // namespace wm
