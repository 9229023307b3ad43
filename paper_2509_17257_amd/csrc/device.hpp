// Internal device-side layout of an H^2 operator and the launchers of each stage.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace h2x {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Raw buffer resource over [p, p + bytes) (no stride or swizzle; a load past the end returns
// zeros); the last descriptor word is the default data format of the gfx9 family.  Loads
// through it take a wave-uniform base in scalar registers and a 32-bit byte offset per lane,
// which leaves out the 64-bit address arithmetic of global loads.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
// cache policy of a buffer load: 0 the default, kBufNT streaming (non-temporal)
constexpr int kBufNT = 2;
template <int POL>
__device__ inline u32x4 buf_ld16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, POL);
}
template <int POL>
__device__ inline float buf_ld4f(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, POL));
}
template <int POL>
__device__ inline u32x2 buf_ld8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, POL);
}

// Tile choices of the matrix-core paths (0: the default rule), filled by the
// autotuner per bucket of the column count: bucket b holds ceil(m / 16) = b + 1
// for b < 4, bucket 4 anything wider.
struct TuneCfg {
    int8_t nj_transfer = 0;  // 16-column tiles per work-group: forward leaf, transfer passes
    int8_t nj_coupling = 0;  // 16-column tiles per work-group: coupling
    int8_t np_leaf = 0;      // 32-column tiles per work-group: leaf stage
    int8_t fuse_up = 0;      // forward leaf and upward pass in one launch: 1 on; 0 (built-in
                             // rule) and 2 off
    int8_t overlap = 0;      // near field on a second stream during the transfer passes and
                             // the coupling: 0 (built-in rule) and 2 off; on with a grid
                             // of 256 (1), 128 (3) or 512 (4) work-groups
    int8_t leaf_kind = 0;    // leaf stage: 0 built-in rule (3 where it applies, else 1), 1 wave-per-term
                             // tiles, 2 rows split over waves, 3 one contraction per leaf
    int8_t split = 0;        // coupling of the deep rows on the second stream beside the upper
                             // transfer levels: 0 built-in rule, 1 on (leaving room on every
                             // CU for a transfer work-group), 2 off, 3 on without the reserve
};
constexpr int kTuneBuckets = 5;
inline int tune_bucket(int64_t m) { return (int)std::min<int64_t>(kTuneBuckets - 1, (m + 15) / 16 - 1); }

// Flat device arrays of one operator, all inside the caller's workspace.
struct DevMat {
    int64_t n = 0;
    int32_t C = 0, L = 0, k = 0, p = 0, depth_max = 0, max_leaf = 0, max_near_rows = 0;
    int32_t leaf_half = 0;  // see Plan::leaf_half
    int64_t n_adm = 0, n_near = 0, near_entries = 0;
    h2x_prec storage = H2X_F64;
    int swz = 0;     // coupling-matrix layout (see s_index)
    int near_t = 0;  // near-field blocks stored transposed (|s| x |t| row-major)
    int mc = 0;      // every stage runs on the matrix cores (FP64, k = 64 or k <= 32)
    int kernel = 0;
    int cplx = 0;                   // complex kernel: S and N hold a real and an imaginary plane
    int64_t s_plane = 0, n_plane = 0;  // elements per plane of S and N
    double ell = 0, shift = 0;

    // topology
    int32_t *first = nullptr, *size = nullptr, *parent = nullptr, *son0 = nullptr, *son1 = nullptr;
    int32_t *leaves = nullptr, *lvl_all = nullptr, *lvl_inner = nullptr;
    int32_t *up_son = nullptr;  // 2 per entry of lvl_inner: its two sons
    int32_t *dn_par = nullptr;  // per entry of lvl_all: its parent (-1 at the root)
    int64_t *adm_ptr = nullptr;  // C + 1
    int32_t *adm_col = nullptr;  // n_adm
    int32_t *adm_row = nullptr;  // n_adm (row cluster of each block)
    int32_t *cpl_order = nullptr;  // C, launch order of the coupling rows
    int32_t *leaf_order = nullptr; // L, launch order of the leaves (one contraction per leaf)
    int32_t *cpl_deep = nullptr, *cpl_shallow = nullptr;  // the same rows in two parts
    int32_t n_deep = 0, n_shallow = 0, split_depth = 0;   // (split_depth 0: no split)
    int64_t *near_ptr = nullptr; // L + 1
    int32_t *near_col = nullptr; // n_near
    int32_t *near_row = nullptr; // n_near (row leaf cluster)
    int64_t *near_off = nullptr; // n_near (offsets in the layout selected by near_t)
    int64_t *vt_off = nullptr;   // L, offsets of the transposed leaf bases (matrix-core layout)
    int64_t *near_off_rm = nullptr;  // n_near, offsets of row-major |t| x |s| blocks (gradient output)
    int64_t *adm_cptr = nullptr, *adm_cblk = nullptr;    // admissible blocks by column cluster
    int64_t *near_cptr = nullptr, *near_cblk = nullptr;  // near-field blocks by column leaf
    int32_t *sys_of = nullptr;   // C, system of each cluster
    int32_t *depth = nullptr;    // C, depth of each cluster
    int64_t *perm = nullptr;     // n
    double *pts = nullptr;       // n x 3 tree order
    double *box = nullptr;       // C x 6
    double *nodes = nullptr;     // C x k x 3

    // operator (element type per `storage`; near field FP64 or FP32)
    void *V = nullptr;   // n x k
    void *E = nullptr;   // C x k x k
    double *E1 = nullptr;  // C x 3 x p x p: one-dimensional factors of the transfer matrices (FP64)
    void *S = nullptr;   // n_adm x k x k
    void *N = nullptr;   // near field (row-major blocks, or transposed and padded when near_t)
    void *Vt = nullptr;  // transposed leaf bases (matrix-core layout only)

    // host copies of the level tables (launch sizes)
    const Plan *plan = nullptr;

    TuneCfg tuned[kTuneBuckets];

    // second stream and fork / join events of the operator (near field concurrent with
    // the transfer passes); null when not created
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

};

inline int s_swizzled(const DevMat &dm) { return dm.swz; }

// Work of clusters whose system has stopped can be left out of a product: flag
// holds one entry per system (nonzero: stopped), sys_of the system of each
// cluster.  A default-constructed Skip leaves nothing out.
struct Skip {
    const int32_t *flag = nullptr;
    const int32_t *sys_of = nullptr;
    __device__ bool operator()(int32_t c) const { return flag && flag[sys_of[c]]; }
};

size_t mat_layout(const Plan &P, h2x_prec storage, DevMat *dm, char *base);

hipError_t launch_fill(const DevMat &dm, hipStream_t st);

size_t matmul_ws_bytes(const DevMat &dm, int64_t m);
// ev (optional): 7 events recorded on the stream: before the first stage, after
// each of the 5 stages, and (ev[6]) after the near field, which the matrix-core
// path fuses into the leaf stage
// skip (optional, device, one flag per system of the plan): clusters of systems
// whose flag is set are left out (their rows of Y are not written); honoured on
// the matrix-core path
hipError_t run_matmul(const DevMat &dm, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                      double *Y, int64_t ldy, bool tree_order, char *ws, hipStream_t st,
                      hipEvent_t *ev = nullptr, const int32_t *skip = nullptr);

// the product with explicit tile choices (the autotuner's candidates)
hipError_t run_matmul_cfg(const DevMat &dm, const TuneCfg &cfg, int64_t m, double alpha, const double *X, int64_t ldx,
                          double beta, double *Y, int64_t ldy, bool tree_order, char *ws, hipStream_t st,
                          hipEvent_t *ev, const int32_t *skip);
size_t autotune_ws_bytes(const DevMat &dm, int64_t m);
h2x_status run_autotune(DevMat &dm, int64_t m, char *ws, size_t ws_bytes, hipStream_t st, h2x_tune_info *info);

size_t cg_ws_bytes(const DevMat &dm, int64_t m);
size_t cg_batch_ws_bytes(const DevMat *const *mats, int32_t nmat, int64_t m);
// hi (optional, one operator and one system only): mixed precision with residual
// replacement -- iterations use mats[0], the residual is recomputed with hi
h2x_status run_block_cg_batch(const DevMat *const *mats, int32_t nmat, const h2x_cg_params &prm, int64_t m,
                              const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                              h2x_cg_info *info, hipStream_t st, const DevMat *hi = nullptr, double delta = 0.0);
size_t mixed_ws_bytes(const DevMat &hi, const DevMat &lo, int64_t m);
h2x_status run_block_cg_mixed(const DevMat &hi, const DevMat &lo, const h2x_cg_params &prm, double delta, int64_t m,
                              const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                              h2x_cg_info *info, hipStream_t st);
h2x_status run_block_cg(const DevMat &dm, const h2x_cg_params &prm, int64_t m, const double *B, int64_t ldb,
                        double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info, hipStream_t st);

size_t gmres_ws_bytes(const DevMat &dm, int64_t m, int ell);

// right-hand-side chunking
size_t solve_ws_bytes(const DevMat &dm, int32_t solver, int64_t m, int32_t restart);
h2x_status choose_chunk(const DevMat &dm, int32_t solver, int32_t restart, int64_t m, size_t mem_bytes, int32_t ncand,
                        const int64_t *cand, const double *ms, int64_t *m_chunk);
size_t product_times_ws_bytes(const DevMat &dm, int32_t ncand, const int64_t *cand);
h2x_status run_product_times(const DevMat &dm, int32_t ncand, const int64_t *cand, int32_t reps, char *ws,
                             size_t ws_bytes, hipStream_t st, double *ms);
h2x_status run_cg_chunked(const DevMat &dm, const h2x_cg_params &prm, int64_t m, int64_t mc, const double *B,
                          int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info,
                          hipStream_t st);
h2x_status run_gmres_chunked(const DevMat &dm, const h2x_gmres_params &prm, int64_t m, int64_t mc, const double *B,
                             int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_gmres_info *info,
                             hipStream_t st);
h2x_status run_block_gmres(const DevMat &dm, const h2x_gmres_params &prm, int64_t m, const double *B, int64_t ldb,
                           double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_gmres_info *info, hipStream_t st);

// forward transformation of X into x-hat (leaves and every cluster at or below the
// shallowest admissible depth); FP64 operators only
hipError_t run_forward_transform(const DevMat &dm, int64_t m, const double *X, int64_t ldx, bool tree_order,
                                 double *xh, int64_t ldh, double *xt_ws, hipStream_t st);
hipError_t run_down_pass(const DevMat &dm, int64_t m, double *yh, int64_t ldh, hipStream_t st);

// adjoint product Y = beta Y + alpha A^T X (column lists, transposed blocks)
hipError_t run_matmul_adjoint(const DevMat &dm, int64_t m, double alpha, const double *X, int64_t ldx, double beta,
                              double *Y, int64_t ldy, char *ws, hipStream_t st);
size_t adjoint_ws_bytes(const DevMat &dm, int64_t m);
size_t grad_ws_bytes(const DevMat &dm, int64_t m);
hipError_t run_grad(const DevMat &dm, int64_t m, const double *X, int64_t ldx, const double *dY, int64_t lddy,
                    double *dS, double *dN, double *dell, double scale, int32_t dell_terms, char *ws,
                    hipStream_t st);
hipError_t refill_ell(DevMat &dm, double ell, hipStream_t st);
hipError_t run_read_coupling(const DevMat &dm, double *out, hipStream_t st);
hipError_t run_write_coupling(const DevMat &dm, const double *in, hipStream_t st);

size_t bcg_ws_bytes(const DevMat &dm, int64_t m);
h2x_status run_block_cg_shared(const DevMat &dm, const h2x_cg_params &prm, int64_t m, const double *B, int64_t ldb,
                               double *X, int64_t ldx, char *ws, size_t ws_bytes, h2x_cg_info *info,
                               hipStream_t st);

size_t refine_ws_bytes(const DevMat &hi, const DevMat &lo, int64_t m);
h2x_status run_refine(const DevMat &hi, const DevMat &lo, const h2x_cg_params &inner, double rtol, int32_t max_outer,
                      int64_t m, const double *B, int64_t ldb, double *X, int64_t ldx, char *ws, size_t ws_bytes,
                      h2x_cg_info *info, hipStream_t st);

}  // namespace h2x

struct h2x_plan {
    h2x::Plan *p;
};

struct h2x_mat {
    const h2x_plan *plan;
    h2x::DevMat dm;
    size_t ws_bytes;
};

struct h2x_batch {
    std::vector<const h2x_mat *> mats;
    std::vector<const h2x::DevMat *> dms;
};
