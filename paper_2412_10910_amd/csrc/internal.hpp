// Internal declarations shared by the host orchestration and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "nnmg.h"

namespace nnmg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

#define NNMG_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::nnmg::fail(NNMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// context and device memory
// ---------------------------------------------------------------------------
struct Ctx {
    int device = 0;
    nnmg_allocator alloc{};
    bool custom = false;
    void* noalloc_scratch = nullptr;  // device address of this device's static scratch array
    void* allocate(size_t bytes);
    void release(void* p);
};

template <class T>
struct DeviceArray {
    Ctx* ctx = nullptr;
    T* ptr = nullptr;
    size_t n = 0;
    DeviceArray() = default;
    DeviceArray(const DeviceArray&) = delete;
    DeviceArray& operator=(const DeviceArray&) = delete;
    DeviceArray(DeviceArray&& o) noexcept { swap(o); }
    DeviceArray& operator=(DeviceArray&& o) noexcept {
        reset();
        swap(o);
        return *this;
    }
    ~DeviceArray() { reset(); }
    void swap(DeviceArray& o) noexcept {
        std::swap(ctx, o.ctx);
        std::swap(ptr, o.ptr);
        std::swap(n, o.n);
    }
    void reset() {
        if (ptr) ctx->release(ptr);
        ptr = nullptr;
        n = 0;
    }
    void alloc(Ctx* c, size_t count) {
        reset();
        ctx = c;
        n = count;
        if (count) ptr = static_cast<T*>(c->allocate(count * sizeof(T)));
    }
    void upload(Ctx* c, const T* host, size_t count) {
        alloc(c, count);
        if (count) NNMG_HIP(hipMemcpy(ptr, host, count * sizeof(T), hipMemcpyHostToDevice));
    }
    void upload(Ctx* c, const std::vector<T>& v) { upload(c, v.data(), v.size()); }
    std::vector<T> download() const {
        std::vector<T> out(n);
        if (n) NNMG_HIP(hipMemcpy(out.data(), ptr, n * sizeof(T), hipMemcpyDeviceToHost));
        return out;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// 1D tables of the Q_k element (Gauss points, Gauss-Lobatto nodes)
// ---------------------------------------------------------------------------
constexpr int kMaxN = 5;

struct Basis1D {
    int n = 0;                      // k + 1
    double gauss[kMaxN]{};          // Gauss-Legendre points on [0,1]
    double weight[kMaxN]{};         // and weights
    double node[kMaxN]{};           // Gauss-Lobatto support points on [0,1]
    double bary[kMaxN]{};           // barycentric weights 1 / prod_{m!=a}(x_a - x_m)
    double S[kMaxN][kMaxN]{};       // S[q][a]  = phi_a(g_q)   nodal basis at Gauss points
    double DS[kMaxN][kMaxN]{};      // DS[q][a] = phi_a'(g_q)
    double D[kMaxN][kMaxN]{};       // D[q][p]  = psi_p'(g_q)  collocation derivative on Gauss points
};

Basis1D make_basis(int degree);

// ---------------------------------------------------------------------------
// a level: one mesh and its Q_k space
// ---------------------------------------------------------------------------
struct Level {
    Ctx* ctx = nullptr;
    std::atomic<int> refs{1};
    int dim = 0, degree = 0, n = 0, q = 0;
    int wg = 64;        // lanes per block of the operator kernel
    int cpb = 0;        // cells per block of the operator kernel
    int64_t nblocks = 0;
    int64_t n_cells = 0, n_dofs = 0, n_free = 0;  // n_dofs = ncomp * n_nodes (vector DoFs interleaved by node)
    int64_t n_nodes = 0;     // scalar Q_k nodes
    int ncomp = 1;           // 1: Laplace; dim: linear elasticity
    int op = 0;              // NNMG_OP_LAPLACE or NNMG_OP_ELASTICITY
    double lam = 1.0, mu = 1.0;  // Lame coefficients of the elasticity operator
    Basis1D basis;

    std::vector<double> vertices;    // [V][dim]
    std::vector<int32_t> cells;      // [C][2^dim]
    std::vector<double> support;     // [N][dim]
    std::vector<int32_t> dofmap;     // [C][q] global DoF of every local node
    std::vector<uint8_t> constrained;  // [n_nodes] node mask (every component of a constrained node is fixed)
    std::vector<int32_t> constrained_idx;  // constrained vector DoFs

    DeviceArray<int32_t> d_dofmap;      // [C][q], -1 for constrained DoFs
    DeviceArray<int32_t> d_dofmap_blk;  // operator layout [blk][n][wg], -1 for constrained / padding
    DeviceArray<double> d_metric64;     // operator layout [blk][M][n][wg] (kept while a precision reads it)
    DeviceArray<float> d_metric32;
    DeviceArray<double> d_coef64;       // [blk][NC][cpb] Q1 map coefficients (mode 1)
    DeviceArray<float> d_coef32;
    DeviceArray<double> d_cellverts;    // [C][2^dim][dim]
    DeviceArray<int32_t> d_constrained;
    std::vector<int32_t> order;         // [nblocks * cpb] cell at each block position, -1 = padding
    DeviceArray<int32_t> d_order;
    DeviceArray<int32_t> d_inv_off;     // [N+1] contributions of DoF i: contrib[off[i] .. off[i+1]) (per-node layout)
    DeviceArray<int32_t> d_pos_blk;     // operator layout: contribution slot of each (lane, node), -1 = none,
                                        // | kMergeNext: add the next cell's first node of the line first
    // Entity-compressed operator indices (3D Laplace, degree >= 3; see
    // build_entity_records in host/level.cpp).  Every local node of a cell
    // lies on one of its 27 mesh entities (8 vertices, 12 edges, 6 faces, the
    // interior), whose DoFs are numbered contiguously in a canonical
    // orientation and whose contribution slots are laid out DoF-major with one
    // slot per writing cell.  Per block position a record of kEntWords words:
    //   [0, 27)   D_e: first DoF of entity e (-1: constrained)
    //   [27, 54)  SR_e: first slot of entity e + this cell's rank among its
    //             writers (-1: constrained, or added by the previous cell)
    //   [54, 61)  8 bits per entity (4 per word): bits 0-3 the number of
    //             writers c_e, bits 4-6 the orientation (1: reverse the first
    //             entity axis, 2: reverse the second, 4: swap them)
    //   61        flags: 1 = the x-min face is added by the previous cell of
    //             the block, 2 = this cell adds the next cell's x-min face
    // Node (local coordinates u, v, w on its entity) then has DoF D_e + m and
    // slot SR_e + m c_e, with m the canonical index of (u, v, w).
    DeviceArray<int32_t> d_ent_rec;     // [blk][kEntWords][cpb]
    DeviceArray<int32_t> d_inv_off_ent; // [N+1] slot offsets of the entity layout
    size_t contrib_len = 0;             // number of contribution slots (the larger of the two layouts)
    DeviceArray<char> d_contrib;        // contribution buffer of the level's own operator calls
    int contrib_rhs = 1;                // right-hand sides d_contrib holds (grown on demand)
    int config_version = 0;             // bumped when the autotuner changes the kernel variant
    // operator variant of each precision ([NNMG_FP64], [NNMG_FP32]; host/tune.cpp)
    struct OpVariant {
        int geometry_mode = 1;  // 0: stored metric per Gauss point, 1: trilinear coefficients
        bool atomic = false;    // float atomics into the output instead of contribution slots
        int index_layout = 0;   // 0: per-node indices and slots (d_dofmap_blk, d_pos_blk), 1: entity records
        int sweep = 0;          // 0: contractions across lanes through LDS, 1: lines swapped through LDS
        int rhs_split = 0;      // several right-hand sides: 0 each block loops over them, 1 one grid row each
        int group = 1;          // layout blocks per workgroup of the slot kernels (1 or 2): cells per workgroup
                                // = group * cpb; the atomic variants run one
    } var[2];
    // the slot offsets the consumers of a `prec` operator product read
    const int32_t* inv_off(int prec) const { return var[prec].index_layout ? d_inv_off_ent.ptr : d_inv_off.ptr; }
    DeviceArray<double> d_diag64;       // operator diagonal, 1 on constrained
    DeviceArray<double> d_dinv64;       // inverse diagonal, 0 on constrained
    DeviceArray<float> d_dinv32;
};

void level_retain(Level* l);
void level_release(Level* l);

// ---------------------------------------------------------------------------
// a transfer between a fine and a coarse level
// ---------------------------------------------------------------------------
struct Transfer {
    Ctx* ctx = nullptr;
    std::atomic<int> refs{1};
    Level* fine = nullptr;
    Level* coarse = nullptr;
    int64_t n_points = 0, n_projected = 0;
    int max_newton = 0;
    int team = 16;  // lanes per coarse cell in the transfer kernels
    std::vector<int32_t> h_point_dof;    // fine DoF per point, fine-DoF order
    std::vector<int32_t> h_point_owner;  // owner per point, fine-DoF order
    std::vector<double> h_point_xi;      // [n_points][dim], fine-DoF order
    DeviceArray<int32_t> d_off;          // [C_coarse + 1] points grouped by owner
    DeviceArray<int32_t> d_fine;         // [n_points] fine DoF, grouped by owner
    DeviceArray<double> d_xi64;          // [dim][n_points], grouped by owner
    DeviceArray<float> d_xi32;
    DeviceArray<int32_t> d_blk_cells;    // [2][n_points / kPointBlock]: owner of the first and last
                                         // point of each block of the point-parallel kernels
    // restriction sums per (coarse cell, node), in slots sorted by coarse DoF
    DeviceArray<int32_t> d_rslot;        // [C_coarse][q] slot of each sum, -1 for constrained DoFs
    DeviceArray<int32_t> d_roff;         // [N_coarse + 1] DoF j sums rbuf[roff[j] .. roff[j+1])
    // nested polynomial transfer (the two levels share the mesh, the coarse degree is lower)
    bool nested_p = false;
    double pmat[kMaxN * kMaxN]{};        // E[i][a] = coarse basis a at fine node i, at i * kMaxN + a
    DeviceArray<int32_t> d_pfdm;         // [C][q_fine]: the fine node a cell writes, -1 if another cell owns it
    size_t n_rslots = 0;                 // restriction slots
    DeviceArray<double> d_rbuf;          // slot values (float64 or float32)
    int rbuf_rhs = 1;                    // right-hand sides d_rbuf holds (grown on demand)
    int config_version = 0;              // bumped when the autotuner changes the team size
};

constexpr int kPointBlock = 256;
constexpr int kMaxRhs = 8;               // right-hand sides one launch can carry (interleaved [DoF][nr])
constexpr int kScal = 8;                 // CG scalars per right-hand side

// grow the level's contribution buffer / the transfer's restriction buffer to
// nr right-hand sides (synchronizes the device when it reallocates)
void level_reserve_rhs(Level& l, int nr);
void transfer_reserve_rhs(Transfer& t, int nr);

// autotuner (host/tune.cpp)
int level_variant(const Level& L, int prec);
void level_set_variant(Level& L, int prec, int v);  // prec -1: both precisions
void level_set_rhs_split(Level& L, int prec, int split);
void level_set_cells_per_block(Level& L, int prec, int cells);  // cells: cpb or 2 cpb
int level_cells_per_block(const Level& L, int prec);
void level_tune(Level& L, int prec, int reps, nnmg_tune_result* res);
void transfer_set_team(Transfer& T, int team);
void transfer_tune(Transfer& T, int prec, int reps, nnmg_tune_result* res);
constexpr int32_t kMergeNext = 1 << 30;  // flag in a contribution slot index (see Level::d_pos_blk)
constexpr int kEntWords = 62;            // words per cell of the entity-compressed operator indices
constexpr int kWaveLanes = 64;           // CDNA wavefront width  // points per block of the point-parallel transfer kernels

void transfer_retain(Transfer* t);
void transfer_release(Transfer* t);

// ---------------------------------------------------------------------------
// kernel launchers (kernels/*.hip)
// ---------------------------------------------------------------------------
void launch_fill(void* x, size_t n, int prec, hipStream_t s);  // prec: 0 double, 1 float
void launch_cast_64_to_32(const double* a, float* b, size_t n, hipStream_t s);
void launch_cast_32_to_64(const float* a, double* b, size_t n, hipStream_t s);
void launch_set_constrained(const int32_t* idx, size_t n, double v, void* dst, int prec, hipStream_t s);
void launch_lincomb(size_t n, double a, const double* x, double b, double* y, hipStream_t s);  // y = a x + b y
void launch_copy_constrained(const int32_t* idx, size_t n, const void* src, void* dst, int prec,
                             hipStream_t s, int nr = 1);

// operator apply: dst += A src over the cells (constrained rows untouched)
void vmult_shape(int dim, int n, int* wg, int* cells_per_block);

// operator application with its contribution slots in a static device array
// (no allocation; see kernels/noalloc.hip)
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
void* noalloc_scratch_init(int device);  // once per device, with the device current
void vmult_noalloc(const Level& L, int prec, const void* src, void* dst, void* scratch_dev, hipStream_t s);
// contrib = the (cell, node) contributions of A src, in DoF-sorted slots
void launch_vmult_contrib(const Level& L, int prec, const void* src, void* contrib, hipStream_t s, int nr = 1);
// consumers of a contribution buffer (kernels/gather.hip); constrained rows are not written
// (nr interleaved right-hand sides; the vectors hold n_dofs * nr values)
void launch_gather(const Level& L, int prec, const void* contrib, void* dst, bool accumulate, hipStream_t s,
                   int nr = 1);
// Chebyshev step modes (kernels/gather.hip, kernels/vector.hip): what the
// previous direction d is, and whether the new one is stored
constexpr int kChebFirst = 1;  // d = 0: the first step from a given x
constexpr int kChebDIsX = 2;   // d = x: the step after a first step from zero, which sets d = x
constexpr int kChebLast = 4;   // the new d is not stored: no later step reads it
void launch_cheb_step_gather(const Level& L, int prec, const void* contrib, const void* f, const void* dinv,
                             void* x, void* d, double c1, double c2, int mode, hipStream_t s, int nr = 1);
void launch_residual_gather(const Level& L, int prec, const void* contrib, const void* f, void* r, hipStream_t s,
                            int nr = 1);
// out[r * kScal] = p_r . q_r; scalar_op >= 0 also forms the CG scalar that
// waits for the sum (0: alpha from p.q; 1: beta and rz from r.z) on the
// scalars at scal
void launch_gather_dot(const Level& L, const double* contrib, const double* p, double* q, double* partial,
                       double* out, hipStream_t s, int nr = 1, double* scal = nullptr, int scalar_op = -1);
// out[r * ostride] = sum of partial[block][r] over m blocks (scalar_op: as above,
// with ostride = kScal)
void launch_sum_partials(const double* partial, size_t m, double* out, hipStream_t s, int nr = 1,
                         size_t ostride = 1, double* scal = nullptr, int scalar_op = -1);
// dst += A src on the unconstrained rows and columns (constrained entries untouched);
// uses `contrib`, else the level's own contribution buffer (one right-hand
// side; not for concurrent calls on one level)
void launch_vmult_cells(const Level& L, int prec, const void* src, void* dst, hipStream_t s, int nr = 1,
                        void* contrib = nullptr);
// geometry, diagonal, right-hand side (setup kernels)
void launch_geometry(Level& L, int* d_bad, hipStream_t s);
void launch_diagonal(const Level& L, double* diag, hipStream_t s);
void launch_invert_diagonal(const Level& L, const double* diag, hipStream_t s);
void launch_assemble_rhs(const Level& L, const double* fq, double* b, hipStream_t s);

// transfer
void launch_locate(int dim, const double* pts, int np, const double* cverts, const double* boxes,
                   const int32_t* boff, const int32_t* bcells, const double* glo, const double* gstep,
                   const int* gnb, double inside_tol, double newton_tol, int newton_max_it,
                   int32_t* owner, double* xi, int32_t* flags, hipStream_t s);
void launch_prolongate(const Transfer& t, int prec, const void* coarse, void* fine, hipStream_t s, int nr = 1);
// coarse = P^T fine (accumulate = false) or coarse += P^T fine; constrained coarse entries untouched
// rbuf: scratch of restriction_scratch_bytes(t, nr) for the per-cell sums, or
// nullptr for the transfer's own buffer (calls on one transfer must then not overlap)
void launch_restrict(const Transfer& t, int prec, const void* fine, void* coarse, bool accumulate, hipStream_t s,
                     int nr = 1, void* rbuf = nullptr);
// coarse = P^T fine, fused with the coarse level's first smoothing step from
// zero: x = dinv * coarse * c0 (launch_cheb_first_zero), for all entries
void launch_restrict_first_zero(const Transfer& t, int prec, const void* fine, void* coarse, const void* dinv,
                                void* x, double c0, hipStream_t s, int nr = 1, void* rbuf = nullptr);
size_t restriction_scratch_bytes(const Transfer& t, int nr);
// nested polynomial transfer (kernels/pmg.hip): fine += P coarse, and the restriction's per-cell sums
void launch_pmg_prolongate(const Transfer& t, int prec, const void* coarse, void* fine, int nr, hipStream_t s);
void launch_pmg_restrict_sums(const Transfer& t, int prec, const void* fine, void* rbuf, int nr, hipStream_t s);
// dst[v] (+)= sum of the run of v's node, for every value v of n * nr (n vector DoFs of ncomp
// components) whose node has one; elem holds one plane of `plane` entries per right-hand side,
// component c of slot k at k * ncomp + c
void launch_gather_runs(size_t n, int ncomp, const int32_t* off, int prec, const void* elem, size_t plane,
                        void* dst, bool accumulate, hipStream_t s, int nr = 1);
// launch_gather_runs into f (not accumulating), then x = dinv * f * c0 for every value
void launch_gather_runs_first_zero(size_t n, int ncomp, const int32_t* off, int prec, const void* elem,
                                   size_t plane, void* f, const void* dinv, void* x, double c0, hipStream_t s,
                                   int nr = 1);
// entries of one right-hand side's plane of a level's contribution buffer
size_t contrib_plane(const Level& L);

// vector kernels for the smoother and CG
// x = dinv * f * c0   (first step from a zero guess; its direction d equals
// x, which the next step reads in its place: kChebDIsX)
void launch_cheb_first_zero(int prec, size_t n, const void* f, const void* dinv, void* x, double c0,
                            hipStream_t s, int nr = 1);
// f32 = (float) f64, then launch_cheb_first_zero on f32 (float32 vectors)
void launch_cast_cheb_first_zero(size_t n, const double* f64, float* f32, const float* dinv, float* x, double c0,
                                 hipStream_t s, int nr = 1);
// r = f - ax; ax = 0; d = c1 d + c2 dinv r (mode: kCheb* above); x += d
void launch_cheb_step(int prec, size_t n, const void* f, void* ax, const void* dinv, void* x, void* d,
                      double c1, double c2, int mode, hipStream_t s, int nr = 1);
// r = f - ax; ax = 0
void launch_residual(int prec, size_t n, const void* f, void* ax, void* r, hipStream_t s);
// y += x
void launch_splitmix_vector(double* v, const uint8_t* mask_free, size_t n, uint64_t seed, hipStream_t s);

// float64 reductions: out = sum_i a_i b_i (two-stage, deterministic)
void launch_dot(const double* a, const double* b, size_t n, double* partial, double* out, hipStream_t s,
                int nr = 1, size_t ostride = 1, double* scal = nullptr, int scalar_op = -1);
// z = (double) z32 (z may be nullptr: not stored), then out = r . z as launch_dot(r, z, ...) computes it
void launch_cast_dot(const double* r, const float* z32, double* z, size_t n, double* partial, double* out,
                     hipStream_t s, int nr = 1, size_t ostride = 1, double* scal = nullptr, int scalar_op = -1);
size_t dot_partials(size_t n);
// CG kernels; scal layout documented in hierarchy.cpp
// (n vector DoFs, nr interleaved right-hand sides, scalars of r at scal + r * kScal)
// r -= alpha q and r.r into rr_out; the matching x += alpha p is left to the next launch_cg_direction
void launch_cg_update(size_t n, double* r, const double* q, const double* scal, double* partial, double* rr_out,
                      hipStream_t s, int nr = 1);
// x += alpha p (the update cg_update left), then p = z + beta p; z = nullptr: the update of x only
void launch_cg_direction(size_t n, const double* z, double* p, double* x, const double* scal, hipStream_t s,
                         int nr = 1);
// the same with z = (double) z32
void launch_cg_direction32(size_t n, const float* z32, double* p, double* x, const double* scal, hipStream_t s,
                           int nr = 1);
void launch_jacobi(size_t n, const double* dinv, const double* r, double* z, hipStream_t s);
void launch_axpy(size_t n, double a_sign, const double* scal_a, int idx, const double* x, double* y,
                 hipStream_t s);

// dense coarse solve
// O[oidx ? oidx[i] : i] = base_i + sign * sum_j M_ij V[vidx ? vidx[j] : j], base_i = B[bidx ? bidx[i] : i] or 0
// (nr interleaved right-hand sides: index i stands for values i nr .. i nr + nr - 1)
void launch_coarse_gemv(const double* M, size_t m, const void* V, int vprec, const int32_t* vidx, const void* B,
                        int bprec, const int32_t* bidx, double sign, void* O, int oprec, const int32_t* oidx,
                        hipStream_t s, int nr = 1);
void launch_gauss_jordan(double* M, size_t m, double* rowbuf, double* colbuf, hipStream_t s);
void launch_column_from_unit(const int32_t* free_idx, size_t m, const double* ax, double* M, size_t col,
                             hipStream_t s);
void launch_set_unit(double* x, size_t n, int64_t idx, double val, hipStream_t s);

}  // namespace nnmg

// the opaque handles of the C ABI are the internal objects themselves
struct nnmg_ctx : nnmg::Ctx {};
struct nnmg_level : nnmg::Level {};
struct nnmg_transfer : nnmg::Transfer {};
