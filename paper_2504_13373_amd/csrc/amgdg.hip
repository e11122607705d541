// C-ABI of the amgdg library: setup (Algorithm 5), V-cycle (Algorithm 2) and
// Krylov drivers on one GPU.  Host code orchestrates; every arithmetic step on
// matrices and vectors is a kernel of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/amgdg.h"
#include "index.h"
#include "kernels.h"

namespace amgdg {

static thread_local std::string g_last_error;

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            throw Error(e_ == hipErrorOutOfMemory ? AMGDG_ENOMEM : AMGDG_EHIP,                        \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                           \
    } while (0)

// ------------------------------------------------------------ device memory
struct DevMem {
    std::vector<void*> blocks;
    std::vector<size_t> sizes;
    ~DevMem() { release(); }
    void release() {
        for (void* p : blocks) (void)hipFree(p);
        blocks.clear();
        sizes.clear();
    }
    template <typename T>
    T* alloc(int64_t n) {
        void* p = nullptr;
        const size_t bytes = sizeof(T) * size_t(std::max<int64_t>(n, 1));
        HIPCHK(hipMalloc(&p, bytes));
        blocks.push_back(p);
        sizes.push_back(bytes);
        return static_cast<T*>(p);
    }
    void zero_all(hipStream_t st) {
        for (size_t i = 0; i < blocks.size(); ++i) HIPCHK(hipMemsetAsync(blocks[i], 0, sizes[i], st));
    }
    // frees one block of this DevMem (nothing if p is not one of them)
    void free(void* p) {
        for (size_t i = 0; i < blocks.size(); ++i)
            if (blocks[i] == p) {
                (void)hipFree(p);
                blocks.erase(blocks.begin() + long(i));
                sizes.erase(sizes.begin() + long(i));
                return;
            }
    }
};

template <typename T>
static T* upload(DevMem& M, const std::vector<T>& v, hipStream_t st) {
    T* p = M.alloc<T>(int64_t(v.size()));
    if (!v.empty()) {
        HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return p;
}

template <typename T>
static std::vector<T> download(const T* d, int64_t n, hipStream_t st) {
    std::vector<T> h(size_t(std::max<int64_t>(n, 0)));
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(h.data(), d, sizeof(T) * size_t(n), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return h;
}

// ------------------------------------------------------------ level data
struct SellStore {
    Sell<double> d;
    Sell<float> f;
    int64_t n_vals = 0;
    const int32_t* pos = nullptr;  // slice position of each block row when the rows are reordered
};

// An operator of the hierarchy in the layout its block shape calls for: the
// sliced row-interleaved layout for tall blocks (br > 4), block CSR with a lane
// group per block row for small blocks (coarse levels, restriction).
struct MatStore {
    bool vec = false;
    SellStore s;
    Bcsr<double> bd;
    Bcsr<float> bf;
    Nbsr<double> nd;  // natural layout of a sliced matrix, for 16-column MFMA tiles
    Nbsr<float> nf;
    int64_t n_vals = 0;
    bool unit = false;  // diagonal blocks implied identity (S = D^{-1} A)
    // tuned launch shapes per column count (0: the default rule): columns per
    // launch, and blocks loaded ahead in the MFMA tiles (per m / 16)
    std::array<int8_t, 65> cap64{}, cap32{};
    std::array<int8_t, 5> mfu64{}, mfu32{};
};

template <typename T>
struct VBuf {
    T *b = nullptr, *u = nullptr, *w = nullptr, *r = nullptr;
    T* cur = nullptr;  // buffer holding u_k during a V-cycle
    T* c = nullptr;    // D_k^{-1} b_k of the V-cycle's level-k right-hand side
};

struct Level {
    int64_t n_units = 0, n = 0, n_agg = 0, nnzb = 0, nT = 0;
    int nb = 0, s = 0, r = 0;
    // Real dofs of each unit (eq:sik chooses them per aggregate): unit u owns
    // the vector rows u*nb + [0, sz[u]); rows beyond sz[u] are padding that
    // every operator keeps zero.  padded: some sz[u] < nb.
    std::vector<int32_t> sz;
    std::vector<int64_t> roff;  // real-dof offset of each unit (level order)
    int32_t* sz_d = nullptr;
    int64_t* roff_d = nullptr;
    int64_t n_real = 0;
    bool padded = false;
    // matrix-free level (eq:matfree1, eq:matfree2): A_k is not kept after the
    // setup; the V-cycle forms A_k u as R_{k-1} A_{k-1} T_{k-1} u
    bool matfree = false;
    double omega = 1.0, rho = std::numeric_limits<double>::quiet_NaN();
    std::vector<int32_t> sweeps;
    double* A_nat = nullptr;
    double* Dinv_nat = nullptr;
    double* Dinv_sell = nullptr;
    float* Dinv_sell32 = nullptr;
    float* Dinv_nat32 = nullptr;
    MatStore A, T, R;
    // the row-scaled operators the V-cycle runs on: S = D^{-1} A (A's pattern)
    // and RD = R D (R's pattern), so that R (b - A u) = RD (D^{-1} b - S u)
    MatStore S, RD;
    double *S_nat = nullptr, *RD_nat = nullptr;
    int64_t nnzb_S = 0;  // stored blocks of S: A's off-diagonal blocks
    // M = R (D - omega A) (R A's pattern): the restriction of the residual after
    // a sweep from the residual before it, R D (c - S u') = M (c - S u) for
    // u' = u + omega (c - S u), so that the last pre-sweep's own residual
    // replaces a residual pass over S.  Kept where it holds no more values
    // than the S and RD reads it replaces (plus a launch's worth).
    MatStore M;
    double* M_nat = nullptr;
    int64_t nM = 0;
    bool has_M = false;
    double *B_in = nullptr, *B_rel = nullptr, *Pu = nullptr, *sv = nullptr, *T_nat = nullptr, *R_nat = nullptr;
};

// Status record of a Work (doubles): [0, 64) ||r||^2 per column from the CG
// update; [64, 96) one int32 error flag per column; [96, 160) ||b||^2 and
// [160, 224) ||b - A x0||^2 of the columns admitted in the iteration;
// [224, 288) true residual norms^2.
constexpr int ST_RR = 0, ST_FLAG = 64, ST_BN = 96, ST_R0 = 160, ST_TR = 224, ST_LEN = 288;
// column masks (int32): direction update, CG update, residual replacement, admission with x0
constexpr int MASK_DIR = 0, MASK_UPD = 64, MASK_REPL = 128, MASK_ADM = 192, MASK_LEN = 256;
// pinned FGMRES records: two step records of 2 * 257 + 1 doubles, 8 residual slots, y (<= 256)
constexpr int GM_H_LEN = 2 * 515 + 8 + 256;

// The device state of one solve, or of one batch of right-hand sides: V-cycle
// vectors per level, Krylov vectors (row-major n x m), reduction scratch, the
// status record and masks with their pinned host mirrors, the captured
// V-cycles and the events the host loop waits on.  A handle owns one for its
// blocking entry points; a server owns one per batch.  One host thread and
// one stream use a Work at a time.
struct Work {
    DevMem mem;
    int m = 0, restart = 0;
    bool mixed = false;
    int64_t bytes = 0;  // device bytes held
    std::vector<VBuf<double>> v64;
    std::vector<VBuf<float>> v32;
    double *kb = nullptr, *kx = nullptr, *kr = nullptr, *kr2 = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr,
           *kt = nullptr;
    double *kgin = nullptr, *kgout = nullptr;  // fixed input/output of the FP64 V-cycle graph
    float *kr32 = nullptr, *kz32 = nullptr;
    double *V = nullptr, *Z = nullptr;  // FGMRES basis
    double *scratch = nullptr, *scal = nullptr, *kpart = nullptr, *stat = nullptr;
    double* kslice = nullptr;  // per-slice partials of the level-0 product A p with p.(A p)
    int32_t* mask = nullptr;
    double* stat_h = nullptr;   // pinned
    int32_t* mask_h = nullptr;  // pinned
    double* gm_h = nullptr;     // pinned FGMRES records (Works with a basis)
    // captured V-cycles, keyed by (precision, columns, input, output)
    struct GraphEntry {
        int prec, m;
        const void* in;
        void* out;
        hipGraph_t g;
        hipGraphExec_t e;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap = nullptr;
    hipEvent_t ev = nullptr;      // status readback of the host loop
    hipEvent_t ev2 = nullptr;     // second readback slot (FGMRES run-ahead)
    hipEvent_t ev_ret = nullptr;  // solutions of retired columns written
    bool use_graph = true;        // per call: off with AMGDG_EAGER
    void drop_graphs() {
        for (auto& e : graphs) {
            (void)hipGraphExecDestroy(e.e);
            (void)hipGraphDestroy(e.g);
        }
        graphs.clear();
    }
    ~Work() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (ev) (void)hipEventDestroy(ev);
        if (ev2) (void)hipEventDestroy(ev2);
        if (ev_ret) (void)hipEventDestroy(ev_ret);
        if (stat_h) (void)hipHostFree(stat_h);
        if (mask_h) (void)hipHostFree(mask_h);
        if (gm_h) (void)hipHostFree(gm_h);
    }
};

struct Ctx {
    DevMem mem;
    DevMem* build_mem = nullptr;  // where build_mat places a layout (nullptr: mem)
    DevMem& bm() { return build_mem ? *build_mem : mem; }
    Plan plan;
    amgdg_params prm{};
    int N = 0;                  // index of the coarsest level
    std::vector<Level> lv;      // N + 1 levels
    int64_t nN = 0;
    double* Ainv = nullptr;
    int64_t* perm_d = nullptr;  // internal unit -> caller element
    std::vector<int32_t> in_rp, in_ci;  // caller's level-0 pattern (for export)
    double* scratch = nullptr;  // reduction partials of the setup
    double* scal = nullptr;     // device scalars of the setup
    int32_t* flag = nullptr;
    bool mixed = false;
    bool lanes_tuned = false;   // lane-group widths fixed by the autotuner
    std::unique_ptr<Work> W0;   // state of the blocking entry points
    ~Ctx() {
        (void)hipDeviceSynchronize();
        W0.reset();
    }
};

static int32_t read_flag(Ctx& C, hipStream_t st) {
    int32_t f = 0;
    HIPCHK(hipMemcpyAsync(&f, C.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemsetAsync(C.flag, 0, sizeof(int32_t), st));
    return f;
}

// Values of one precision in the sliced layout (the offsets depend on the
// vector width, so FP64 and FP32 copies each have their own).
template <typename T>
static void sell_values(Ctx& C, Sell<T>& d, int64_t ns, const std::vector<int32_t>& K,
                        const std::vector<int64_t>& slot_src, const std::vector<int32_t>& slot_k,
                        const std::vector<int32_t>& slot_g, const std::vector<int32_t>& slot_s, const double* nat_d,
                        hipStream_t st) {
    constexpr int VW = 16 / int(sizeof(T));
    std::vector<int64_t> voff(ns + 1), base(slot_s.size());
    int64_t v = 0;
    int32_t tpad = 0;
    for (int64_t s = 0; s < ns; ++s) {
        voff[s] = v;
        const int32_t tq = (K[s] * d.bc + VW - 1) / VW;
        tpad = std::max(tpad, tq * VW);
        v += int64_t(tq) * VW * d.L;
    }
    voff[ns] = v;
    for (size_t q = 0; q < slot_s.size(); ++q) base[q] = voff[slot_s[q]];
    d.tpad = std::max<int32_t>(tpad, VW);
    d.brpad = (d.br + VW - 1) / VW * VW;
    d.voff = upload(C.bm(), voff, st);
    T* vals = C.bm().alloc<T>(v);
    HIPCHK(hipMemsetAsync(vals, 0, sizeof(T) * size_t(std::max<int64_t>(v, 1)), st));
    {
        DevMem tmp;
        const int64_t* src = upload(tmp, slot_src, st);
        const int64_t* bs = upload(tmp, base, st);
        const int32_t* sk = upload(tmp, slot_k, st);
        const int32_t* sg = upload(tmp, slot_g, st);
        HIPCHK(launch_to_sell_vals<T>(nat_d, src, bs, sk, sg, int64_t(slot_s.size()), d.L, d.br, d.bc, vals, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    d.vals = vals;
}

// Builds the sliced layout of a natural BSR matrix (row-major br x bc blocks)
// whose pattern (rp, ci) is on the host and values nat_d on the device.
static void build_sell(Ctx& C, SellStore& S, int64_t n_brow, int br, int bc, const std::vector<int32_t>& rp,
                       const std::vector<int32_t>& ci, const double* nat_d, bool f32, hipStream_t st) {
    if (br < 1 || br > 64) throw Error(AMGDG_EUNSUPPORTED, "block size must be 1..64");
    auto len = [&](int64_t row) { return row < n_brow ? rp[row + 1] - rp[row] : 0; };
    int32_t longest = 0;
    for (int64_t row = 0; row < n_brow; ++row) longest = std::max(longest, len(row));
    // floor(64 / br) block rows per wavefront, fewer for long rows (the x
    // staging of a slice must fit LDS)
    const int G = sell_rows_per_wave(br, bc, longest), L = G * br;
    const int64_t ns = (n_brow + G - 1) / G;
    // Slot counts with the rows in order, and with the rows sorted by length
    // (longest first, stable) within windows of 8 slices; the sorted order is
    // kept for the square-block level operators when it cuts the padded slots
    // by more than 5% (rows of varying length, such as LDG's neighbours of
    // neighbours).  The prolongation's short rows stay in order: there the
    // scattered row writes cost more than the padding.
    std::vector<int32_t> order(static_cast<size_t>(ns * G));
    for (int64_t q = 0; q < ns * G; ++q) order[q] = int32_t(std::min<int64_t>(q, n_brow));
    auto slots = [&](const std::vector<int32_t>& ord) {
        int64_t tot = 0;
        for (int64_t s = 0; s < ns; ++s) {
            int32_t kmax = 0;
            for (int g = 0; g < G; ++g) kmax = std::max(kmax, len(ord[s * G + g]));
            tot += int64_t(kmax) * G;
        }
        return tot;
    };
    const int64_t plain = slots(order);
    std::vector<int32_t> sorted = order;
    const int64_t win = int64_t(8) * G;
    for (int64_t w0 = 0; w0 < ns * G; w0 += win) {
        const auto b = sorted.begin() + w0, e = sorted.begin() + std::min(w0 + win, ns * G);
        std::stable_sort(b, e, [&](int32_t x, int32_t y) { return len(x) > len(y); });
    }
    const bool use_sorted = br == bc && slots(sorted) * 20 < plain * 19;
    if (use_sorted) order.swap(sorted);
    std::vector<int32_t> coff(ns + 1), K(ns), cols, slot_k, slot_g, slot_s;
    std::vector<int64_t> slot_src;
    int32_t c = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int32_t kmax = 0;
        for (int g = 0; g < G; ++g) kmax = std::max(kmax, len(order[s * G + g]));
        K[s] = kmax;
        coff[s] = c;
        for (int kk = 0; kk < kmax; ++kk)
            for (int g = 0; g < G; ++g) {
                const int64_t row = order[s * G + g];
                int64_t blk = -1;
                int32_t col = 0;
                if (row < n_brow && kk < rp[row + 1] - rp[row]) {
                    blk = rp[row] + kk;
                    col = ci[blk];
                }
                cols.push_back(col);
                slot_src.push_back(blk);
                slot_k.push_back(kk);
                slot_g.push_back(g);
                slot_s.push_back(int32_t(s));
            }
        c += kmax * G;
        if (c < 0) throw Error(AMGDG_EUNSUPPORTED, "matrix too large for int32 slot indexing");
    }
    coff[ns] = c;
    Sell<double> d;
    d.n_brow = int32_t(n_brow);
    d.br = br;
    d.bc = bc;
    d.G = G;
    d.L = L;
    d.n_slices = int32_t(ns);
    d.coff = upload(C.bm(), coff, st);
    d.K = upload(C.bm(), K, st);
    d.cols = upload(C.bm(), cols, st);
    if (use_sorted) {
        d.rows = upload(C.bm(), order, st);
        std::vector<int32_t> pos(static_cast<size_t>(n_brow));
        for (int64_t q = 0; q < ns * G; ++q)
            if (order[q] < n_brow) pos[order[q]] = int32_t(q);
        S.pos = upload(C.bm(), pos, st);
    }
    Sell<float> f;
    f.n_brow = d.n_brow;
    f.br = br;
    f.bc = bc;
    f.G = G;
    f.L = L;
    f.n_slices = d.n_slices;
    f.coff = d.coff;
    f.K = d.K;
    f.cols = d.cols;
    f.rows = d.rows;
    sell_values<double>(C, d, ns, K, slot_src, slot_k, slot_g, slot_s, nat_d, st);
    if (f32) sell_values<float>(C, f, ns, K, slot_src, slot_k, slot_g, slot_s, nat_d, st);
    S.d = d;
    S.f = f;
    int64_t nv = 0;
    for (int64_t s = 0; s < ns; ++s) nv += int64_t(K[s]) * bc * L;
    S.n_vals = nv;
}

template <typename T>
static T* sell_dinv(Ctx& C, const Sell<T>& A, const int32_t* pos, const double* dinv_nat, hipStream_t st) {
    const int64_t cnt = int64_t(A.n_slices) * A.brpad * A.L;
    T* out = C.bm().alloc<T>(cnt);
    HIPCHK(hipMemsetAsync(out, 0, sizeof(T) * size_t(std::max<int64_t>(cnt, 1)), st));
    HIPCHK(launch_dinv_to_sell<T>(dinv_nat, A.n_brow, A.br, A.G, A.L, A.brpad, out, st, pos));
    return out;
}

static void build_mat_layouts(Ctx& C, MatStore& M, int64_t n_brow, int br, int bc, const std::vector<int32_t>& rp,
                              const std::vector<int32_t>& ci, const double* nat_d, bool f32, hipStream_t st);

// unit: a square operator whose diagonal blocks are the identity and are not
// among (rp, ci, nat_d); every layout's products add the row's own x entries
static void build_mat(Ctx& C, MatStore& M, int64_t n_brow, int br, int bc, const std::vector<int32_t>& rp,
                      const std::vector<int32_t>& ci, const double* nat_d, bool f32, hipStream_t st,
                      bool unit = false) {
    build_mat_layouts(C, M, n_brow, br, bc, rp, ci, nat_d, f32, st);
    const int32_t u = unit ? 1 : 0;
    M.bd.unit = M.bf.unit = M.nd.unit = M.nf.unit = M.s.d.unit = M.s.f.unit = u;
    M.unit = unit;
}

static void build_mat_layouts(Ctx& C, MatStore& M, int64_t n_brow, int br, int bc, const std::vector<int32_t>& rp,
                              const std::vector<int32_t>& ci, const double* nat_d, bool f32, hipStream_t st) {
    if (br <= BCSR_MAXBR) {
        M.vec = true;
        const int64_t nnzb = int64_t(ci.size());
        const double avg = n_brow > 0 ? double(nnzb) / double(n_brow) : 1.0;
        int P = 4;
        while (P < avg && P < 64) P *= 2;
        // rows of many entries: lanes over the entries, a wavefront per block
        // row, or a workgroup where that leaves fewer than 16 wavefronts per CU
        const double entries = avg * bc;
        if (entries >= 96) P = (entries >= 128 && n_brow < 4096) ? 256 : 128;
        Bcsr<double> d;
        d.n_brow = int32_t(n_brow);
        d.br = br;
        d.bc = bc;
        d.P = P;
        d.rp = upload(C.bm(), rp, st);
        d.ci = upload(C.bm(), ci, st);
        d.vals = nat_d;
        M.bd = d;
        M.bf.n_brow = d.n_brow;
        M.bf.br = br;
        M.bf.bc = bc;
        M.bf.P = P;
        M.bf.rp = d.rp;
        M.bf.ci = d.ci;
        M.n_vals = nnzb * br * bc;
        if (f32) {
            float* fv = C.bm().alloc<float>(M.n_vals);
            HIPCHK(launch_f64_to_f32(nat_d, fv, M.n_vals, st));
            M.bf.vals = fv;
        }
        // the same natural blocks, read by the MFMA tiles at multiples of 16 columns
        if (bc <= NBSR_MAXB) {
            M.nd.n_brow = d.n_brow, M.nd.br = br, M.nd.bc = bc, M.nd.rp = d.rp, M.nd.ci = d.ci, M.nd.vals = nat_d;
            M.nf.n_brow = d.n_brow, M.nf.br = br, M.nf.bc = bc, M.nf.rp = d.rp, M.nf.ci = d.ci, M.nf.vals = M.bf.vals;
        }
    } else {
        M.vec = false;
        build_sell(C, M.s, n_brow, br, bc, rp, ci, nat_d, f32, st);
        M.n_vals = M.s.n_vals;
        if (br <= NBSR_MAXB && bc <= NBSR_MAXB) {
            Nbsr<double> d;
            d.n_brow = int32_t(n_brow);
            d.br = br;
            d.bc = bc;
            d.rp = upload(C.bm(), rp, st);
            d.ci = upload(C.bm(), ci, st);
            d.vals = nat_d;
            M.nd = d;
            if (f32) {
                const int64_t nv = int64_t(ci.size()) * br * bc;
                float* fv = C.bm().alloc<float>(nv);
                HIPCHK(launch_f64_to_f32(nat_d, fv, nv, st));
                M.nf.n_brow = d.n_brow;
                M.nf.br = br;
                M.nf.bc = bc;
                M.nf.rp = d.rp;
                M.nf.ci = d.ci;
                M.nf.vals = fv;
            }
        }
    }
}

template <typename T>
static const Sell<T>& sel(const SellStore& S);
template <>
const Sell<double>& sel<double>(const SellStore& S) { return S.d; }
template <>
const Sell<float>& sel<float>(const SellStore& S) { return S.f; }
template <typename T>
static const Bcsr<T>& bsel(const MatStore& M);
template <>
const Bcsr<double>& bsel<double>(const MatStore& M) { return M.bd; }
template <>
const Bcsr<float>& bsel<float>(const MatStore& M) { return M.bf; }

template <typename T>
static const T* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) { return L.A.vec ? L.Dinv_nat : L.Dinv_sell; }
template <>
const float* dinv_of<float>(const Level& L) { return L.A.vec ? L.Dinv_nat32 : L.Dinv_sell32; }

template <typename T>
static const Nbsr<T>& nsel(const MatStore& M);
template <>
const Nbsr<double>& nsel<double>(const MatStore& M) { return M.nd; }
template <>
const Nbsr<float>& nsel<float>(const MatStore& M) { return M.nf; }

template <typename T>
static const T* dinv_nat_of(const Level& L);
template <>
const double* dinv_nat_of<double>(const Level& L) { return L.Dinv_nat; }
template <>
const float* dinv_nat_of<float>(const Level& L) { return L.Dinv_nat32; }

// 16-column tiles go through the MFMA kernel (blocks up to 16 x 16): for a
// sliced (tall-block) matrix one read of it per 16 columns instead of one per
// 4 (FP64) or 8 (FP32) columns; for the block-CSR operators 16-value x rows
// loaded by 16 lanes and one wavefront per block row.
template <typename T>
static bool use_mfma(const MatStore& M, int m) {
    return m % MFMA_COLS == 0 && nsel<T>(M).vals != nullptr;
}
template <typename T>
static int cap_of(const MatStore& M, int m) {
    return m <= 64 ? (sizeof(T) == 8 ? M.cap64[m] : M.cap32[m]) : 0;
}
template <typename T>
static int mfu_of(const MatStore& M, int m) {
    return m / MFMA_COLS <= 4 ? (sizeof(T) == 8 ? M.mfu64[m / MFMA_COLS] : M.mfu32[m / MFMA_COLS]) : 0;
}

// omega is read by S_SWEEP and S_SWEEP_R only; y2 (S_SWEEP_R only) receives b - A x
template <typename T>
static void mat_spmv(int mode, const MatStore& M, const T* x, const T* b, T* y, int m, hipStream_t st,
                     T omega = T(0), T* y2 = nullptr, bool rev = false) {
    if (M.vec && !use_mfma<T>(M, m))
        HIPCHK(launch_bspmv<T>(mode, bsel<T>(M), x, b, y, m, st, cap_of<T>(M, m), omega, nullptr, y2));
    else if (use_mfma<T>(M, m))
        HIPCHK(launch_mfma<T>(mode == AX        ? MF_AX
                              : mode == B_MINUS ? MF_BMINUS
                              : mode == B_PLUS  ? MF_BPLUS
                              : mode == S_SWEEP_R ? MF_SSWEEP_R
                                                    : MF_SSWEEP,
                              nsel<T>(M), nullptr, x, b, y, omega, m, st, mfu_of<T>(M, m), y2));
    else {
        Sell<T> A = sel<T>(M.s);
        A.rev = rev ? 1 : 0;
        HIPCHK(launch_spmv<T>(mode, A, x, b, y, m, st, cap_of<T>(M, m), omega, y2));
    }
}

// y2 (SWEEP0 only, may be null) receives D^{-1} b
template <typename T>
static void mat_sweep(int mode, const Level& L, const T* x, const T* b, T* y, T omega, int m, const int32_t* mask,
                      hipStream_t st, T* y2 = nullptr) {
    if (L.A.vec)
        HIPCHK(launch_bsweep<T>(mode, bsel<T>(L.A), dinv_of<T>(L), x, b, y, omega, m, mask, st, cap_of<T>(L.A, m), y2));
    else if ((mode == SWEEP || mode == SWEEP0) && use_mfma<T>(L.A, m) && dinv_nat_of<T>(L))
        HIPCHK(launch_mfma<T>(mode == SWEEP ? MF_SWEEP : MF_SWEEP0, nsel<T>(L.A), dinv_nat_of<T>(L), x, b, y, omega, m,
                              st, mfu_of<T>(L.A, m), y2));
    else
        HIPCHK(launch_sweep<T>(mode, sel<T>(L.A.s), dinv_of<T>(L), x, b, y, omega, m, mask, st, cap_of<T>(L.A, m),
                               y2));
}


// y = omega D'^{-1} (R x), y2 = D'^{-1} (R x) with D'^{-1} and omega of the level
// R restricts to (its first sweep from zero on the right-hand side R x), when
// R is stored as block CSR or runs on the MFMA tiles; false if not possible.
template <typename T>
static bool restrict_start(const MatStore& R, const Level& Ln, const T* x, T* y, T* y2, int m, hipStream_t st) {
    const T* dinv = dinv_nat_of<T>(Ln);
    if (!dinv) return false;
    if (use_mfma<T>(R, m))
        HIPCHK(launch_mfma<T>(MF_RDINV, nsel<T>(R), dinv, x, nullptr, y, T(Ln.omega), m, st, mfu_of<T>(R, m), y2));
    else if (R.vec)
        HIPCHK(launch_bspmv<T>(AX_DSCALE, bsel<T>(R), x, nullptr, y, m, st, cap_of<T>(R, m), T(Ln.omega), dinv, y2));
    else
        return false;
    return true;
}

// blocking dot products through the partials buffer `part` and device scalars `out`
static double dot1(double* part, double* out, const double* a, const double* b, int64_t n, hipStream_t st) {
    HIPCHK(launch_dot<double>(a, b, n, 1, part, out, st));
    double h = 0;
    HIPCHK(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

static std::vector<double> dotm(double* part, double* out, const double* a, const double* b, int64_t n, int m,
                                hipStream_t st) {
    HIPCHK(launch_dot<double>(a, b, n, m, part, out, st));
    std::vector<double> h(m);
    HIPCHK(hipMemcpyAsync(h.data(), out, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

// Algorithm 4 with P(A_k) = D_k: x unit, q times x <- D^{-1} A x / ||.||, returns ||D^{-1} A x||.
static double power_rho(Ctx& C, Level& L, int k, hipStream_t st) {
    DevMem tmp;
    double* x = tmp.alloc<double>(L.n);
    double* y = tmp.alloc<double>(L.n);
    if (L.padded)
        HIPCHK(launch_uniform_padded(C.prm.pow_seed + uint64_t(k), L.roff_d, L.sz_d, L.n_units, L.nb, x, st));
    else
        HIPCHK(launch_uniform(C.prm.pow_seed + uint64_t(k), k == 0 ? C.perm_d : nullptr, L.n_units, L.nb, x, st));
    HIPCHK(launch_dot<double>(x, x, L.n, 1, C.scratch, C.scal, st));
    HIPCHK(launch_scale_by_inv_norm(x, L.n, C.scal, st));
    for (int it = 0; it < C.prm.q_power; ++it) {
        mat_sweep<double>(DINVA, L, x, nullptr, y, -1.0, 1, nullptr, st);
        HIPCHK(launch_dot<double>(y, y, L.n, 1, C.scratch, C.scal, st));
        HIPCHK(launch_scale_by_inv_norm(y, L.n, C.scal, st));
        std::swap(x, y);
    }
    mat_sweep<double>(DINVA, L, x, nullptr, y, -1.0, 1, nullptr, st);
    return std::sqrt(dot1(C.scratch, C.scal, y, y, L.n, st));
}

// eq:bsmooth for all r columns at once: a column stops (mask 0, frozen) after
// the sweep whose norm ratio ||x^(m)|| / ||x^(m+1)|| is below 1 + gamma, or at relax_max.
static void relax_candidates(Ctx& C, Level& L, double* B, hipStream_t st) {
    const int r = L.r;
    DevMem tmp;
    double* X = B;
    double* Y = tmp.alloc<double>(L.n * r);
    int32_t* mask = tmp.alloc<int32_t>(r);
    std::vector<int32_t> act(r, 1);
    L.sweeps.assign(r, 0);
    std::vector<double> nx = dotm(C.scratch, C.scal, X, X, L.n, r, st);
    HIPCHK(hipMemcpyAsync(mask, act.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, st));
    const double thr = 1.0 + C.prm.gamma;
    for (int sweep = 0; sweep < C.prm.relax_max; ++sweep) {
        mat_sweep<double>(RELAX, L, X, nullptr, Y, L.omega, r, mask, st);
        std::vector<double> ny = dotm(C.scratch, C.scal, Y, Y, L.n, r, st);
        std::swap(X, Y);
        bool any = false;
        for (int c = 0; c < r; ++c) {
            if (!act[c]) continue;
            L.sweeps[c]++;
            const double ratio = std::sqrt(nx[c]) / std::sqrt(ny[c]);
            if (ratio < thr || L.sweeps[c] >= C.prm.relax_max) act[c] = 0;
            nx[c] = ny[c];
            any = any || act[c];
        }
        HIPCHK(hipMemcpyAsync(mask, act.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!any) break;
    }
    if (X != B) HIPCHK(hipMemcpyAsync(B, X, sizeof(double) * L.n * r, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
}

static void check_finite_host(const double* v, int64_t n, const char* what) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) throw Error(AMGDG_ENAN, std::string(what) + " contains NaN or Inf");
}

static void setup_impl(Ctx& C, int64_t n_elem, int32_t nb, const int32_t* row_ptr, const int32_t* col_idx,
                       const double* vals, int64_t nnzb, const int32_t* agg_of_elem, const double* B1,
                       hipStream_t st) {
    const amgdg_params& p = C.prm;
    if (nb < 1 || nb > 64) throw Error(AMGDG_EUNSUPPORTED, "nb must be 1..64");
    if (p.n_levels < 1) throw Error(AMGDG_EINVAL, "n_levels must be >= 1");
    if (p.n_levels > 1 && (p.r < 1 || p.r > 64)) throw Error(AMGDG_EUNSUPPORTED, "r must be 1..64");
    if (!(p.delta >= 0.0)) throw Error(AMGDG_EINVAL, "delta must be >= 0");
    if (p.matfree_levels < 0 || (p.matfree_levels > 0 && p.matfree_levels > p.n_levels - 2))
        throw Error(AMGDG_EINVAL, "matfree_levels must be 0..n_levels-2");
    if (p.t_pre < 0 || p.t_post < 0 || p.q_power < 0 || p.relax_max < 1 || !(p.n_cut > 0))
        throw Error(AMGDG_EINVAL, "bad smoothing or coarsening parameters");
    if (p.b_update != 0) throw Error(AMGDG_EUNSUPPORTED, "only B^{k+1} = R B^k is implemented");
    if (!vals) throw Error(AMGDG_EINVAL, "vals is NULL");
    check_finite_host(vals, nnzb * nb * nb, "A");
    try {
        build_plan(C.plan, n_elem, row_ptr, col_idx, nnzb, p.n_levels, agg_of_elem, p.hstar_smooth != 0);
    } catch (const std::invalid_argument& e) {
        throw Error(AMGDG_EINVAL, e.what());
    }
    C.in_rp.assign(row_ptr, row_ptr + n_elem + 1);
    C.in_ci.assign(col_idx, col_idx + nnzb);
    C.N = p.n_levels - 1;
    C.mixed = p.mixed != 0;
    C.lv.assign(C.N + 1, Level());
    C.scratch = C.mem.alloc<double>(int64_t(DOT_PARTS) * 64 + 1024);
    C.scal = C.mem.alloc<double>(2048);
    C.flag = C.mem.alloc<int32_t>(4);
    HIPCHK(hipMemsetAsync(C.flag, 0, 4 * sizeof(int32_t), st));
    C.perm_d = upload(C.mem, C.plan.perm, st);

    // level-0 values in internal order
    {
        const int64_t per = int64_t(nb) * nb;
        std::vector<double> a0(size_t(nnzb * per));
        for (int64_t b = 0; b < nnzb; ++b)
            std::memcpy(&a0[size_t(b * per)], vals + C.plan.A0_src[b] * per, sizeof(double) * per);
        C.lv[0].A_nat = upload(C.mem, a0, st);
    }

    // B^1 in internal order
    double* B = nullptr;
    const int r = p.r;
    if (C.N > 0) {
        B = C.mem.alloc<double>(n_elem * nb * r);
        if (B1) {
            check_finite_host(B1, n_elem * nb * r, "B1");
            std::vector<double> h(size_t(n_elem * nb * r));
            const int64_t per = int64_t(nb) * r;
            for (int64_t u = 0; u < n_elem; ++u)
                std::memcpy(&h[size_t(u * per)], B1 + C.plan.perm[u] * per, sizeof(double) * per);
            HIPCHK(hipMemcpyAsync(B, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        } else {
            HIPCHK(launch_normal(p.b1_seed, C.perm_d, n_elem, nb, r, B, st));
        }
    }

    int cur_nb = nb;
    std::vector<int32_t> cur_sz(size_t(n_elem), nb);
    for (int k = 0; k <= C.N; ++k) {
        Level& L = C.lv[k];
        const bool coarsest = (k == C.N);
        const std::vector<int32_t>& Arp = coarsest ? C.plan.AN_rp : C.plan.lv[k].A_rp;
        const std::vector<int32_t>& Aci = coarsest ? C.plan.AN_ci : C.plan.lv[k].A_ci;
        L.n_units = int64_t(Arp.size()) - 1;
        L.nb = cur_nb;
        L.n = L.n_units * L.nb;
        L.nnzb = int64_t(Aci.size());
        L.sz = cur_sz;
        L.roff.assign(size_t(L.n_units) + 1, 0);
        for (int64_t u = 0; u < L.n_units; ++u) L.roff[u + 1] = L.roff[u] + L.sz[u];
        L.n_real = L.roff[L.n_units];
        L.padded = L.n_real != L.n;
        L.sz_d = upload(C.mem, L.sz, st);
        L.roff_d = upload(C.mem, L.roff, st);
        if (coarsest) {
            C.nN = L.n;
            if (C.nN > 20000) throw Error(AMGDG_EUNSUPPORTED, "coarsest level too large for a dense inverse");
            DevMem tmp;
            int32_t* rp_d = upload(tmp, Arp, st);
            int32_t* ci_d = upload(tmp, Aci, st);
            C.Ainv = C.mem.alloc<double>(C.nN * C.nN);
            HIPCHK(launch_dense_from_bsr(L.A_nat, rp_d, ci_d, L.n_units, L.nb, L.nnzb, C.Ainv, st));
            double* am = tmp.alloc<double>(1 + DOT_PARTS);
            HIPCHK(launch_absmax(C.Ainv, C.nN * C.nN, am, st));
            int32_t* piv = tmp.alloc<int32_t>(C.nN);
            double* rowc = tmp.alloc<double>(C.nN);
            double* colc = tmp.alloc<double>(C.nN);
            HIPCHK(launch_gj_invert(C.Ainv, C.nN, piv, C.flag, am, double(C.nN) * 2.220446049250313e-16, rowc, colc, st));
            if (read_flag(C, st)) throw Error(AMGDG_ESINGULAR, "coarsest matrix is singular to working precision");
            break;
        }
        const LevelPattern& P = C.plan.lv[k];
        L.n_agg = P.n_agg;
        L.r = r;
        // On a matrix-free level (1 <= k <= matfree_levels) A_k's layouts serve
        // the setup's power iteration and relaxation only: they are built in
        // FP64 into `setup_only` and freed with A_k's values at the end of this
        // level; S_k = D_k^{-1} A_k is not formed.
        L.matfree = k >= 1 && k <= p.matfree_levels;
        DevMem setup_only;
        // D_k^{-1}
        {
            DevMem tmp;
            int32_t* dpos = upload(tmp, P.A_diag, st);
            L.Dinv_nat = C.mem.alloc<double>(L.n_units * L.nb * L.nb);
            HIPCHK(launch_block_inverse(L.A_nat, dpos, L.n_units, L.nb, L.Dinv_nat, C.flag, st));
            if (read_flag(C, st))
                throw Error(AMGDG_ESINGULAR, "diagonal block singular to working precision on level " + std::to_string(k));
        }
        if (L.matfree) C.build_mem = &setup_only;
        build_mat(C, L.A, L.n_units, L.nb, L.nb, P.A_rp, P.A_ci, L.A_nat, C.mixed && !L.matfree, st);
        if (!L.matfree) {
            // S = D^{-1} A without its diagonal blocks, D^{-1} A_ee = I: a sweep
            // u + omega (c - S u) reads the off-diagonal blocks and u itself
            DevMem tmp;
            int32_t* rp_d = upload(tmp, P.A_rp, st);
            double* S_full = tmp.alloc<double>(L.nnzb * L.nb * L.nb);
            HIPCHK(launch_row_scale(L.A_nat, rp_d, L.n_units, L.nb, L.Dinv_nat, S_full, st));
            std::vector<int32_t> srp(size_t(L.n_units) + 1, 0), sci, src;
            sci.reserve(size_t(L.nnzb - L.n_units));
            src.reserve(size_t(L.nnzb - L.n_units));
            for (int64_t e = 0; e < L.n_units; ++e) {
                for (int32_t a = P.A_rp[e]; a < P.A_rp[e + 1]; ++a)
                    if (a != P.A_diag[e]) {
                        sci.push_back(P.A_ci[a]);
                        src.push_back(a);
                    }
                srp[e + 1] = int32_t(sci.size());
            }
            L.nnzb_S = int64_t(sci.size());
            int32_t* src_d = upload(tmp, src, st);
            L.S_nat = C.mem.alloc<double>(L.nnzb_S * L.nb * L.nb);
            HIPCHK(launch_gather_blocks(S_full, src_d, L.nnzb_S, L.nb * L.nb, L.S_nat, st));
            HIPCHK(hipStreamSynchronize(st));
            build_mat(C, L.S, L.n_units, L.nb, L.nb, srp, sci, L.S_nat, C.mixed, st, true);
        }
        if (!L.A.vec) {
            L.Dinv_sell = sell_dinv<double>(C, L.A.s.d, L.A.s.pos, L.Dinv_nat, st);
            if (C.mixed && !L.matfree) L.Dinv_sell32 = sell_dinv<float>(C, L.A.s.f, L.A.s.pos, L.Dinv_nat, st);
        }
        C.build_mem = nullptr;
        if (C.mixed) {
            L.Dinv_nat32 = C.mem.alloc<float>(L.n_units * L.nb * L.nb);
            HIPCHK(launch_f64_to_f32(L.Dinv_nat, L.Dinv_nat32, L.n_units * L.nb * L.nb, st));
        }
        // omega_k
        if (p.omega_fixed > 0) {
            L.omega = p.omega_fixed;
        } else {
            L.rho = power_rho(C, L, k, st);
            if (!(L.rho > 0) || !std::isfinite(L.rho)) throw Error(AMGDG_ENAN, "power iteration gave rho <= 0");
            L.omega = (4.0 / 3.0) / L.rho;
        }
        // relaxation of the candidates
        L.B_in = C.mem.alloc<double>(L.n * r);
        HIPCHK(hipMemcpyAsync(L.B_in, B, sizeof(double) * L.n * r, hipMemcpyDeviceToDevice, st));
        relax_candidates(C, L, B, st);
        L.B_rel = B;
        // coarse sizes s_J (eq:sik): the h-step count from the aggregate's real
        // dofs, or, for an aggregate that equals its only child (h*-step), the
        // count of singular values above delta times the largest, decided on
        // the device with the SVD
        std::vector<int32_t> sJ(size_t(P.n_agg));
        int smax_possible = 0;
        bool all_h = true;
        for (int64_t J = 0; J < P.n_agg; ++J) {
            int64_t rows = 0;
            for (int32_t u = P.first_child[J]; u < P.first_child[J + 1]; ++u) rows += L.sz[u];
            const int64_t cap = std::min<int64_t>(rows, r);
            if (P.first_child[J + 1] - P.first_child[J] == 1) {
                sJ[J] = -1;
                all_h = false;
                smax_possible = std::max<int>(smax_possible, int(cap));
            } else {
                sJ[J] = int32_t(std::min<int64_t>((int64_t)std::ceil(double(rows) / p.n_cut), cap));
                smax_possible = std::max<int>(smax_possible, sJ[J]);
            }
            if (rows > 1024) throw Error(AMGDG_EUNSUPPORTED, "aggregate with more than 1024 dofs");
        }
        bool uniform_s = all_h;
        for (int64_t J = 1; J < P.n_agg && uniform_s; ++J) uniform_s = sJ[J] == sJ[0];
        int64_t max_rows = 0;
        for (int64_t J = 0; J < P.n_agg; ++J)
            max_rows = std::max<int64_t>(max_rows, int64_t(P.first_child[J + 1] - P.first_child[J]) * L.nb);
        DevMem tmp;
        int32_t* fc = upload(tmp, P.first_child, st);
        L.sv = C.mem.alloc<double>(P.n_agg * r);
        int s = 0;
        if (uniform_s && !L.padded && r <= 16 && max_rows <= 128 && P.n_agg > 0) {
            // one wavefront per aggregate, registers only (r <= 16, <= 128 rows)
            s = sJ[0];
            L.Pu = C.mem.alloc<double>(L.n * s);
            HIPCHK(launch_svd(B, r, fc, P.n_agg, L.nb, s, L.Pu, L.sv, C.flag, st));
            const int32_t f = read_flag(C, st);
            if (f & 4) throw Error(AMGDG_ESINGULAR, "candidate block of an aggregate is rank deficient");
        } else {
            // general form: one workgroup per aggregate, columns in global memory
            std::vector<int64_t> woff(size_t(P.n_agg) + 1, 0);
            for (int64_t J = 0; J < P.n_agg; ++J) {
                int64_t nr = 0;
                for (int32_t u = P.first_child[J]; u < P.first_child[J + 1]; ++u) nr += L.sz[u];
                woff[J + 1] = woff[J] + nr * r + (nr < r ? nr * nr : 0);
            }
            const int spad0 = std::max(smax_possible, 1);
            double* Pw = tmp.alloc<double>(L.n * spad0);
            HIPCHK(hipMemsetAsync(Pw, 0, sizeof(double) * size_t(L.n * spad0), st));
            int32_t* sJ_d = upload(tmp, sJ, st);
            const int64_t* woff_d = upload(tmp, woff, st);
            double* work = tmp.alloc<double>(woff[P.n_agg]);
            HIPCHK(launch_svd_gen(B, r, fc, L.sz_d, L.nb, P.n_agg, sJ_d, p.delta, spad0, work, woff_d, Pw, L.sv,
                                  C.flag, st));
            const int32_t f = read_flag(C, st);
            if (f & 2) throw Error(AMGDG_EUNSUPPORTED, "aggregate SVD outside the supported sizes");
            if (f & 4) throw Error(AMGDG_ESINGULAR, "candidate block of an aggregate is rank deficient");
            sJ = download(sJ_d, P.n_agg, st);
            for (int64_t J = 0; J < P.n_agg; ++J) {
                if (sJ[J] < 1) throw Error(AMGDG_ESINGULAR, "an aggregate keeps no coarse vector");
                s = std::max<int>(s, sJ[J]);
            }
            L.Pu = C.mem.alloc<double>(L.n * s);
            HIPCHK(hipMemcpy2DAsync(L.Pu, sizeof(double) * s, Pw, sizeof(double) * spad0, sizeof(double) * s,
                                    size_t(L.n), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        if (s > 64) throw Error(AMGDG_EUNSUPPORTED, "coarse block size above 64");
        L.s = s;
        cur_sz = sJ;
        // T = P~ - omega D^{-1} A P~ ; R = T^T
        L.nT = int64_t(P.T_ci.size());
        {
            int32_t* A_ci = upload(tmp, P.A_ci, st);
            int32_t* T_row = upload(tmp, P.T_row, st);
            int32_t* T_ci = upload(tmp, P.T_ci, st);
            int32_t* Tm_ptr = upload(tmp, P.Tm_ptr, st);
            int32_t* Tm_a = upload(tmp, P.Tm_a, st);
            int32_t* agg = upload(tmp, P.agg, st);
            double* W = tmp.alloc<double>(L.nT * L.nb * s);
            L.T_nat = C.mem.alloc<double>(L.nT * L.nb * s);
            HIPCHK(launch_T_build(L.A_nat, A_ci, T_row, T_ci, Tm_ptr, Tm_a, agg, L.nT, L.nb, s, L.Pu, L.Dinv_nat,
                                  L.omega, W, L.T_nat, st));
            int32_t* R_t = upload(tmp, P.R_t, st);
            L.R_nat = C.mem.alloc<double>(L.nT * L.nb * s);
            HIPCHK(launch_R_from_T(L.T_nat, R_t, L.nT, L.nb, s, L.R_nat, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        build_mat(C, L.T, L.n_units, L.nb, s, P.T_rp, P.T_ci, L.T_nat, C.mixed, st);
        build_mat(C, L.R, P.n_agg, s, L.nb, P.R_rp, P.R_ci, L.R_nat, C.mixed, st);
        {
            DevMem t1;
            int32_t* rci = upload(t1, P.R_ci, st);
            int32_t* dpos = upload(t1, P.A_diag, st);
            L.RD_nat = C.mem.alloc<double>(L.nT * L.nb * s);
            HIPCHK(launch_right_diag(L.R_nat, rci, L.nT, L.nb, s, L.A_nat, dpos, L.RD_nat, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        build_mat(C, L.RD, P.n_agg, s, L.nb, P.R_rp, P.R_ci, L.RD_nat, C.mixed, st);
        // M = R (D - omega A), where it reads no more values than the residual
        // pass over S and the RD product it replaces (plus 2^21, about a
        // launch's latency at full bandwidth), and where it is stored as block
        // CSR (s <= 4), whose entry-wise kernel reads its long rows at full
        // width; a sliced M (larger coarse blocks) would stage rows one
        // neighbour layer longer than R D's, in chunks, which measured slower
        // on the hexahedral hierarchies
        const bool try_M = p.restrict_resid && p.t_pre >= 1 && !L.matfree && s <= BCSR_MAXBR;
        if (try_M) symbolic_M(C.plan.lv[k]);
        L.nM = int64_t(P.M_ci.size());
        if (try_M && L.nM * s * L.nb <= L.nnzb * L.nb * L.nb + L.nT * s * L.nb + (int64_t(1) << 21)) {
            DevMem t1;
            int32_t* rci = upload(t1, P.R_ci, st);
            int32_t* mci = upload(t1, P.M_ci, st);
            int64_t* mpp = upload(t1, P.M_pp, st);
            int32_t* mpr = upload(t1, P.M_pr, st);
            int32_t* mpa = upload(t1, P.M_pa, st);
            L.M_nat = C.mem.alloc<double>(L.nM * s * L.nb);
            HIPCHK(launch_restrict_resid(L.R_nat, L.A_nat, rci, mci, mpp, mpr, mpa, L.nM, L.nb, s, L.omega, L.M_nat,
                                         st));
            HIPCHK(hipStreamSynchronize(st));
            build_mat(C, L.M, P.n_agg, s, L.nb, P.M_rp, P.M_ci, L.M_nat, C.mixed, st);
            L.has_M = true;
        }
        if (try_M) {  // the pairs served the numeric phase only
            LevelPattern& Pm = C.plan.lv[k];
            std::vector<int64_t>().swap(Pm.M_pp);
            std::vector<int32_t>().swap(Pm.M_pr);
            std::vector<int32_t>().swap(Pm.M_pa);
        }
        // A_{k+1} = R (A T)
        Level& Ln = C.lv[k + 1];
        {
            DevMem t2;
            const int64_t nAT = int64_t(P.AT_ci.size());
            double* ATv = t2.alloc<double>(nAT * L.nb * s);
            int64_t* pp = upload(t2, P.AT_pp, st);
            int32_t* pa = upload(t2, P.AT_pa, st);
            int32_t* pt = upload(t2, P.AT_pt, st);
            HIPCHK(launch_AT(L.A_nat, L.T_nat, pp, pa, pt, nAT, L.nb, s, ATv, st));
            const int64_t nC = int64_t(P.C_ci.size());
            Ln.A_nat = C.mem.alloc<double>(nC * s * s);
            int64_t* cpp = upload(t2, P.C_pp, st);
            int32_t* cpt = upload(t2, P.C_pt, st);
            int32_t* cpu = upload(t2, P.C_pu, st);
            HIPCHK(launch_galerkin(L.T_nat, ATv, cpp, cpt, cpu, nC, L.nb, s, Ln.A_nat, st));
            // coarse units with s_J < s: unit diagonal on their padding rows
            bool pad_next = false;
            for (int32_t v : cur_sz) pad_next = pad_next || v < s;
            if (pad_next) {
                const std::vector<int32_t>& dg = (k + 1 < C.N) ? C.plan.lv[k + 1].A_diag : C.plan.AN_diag;
                int32_t* dg_d = upload(t2, dg, st);
                int32_t* sz_d = upload(t2, cur_sz, st);
                HIPCHK(launch_pad_diag(Ln.A_nat, dg_d, P.n_agg, s, sz_d, st));
            }
            HIPCHK(hipStreamSynchronize(st));
        }
        // B^{k+1} = R B^k
        if (k + 1 < C.N) {
            double* Bn = C.mem.alloc<double>(P.n_agg * s * r);
            mat_spmv<double>(AX, L.R, B, nullptr, Bn, r, st);
            B = Bn;
        }
        cur_nb = s;
        HIPCHK(hipStreamSynchronize(st));
        if (L.matfree) {
            // A_k's values and layouts go; D_k^{-1} (natural, FP64 and FP32), T_k,
            // R_k and R_k D_k stay
            C.mem.free(L.A_nat);
            L.A_nat = nullptr;
            L.A = MatStore();
            L.Dinv_sell = nullptr;
        }
    }
    HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------ workspaces

// Lays out the device buffers of a Work of m columns (restart > 0: with a
// restarted-FGMRES basis).  With W == nullptr only the byte count is formed.
static int64_t work_layout(const Ctx& C, Work* W, int m, int restart) {
    int64_t bytes = 0;
    auto get = [&](auto tag, int64_t n) {
        using T = decltype(tag);
        bytes += (int64_t(sizeof(T)) * std::max<int64_t>(n, 1) + 255) / 256 * 256;
        return W ? W->mem.alloc<T>(n) : static_cast<T*>(nullptr);
    };
    const double d = 0.0;
    const float f = 0.0f;
    const int32_t i = 0;
    if (W) {
        W->v64.assign(C.N + 1, VBuf<double>());
        W->v32.assign(C.N + 1, VBuf<float>());
    }
    for (int k = 0; k <= C.N; ++k) {
        const int64_t cnt = C.lv[k].n * m;
        double* b = get(d, cnt);
        double* u = get(d, cnt);
        double* w = get(d, cnt);
        double* r = get(d, cnt);
        double* c = k < C.N ? get(d, cnt) : nullptr;
        if (W) W->v64[k] = VBuf<double>{b, u, w, r, nullptr, c};
        if (C.mixed) {
            float* bf = get(f, cnt);
            float* uf = get(f, cnt);
            float* wf = get(f, cnt);
            float* rf = get(f, cnt);
            float* cf = k < C.N ? get(f, cnt) : nullptr;
            if (W) W->v32[k] = VBuf<float>{bf, uf, wf, rf, nullptr, cf};
        }
    }
    const int64_t n = C.lv[0].n * m;
    double* kv[10];
    for (double*& p : kv) p = get(d, n);
    float* kr32 = C.mixed ? get(f, n) : nullptr;
    float* kz32 = C.mixed ? get(f, n) : nullptr;
    double* V = restart > 0 ? get(d, C.lv[0].n * (restart + 1)) : nullptr;
    double* Z = restart > 0 ? get(d, C.lv[0].n * restart) : nullptr;
    double* scratch = get(d, int64_t(DOT_PARTS) * 64 + 1024);
    double* scal = get(d, 2048);
    double* kpart = get(d, 2 * 16 * (KRY_BLOCKS + 1) + 64);
    // partials of p.(A p): per sliced workgroup (8 columns at a time), or per
    // workgroup of the FP64 tiles (16 columns at a time)
    const MatStore& A0 = C.lv[0].A;
    const int64_t n_sp = std::max<int64_t>(A0.vec ? 1 : int64_t(A0.s.d.n_slices) * 8,
                                           use_mfma<double>(A0, m) ? mfma_dot_parts(int64_t(A0.nd.n_brow)) : 0);
    double* kslice = get(d, n_sp);
    double* stat = get(d, ST_LEN);
    int32_t* mask = get(i, MASK_LEN);
    if (W) {
        W->kb = kv[0], W->kx = kv[1], W->kr = kv[2], W->kr2 = kv[3], W->kz = kv[4];
        W->kp = kv[5], W->kq = kv[6], W->kt = kv[7], W->kgin = kv[8], W->kgout = kv[9];
        W->kr32 = kr32, W->kz32 = kz32;
        W->V = V, W->Z = Z;
        W->scratch = scratch, W->scal = scal, W->kpart = kpart, W->stat = stat, W->mask = mask;
        W->kslice = kslice;
    }
    return bytes;
}

static int64_t work_bytes(const Ctx& C, int m, int restart) { return work_layout(C, nullptr, m, restart); }

// (Re)allocates W for m columns and zeroes it: no column ever holds a value
// that was not written by this library.
static void work_init(Ctx& C, Work& W, int m, int restart, hipStream_t st) {
    if (W.m > 0) HIPCHK(hipStreamSynchronize(st));
    W.drop_graphs();
    W.mem.release();
    W.m = 0;
    W.bytes = work_layout(C, &W, m, restart);
    W.mem.zero_all(st);
    if (!W.stat_h) {
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&W.stat_h), ST_LEN * sizeof(double), hipHostMallocDefault));
        std::memset(W.stat_h, 0, ST_LEN * sizeof(double));
    }
    if (!W.mask_h) {
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&W.mask_h), MASK_LEN * sizeof(int32_t), hipHostMallocDefault));
        std::memset(W.mask_h, 0, MASK_LEN * sizeof(int32_t));
    }
    if (restart > 0 && !W.gm_h) {
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&W.gm_h), GM_H_LEN * sizeof(double), hipHostMallocDefault));
        std::memset(W.gm_h, 0, GM_H_LEN * sizeof(double));
    }
    if (!W.ev) HIPCHK(hipEventCreateWithFlags(&W.ev, hipEventDisableTiming));
    if (!W.ev2) HIPCHK(hipEventCreateWithFlags(&W.ev2, hipEventDisableTiming));
    if (!W.ev_ret) HIPCHK(hipEventCreateWithFlags(&W.ev_ret, hipEventDisableTiming));
    HIPCHK(hipStreamSynchronize(st));
    W.m = m;
    W.restart = restart;
    W.mixed = C.mixed;
}

// The handle's own Work, grown to at least m columns (and an FGMRES basis of
// `restart` vectors) when needed.
static Work& default_work(Ctx& C, int m, int restart, hipStream_t st) {
    if (!C.W0) C.W0 = std::make_unique<Work>();
    Work& W = *C.W0;
    if (W.m >= m && W.restart >= restart) return W;
    work_init(C, W, std::max(m, W.m), std::max(restart, W.restart), st);
    return W;
}

// ------------------------------------------------------------ V-cycle

template <typename T>
static VBuf<T>& vbuf(Work& W, int k);
template <>
VBuf<double>& vbuf<double>(Work& W, int k) { return W.v64[k]; }
template <>
VBuf<float>& vbuf<float>(Work& W, int k) { return W.v32[k]; }

template <typename T>
static VBuf<T>* vbufs(Work& W) {
    return &vbuf<T>(W, 0);
}

template <typename T>
static void coarse_solve(Ctx& C, const T* b, T* u, int m, hipStream_t st) {
    HIPCHK(launch_gemv<T>(C.Ainv, b, u, C.nN, m, st));
}

// q = A_k u on a matrix-free level k (eq:matfree2 unrolled one level at a
// time: A_k = R_{k-1} A_{k-1} T_{k-1}, with A_{k-1} formed the same way when it
// is not stored either).  The products use level k-1's free vectors: the one
// of u/w that does not hold u_{k-1}, and r (its residual has been restricted).
template <typename T>
static void matfree_apply(Ctx& C, VBuf<T>* VB, int k, const T* u, T* q, int m, hipStream_t st) {
    Level& Lp = C.lv[k - 1];
    VBuf<T>& Vp = VB[k - 1];
    T* t = (Vp.cur == Vp.u) ? Vp.w : Vp.u;
    T* t2 = Vp.r;
    mat_spmv<T>(AX, Lp.T, u, nullptr, t, m, st);
    if (Lp.matfree) matfree_apply<T>(C, VB, k - 1, t, t2, m, st);
    else mat_spmv<T>(AX, Lp.A, t, nullptr, t2, m, st);
    mat_spmv<T>(AX, Lp.R, t2, nullptr, q, m, st);
}

// z0 = V(b0), internal order, m columns (Algorithm 2, one pass from u = 0).
// VB holds the level vectors of levels 0..N (the V-cycle's only workspace).
template <typename T>
static void vcycle_impl(Ctx& C, VBuf<T>* VB, const T* b0, T* z0, int m, hipStream_t st) {
    const int N = C.N;
    const int tpre = C.prm.t_pre, tpost = C.prm.t_post;
    auto vb = [&](int k) -> VBuf<T>& { return VB[k]; };
    if (N == 0) {
        coarse_solve<T>(C, b0, z0, m, st);
        return;
    }
    bool started = false;  // level k's first sweep was done by the restriction into it
    // Consecutive passes over a level's S go in opposite directions (Sell::rev):
    // each starts on the part of S that the memory-side cache took in last
    std::vector<int> s_pass(size_t(N), 0);
    for (int k = 0; k < N; ++k) {
        Level& L = C.lv[k];
        VBuf<T>& V = vb(k);
        const T* bk = (k == 0) ? b0 : V.b;
        T* cur = V.u;
        T* oth = V.w;
        const T om = T(L.omega);
        // Every sweep after the first runs on S = D^{-1} A with c = D^{-1} b:
        // u + omega D^{-1} (b - A u) = u + omega (c - S u), one matrix read
        // instead of A and D^{-1}.  The first sweep (from u = 0) also writes c.
        if (L.matfree) {
            // the same sweeps with A_k u formed by matfree_apply into V.r:
            // u + omega (c - D^{-1} A_k u); the residual D^{-1} (b - A_k u) goes to
            // the free one of u/w and is restricted by R D like S's residual
            const T* dinv = dinv_nat_of<T>(L);
            if (tpre == 0) {
                HIPCHK(hipMemsetAsync(cur, 0, sizeof(T) * L.n * m, st));
                HIPCHK(launch_bdiag<T>(BD_START, dinv, bk, nullptr, nullptr, oth, V.c, T(1), L.n_units, L.nb, m, st));
            } else {
                if (!started)
                    HIPCHK(launch_bdiag<T>(BD_START, dinv, bk, nullptr, nullptr, cur, V.c, om, L.n_units, L.nb, m, st));
                for (int t = 1; t < tpre; ++t) {
                    V.cur = cur;
                    matfree_apply<T>(C, VB, k, cur, V.r, m, st);
                    HIPCHK(launch_bdiag<T>(BD_SWEEP, dinv, V.r, V.c, cur, oth, nullptr, om, L.n_units, L.nb, m, st));
                    std::swap(cur, oth);
                }
            }
            V.cur = cur;
            matfree_apply<T>(C, VB, k, cur, V.r, m, st);
            HIPCHK(launch_bdiag<T>(BD_RESID, dinv, V.r, V.c, nullptr, oth, nullptr, om, L.n_units, L.nb, m, st));
            VBuf<T>& Vn = vb(k + 1);
            started = k + 1 < N && tpre > 0 && restrict_start<T>(L.RD, C.lv[k + 1], oth, Vn.u, Vn.c, m, st);
            if (!started) mat_spmv<T>(AX, L.RD, oth, nullptr, Vn.b, m, st);
            continue;
        }
        // With M = R (D - omega A) the last pre-sweep also writes the residual
        // e = c - S u of the iterate it starts from, and R (b - A u') = M e for
        // the iterate u' it writes; after a single sweep from zero e is c.  On
        // the 16-column tiles (one wavefront per block row) M serves only levels
        // with at least 2,048 coarse block rows: below that its long rows leave
        // the tiles with too few wavefronts (the 3D hierarchy's last restriction
        // took 722 us through M at 16 columns)
        const bool via_M = L.has_M && tpre >= 1 && (!use_mfma<T>(L.M, m) || L.n_agg >= 2048);
        const T* e = V.c;
        if (tpre == 0) {
            HIPCHK(hipMemsetAsync(cur, 0, sizeof(T) * L.n * m, st));
            mat_sweep<T>(SWEEP0, L, nullptr, bk, V.c, T(1), m, nullptr, st);
        } else {
            if (!started) mat_sweep<T>(SWEEP0, L, nullptr, bk, cur, om, m, nullptr, st, V.c);
            for (int t = 1; t < tpre; ++t) {
                const bool rev = (s_pass[k]++ & 1) != 0;
                if (via_M && t == tpre - 1) {
                    mat_spmv<T>(S_SWEEP_R, L.S, cur, V.c, oth, m, st, om, V.r, rev);
                    e = V.r;
                } else {
                    mat_spmv<T>(S_SWEEP, L.S, cur, V.c, oth, m, st, om, nullptr, rev);
                }
                std::swap(cur, oth);
            }
        }
        V.cur = cur;
        // R (b - A u) = RD (c - S u), or M e
        const MatStore& Rk = via_M ? L.M : L.RD;
        if (!via_M) {
            mat_spmv<T>(B_MINUS, L.S, cur, V.c, V.r, m, st, T(0), nullptr, (s_pass[k]++ & 1) != 0);
            e = V.r;
        }
        // Into a non-coarsest level the restriction also takes that level's first
        // sweep: it writes omega D^{-1} b_{k+1} and c_{k+1} = D^{-1} b_{k+1} (the
        // same operations as the first sweep on the stored b_{k+1}); b_{k+1}
        // itself is not needed then.
        VBuf<T>& Vn = vb(k + 1);
        started = k + 1 < N && tpre > 0 && restrict_start<T>(Rk, C.lv[k + 1], e, Vn.u, Vn.c, m, st);
        if (!started) mat_spmv<T>(AX, Rk, e, nullptr, Vn.b, m, st);
    }
    {
        VBuf<T>& V = vb(N);
        coarse_solve<T>(C, V.b, V.u, m, st);
        V.cur = V.u;
    }
    for (int k = N - 1; k >= 0; --k) {
        Level& L = C.lv[k];
        VBuf<T>& V = vb(k);
        const T om = T(L.omega);
        T* cur = V.cur;
        auto other = [&](T* c) { return c == V.u ? V.w : V.u; };
        T* dst = (k == 0 && tpost == 0) ? z0 : other(cur);
        mat_spmv<T>(B_PLUS, L.T, vb(k + 1).cur, cur, dst, m, st);
        cur = dst;
        for (int t = 0; t < tpost; ++t) {
            dst = (k == 0 && t == tpost - 1) ? z0 : other(cur);
            if (L.matfree) {
                V.cur = cur;
                matfree_apply<T>(C, VB, k, cur, V.r, m, st);
                HIPCHK(launch_bdiag<T>(BD_SWEEP, dinv_nat_of<T>(L), V.r, V.c, cur, dst, nullptr, om, L.n_units, L.nb,
                                       m, st));
            } else {
                mat_spmv<T>(S_SWEEP, L.S, cur, V.c, dst, m, st, om, nullptr, (s_pass[k]++ & 1) != 0);
            }
            cur = dst;
        }
        V.cur = cur;
    }
}

// Whether a call replays the captured V-cycle (flags without AMGDG_EAGER).
// The graph's start and end leave the device idle for a few microseconds each;
// where one pass over the level-0 operator S reads 128 MB or more, the host
// queues the V-cycle's kernels one by one long before the device reaches them,
// so those V-cycles are launched eagerly.
static bool graph_for(const Ctx& C, int flags, int prec_bytes) {
    if (flags & AMGDG_EAGER) return false;
    const Level& L = C.lv[0];
    const double s_bytes = double(L.nnzb_S) * L.nb * L.nb * prec_bytes;
    return s_bytes < 128.0 * (1 << 20);
}

// The V-cycle as a captured HIP graph: its ~40 launches (most of them small
// coarse-level kernels) are submitted as one graph launch, so the host no
// longer paces the coarse levels.  The graph is captured on the Work's private
// stream the first time a (precision, m, input, output) combination is seen and
// replayed on the caller's stream; reallocating the Work drops the cache.  It
// holds only kernel nodes (no memset or copy nodes).
template <typename T>
static void vcycle_run(Ctx& C, Work& W, const T* b0, T* z0, int m, hipStream_t st, bool allow_graph) {
    if (!allow_graph || C.prm.t_pre == 0 || C.N == 0) {
        vcycle_impl<T>(C, vbufs<T>(W), b0, z0, m, st);
        return;
    }
    const int prec = int(sizeof(T));
    for (auto& e : W.graphs)
        if (e.prec == prec && e.m == m && e.in == b0 && e.out == z0) {
            HIPCHK(hipGraphLaunch(e.e, st));
            return;
        }
    if (W.graphs.size() >= 8) {
        HIPCHK(hipStreamSynchronize(st));
        W.drop_graphs();
    }
    if (!W.cap) HIPCHK(hipStreamCreateWithFlags(&W.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(W.cap, hipStreamCaptureModeThreadLocal));
    try {
        vcycle_impl<T>(C, vbufs<T>(W), b0, z0, m, W.cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(W.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(W.cap, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        HIPCHK(err);
    }
    W.graphs.push_back({prec, m, b0, z0, g, ex});
    HIPCHK(hipGraphLaunch(ex, st));
}

// ------------------------------------------------------------ Krylov helpers

struct KrylovState {
    std::vector<int32_t> its;
    std::vector<double> rel;
    std::vector<double> bnorm;
};

// z = V(r) in FP64 for arbitrary r, z: through the graph's fixed buffers.
static void precond_fp64(Ctx& C, Work& W, const double* r, double* z, int m, hipStream_t st) {
    if (!W.use_graph) {
        vcycle_impl<double>(C, vbufs<double>(W), r, z, m, st);
        return;
    }
    const size_t bytes = sizeof(double) * size_t(C.lv[0].n) * m;
    if (r != W.kgin) HIPCHK(hipMemcpyAsync(W.kgin, r, bytes, hipMemcpyDeviceToDevice, st));
    vcycle_run<double>(C, W, W.kgin, W.kgout, m, st, true);
    if (z != W.kgout) HIPCHK(hipMemcpyAsync(z, W.kgout, bytes, hipMemcpyDeviceToDevice, st));
}

static void precond(Ctx& C, Work& W, const double* r, double* z, int m, int precision, hipStream_t st) {
    const int64_t n = C.lv[0].n;
    if (precision == AMGDG_MIXED) {
        HIPCHK((launch_convert<double, float>(r, W.kr32, n * m, st)));
        vcycle_run<float>(C, W, W.kr32, W.kz32, m, st, W.use_graph);
        HIPCHK((launch_convert<float, double>(W.kz32, z, n * m, st)));
    } else {
        precond_fp64(C, W, r, z, m, st);
    }
}

// true residual W.kt = b - A x and its per-column norms^2
static std::vector<double> true_res(Ctx& C, Work& W, const double* b, const double* x, int m, hipStream_t st) {
    Level& L = C.lv[0];
    mat_spmv<double>(B_MINUS, L.A, x, b, W.kt, m, st);
    return dotm(W.scratch, W.scal, W.kt, W.kt, L.n, m, st);
}

static void check_nan(const std::vector<double>& v, const char* what) {
    for (double d : v)
        if (!std::isfinite(d)) throw Error(AMGDG_ENAN, std::string("NaN or Inf in ") + what);
}

// ------------------------------------------------------------ CG batch engine

static constexpr double kReplaceDrop = 1e-6;
using Clock = std::chrono::steady_clock;

// A right-hand side waiting for, or holding, a column of a batch.
struct Rhs {
    int64_t tag = 0;
    const double* b = nullptr;   // caller's b (column start); rows `ld` apart
    double* x = nullptr;         // caller's x, same addressing
    const double* x0 = nullptr;  // initial guess, same addressing, or NULL (x0 = 0)
    int64_t ld = 1;
    double tol = 1e-8;
    int32_t maxit = 1000;
    bool internal = false;       // rows already in internal order
    Clock::time_point t_submit;
};

// How a right-hand side left its batch.
struct Outcome {
    int64_t tag = 0;
    int rc = AMGDG_OK;
    int32_t its = 0;
    double rel = 0.0;
    double latency = 0.0;  // seconds from submission to the host seeing x written
    Clock::time_point t_submit;
};

// Preconditioned CG (flexible = false) or flexible CG with residual replacement
// (flexible = true, Polak-Ribiere beta) on up to m right-hand sides at once,
// the columns of one Work.  Columns are independent: each kernel computes
// column c from column c only, and every reduction adds in an order fixed by n
// alone, so a right-hand side gets bit-identical iterates whatever shares the
// batch and whichever column it occupies.  Columns join between iterations
// (admit) and leave when they converge, fail or reach their iteration limit
// (retire).  A column spends the iteration in which it joins with
// alpha = beta = 0: that iteration forms z = M r0 and r0.z, and its direction
// update sets p = z, which is the method's start.
//
// Host loop, per iteration: the fused update of x and r (with ||r||^2 and, for
// the FP32 V-cycle, the FP32 copy of r); the status record is copied to pinned
// memory behind an event; the preconditioner of the new residual and the new
// r.z are queued at once (run-ahead, so the GPU does not wait for the host);
// when the event has passed, the host reads the status, retires and admits
// columns and queues the new direction, q = A p and p.q.  A column whose
// recursive residual meets its tolerance, has dropped by kReplaceDrop since its
// last replacement (flexible) or reaches its iteration limit is first checked
// against its true residual b - A x (one more readback); in the flexible
// method a true residual above the tolerance replaces the recursive one.
// What a batch runs: right-hand sides are admitted into its columns, the
// engine queues its work on its stream and the host advances it whenever the
// event it waits on has passed.  An outcome moves to `done` once the solution
// of its retired right-hand side is written (W->ev_ret).
struct Engine {
    Ctx* C = nullptr;
    Work* W = nullptr;
    hipStream_t st = nullptr;
    bool fail_fast = false;  // an error fails the call instead of one column
    std::vector<Outcome> retiring;
    std::vector<Outcome> done;
    virtual ~Engine() = default;
    virtual int free_slot() const = 0;
    virtual void admit(int slot, const Rhs& rq) = 0;
    virtual int busy() const = 0;        // right-hand sides admitted and not retired
    virtual bool idle() const = 0;       // no event to wait for
    virtual void start() = 0;            // queues admitted work on an idle engine
    virtual hipEvent_t waiting() const = 0;
    virtual void process() = 0;          // called once the awaited event has passed
    bool ready() const {
        if (idle()) return false;
        const hipError_t e = hipEventQuery(waiting());
        if (e == hipSuccess) return true;
        if (e != hipErrorNotReady) HIPCHK(e);
        return false;
    }
    void collect(bool blocking) {
        if (retiring.empty()) return;
        if (blocking) {
            HIPCHK(hipEventSynchronize(W->ev_ret));
        } else {
            const hipError_t e = hipEventQuery(W->ev_ret);
            if (e == hipErrorNotReady) return;
            HIPCHK(e);
        }
        const Clock::time_point now = Clock::now();
        for (Outcome& o : retiring) {
            o.latency = std::chrono::duration<double>(now - o.t_submit).count();
            done.push_back(o);
        }
        retiring.clear();
    }
    // blocking driver: runs until every admitted right-hand side has left
    void run() {
        if (idle()) start();
        while (!idle()) {
            HIPCHK(hipEventSynchronize(waiting()));
            process();
        }
        collect(true);
    }
};

struct CgBatch : Engine {
    enum { EMPTY = 0, STARTING = 1, RUNNING = 2 };
    enum { IDLE = 0, WAIT_STATUS = 1, WAIT_TRUE = 2 };
    struct Col {
        int state = EMPTY;
        bool upd = false;    // active in the update of the iteration in flight
        bool check = false;  // waiting for its true residual
        Rhs rq;
        int32_t its = 0;
        double bnorm = 1.0, rel = 0.0, anchor = 1.0;
    };
    int m = 0;
    bool flexible = false, mixed = false;
    int phase = IDLE;
    std::vector<Col> col;
    std::vector<int> pending;               // admitted, not yet queued
    std::vector<std::pair<int, Outcome>> leaving;  // retired in this host step
    double *r = nullptr, *rn = nullptr;
    double *d_pq = nullptr, *d_rz = nullptr, *d_rz2 = nullptr, *d_zro = nullptr;
    int32_t* flags_d = nullptr;
    int32_t last_upd[64], last_dir[64];

    void init(Ctx& c, Work& w, hipStream_t s, int width, bool flex, bool mix, bool ff) {
        C = &c;
        W = &w;
        st = s;
        m = width;
        flexible = flex;
        mixed = mix;
        fail_fast = ff;
        phase = IDLE;
        col.assign(m, Col());
        pending.clear();
        leaving.clear();
        retiring.clear();
        done.clear();
        r = W->kr;
        rn = W->kr2;
        d_pq = W->scal;
        d_rz = W->scal + 64;
        d_rz2 = W->scal + 128;
        d_zro = W->scal + 192;
        flags_d = reinterpret_cast<int32_t*>(W->stat + ST_FLAG);
        std::fill(last_upd, last_upd + 64, -1);
        std::fill(last_dir, last_dir + 64, -1);
    }

    int free_slot() const override {
        for (int c = 0; c < m; ++c)
            if (col[c].state == EMPTY && std::find(pending.begin(), pending.end(), c) == pending.end()) return c;
        return -1;
    }
    int busy() const override {
        int k = int(pending.size());
        for (const Col& c : col) k += c.state != EMPTY;
        return k;
    }
    bool idle() const override { return phase == IDLE; }
    hipEvent_t waiting() const override { return W->ev; }
    void start() override {
        if (phase == IDLE && !pending.empty()) issue();
    }
    void admit(int slot, const Rhs& rq) override {
        col[slot].rq = rq;
        pending.push_back(slot);
    }

    void apply_M(double* rz_out, const double* r_old, double* zro) {
        const int64_t n = C->lv[0].n;
        if (mixed) vcycle_run<float>(*C, *W, W->kr32, W->kz32, m, st, W->use_graph);
        else if (!flexible) vcycle_run<double>(*C, *W, r, W->kz, m, st, W->use_graph);  // r, z fixed buffers
        else precond_fp64(*C, *W, r, W->kz, m, st);
        // mixed: the FP64 z is never stored; the direction update reads z32 itself
        HIPCHK(launch_zdots(mixed ? W->kz32 : nullptr, mixed ? nullptr : W->kz, r, r_old, n, m, W->kpart, rz_out, zro,
                            st));
    }

    // uploads mask region `off` from the pinned mirror if it differs from `last`
    void upload_mask(int off, int32_t* last) {
        bool same = true;
        for (int c = 0; c < m; ++c) same = same && last[c] == W->mask_h[off + c];
        if (same) return;
        HIPCHK(hipMemcpyAsync(W->mask + off, W->mask_h + off, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        for (int c = 0; c < m; ++c) last[c] = W->mask_h[off + c];
    }

    // queues admissions and the next iteration (update, status readback, run-ahead M)
    void issue() {
        const Level& L = C->lv[0];
        const int64_t n = L.n;
        if (!pending.empty()) {
            bool any_x0 = false;
            for (int c : pending) {
                const Rhs& q = col[c].rq;
                HIPCHK(launch_admit(q.b, q.ld, q.x0, q.ld, q.internal ? nullptr : C->perm_d, L.n_units, L.nb, W->kb,
                                    W->kx, r, W->kp, W->kq, m, c, flags_d, st));
                any_x0 = any_x0 || q.x0;
            }
            HIPCHK(launch_dot_tail(W->kb, W->kb, n, m, W->kpart, W->stat + ST_BN, st));
            if (any_x0) {
                // r = b - A x0 for the admitted columns with an initial guess
                for (int c = 0; c < m; ++c) W->mask_h[MASK_ADM + c] = 0;
                for (int c : pending) W->mask_h[MASK_ADM + c] = col[c].rq.x0 ? 1 : 0;
                HIPCHK(hipMemcpyAsync(W->mask + MASK_ADM, W->mask_h + MASK_ADM, sizeof(int32_t) * m,
                                      hipMemcpyHostToDevice, st));
                mat_spmv<double>(B_MINUS, L.A, W->kx, W->kb, W->kt, m, st);
                HIPCHK(launch_copy_cols(W->kt, r, n, m, W->mask + MASK_ADM, st));
                HIPCHK(launch_dot_tail(r, r, n, m, W->kpart, W->stat + ST_R0, st));
            }
            for (int c : pending) {
                col[c].state = STARTING;
                col[c].its = 0;
            }
            pending.clear();
        }
        for (int c = 0; c < m; ++c) {
            col[c].upd = col[c].state == RUNNING;
            W->mask_h[MASK_UPD + c] = col[c].upd ? 1 : 0;
        }
        upload_mask(MASK_UPD, last_upd);
        HIPCHK(launch_cg_update(W->kx, r, flexible ? rn : r, W->kp, W->kq, mixed ? W->kr32 : nullptr, n, m, d_rz, d_pq,
                                W->mask + MASK_UPD, W->kpart, W->stat + ST_RR, flags_d, st, W->stat, W->stat_h, ST_TR));
        if (flexible) std::swap(r, rn);  // r: new residual, rn: previous
        // (the update's last finalize has mirrored the status record [0, ST_TR) to stat_h)
        HIPCHK(hipEventRecord(W->ev, st));
        apply_M(d_rz2, flexible ? rn : nullptr, flexible ? d_zro : nullptr);
        phase = WAIT_STATUS;
    }

    void retire(int c, int rc, double rel) {
        Col& k = col[c];
        if (fail_fast && rc != AMGDG_OK && rc != AMGDG_ENOCONV) {
            (void)hipStreamSynchronize(st);
            phase = IDLE;
            throw Error(rc, rc == AMGDG_EBREAKDOWN ? "CG breakdown: p^T A p <= 0 (matrix or preconditioner not SPD)"
                                                   : "NaN or Inf in CG (right-hand side or iterate)");
        }
        Outcome o;
        o.tag = k.rq.tag;
        o.rc = rc;
        o.its = k.its;
        o.rel = rel;
        o.t_submit = k.rq.t_submit;
        leaving.push_back({c, o});
        k.state = EMPTY;
        k.upd = false;
        k.check = false;
    }

    // handles the phase whose event has passed and queues what follows
    void process() override {
        if (phase == WAIT_STATUS) {
            const int32_t* fl = reinterpret_cast<const int32_t*>(W->stat_h + ST_FLAG);
            bool need_true = false;
            for (int c = 0; c < m; ++c) {
                Col& k = col[c];
                if (k.state == STARTING) {
                    const double bn2 = W->stat_h[ST_BN + c];
                    const double r02 = k.rq.x0 ? W->stat_h[ST_R0 + c] : bn2;
                    if (!std::isfinite(bn2) || !std::isfinite(r02)) {
                        retire(c, AMGDG_ENAN, std::numeric_limits<double>::quiet_NaN());
                        continue;
                    }
                    k.bnorm = std::sqrt(bn2) > 0 ? std::sqrt(bn2) : 1.0;
                    k.rel = std::sqrt(r02) / k.bnorm;
                    k.anchor = k.rel;
                    if (k.rel <= k.rq.tol) retire(c, AMGDG_OK, k.rel);
                    else if (k.rq.maxit <= 0) retire(c, AMGDG_ENOCONV, k.rel);
                    else k.state = RUNNING;
                } else if (k.state == RUNNING && k.upd) {
                    if (fl[c]) {
                        retire(c, (fl[c] & 1) ? AMGDG_EBREAKDOWN : AMGDG_ENAN, k.rel);
                        continue;
                    }
                    ++k.its;
                    k.rel = std::sqrt(W->stat_h[ST_RR + c]) / k.bnorm;
                    k.check = k.rel <= k.rq.tol || (flexible && k.rel <= k.anchor * kReplaceDrop) ||
                              k.its >= k.rq.maxit;
                    need_true = need_true || k.check;
                }
            }
            if (need_true) {
                const int64_t n = C->lv[0].n;
                mat_spmv<double>(B_MINUS, C->lv[0].A, W->kx, W->kb, W->kt, m, st);
                HIPCHK(launch_dot_tail(W->kt, W->kt, n, m, W->kpart, W->stat + ST_TR, st));
                HIPCHK(hipMemcpyAsync(W->stat_h + ST_TR, W->stat + ST_TR, sizeof(double) * m, hipMemcpyDeviceToHost,
                                      st));
                HIPCHK(hipEventRecord(W->ev, st));
                phase = WAIT_TRUE;
                return;
            }
        } else if (phase == WAIT_TRUE) {
            bool any_repl = false;
            for (int c = 0; c < m; ++c) W->mask_h[MASK_REPL + c] = 0;
            for (int c = 0; c < m; ++c) {
                Col& k = col[c];
                if (!(k.state == RUNNING && k.check)) continue;
                k.check = false;
                const double t = std::sqrt(W->stat_h[ST_TR + c]) / k.bnorm;
                if (!std::isfinite(t)) retire(c, AMGDG_ENAN, t);
                else if (t <= k.rq.tol) retire(c, AMGDG_OK, t);
                else if (k.its >= k.rq.maxit) retire(c, AMGDG_ENOCONV, t);
                else if (flexible) {
                    W->mask_h[MASK_REPL + c] = 1;  // the true residual takes the place of the recursive one
                    k.anchor = t;
                    any_repl = true;
                }
            }
            if (any_repl) {
                const int64_t n = C->lv[0].n;
                HIPCHK(hipMemcpyAsync(W->mask + MASK_REPL, W->mask_h + MASK_REPL, sizeof(int32_t) * m,
                                      hipMemcpyHostToDevice, st));
                HIPCHK(launch_copy_cols(W->kt, r, n, m, W->mask + MASK_REPL, st));
                if (mixed) HIPCHK((launch_convert<double, float>(r, W->kr32, n * m, st)));
                apply_M(d_rz2, flexible ? rn : nullptr, flexible ? d_zro : nullptr);
            }
        } else {
            return;
        }
        advance();
    }

    // x of the columns retired in this host step goes out; the direction
    // update and the next iteration are queued
    void advance() {
        if (!leaving.empty()) {
            const Level& L = C->lv[0];
            for (auto& pr : leaving) {
                const Rhs& q = col[pr.first].rq;
                HIPCHK(launch_scatter_col(W->kx + pr.first, m, q.x, q.ld, q.internal ? nullptr : C->perm_d, L.n_units,
                                          L.nb, st));
                retiring.push_back(pr.second);
            }
            leaving.clear();
            HIPCHK(hipEventRecord(W->ev_ret, st));
        }
        bool running = false;
        for (const Col& k : col) running = running || k.state == RUNNING;
        if (!running && pending.empty()) {
            phase = IDLE;
            return;
        }
        if (running) {
            const int64_t n = C->lv[0].n;
            for (int c = 0; c < m; ++c) W->mask_h[MASK_DIR + c] = (col[c].state == RUNNING && col[c].upd) ? 1 : 0;
            upload_mask(MASK_DIR, last_dir);
            HIPCHK(launch_cg_dir(W->kp, mixed ? nullptr : W->kz, n, m, d_rz2, flexible ? d_zro : nullptr, d_rz,
                                 W->mask + MASK_DIR, st, mixed ? W->kz32 : nullptr));
            std::swap(d_rz, d_rz2);
            const MatStore& A0 = C->lv[0].A;
            if (!A0.vec && !use_mfma<double>(A0, m)) {
                // q = A p with p.q from per-slice partials of the product itself
                HIPCHK(launch_spmv_dot(sel<double>(A0.s), W->kp, W->kq, m, W->kslice, d_pq, st, cap_of<double>(A0, m)));
            } else if (use_mfma<double>(A0, m)) {
                // the same on the FP64 tiles: per-workgroup partials of p.q
                HIPCHK(launch_mfma_dot(nsel<double>(A0), W->kp, W->kq, m, W->kslice, W->kpart, d_pq, st,
                                       mfu_of<double>(A0, m)));
            } else {
                mat_spmv<double>(AX, A0, W->kp, nullptr, W->kq, m, st);
                HIPCHK(launch_dot_tail(W->kp, W->kq, n, m, W->kpart, d_pq, st));
            }
        }
        issue();
    }
};

// ------------------------------------------------------------ solvers

static int solve_stationary(Ctx& C, Work& W, int m, int precision, double tol, int maxit, KrylovState& S,
                            hipStream_t st) {
    Level& L = C.lv[0];
    const int64_t n = L.n;
    std::vector<int32_t> act(m, 1);
    S.its.assign(m, 0);
    S.rel.assign(m, 0.0);
    std::vector<double> rr = true_res(C, W, W.kb, W.kx, m, st);
    for (int it = 1; it <= maxit; ++it) {
        HIPCHK(hipMemcpyAsync(W.kr, W.kt, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
        precond(C, W, W.kr, W.kz, m, precision, st);
        // x += z for active columns: alpha = active
        std::vector<double> a(m);
        for (int c = 0; c < m; ++c) a[c] = act[c] ? 1.0 : 0.0;
        HIPCHK(hipMemcpyAsync(W.scal + 1024, a.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        HIPCHK(launch_axpby_dev(W.kz, W.kx, n, m, W.scal + 1024, 1.0, 1.0, st));
        HIPCHK(hipStreamSynchronize(st));
        rr = true_res(C, W, W.kb, W.kx, m, st);
        check_nan(rr, "residual");
        bool any = false;
        for (int c = 0; c < m; ++c)
            if (act[c]) {
                S.its[c] = it;
                S.rel[c] = std::sqrt(rr[c]) / S.bnorm[c];
                if (S.rel[c] <= tol) act[c] = 0;
                any = any || act[c];
            }
        if (!any) return AMGDG_OK;
    }
    return AMGDG_ENOCONV;
}

// Right-preconditioned restarted FGMRES(restart) on one right-hand side: the
// preconditioned vectors z_j = M(v_j) are kept, so M may change between steps
// (as the FP32 V-cycle's rounding does), and every restart begins from the
// true FP64 residual, which makes the mixed-precision variant iterative
// refinement with an FGMRES inner solver.  Arnoldi uses classical Gram-Schmidt
// applied twice.  A step needs no host value: both passes' coefficients and
// the new vector's norm stay on the device, which also normalises the vector,
// so the host queues step j + 1 before it reads step j (a two-slot ring of
// pinned records) and only applies the Givens rotations and the stopping test.
// A cycle ends when the least-squares residual meets the tolerance, the basis
// is full or the iteration limit is reached; then x += Z y and the true
// residual decides between stopping and restarting.
struct GmresRun : Engine {
    enum { IDLE = 0, WAIT_STEP = 1, WAIT_RES = 2 };
    // device scalars (W->scal) and the pinned record of a step
    static constexpr int H1 = 0, H2 = 257, NRM = 514, REC = 515, YD = 1024, BN = 1536, RR = 1537;
    // pinned layout (W->gm_h): two step records, then ||b||^2 and ||r||^2, then y
    static constexpr int RES = 2 * REC, YH = 2 * REC + 8;
    int restart = 30;
    bool mixed = false;
    int phase = IDLE;
    bool pend = false, has = false, first = true;
    Rhs rq;
    int32_t total = 0, cyc0 = 0;
    int j = 0, queued = 0;
    double bnorm = 1.0;
    std::vector<double> H, cs, sn, g, y;

    void init(Ctx& c, Work& w, hipStream_t s, int rst, bool mix, bool ff) {
        C = &c;
        W = &w;
        st = s;
        restart = rst;
        mixed = mix;
        fail_fast = ff;
        phase = IDLE;
        pend = has = false;
        H.assign(size_t(restart + 1) * restart, 0.0);
        cs.assign(restart, 0.0);
        sn.assign(restart, 0.0);
        g.assign(restart + 1, 0.0);
        y.assign(restart, 0.0);
    }
    int free_slot() const override { return (pend || has) ? -1 : 0; }
    void admit(int, const Rhs& q) override {
        rq = q;
        pend = true;
    }
    int busy() const override { return (pend || has) ? 1 : 0; }
    bool idle() const override { return phase == IDLE; }
    hipEvent_t waiting() const override {
        return (phase == WAIT_STEP && (j & 1)) ? W->ev2 : W->ev;
    }
    double& Hat(int i, int k) { return H[size_t(i) * restart + k]; }

    void start() override {
        if (!pend) return;
        pend = false;
        has = true;
        first = true;
        total = 0;
        const Level& L = C->lv[0];
        int32_t* flags_d = reinterpret_cast<int32_t*>(W->stat + ST_FLAG);
        HIPCHK(launch_admit(rq.b, rq.ld, rq.x0, rq.ld, rq.internal ? nullptr : C->perm_d, L.n_units, L.nb, W->kb,
                            W->kx, W->kt, W->kp, W->kq, 1, 0, flags_d, st));
        HIPCHK(launch_dot<double>(W->kb, W->kb, L.n, 1, W->scratch, W->scal + BN, st));
        queue_residual();
    }

    // t = b - A x, ||t||^2 and (first time) ||b||^2 to the host
    void queue_residual() {
        const Level& L = C->lv[0];
        mat_spmv<double>(B_MINUS, L.A, W->kx, W->kb, W->kt, 1, st);
        HIPCHK(launch_dot<double>(W->kt, W->kt, L.n, 1, W->scratch, W->scal + RR, st));
        HIPCHK(hipMemcpyAsync(W->gm_h + RES, W->scal + BN, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(W->ev, st));
        phase = WAIT_RES;
    }

    // Arnoldi step k of the cycle: z_k = M v_k, w = A z_k, CGS2, ||w||, v_{k+1} = w / ||w||
    void queue_step() {
        const int k = queued;
        if (k >= restart || cyc0 + k >= rq.maxit) return;
        const int64_t n = C->lv[0].n;
        double* vk = W->V + int64_t(k) * n;
        double* zk = W->Z + int64_t(k) * n;
        double* w = W->V + int64_t(k + 1) * n;
        precond(*C, *W, vk, zk, 1, mixed ? AMGDG_MIXED : AMGDG_FP64, st);
        mat_spmv<double>(AX, C->lv[0].A, zk, nullptr, w, 1, st);
        HIPCHK(launch_multidot(W->V, n, k + 1, w, n, W->scratch, W->scal + H1, st));
        HIPCHK(launch_multi_axpy(W->V, n, k + 1, W->scal + H1, w, n, -1.0, st));
        HIPCHK(launch_multidot(W->V, n, k + 1, w, n, W->scratch, W->scal + H2, st));
        HIPCHK(launch_multi_axpy(W->V, n, k + 1, W->scal + H2, w, n, -1.0, st));
        HIPCHK(launch_dot<double>(w, w, n, 1, W->scratch, W->scal + NRM, st));
        HIPCHK(hipMemcpyAsync(W->gm_h + (k & 1) * REC, W->scal, REC * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord((k & 1) ? W->ev2 : W->ev, st));
        HIPCHK(launch_scale_by_inv_norm(w, n, W->scal + NRM, st));
        ++queued;
    }

    void retire(int rc, double rel) {
        if (fail_fast && rc != AMGDG_OK && rc != AMGDG_ENOCONV) {
            (void)hipStreamSynchronize(st);
            phase = IDLE;
            has = false;
            throw Error(rc, rc == AMGDG_EBREAKDOWN ? "GMRES breakdown" : "NaN or Inf in GMRES (right-hand side or iterate)");
        }
        const Level& L = C->lv[0];
        HIPCHK(launch_scatter_col(W->kx, 1, rq.x, rq.ld, rq.internal ? nullptr : C->perm_d, L.n_units, L.nb, st));
        HIPCHK(hipEventRecord(W->ev_ret, st));
        Outcome o;
        o.tag = rq.tag;
        o.rc = rc;
        o.its = total;
        o.rel = rel;
        o.t_submit = rq.t_submit;
        retiring.push_back(o);
        has = false;
        phase = IDLE;
        if (pend) start();
    }

    void process() override {
        if (phase == WAIT_RES) {
            if (first) {
                const double bn2 = W->gm_h[RES];
                if (!std::isfinite(bn2)) return retire(AMGDG_ENAN, std::numeric_limits<double>::quiet_NaN());
                bnorm = std::sqrt(bn2) > 0 ? std::sqrt(bn2) : 1.0;
                first = false;
            }
            const double rr = W->gm_h[RES + 1];
            if (!std::isfinite(rr)) return retire(AMGDG_ENAN, rr);
            const double beta = std::sqrt(rr);
            const double rel = beta / bnorm;
            if (rel <= rq.tol) return retire(AMGDG_OK, rel);
            if (total >= rq.maxit) return retire(AMGDG_ENOCONV, rel);
            HIPCHK(launch_axpby_dev(W->kt, W->V, C->lv[0].n, 1, nullptr, 1.0 / beta, 0.0, st));
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            cyc0 = total;
            j = 0;
            queued = 0;
            queue_step();
            queue_step();  // run-ahead
            phase = WAIT_STEP;
            return;
        }
        if (phase != WAIT_STEP) return;
        const double* rec = W->gm_h + (j & 1) * REC;
        const double hn = std::sqrt(rec[NRM]);
        bool finite = std::isfinite(hn);
        for (int i = 0; i <= j; ++i) {
            Hat(i, j) = rec[H1 + i] + rec[H2 + i];
            finite = finite && std::isfinite(Hat(i, j));
        }
        if (!finite) return retire(AMGDG_ENAN, std::numeric_limits<double>::quiet_NaN());
        Hat(j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
            Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
            Hat(i, j) = t;
        }
        const double den = std::hypot(Hat(j, j), Hat(j + 1, j));
        if (!(den > 0)) return retire(AMGDG_EBREAKDOWN, std::numeric_limits<double>::quiet_NaN());
        cs[j] = Hat(j, j) / den;
        sn[j] = Hat(j + 1, j) / den;
        Hat(j, j) = den;
        Hat(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++total;
        const int jend = j + 1;
        if (std::fabs(g[j + 1]) <= rq.tol * bnorm || jend == restart || total >= rq.maxit) {
            // x += Z y with H[:jend, :jend] y = g[:jend]
            for (int i = jend - 1; i >= 0; --i) {
                double s = g[i];
                for (int l = i + 1; l < jend; ++l) s -= Hat(i, l) * y[l];
                y[i] = s / Hat(i, i);
            }
            std::memcpy(W->gm_h + YH, y.data(), sizeof(double) * jend);
            HIPCHK(hipMemcpyAsync(W->scal + YD, W->gm_h + YH, sizeof(double) * jend, hipMemcpyHostToDevice, st));
            HIPCHK(launch_multi_axpy(W->Z, C->lv[0].n, jend, W->scal + YD, W->kx, C->lv[0].n, 1.0, st));
            queue_residual();
            return;
        }
        ++j;
        queue_step();  // keeps one step queued ahead of the one awaited
    }
};

static void check_solve_args(const Ctx& C, int m, int method, int precision) {
    if (C.N == 0) throw Error(AMGDG_EUNSUPPORTED, "Krylov solve needs at least two levels");
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    if (precision != AMGDG_FP64 && precision != AMGDG_MIXED) throw Error(AMGDG_EINVAL, "bad precision");
    if (precision == AMGDG_MIXED && !C.mixed) throw Error(AMGDG_EINVAL, "mixed precision needs params.mixed = 1");
    if (method < AMGDG_STATIONARY || method > AMGDG_FGMRES) throw Error(AMGDG_EINVAL, "bad method");
}

static int solve_impl(Ctx& C, int m, const double* b_dev, double* x_dev, int method, int precision, double rtol,
                      int max_it, int restart, int flags, amgdg_solve_stats* stats, hipStream_t st) {
    check_solve_args(C, m, method, precision);
    if (!b_dev || !x_dev) throw Error(AMGDG_EINVAL, "b or x is NULL");
    if (method == AMGDG_FGMRES && (m != 1 || restart < 1 || restart > 256))
        throw Error(AMGDG_EUNSUPPORTED, "FGMRES: m = 1 and 1 <= restart <= 256");
    const auto t0 = Clock::now();
    Work& W = default_work(C, m, method == AMGDG_FGMRES ? restart : 0, st);
    W.use_graph = graph_for(C, flags, precision == AMGDG_MIXED ? 4 : 8);
    Level& L = C.lv[0];
    const int64_t n = L.n;
    const bool internal = flags & AMGDG_INTERNAL_ORDER;
    std::vector<int32_t> its(m, 0);
    std::vector<double> rel(m, 0.0);
    int rc = AMGDG_OK;
    if (method != AMGDG_STATIONARY) {
        CgBatch cg;
        GmresRun gm;
        Engine* E = &cg;
        if (method == AMGDG_FGMRES) {
            gm.init(C, W, st, restart, precision == AMGDG_MIXED, true);
            E = &gm;
        } else {
            cg.init(C, W, st, m, method == AMGDG_FCG, precision == AMGDG_MIXED, true);
        }
        for (int c = 0; c < m; ++c) {
            Rhs q;
            q.tag = c;
            q.b = b_dev + c;
            q.x = x_dev + c;
            q.x0 = (flags & AMGDG_X0) ? x_dev + c : nullptr;
            q.ld = m;
            q.tol = rtol;
            q.maxit = max_it;
            q.internal = internal;
            q.t_submit = t0;
            E->admit(c, q);
        }
        E->run();
        for (const Outcome& o : E->done) {
            its[o.tag] = o.its;
            rel[o.tag] = o.rel;
            if (o.rc != AMGDG_OK) rc = AMGDG_ENOCONV;
        }
    } else {
        if (internal) HIPCHK(hipMemcpyAsync(W.kb, b_dev, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
        else HIPCHK((launch_permute<double, double>(b_dev, W.kb, C.perm_d, L.n_units, L.nb, m, 1, st)));
        if (flags & AMGDG_X0) {
            if (internal) HIPCHK(hipMemcpyAsync(W.kx, x_dev, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
            else HIPCHK((launch_permute<double, double>(x_dev, W.kx, C.perm_d, L.n_units, L.nb, m, 1, st)));
        } else {
            HIPCHK(hipMemsetAsync(W.kx, 0, sizeof(double) * n * m, st));
        }
        KrylovState S;
        S.bnorm = dotm(W.scratch, W.scal, W.kb, W.kb, n, m, st);
        check_nan(S.bnorm, "b");
        for (double& v : S.bnorm) v = std::sqrt(v) > 0 ? std::sqrt(v) : 1.0;
        rc = solve_stationary(C, W, m, precision, rtol, max_it, S, st);
        // final true residuals
        std::vector<double> tr = true_res(C, W, W.kb, W.kx, m, st);
        if (internal) HIPCHK(hipMemcpyAsync(x_dev, W.kx, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
        else HIPCHK((launch_permute<double, double>(W.kx, x_dev, C.perm_d, L.n_units, L.nb, m, 0, st)));
        HIPCHK(hipStreamSynchronize(st));
        for (int c = 0; c < m; ++c) {
            its[c] = S.its[c];
            rel[c] = std::sqrt(tr[c]) / S.bnorm[c];
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        int all = 1, mx = 0;
        for (int c = 0; c < m; ++c) {
            stats->iterations[c] = its[c];
            stats->rel_residual[c] = rel[c];
            mx = std::max(mx, its[c]);
            if (!(rel[c] <= rtol)) all = 0;
        }
        stats->max_iterations = mx;
        stats->all_converged = all;
        stats->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    }
    return rc;
}

// ------------------------------------------------------------ serving

// Continuous batching.  Requests on the same (handle, method, precision,
// restart) share a batch: CG requests the `width` columns of one CgBatch,
// where a request takes a free column between iterations and leaves it when
// done, so the level operators are read once per iteration for every request
// of the batch; an FGMRES request a batch of its own (one column and its
// Krylov basis).  Batches run on streams of their own, so their work overlaps
// on the device, and are created while the device bytes of all batch
// workspaces stay within the budget; an idle batch of another key is released
// to make room.  Requests wait in submission order; one that cannot be placed
// does not hold back requests that can.
struct Request {
    Ctx* C = nullptr;
    int method = AMGDG_PCG, precision = AMGDG_FP64, restart = 0;
    Rhs rq;
};

struct ServerBatch {
    Ctx* C = nullptr;
    int method = 0, precision = 0, restart = 0;
    hipStream_t st = nullptr;
    Work W;
    std::unique_ptr<Engine> eng;
    ~ServerBatch() {
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    }
    bool same_key(const Request& r) const {
        return C == r.C && method == r.method && precision == r.precision && restart == r.restart;
    }
};

struct Server {
    int width = 4;
    int64_t budget = 0, used = 0;
    std::deque<Request> queue;
    std::vector<std::unique_ptr<ServerBatch>> batches;
    std::vector<Outcome> done;

    static int batch_width(int method, int width) { return method == AMGDG_FGMRES ? 1 : width; }
    static int64_t batch_bytes(const Ctx& C, int method, int width, int restart) {
        return work_bytes(C, batch_width(method, width), method == AMGDG_FGMRES ? restart : 0);
    }
    static bool idle(const ServerBatch& b) { return b.eng->idle() && b.eng->busy() == 0 && b.eng->retiring.empty(); }

    ServerBatch* create(const Request& r) {
        const int64_t need = batch_bytes(*r.C, r.method, width, r.restart);
        if (used + need > budget) {
            // release idle batches of other keys, oldest first
            for (size_t i = 0; i < batches.size() && used + need > budget;) {
                ServerBatch& b = *batches[i];
                if (idle(b) && !b.same_key(r)) {
                    used -= b.W.bytes;
                    batches.erase(batches.begin() + i);
                } else {
                    ++i;
                }
            }
        }
        if (used + need > budget) return nullptr;
        auto b = std::make_unique<ServerBatch>();
        b->C = r.C;
        b->method = r.method;
        b->precision = r.precision;
        b->restart = r.restart;
        HIPCHK(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
        const bool fgm = r.method == AMGDG_FGMRES;
        work_init(*r.C, b->W, batch_width(r.method, width), fgm ? r.restart : 0, b->st);
        b->W.use_graph = true;
        if (fgm) {
            auto e = std::make_unique<GmresRun>();
            e->init(*r.C, b->W, b->st, r.restart, r.precision == AMGDG_MIXED, false);
            b->eng = std::move(e);
        } else {
            auto e = std::make_unique<CgBatch>();
            e->init(*r.C, b->W, b->st, width, r.method == AMGDG_FCG, r.precision == AMGDG_MIXED, false);
            b->eng = std::move(e);
        }
        used += b->W.bytes;
        batches.push_back(std::move(b));
        return batches.back().get();
    }

    void admit_queued() {
        std::vector<ServerBatch*> kick;
        for (auto it = queue.begin(); it != queue.end();) {
            ServerBatch* tgt = nullptr;
            for (auto& b : batches)
                if (b->same_key(*it) && b->eng->free_slot() >= 0) {
                    tgt = b.get();
                    break;
                }
            if (!tgt) tgt = create(*it);
            if (!tgt) {
                ++it;
                continue;
            }
            tgt->eng->admit(tgt->eng->free_slot(), it->rq);
            if (tgt->eng->idle() && std::find(kick.begin(), kick.end(), tgt) == kick.end()) kick.push_back(tgt);
            it = queue.erase(it);
        }
        for (ServerBatch* b : kick) b->eng->start();
    }

    int64_t pending() const {
        int64_t k = int64_t(queue.size());
        for (auto& b : batches) k += b->eng->busy() + int64_t(b->eng->retiring.size());
        return k;
    }

    void step(bool wait) {
        admit_queued();
        while (true) {
            bool progressed = false;
            for (auto& b : batches) {
                Engine& e = *b->eng;
                if (e.ready()) {
                    e.process();
                    progressed = true;
                }
                const size_t before = e.done.size();
                e.collect(false);
                if (e.done.size() != before) progressed = true;
                for (Outcome& o : e.done) done.push_back(o);
                e.done.clear();
            }
            if (progressed) admit_queued();
            if (!wait || progressed || pending() == 0) return;
            bool in_flight = false;
            for (auto& b : batches) in_flight = in_flight || !b->eng->idle() || !b->eng->retiring.empty();
            if (!in_flight) return;  // queued requests that no budget can place
            std::this_thread::yield();
        }
    }
};

// ------------------------------------------------------------ autotuner

// Picks launch shapes for m columns by timing the candidates on the
// operators the V-cycle runs (HIP events on the handle's vectors: S_k =
// D^{-1} A_k in its sweep, T_k and R_k D in their products; A_k and R_k, which
// have the same shapes, take the same choices):
//   - columns per launch of the sliced and block-CSR kernels (1, 2, 4, 8(, 16));
//   - blocks loaded ahead in the MFMA tiles (1, 2, 4) when m is a multiple of 16;
//   - with `lanes`, the lanes per block row of every block-CSR operator
//     (4 .. 64, timed at one column), once per handle.
// The first two leave every column's arithmetic unchanged; the lane-group
// width changes the summation order (hence rounding) and is therefore chosen
// once, before use, and then applies to every column count.
static void autotune_impl(Ctx& C, int m, bool lanes, hipStream_t st) {
    if (C.N == 0) return;
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    if (lanes && C.lanes_tuned) throw Error(AMGDG_EINVAL, "lane-group widths are already tuned for this handle");
    Work& W = default_work(C, std::max(m, 1), 0, st);
    W.drop_graphs();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    // average time of `launch`: one warm-up, then repetitions spanning at least
    // about 0.2 ms (3 .. 200 launches), so that small coarse-level kernels are
    // timed above the event resolution
    auto timed = [&](auto&& launch) {
        launch();
        HIPCHK(hipEventRecord(e0, st));
        launch();
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float one = 0.f;
        HIPCHK(hipEventElapsedTime(&one, e0, e1));
        const int reps = std::max(3, std::min(200, int(0.2f / std::max(one, 1e-4f))));
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) launch();
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        return ms / float(reps);
    };
    for (int k = 0; k < C.N; ++k) {
        Level& L = C.lv[k];
        struct Op {
            MatStore* M;
            MatStore* twin;
            int kin, kout;
        } ops[4] = {{&L.S, &L.A, k, k}, {&L.T, nullptr, k + 1, k}, {&L.RD, &L.R, k, k + 1}, {&L.M, nullptr, k, k + 1}};
        for (Op& o : ops) {
            if (o.M == &L.S && L.matfree) continue;  // no S_k on a matrix-free level
            if (o.M == &L.M && !L.has_M) continue;
            MatStore& M = *o.M;
            // S_k is timed in its block-Jacobi sweep (2 nu - 1 of them per level
            // and cycle), T_k and R_k D in their products
            auto run = [&](auto tag, int cols) {
                using T = decltype(tag);
                VBuf<T>& vin = vbuf<T>(W, o.kin);
                VBuf<T>& vout = vbuf<T>(W, o.kout);
                if (o.M == &L.S) mat_spmv<T>(S_SWEEP, M, vin.u, vin.b, vout.w, cols, st, T(L.omega));
                else mat_spmv<T>(AX, M, vin.u, nullptr, vout.w, cols, st);
            };
            auto tune_type = [&](auto tag) {
                using T = decltype(tag);
                if (sizeof(T) == 4 && !C.mixed) return;
                auto& cap = sizeof(T) == 8 ? M.cap64 : M.cap32;
                auto& mfu = sizeof(T) == 8 ? M.mfu64 : M.mfu32;
                if (use_mfma<T>(M, m)) {
                    int best = 0;
                    float bt = 0.f;
                    for (int u : {1, 2, 3, 4}) {
                        mfu[m / MFMA_COLS] = int8_t(u);
                        const float t = timed([&] { run(tag, m); });
                        if (best == 0 || t < bt) best = u, bt = t;
                    }
                    mfu[m / MFMA_COLS] = int8_t(best);
                } else if (m > 1) {
                    int best = 0;
                    float bt = 0.f;
                    for (int c : {1, 2, 4, 8, 16}) {
                        if (!M.vec && c == 16) continue;
                        cap[m] = int8_t(c);
                        const float t = timed([&] { run(tag, m); });
                        if (best == 0 || t < bt) best = c, bt = t;
                    }
                    cap[m] = int8_t(best);
                }
            };
            if (lanes && M.vec) {
                int best = 0;
                float bt = 0.f;
                for (int P : {4, 8, 16, 32, 64, 128, 256}) {
                    M.bd.P = M.bf.P = P;
                    const float t = C.mixed ? timed([&] { run(0.0f, 1); }) : timed([&] { run(0.0, 1); });
                    if (best == 0 || t < bt) best = P, bt = t;
                }
                M.bd.P = M.bf.P = best;
            }
            tune_type(0.0);
            tune_type(0.0f);
            if (o.twin) {
                MatStore& Tw = *o.twin;
                Tw.cap64 = M.cap64, Tw.cap32 = M.cap32, Tw.mfu64 = M.mfu64, Tw.mfu32 = M.mfu32;
                Tw.bd.P = Tw.bf.P = M.bd.P;
            }
        }
    }
    if (lanes) C.lanes_tuned = true;
    HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------ single steps

template <typename T>
static int apply_impl(Ctx& C, int k, int op, int m, const T* x, const T* b, T* y, int flags, hipStream_t st) {
    if (k < 0 || k > C.N) throw Error(AMGDG_EINVAL, "bad level");
    if (op != AMGDG_OP_COARSE && k == C.N) throw Error(AMGDG_EINVAL, "operation needs a non-coarsest level");
    if (op == AMGDG_OP_COARSE && k != C.N) throw Error(AMGDG_EINVAL, "AMGDG_OP_COARSE works on the coarsest level");
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    if (sizeof(T) == 4 && !C.mixed) throw Error(AMGDG_EINVAL, "FP32 operators not built (params.mixed = 0)");
    Work& W = default_work(C, m, 0, st);
    Level& L = C.lv[k];
    const bool perm = (k == 0) && !(flags & AMGDG_INTERNAL_ORDER);
    VBuf<T>& V = vbuf<T>(W, k);
    const int64_t nun = L.n_units;
    auto in = [&](const T* p, T* tmp) -> const T* {
        if (!p) return nullptr;
        if (!perm) return p;
        HIPCHK((launch_permute<T, T>(p, tmp, C.perm_d, nun, L.nb, m, 1, st)));
        return tmp;
    };
    // Only the arguments an operation reads are touched: b is not read by SPMV,
    // RESTRICT and COARSE, x is not read by SWEEP0.  Level-0 arguments are
    // gathered into internal order; the coarse x of PROLONG and the coarse y of
    // RESTRICT are not level-0 arrays and are used as they are.
    const bool uses_b = (op == AMGDG_OP_SWEEP || op == AMGDG_OP_SWEEP0 || op == AMGDG_OP_RESIDUAL ||
                         op == AMGDG_OP_PROLONG || op == AMGDG_OP_SWEEP_SCALED ||
                         op == AMGDG_OP_SWEEP_SCALED_RESID);
    const bool uses_x = (op != AMGDG_OP_SWEEP0);
    if ((uses_b && !b) || (uses_x && !x)) throw Error(AMGDG_EINVAL, "missing input array");
    if (L.matfree && (op == AMGDG_OP_SPMV || op == AMGDG_OP_RESIDUAL || op == AMGDG_OP_SWEEP ||
                      op == AMGDG_OP_SWEEP0 || op == AMGDG_OP_SWEEP_SCALED || op == AMGDG_OP_SWEEP_SCALED_RESID))
        throw Error(AMGDG_EUNSUPPORTED, "A_k is not stored on a matrix-free level");
    if (op == AMGDG_OP_RESTRICT_RESID && !L.has_M) throw Error(AMGDG_EUNSUPPORTED, "this level keeps no M_k");
    const bool fine_out = (op != AMGDG_OP_RESTRICT && op != AMGDG_OP_RESTRICT_SCALED && op != AMGDG_OP_RESTRICT_RESID);
    const bool fine_x = (op != AMGDG_OP_PROLONG);
    T* out = (perm && fine_out) ? V.u : y;
    const T* xi = !uses_x ? nullptr : (fine_x ? in(x, V.b) : x);
    const T* bi = uses_b ? in(b, V.r) : nullptr;
    switch (op) {
        case AMGDG_OP_SPMV: mat_spmv<T>(AX, L.A, xi, nullptr, out, m, st); break;
        case AMGDG_OP_RESIDUAL: mat_spmv<T>(B_MINUS, L.A, xi, bi, out, m, st); break;
        case AMGDG_OP_SWEEP: mat_sweep<T>(SWEEP, L, xi, bi, out, T(L.omega), m, nullptr, st); break;
        case AMGDG_OP_SWEEP0: mat_sweep<T>(SWEEP0, L, nullptr, bi, out, T(L.omega), m, nullptr, st); break;
        case AMGDG_OP_RESTRICT: mat_spmv<T>(AX, L.R, xi, nullptr, out, m, st); break;
        case AMGDG_OP_PROLONG: mat_spmv<T>(B_PLUS, L.T, xi, bi, out, m, st); break;
        case AMGDG_OP_COARSE: coarse_solve<T>(C, xi, out, m, st); break;
        case AMGDG_OP_SWEEP_SCALED: mat_spmv<T>(S_SWEEP, L.S, xi, bi, out, m, st, T(L.omega)); break;
        case AMGDG_OP_RESTRICT_SCALED: mat_spmv<T>(AX, L.RD, xi, nullptr, out, m, st); break;
        case AMGDG_OP_RESTRICT_RESID: mat_spmv<T>(AX, L.M, xi, nullptr, out, m, st); break;
        case AMGDG_OP_SWEEP_SCALED_RESID: {
            // the residual half goes through V.w (internal order) when level-0 rows are permuted
            T* out2 = perm ? V.w : y + L.n * m;
            mat_spmv<T>(S_SWEEP_R, L.S, xi, bi, out, m, st, T(L.omega), out2);
            if (perm) HIPCHK((launch_permute<T, T>(out2, y + L.n * m, C.perm_d, nun, L.nb, m, 0, st)));
            break;
        }
        default: throw Error(AMGDG_EINVAL, "bad op");
    }
    if (perm && fine_out) HIPCHK((launch_permute<T, T>(out, y, C.perm_d, nun, L.nb, m, 0, st)));
    return AMGDG_OK;
}

// ------------------------------------------------------------ exports

static void need(int64_t bytes, int64_t have) {
    if (have < bytes) throw Error(AMGDG_EINVAL, "export buffer too small: need " + std::to_string(bytes) + " bytes");
}

// rows of unit-blocked arrays (per_unit values each) from internal to caller order
static void unperm_rows(const Ctx& C, int k, std::vector<double>& h, int64_t per_unit) {
    if (k != 0) return;
    std::vector<double> o(h.size());
    for (size_t u = 0; u < C.plan.perm.size(); ++u)
        std::memcpy(&o[size_t(C.plan.perm[u] * per_unit)], &h[size_t(u * per_unit)], sizeof(double) * per_unit);
    h.swap(o);
}

// pattern + values of a block matrix with rows in internal order -> caller order
// (rows permuted for level 0; for R at level 0 the columns are level-0 units).
static void export_matrix(const Ctx& C, int k, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                          const std::vector<double>& vals, int64_t per, bool perm_rows, bool perm_cols,
                          std::vector<int32_t>& orp, std::vector<int32_t>& oci, std::vector<double>& ovals) {
    const int64_t nr = int64_t(rp.size()) - 1;
    orp.assign(nr + 1, 0);
    oci.clear();
    ovals.clear();
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t re = 0; re < nr; ++re) {
        const int64_t ri = (perm_rows && k == 0) ? C.plan.iperm[re] : re;
        row.clear();
        for (int32_t b = rp[ri]; b < rp[ri + 1]; ++b) {
            const int32_t c = (perm_cols && k == 0) ? int32_t(C.plan.perm[ci[b]]) : ci[b];
            row.push_back({c, b});
        }
        std::sort(row.begin(), row.end());
        for (auto& pr : row) {
            oci.push_back(pr.first);
            ovals.insert(ovals.end(), vals.begin() + pr.second * per, vals.begin() + (pr.second + 1) * per);
        }
        orp[re + 1] = int32_t(oci.size());
    }
}

template <typename V>
static void copy_out(const std::vector<V>& v, void* buf, int64_t bytes) {
    const int64_t need_b = int64_t(v.size() * sizeof(V));
    need(need_b, bytes);
    if (need_b) std::memcpy(buf, v.data(), size_t(need_b));
}

static int export_impl(Ctx& C, int k, int what, void* buf, int64_t bytes, hipStream_t st) {
    if (k < 0 || k > C.N) throw Error(AMGDG_EINVAL, "bad level");
    if (!buf) throw Error(AMGDG_EINVAL, "buffer is NULL");
    Level& L = C.lv[k];
    const bool coarsest = (k == C.N);
    if (what == AMGDG_PERM) {
        if (k != 0) throw Error(AMGDG_EINVAL, "PERM is a level-0 item");
        copy_out(C.plan.perm, buf, bytes);
        return AMGDG_OK;
    }
    if (what == AMGDG_UNIT_DOFS) {  // every level-0 unit holds nb dofs, so caller order needs no permutation
        copy_out(L.sz, buf, bytes);
        return AMGDG_OK;
    }
    if (what == AMGDG_A_ROWPTR || what == AMGDG_A_COLIDX || what == AMGDG_A_VALS) {
        const std::vector<int32_t>& rp = coarsest ? C.plan.AN_rp : C.plan.lv[k].A_rp;
        const std::vector<int32_t>& ci = coarsest ? C.plan.AN_ci : C.plan.lv[k].A_ci;
        const int64_t per = int64_t(L.nb) * L.nb;
        if (what == AMGDG_A_VALS && !L.A_nat) throw Error(AMGDG_EUNSUPPORTED, "A_k is not stored on a matrix-free level");
        std::vector<double> v = download(L.A_nat, int64_t(ci.size()) * per, st);
        std::vector<int32_t> orp, oci;
        std::vector<double> ov;
        export_matrix(C, k, rp, ci, v, per, true, true, orp, oci, ov);
        if (what == AMGDG_A_ROWPTR) copy_out(orp, buf, bytes);
        else if (what == AMGDG_A_COLIDX) copy_out(oci, buf, bytes);
        else copy_out(ov, buf, bytes);
        return AMGDG_OK;
    }
    if (coarsest) throw Error(AMGDG_EINVAL, "item not defined on the coarsest level");
    const LevelPattern& P = C.plan.lv[k];
    const int nb = L.nb, s = L.s, r = L.r;
    switch (what) {
        case AMGDG_T_ROWPTR:
        case AMGDG_T_COLIDX:
        case AMGDG_T_VALS: {
            std::vector<double> v = download(L.T_nat, L.nT * nb * s, st);
            std::vector<int32_t> orp, oci;
            std::vector<double> ov;
            export_matrix(C, k, P.T_rp, P.T_ci, v, int64_t(nb) * s, true, false, orp, oci, ov);
            if (what == AMGDG_T_ROWPTR) copy_out(orp, buf, bytes);
            else if (what == AMGDG_T_COLIDX) copy_out(oci, buf, bytes);
            else copy_out(ov, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_R_ROWPTR:
        case AMGDG_R_COLIDX:
        case AMGDG_R_VALS: {
            std::vector<double> v = download(L.R_nat, L.nT * nb * s, st);
            std::vector<int32_t> orp, oci;
            std::vector<double> ov;
            export_matrix(C, k, P.R_rp, P.R_ci, v, int64_t(nb) * s, false, true, orp, oci, ov);
            if (what == AMGDG_R_ROWPTR) copy_out(orp, buf, bytes);
            else if (what == AMGDG_R_COLIDX) copy_out(oci, buf, bytes);
            else copy_out(ov, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_DINV: {
            std::vector<double> v = download(L.Dinv_nat, L.n_units * nb * nb, st);
            unperm_rows(C, k, v, int64_t(nb) * nb);
            copy_out(v, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_B_RELAXED:
        case AMGDG_B_INPUT: {
            std::vector<double> v = download(what == AMGDG_B_RELAXED ? L.B_rel : L.B_in, L.n * r, st);
            unperm_rows(C, k, v, int64_t(nb) * r);
            copy_out(v, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_PTILDE: {
            std::vector<double> v = download(L.Pu, L.n * s, st);
            unperm_rows(C, k, v, int64_t(nb) * s);
            copy_out(v, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_SVALS: {
            std::vector<double> v = download(L.sv, L.n_agg * r, st);
            copy_out(v, buf, bytes);
            return AMGDG_OK;
        }
        case AMGDG_M_ROWPTR:
        case AMGDG_M_COLIDX:
        case AMGDG_M_VALS: {
            if (!L.has_M) throw Error(AMGDG_EUNSUPPORTED, "this level keeps no M_k (its pattern: amgdg_plan_export)");
            std::vector<double> v = download(L.M_nat, L.nM * nb * s, st);
            std::vector<int32_t> orp, oci;
            std::vector<double> ov;
            export_matrix(C, k, P.M_rp, P.M_ci, v, int64_t(nb) * s, false, true, orp, oci, ov);
            if (what == AMGDG_M_ROWPTR) copy_out(orp, buf, bytes);
            else if (what == AMGDG_M_COLIDX) copy_out(oci, buf, bytes);
            else copy_out(ov, buf, bytes);
            return AMGDG_OK;
        }

        default: throw Error(AMGDG_EINVAL, "unknown export item");
    }
}

// ------------------------------------------------------------ plan queries

static void plan_item(Plan& P, int k, int what, std::vector<int32_t>& out32, std::vector<int64_t>& out64) {
    out32.clear();
    out64.clear();
    const int N = P.n_levels - 1;
    if (k < 0 || k > N) throw Error(AMGDG_EINVAL, "bad level");
    if (what == AMGDG_PERM) {
        if (k != 0) throw Error(AMGDG_EINVAL, "PERM is a level-0 item");
        out64 = P.perm;
        return;
    }
    auto rows_caller = [&](const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, bool prow, bool pcol,
                           std::vector<int32_t>& orp, std::vector<int32_t>& oci) {
        const int64_t nr = int64_t(rp.size()) - 1;
        orp.assign(nr + 1, 0);
        oci.clear();
        std::vector<int32_t> row;
        for (int64_t re = 0; re < nr; ++re) {
            const int64_t ri = (prow && k == 0) ? P.iperm[re] : re;
            row.clear();
            for (int32_t b = rp[ri]; b < rp[ri + 1]; ++b) row.push_back((pcol && k == 0) ? int32_t(P.perm[ci[b]]) : ci[b]);
            std::sort(row.begin(), row.end());
            oci.insert(oci.end(), row.begin(), row.end());
            orp[re + 1] = int32_t(oci.size());
        }
    };
    std::vector<int32_t> orp, oci;
    if (what == AMGDG_A_ROWPTR || what == AMGDG_A_COLIDX) {
        const std::vector<int32_t>& rp = (k == N) ? P.AN_rp : P.lv[k].A_rp;
        const std::vector<int32_t>& ci = (k == N) ? P.AN_ci : P.lv[k].A_ci;
        rows_caller(rp, ci, true, true, orp, oci);
    } else if (k == N) {
        throw Error(AMGDG_EINVAL, "item not defined on the coarsest level");
    } else if (what == AMGDG_T_ROWPTR || what == AMGDG_T_COLIDX) {
        rows_caller(P.lv[k].T_rp, P.lv[k].T_ci, true, false, orp, oci);
    } else if (what == AMGDG_R_ROWPTR || what == AMGDG_R_COLIDX) {
        rows_caller(P.lv[k].R_rp, P.lv[k].R_ci, false, true, orp, oci);
    } else if (what == AMGDG_M_ROWPTR || what == AMGDG_M_COLIDX) {
        symbolic_M(P.lv[k]);
        rows_caller(P.lv[k].M_rp, P.lv[k].M_ci, false, true, orp, oci);
    } else {
        throw Error(AMGDG_EINVAL, "unknown plan item");
    }
    out32 = (what == AMGDG_A_ROWPTR || what == AMGDG_T_ROWPTR || what == AMGDG_R_ROWPTR || what == AMGDG_M_ROWPTR)
                ? orp
                : oci;
}

// ------------------------------------------------------------ allocation-free V-cycle
// The workspace of amgdg_vcycle_static: one array in device memory per GPU,
// part of the library's code object, held until the process ends.  On the
// host its name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is handed to kernels.
constexpr size_t STATIC_WS_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

static std::mutex g_ws_mu;
static unsigned char* g_ws_ptr[64];

static unsigned char* static_workspace() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw Error(AMGDG_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (!g_ws_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(AMGDG_EHIP, "hipGetSymbolAddress returned NULL for the static workspace");
        g_ws_ptr[dev] = static_cast<unsigned char*>(p);
    }
    return g_ws_ptr[dev];
}

// Carves the V-cycle's level vectors (and, for caller-order vectors, the two
// permuted copies of level 0) out of `base`; returns the bytes needed.  With
// base == nullptr only the size is formed.  Level 0: u, w, r, c; levels
// 1..N-1: b, u, w, r, c; level N: b, u (what vcycle_impl reads and writes).
template <typename T>
static int64_t static_layout(const Ctx& C, int m, bool caller_order, unsigned char* base, VBuf<T>* V, T** kr,
                             T** kz) {
    int64_t off = 0;
    auto get = [&](int64_t n) -> T* {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (int64_t(sizeof(T)) * std::max<int64_t>(n, 1) + 255) / 256 * 256;
        return p;
    };
    const int N = C.N;
    for (int k = 0; k <= N; ++k) {
        const int64_t cnt = C.lv[k].n * m;
        VBuf<T> v;
        if (k > 0) v.b = get(cnt);
        v.u = get(cnt);
        if (k < N) {
            v.w = get(cnt);
            v.r = get(cnt);
            v.c = get(cnt);
        }
        if (V) V[k] = v;
    }
    if (caller_order) {
        T* a = get(C.lv[0].n * m);
        T* b = get(C.lv[0].n * m);
        if (kr) *kr = a;
        if (kz) *kz = b;
    }
    return off;
}

constexpr int STATIC_MAX_LEVELS = 64;

template <typename T>
static void vcycle_static_impl(Ctx& C, int m, const T* r, T* z, bool internal, hipStream_t st) {
    if (C.N + 1 > STATIC_MAX_LEVELS) throw Error(AMGDG_EUNSUPPORTED, "more than 64 levels");
    const int64_t need = static_layout<T>(C, m, !internal, nullptr, nullptr, nullptr, nullptr);
    if (need > int64_t(STATIC_WS_BYTES))
        throw Error(AMGDG_EUNSUPPORTED, "this V-cycle needs " + std::to_string(need) + " bytes of workspace; the "
                                            "static workspace holds " + std::to_string(STATIC_WS_BYTES));
    unsigned char* base = static_workspace();
    VBuf<T> V[STATIC_MAX_LEVELS];
    T *kr = nullptr, *kz = nullptr;
    static_layout<T>(C, m, !internal, base, V, &kr, &kz);
    const Level& L = C.lv[0];
    if (internal) {
        vcycle_impl<T>(C, V, r, z, m, st);
    } else {
        HIPCHK((launch_permute<T, T>(r, kr, C.perm_d, L.n_units, L.nb, m, 1, st)));
        vcycle_impl<T>(C, V, kr, kz, m, st);
        HIPCHK((launch_permute<T, T>(kz, z, C.perm_d, L.n_units, L.nb, m, 0, st)));
    }
}

}  // namespace amgdg

// ============================================================ C ABI

using namespace amgdg;

struct amgdg_ctx {
    Ctx c;
};
struct amgdg_plan_s {
    Plan p;
};
struct amgdg_server_s {
    Server s;
};

#define ABI_BEGIN try {
#define ABI_END                                                        \
    }                                                                  \
    catch (const Error& e) {                                           \
        g_last_error = e.what();                                       \
        return e.code;                                                 \
    }                                                                  \
    catch (const std::bad_alloc&) {                                    \
        g_last_error = "host allocation failed";                       \
        return AMGDG_ENOMEM;                                           \
    }                                                                  \
    catch (const std::invalid_argument& e) {                           \
        g_last_error = e.what();                                       \
        return AMGDG_EINVAL;                                           \
    }                                                                  \
    catch (const std::exception& e) {                                  \
        g_last_error = e.what();                                       \
        return AMGDG_EINVAL;                                           \
    }

extern "C" {

void amgdg_default_params(amgdg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_levels = 2;
    p->r = 3;
    p->t_pre = 3;
    p->t_post = 3;
    p->q_power = 3;
    p->relax_max = 100;
    p->omega_fixed = 0.0;
    p->gamma = 0.03;
    p->n_cut = 3.0;
    p->b_update = 0;
    p->mixed = 0;
    p->pow_seed = 3;
    p->b1_seed = 2;
    p->delta = 1e-3;
    p->hstar_smooth = 0;
    p->matfree_levels = 0;
    p->restrict_resid = 1;
}

const char* amgdg_last_error(void) { return g_last_error.c_str(); }

int amgdg_partition_rcb(int64_t n_elem, int32_t dim, const double* centroids, int32_t n_levels, int32_t bisections,
                        int32_t* agg_out, int64_t* leaf_order) {
    ABI_BEGIN
    if (n_levels > 1 && !agg_out) throw Error(AMGDG_EINVAL, "agg_out is NULL");
    rcb_partition(n_elem, dim, centroids, n_levels, bisections, agg_out, leaf_order);
    return AMGDG_OK;
    ABI_END
}

int amgdg_plan_create(amgdg_plan* out, int64_t n_elem, const int32_t* row_ptr, const int32_t* col_idx, int64_t nnzb,
                      int32_t n_levels, const int32_t* agg_of_elem) {
    ABI_BEGIN
    if (!out) throw Error(AMGDG_EINVAL, "out is NULL");
    auto p = std::make_unique<amgdg_plan_s>();
    build_plan(p->p, n_elem, row_ptr, col_idx, nnzb, n_levels, agg_of_elem);
    *out = p.release();
    return AMGDG_OK;
    ABI_END
}

void amgdg_plan_destroy(amgdg_plan p) { delete p; }

int amgdg_plan_size(amgdg_plan p, int32_t k, int32_t what, int64_t* count) {
    ABI_BEGIN
    if (!p || !count) throw Error(AMGDG_EINVAL, "NULL argument");
    std::vector<int32_t> a;
    std::vector<int64_t> b;
    plan_item(p->p, k, what, a, b);
    *count = int64_t(what == AMGDG_PERM ? b.size() : a.size());
    return AMGDG_OK;
    ABI_END
}

int amgdg_plan_export(amgdg_plan p, int32_t k, int32_t what, void* host_buf, int64_t bytes) {
    ABI_BEGIN
    if (!p || !host_buf) throw Error(AMGDG_EINVAL, "NULL argument");
    std::vector<int32_t> a;
    std::vector<int64_t> b;
    plan_item(p->p, k, what, a, b);
    if (what == AMGDG_PERM) copy_out(b, host_buf, bytes);
    else copy_out(a, host_buf, bytes);
    return AMGDG_OK;
    ABI_END
}

int amgdg_setup(amgdg_handle* out, int64_t n_elem, int32_t nb, const int32_t* row_ptr, const int32_t* col_idx,
                const double* vals, int64_t nnzb, const int32_t* adj_ptr, const int32_t* adj_idx,
                const int32_t* agg_of_elem, const amgdg_params* p, const double* B1, void* stream) {
    ABI_BEGIN
    if (!out) throw Error(AMGDG_EINVAL, "out is NULL");
    *out = nullptr;
    if (adj_ptr && adj_idx) {
        for (int64_t e = 0; e < n_elem; ++e) {
            if (adj_ptr[e + 1] < adj_ptr[e]) throw Error(AMGDG_EINVAL, "adjacency pointer not monotone");
            for (int32_t a = adj_ptr[e]; a < adj_ptr[e + 1]; ++a)
                if (adj_idx[a] < 0 || adj_idx[a] >= n_elem || adj_idx[a] == e)
                    throw Error(AMGDG_EINVAL, "adjacency index out of range");
        }
    }
    auto h = std::make_unique<amgdg_ctx>();
    if (p) h->c.prm = *p;
    else amgdg_default_params(&h->c.prm);
    setup_impl(h->c, n_elem, nb, row_ptr, col_idx, vals, nnzb, agg_of_elem, B1, hipStream_t(stream));
    *out = h.release();
    return AMGDG_OK;
    ABI_END
}

int amgdg_destroy(amgdg_handle h) {
    ABI_BEGIN
    if (h) {
        (void)hipDeviceSynchronize();
        delete h;
    }
    return AMGDG_OK;
    ABI_END
}

int amgdg_num_levels(amgdg_handle h) { return h ? h->c.N + 1 : 0; }

int amgdg_level_info_get(amgdg_handle h, int32_t k, amgdg_level_info* out) {
    ABI_BEGIN
    if (!h || !out) throw Error(AMGDG_EINVAL, "NULL argument");
    Ctx& C = h->c;
    if (k < 0 || k > C.N) throw Error(AMGDG_EINVAL, "bad level");
    const Level& L = C.lv[k];
    std::memset(out, 0, sizeof(*out));
    out->n_units = L.n_units;
    out->nb = L.nb;
    out->s = (k < C.N) ? L.s : 0;
    out->n = L.n;
    out->nnzb = L.nnzb;
    out->nnzb_T = (k < C.N) ? L.nT : 0;
    out->n_agg = (k < C.N) ? L.n_agg : 0;
    out->omega = L.omega;
    out->rho = L.rho;
    out->r = (k < C.N) ? L.r : 0;
    for (size_t i = 0; i < L.sweeps.size() && i < 64; ++i) out->sweeps[i] = L.sweeps[i];
    out->n_dofs = L.n_real;
    out->matfree = L.matfree ? 1 : 0;
    int64_t tot = 0;
    for (size_t i = 0; i < C.mem.sizes.size(); ++i) tot += int64_t(C.mem.sizes[i]);
    out->bytes_handle = tot;
    out->bytes_A = L.A.n_vals * 8;
    out->bytes_Dinv = (k < C.N) ? L.n_units * L.nb * L.nb * 8 : 0;
    out->bytes_T = L.T.n_vals * 8;
    out->bytes_R = L.R.n_vals * 8;
    out->nnzb_M = L.has_M ? L.nM : 0;
    out->nnzb_S = (k < C.N) ? L.nnzb_S : 0;
    out->restrict_resid = L.has_M ? 1 : 0;
    out->bytes_M = L.has_M ? L.M.n_vals * 8 : 0;
    return AMGDG_OK;
    ABI_END
}

int amgdg_export_level(amgdg_handle h, int32_t k, int32_t what, void* host_buf, int64_t bytes, void* stream) {
    ABI_BEGIN
    if (!h) throw Error(AMGDG_EINVAL, "NULL handle");
    return export_impl(h->c, k, what, host_buf, bytes, hipStream_t(stream));
    ABI_END
}

int amgdg_solve(amgdg_handle h, int32_t m, const double* b_dev, double* x_dev, int32_t method, int32_t precision,
                double rtol, int32_t max_it, int32_t restart, int32_t flags, amgdg_solve_stats* stats, void* stream) {
    ABI_BEGIN
    if (!h) throw Error(AMGDG_EINVAL, "NULL handle");
    return solve_impl(h->c, m, b_dev, x_dev, method, precision, rtol, max_it, restart, flags, stats,
                      hipStream_t(stream));
    ABI_END
}

int amgdg_vcycle(amgdg_handle h, int32_t m, const void* r_dev, void* z_dev, int32_t precision, int32_t flags,
                 void* stream) {
    ABI_BEGIN
    if (!h || !r_dev || !z_dev) throw Error(AMGDG_EINVAL, "NULL argument");
    Ctx& C = h->c;
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    hipStream_t st = hipStream_t(stream);
    if (precision == AMGDG_MIXED && !C.mixed) throw Error(AMGDG_EINVAL, "mixed precision needs params.mixed = 1");
    Work& W = default_work(C, m, 0, st);
    Level& L = C.lv[0];
    const bool internal = flags & AMGDG_INTERNAL_ORDER;
    const bool graph = graph_for(C, flags, precision == AMGDG_MIXED ? 4 : 8);
    if (precision == AMGDG_FP64) {
        const double* r = static_cast<const double*>(r_dev);
        double* z = static_cast<double*>(z_dev);
        if (internal) {
            vcycle_run<double>(C, W, r, z, m, st, graph);
        } else {
            HIPCHK((launch_permute<double, double>(r, W.kr, C.perm_d, L.n_units, L.nb, m, 1, st)));
            vcycle_run<double>(C, W, W.kr, W.kz, m, st, graph);
            HIPCHK((launch_permute<double, double>(W.kz, z, C.perm_d, L.n_units, L.nb, m, 0, st)));
        }
    } else if (precision == AMGDG_MIXED) {
        const float* r = static_cast<const float*>(r_dev);
        float* z = static_cast<float*>(z_dev);
        if (internal) {
            vcycle_run<float>(C, W, r, z, m, st, graph);
        } else {
            HIPCHK((launch_permute<float, float>(r, W.kr32, C.perm_d, L.n_units, L.nb, m, 1, st)));
            vcycle_run<float>(C, W, W.kr32, W.kz32, m, st, graph);
            HIPCHK((launch_permute<float, float>(W.kz32, z, C.perm_d, L.n_units, L.nb, m, 0, st)));
        }
    } else {
        throw Error(AMGDG_EINVAL, "bad precision");
    }
    return AMGDG_OK;
    ABI_END
}

int amgdg_vcycle_static(amgdg_handle h, int32_t m, const void* r_dev, void* z_dev, int32_t precision, int32_t flags,
                        void* stream) {
    ABI_BEGIN
    if (!h || !r_dev || !z_dev) throw Error(AMGDG_EINVAL, "NULL argument");
    Ctx& C = h->c;
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    if (precision == AMGDG_MIXED && !C.mixed) throw Error(AMGDG_EINVAL, "mixed precision needs params.mixed = 1");
    const bool internal = flags & AMGDG_INTERNAL_ORDER;
    hipStream_t st = hipStream_t(stream);
    if (precision == AMGDG_FP64)
        vcycle_static_impl<double>(C, m, static_cast<const double*>(r_dev), static_cast<double*>(z_dev), internal, st);
    else if (precision == AMGDG_MIXED)
        vcycle_static_impl<float>(C, m, static_cast<const float*>(r_dev), static_cast<float*>(z_dev), internal, st);
    else
        throw Error(AMGDG_EINVAL, "bad precision");
    return AMGDG_OK;
    ABI_END
}

int amgdg_apply(amgdg_handle h, int32_t k, int32_t op, int32_t m, int32_t precision, const void* x, const void* b,
                void* y, int32_t flags, void* stream) {
    ABI_BEGIN
    if (!h || !y) throw Error(AMGDG_EINVAL, "NULL argument");
    if (op == AMGDG_OP_COARSE) {
        return apply_impl<double>(h->c, k, op, m, static_cast<const double*>(x), nullptr, static_cast<double*>(y),
                                  flags, hipStream_t(stream));
    }
    if (precision == AMGDG_FP64)
        return apply_impl<double>(h->c, k, op, m, static_cast<const double*>(x), static_cast<const double*>(b),
                                  static_cast<double*>(y), flags, hipStream_t(stream));
    if (precision == AMGDG_MIXED)
        return apply_impl<float>(h->c, k, op, m, static_cast<const float*>(x), static_cast<const float*>(b),
                                 static_cast<float*>(y), flags, hipStream_t(stream));
    throw Error(AMGDG_EINVAL, "bad precision");
    ABI_END
}

int amgdg_batch_bytes(amgdg_handle h, int32_t width, int32_t restart, int64_t* bytes) {
    ABI_BEGIN
    if (!h || !bytes) throw Error(AMGDG_EINVAL, "NULL argument");
    if (width < 1 || width > 64) throw Error(AMGDG_EUNSUPPORTED, "width must be 1..64");
    if (restart < 0 || restart > 256) throw Error(AMGDG_EUNSUPPORTED, "restart must be 0..256");
    *bytes = work_bytes(h->c, width, restart);
    return AMGDG_OK;
    ABI_END
}

int amgdg_server_create(amgdg_server* out, int32_t width, int64_t hbm_budget_bytes) {
    ABI_BEGIN
    if (!out) throw Error(AMGDG_EINVAL, "out is NULL");
    *out = nullptr;
    if (width < 1 || width > 64) throw Error(AMGDG_EUNSUPPORTED, "width must be 1..64");
    if (hbm_budget_bytes <= 0) throw Error(AMGDG_EINVAL, "budget must be positive");
    auto s = std::make_unique<amgdg_server_s>();
    s->s.width = width;
    s->s.budget = hbm_budget_bytes;
    *out = s.release();
    return AMGDG_OK;
    ABI_END
}

int amgdg_server_submit(amgdg_server s, amgdg_handle h, const double* b_dev, double* x_dev, int32_t method,
                        int32_t precision, double rtol, int32_t max_it, int32_t restart, int32_t flags,
                        int64_t tag) {
    ABI_BEGIN
    if (!s || !h || !b_dev || !x_dev) throw Error(AMGDG_EINVAL, "NULL argument");
    Ctx& C = h->c;
    check_solve_args(C, 1, method, precision);
    if (method == AMGDG_STATIONARY) throw Error(AMGDG_EUNSUPPORTED, "the server runs PCG, FCG and FGMRES");
    if (method == AMGDG_FGMRES && (restart < 1 || restart > 256))
        throw Error(AMGDG_EUNSUPPORTED, "FGMRES: 1 <= restart <= 256");
    if (max_it < 0 || !(rtol >= 0)) throw Error(AMGDG_EINVAL, "bad rtol or max_it");
    if (flags & ~(AMGDG_X0 | AMGDG_INTERNAL_ORDER)) throw Error(AMGDG_EINVAL, "bad flags");
    const int64_t need = Server::batch_bytes(C, method, s->s.width, restart);
    if (need > s->s.budget)
        throw Error(AMGDG_ENOMEM, "a batch on this handle needs " + std::to_string(need) + " bytes, over the budget");
    Request r;
    r.C = &C;
    r.method = method;
    r.precision = precision;
    r.restart = method == AMGDG_FGMRES ? restart : 0;
    r.rq.tag = tag;
    r.rq.b = b_dev;
    r.rq.x = x_dev;
    r.rq.x0 = (flags & AMGDG_X0) ? x_dev : nullptr;
    r.rq.ld = 1;
    r.rq.tol = rtol;
    r.rq.maxit = max_it;
    r.rq.internal = flags & AMGDG_INTERNAL_ORDER;
    r.rq.t_submit = Clock::now();
    s->s.queue.push_back(r);
    return AMGDG_OK;
    ABI_END
}

int amgdg_server_step(amgdg_server s, int32_t wait, int64_t* n_pending) {
    ABI_BEGIN
    if (!s) throw Error(AMGDG_EINVAL, "NULL server");
    s->s.step(wait != 0);
    if (n_pending) *n_pending = s->s.pending();
    return AMGDG_OK;
    ABI_END
}

int amgdg_server_poll(amgdg_server s, int32_t capacity, int64_t* tags, int32_t* status, int32_t* iterations,
                      double* rel_residual, double* latency_s, int32_t* n_done) {
    ABI_BEGIN
    if (!s || !n_done || (capacity > 0 && !tags)) throw Error(AMGDG_EINVAL, "NULL argument");
    std::vector<Outcome>& d = s->s.done;
    const int32_t k = int32_t(std::min<int64_t>(std::max(capacity, 0), int64_t(d.size())));
    for (int32_t i = 0; i < k; ++i) {
        tags[i] = d[i].tag;
        if (status) status[i] = d[i].rc;
        if (iterations) iterations[i] = d[i].its;
        if (rel_residual) rel_residual[i] = d[i].rel;
        if (latency_s) latency_s[i] = d[i].latency;
    }
    d.erase(d.begin(), d.begin() + k);
    *n_done = k;
    return AMGDG_OK;
    ABI_END
}

int amgdg_server_destroy(amgdg_server s) {
    ABI_BEGIN
    delete s;
    return AMGDG_OK;
    ABI_END
}

int amgdg_autotune(amgdg_handle h, int32_t m, int32_t flags, void* stream) {
    ABI_BEGIN
    if (!h) throw Error(AMGDG_EINVAL, "NULL handle");
    if (flags & ~AMGDG_TUNE_LANES) throw Error(AMGDG_EINVAL, "bad flags");
    autotune_impl(h->c, m, (flags & AMGDG_TUNE_LANES) != 0, hipStream_t(stream));
    return AMGDG_OK;
    ABI_END
}

int amgdg_tuning_get(amgdg_handle h, int32_t k, int32_t m, int32_t* out) {
    ABI_BEGIN
    if (!h || !out) throw Error(AMGDG_EINVAL, "NULL argument");
    Ctx& C = h->c;
    if (k < 0 || k >= C.N) throw Error(AMGDG_EINVAL, "bad level (no transfer operators on the coarsest level)");
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    const Level& L = C.lv[k];
    const MatStore* ms[3] = {&L.A, &L.T, &L.R};
    for (int i = 0; i < 3; ++i) {
        const MatStore& M = *ms[i];
        out[i] = M.vec ? M.bd.P : 0;
        out[3 + i] = M.cap64[m];
        out[6 + i] = M.cap32[m];
        out[9 + i] = m / MFMA_COLS <= 4 ? M.mfu64[m / MFMA_COLS] : 0;
        out[12 + i] = m / MFMA_COLS <= 4 ? M.mfu32[m / MFMA_COLS] : 0;
    }
    out[15] = C.lanes_tuned ? 1 : 0;
    return AMGDG_OK;
    ABI_END
}

}  // extern "C"
