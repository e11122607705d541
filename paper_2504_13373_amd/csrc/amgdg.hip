// C-ABI of the amgdg library: setup (Algorithm 5), V-cycle (Algorithm 2) and
// Krylov drivers on one GPU.  Host code orchestrates; every arithmetic step on
// matrices and vectors is a kernel of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <stdexcept>
#include <string>
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
    ~DevMem() { release(); }
    void release() {
        for (void* p : blocks) (void)hipFree(p);
        blocks.clear();
    }
    template <typename T>
    T* alloc(int64_t n) {
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, sizeof(T) * size_t(std::max<int64_t>(n, 1))));
        blocks.push_back(p);
        return static_cast<T*>(p);
    }
    void free(void* p) {
        auto it = std::find(blocks.begin(), blocks.end(), p);
        if (it != blocks.end()) {
            (void)hipFree(p);
            blocks.erase(it);
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
};

// An operator of the hierarchy in the layout its block shape calls for: the
// sliced row-interleaved layout for tall blocks (br > 4), block CSR with a lane
// group per block row for small blocks (coarse levels, restriction).
struct MatStore {
    bool vec = false;
    SellStore s;
    Bcsr<double> bd;
    Bcsr<float> bf;
    int64_t n_vals = 0;
};

template <typename T>
struct VBuf {
    T *b = nullptr, *u = nullptr, *w = nullptr, *r = nullptr;
    T* cur = nullptr;  // buffer holding u_k during a V-cycle
};

struct Level {
    int64_t n_units = 0, n = 0, n_agg = 0, nnzb = 0, nT = 0;
    int nb = 0, s = 0, r = 0;
    double omega = 1.0, rho = std::numeric_limits<double>::quiet_NaN();
    std::vector<int32_t> sweeps;
    double* A_nat = nullptr;
    double* Dinv_nat = nullptr;
    double* Dinv_sell = nullptr;
    float* Dinv_sell32 = nullptr;
    float* Dinv_nat32 = nullptr;
    MatStore A, T, R;
    double *B_in = nullptr, *B_rel = nullptr, *Pu = nullptr, *sv = nullptr, *T_nat = nullptr, *R_nat = nullptr;
    VBuf<double> v64;
    VBuf<float> v32;
};

struct Ctx {
    DevMem mem;
    DevMem ws;  // workspaces, reallocated when m grows
    Plan plan;
    amgdg_params prm{};
    int N = 0;                  // index of the coarsest level
    std::vector<Level> lv;      // N + 1 levels
    int64_t nN = 0;
    double* Ainv = nullptr;
    int64_t* perm_d = nullptr;  // internal unit -> caller element
    std::vector<int32_t> in_rp, in_ci;  // caller's level-0 pattern (for export)
    double* scratch = nullptr;  // reduction partials: DOT_PARTS * 64 + more
    double* scal = nullptr;     // device scalars (256)
    int32_t* flag = nullptr;
    int ws_m = 0;
    bool mixed = false;
    // coarse mixed conversion buffers
    double *cin = nullptr, *cout = nullptr;
    // Krylov workspace
    int kr_m = 0, kr_restart = 0;
    double *kb = nullptr, *kx = nullptr, *kr = nullptr, *kr2 = nullptr, *kz = nullptr, *kp = nullptr, *kq = nullptr,
           *kt = nullptr;
    float *kr32 = nullptr, *kz32 = nullptr;
    double *kgin = nullptr, *kgout = nullptr;  // fixed input/output of the FP64 V-cycle graph
    double *V = nullptr, *Z = nullptr;
    int32_t* active_d = nullptr;
    // fused Krylov steps: partial sums, arrival counter, status record (rr[0..64), flag)
    double* kpart = nullptr;
    unsigned* counter = nullptr;
    double* stat = nullptr;
    double* stat_h = nullptr;  // pinned host mirror of stat
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
    hipEvent_t ev = nullptr;  // status readback of the Krylov loop
    bool use_graph = true;  // per call: off with AMGDG_EAGER
    void drop_graphs() {
        for (auto& e : graphs) {
            (void)hipGraphExecDestroy(e.e);
            (void)hipGraphDestroy(e.g);
        }
        graphs.clear();
    }
    ~Ctx() {
        (void)hipDeviceSynchronize();
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (ev) (void)hipEventDestroy(ev);
        if (stat_h) (void)hipHostFree(stat_h);
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
    d.voff = upload(C.mem, voff, st);
    T* vals = C.mem.alloc<T>(v);
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
    const int G = 64 / br, L = G * br;
    const int64_t ns = (n_brow + G - 1) / G;
    std::vector<int32_t> coff(ns + 1), K(ns), cols, slot_k, slot_g, slot_s;
    std::vector<int64_t> slot_src;
    int32_t c = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int32_t kmax = 0;
        for (int g = 0; g < G; ++g) {
            const int64_t row = s * G + g;
            if (row < n_brow) kmax = std::max(kmax, rp[row + 1] - rp[row]);
        }
        K[s] = kmax;
        coff[s] = c;
        for (int kk = 0; kk < kmax; ++kk)
            for (int g = 0; g < G; ++g) {
                const int64_t row = s * G + g;
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
    d.coff = upload(C.mem, coff, st);
    d.K = upload(C.mem, K, st);
    d.cols = upload(C.mem, cols, st);
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
    sell_values<double>(C, d, ns, K, slot_src, slot_k, slot_g, slot_s, nat_d, st);
    if (f32) sell_values<float>(C, f, ns, K, slot_src, slot_k, slot_g, slot_s, nat_d, st);
    S.d = d;
    S.f = f;
    int64_t nv = 0;
    for (int64_t s = 0; s < ns; ++s) nv += int64_t(K[s]) * bc * L;
    S.n_vals = nv;
}

template <typename T>
static T* sell_dinv(Ctx& C, const Sell<T>& A, const double* dinv_nat, hipStream_t st) {
    const int64_t cnt = int64_t(A.n_slices) * A.brpad * A.L;
    T* out = C.mem.alloc<T>(cnt);
    HIPCHK(hipMemsetAsync(out, 0, sizeof(T) * size_t(std::max<int64_t>(cnt, 1)), st));
    HIPCHK(launch_dinv_to_sell<T>(dinv_nat, A.n_brow, A.br, A.G, A.L, A.brpad, out, st));
    return out;
}

static void build_mat(Ctx& C, MatStore& M, int64_t n_brow, int br, int bc, const std::vector<int32_t>& rp,
                      const std::vector<int32_t>& ci, const double* nat_d, bool f32, hipStream_t st) {
    if (br <= BCSR_MAXBR) {
        M.vec = true;
        const int64_t nnzb = int64_t(ci.size());
        const double avg = n_brow > 0 ? double(nnzb) / double(n_brow) : 1.0;
        int P = 4;
        while (P < avg && P < 64) P *= 2;
        Bcsr<double> d;
        d.n_brow = int32_t(n_brow);
        d.br = br;
        d.bc = bc;
        d.P = P;
        d.rp = upload(C.mem, rp, st);
        d.ci = upload(C.mem, ci, st);
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
            float* fv = C.mem.alloc<float>(M.n_vals);
            HIPCHK(launch_f64_to_f32(nat_d, fv, M.n_vals, st));
            M.bf.vals = fv;
        }
    } else {
        M.vec = false;
        build_sell(C, M.s, n_brow, br, bc, rp, ci, nat_d, f32, st);
        M.n_vals = M.s.n_vals;
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
static void mat_spmv(int mode, const MatStore& M, const T* x, const T* b, T* y, int m, hipStream_t st) {
    if (M.vec) HIPCHK(launch_bspmv<T>(mode, bsel<T>(M), x, b, y, m, st));
    else HIPCHK(launch_spmv<T>(mode, sel<T>(M.s), x, b, y, m, st));
}

template <typename T>
static void mat_sweep(int mode, const Level& L, const T* x, const T* b, T* y, T omega, int m, const int32_t* mask,
                      hipStream_t st) {
    if (L.A.vec) HIPCHK(launch_bsweep<T>(mode, bsel<T>(L.A), dinv_of<T>(L), x, b, y, omega, m, mask, st));
    else HIPCHK(launch_sweep<T>(mode, sel<T>(L.A.s), dinv_of<T>(L), x, b, y, omega, m, mask, st));
}


static double dot1(Ctx& C, const double* a, const double* b, int64_t n, hipStream_t st) {
    HIPCHK(launch_dot<double>(a, b, n, 1, C.scratch, C.scal, st));
    double h = 0;
    HIPCHK(hipMemcpyAsync(&h, C.scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

static std::vector<double> dotm(Ctx& C, const double* a, const double* b, int64_t n, int m, hipStream_t st) {
    HIPCHK(launch_dot<double>(a, b, n, m, C.scratch, C.scal, st));
    std::vector<double> h(m);
    HIPCHK(hipMemcpyAsync(h.data(), C.scal, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

// Algorithm 4 with P(A_k) = D_k: x unit, q times x <- D^{-1} A x / ||.||, returns ||D^{-1} A x||.
static double power_rho(Ctx& C, Level& L, int k, hipStream_t st) {
    DevMem tmp;
    double* x = tmp.alloc<double>(L.n);
    double* y = tmp.alloc<double>(L.n);
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
    return std::sqrt(dot1(C, y, y, L.n, st));
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
    std::vector<double> nx = dotm(C, X, X, L.n, r, st);
    HIPCHK(hipMemcpyAsync(mask, act.data(), sizeof(int32_t) * r, hipMemcpyHostToDevice, st));
    const double thr = 1.0 + C.prm.gamma;
    for (int sweep = 0; sweep < C.prm.relax_max; ++sweep) {
        mat_sweep<double>(RELAX, L, X, nullptr, Y, L.omega, r, mask, st);
        std::vector<double> ny = dotm(C, Y, Y, L.n, r, st);
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
    if (nb < 1 || nb > 16) throw Error(AMGDG_EUNSUPPORTED, "nb must be 1..16");
    if (p.n_levels < 1) throw Error(AMGDG_EINVAL, "n_levels must be >= 1");
    if (p.n_levels > 1 && (p.r < 1 || p.r > 8)) throw Error(AMGDG_EUNSUPPORTED, "r must be 1..8");
    if (p.t_pre < 0 || p.t_post < 0 || p.q_power < 0 || p.relax_max < 1 || !(p.n_cut > 0))
        throw Error(AMGDG_EINVAL, "bad smoothing or coarsening parameters");
    if (p.b_update != 0) throw Error(AMGDG_EUNSUPPORTED, "only B^{k+1} = R B^k is implemented");
    if (!vals) throw Error(AMGDG_EINVAL, "vals is NULL");
    check_finite_host(vals, nnzb * nb * nb, "A");
    try {
        build_plan(C.plan, n_elem, row_ptr, col_idx, nnzb, p.n_levels, agg_of_elem);
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
    C.kpart = C.mem.alloc<double>(2 * 16 * (KRY_BLOCKS + 1) + 64);
    C.counter = C.mem.alloc<unsigned>(1);
    HIPCHK(hipMemsetAsync(C.counter, 0, sizeof(unsigned), st));
    C.stat = C.mem.alloc<double>(65);
    HIPCHK(hipMemsetAsync(C.stat, 0, 65 * sizeof(double), st));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&C.stat_h), 65 * sizeof(double), hipHostMallocDefault));
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
    for (int k = 0; k <= C.N; ++k) {
        Level& L = C.lv[k];
        const bool coarsest = (k == C.N);
        const std::vector<int32_t>& Arp = coarsest ? C.plan.AN_rp : C.plan.lv[k].A_rp;
        const std::vector<int32_t>& Aci = coarsest ? C.plan.AN_ci : C.plan.lv[k].A_ci;
        L.n_units = int64_t(Arp.size()) - 1;
        L.nb = cur_nb;
        L.n = L.n_units * L.nb;
        L.nnzb = int64_t(Aci.size());
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
        // D_k^{-1}
        {
            DevMem tmp;
            int32_t* dpos = upload(tmp, P.A_diag, st);
            L.Dinv_nat = C.mem.alloc<double>(L.n_units * L.nb * L.nb);
            HIPCHK(launch_block_inverse(L.A_nat, dpos, L.n_units, L.nb, L.Dinv_nat, C.flag, st));
            if (read_flag(C, st))
                throw Error(AMGDG_ESINGULAR, "diagonal block singular to working precision on level " + std::to_string(k));
        }
        build_mat(C, L.A, L.n_units, L.nb, L.nb, P.A_rp, P.A_ci, L.A_nat, C.mixed, st);
        if (!L.A.vec) {
            L.Dinv_sell = sell_dinv<double>(C, L.A.s.d, L.Dinv_nat, st);
            if (C.mixed) L.Dinv_sell32 = sell_dinv<float>(C, L.A.s.f, L.Dinv_nat, st);
        } else if (C.mixed) {
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
        // coarse block size (eq:sik, h-step)
        int s = -1;
        for (int64_t J = 0; J < P.n_agg; ++J) {
            const int64_t rows = int64_t(P.first_child[J + 1] - P.first_child[J]) * L.nb;
            const int64_t sj = std::min<int64_t>({(int64_t)std::ceil(double(rows) / p.n_cut), rows, (int64_t)r});
            if (s < 0) s = int(sj);
            else if (s != sj) throw Error(AMGDG_EUNSUPPORTED, "coarse block size differs between aggregates");
        }
        L.s = s;
        // P~ by SVD
        DevMem tmp;
        int32_t* fc = upload(tmp, P.first_child, st);
        L.Pu = C.mem.alloc<double>(L.n * s);
        L.sv = C.mem.alloc<double>(P.n_agg * r);
        HIPCHK(launch_svd(B, r, fc, P.n_agg, L.nb, s, L.Pu, L.sv, C.flag, st));
        {
            const int32_t f = read_flag(C, st);
            if (f & 2) throw Error(AMGDG_EUNSUPPORTED, "aggregate with more than 128 rows");
            if (f & 4) throw Error(AMGDG_ESINGULAR, "candidate block of an aggregate is rank deficient");
        }
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
    }
    HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------ workspaces

static void ensure_ws(Ctx& C, int m, hipStream_t st) {
    if (m <= C.ws_m) return;
    HIPCHK(hipStreamSynchronize(st));
    C.drop_graphs();
    C.ws.release();
    for (int k = 0; k <= C.N; ++k) {
        Level& L = C.lv[k];
        const int64_t cnt = L.n * m;
        L.v64.b = C.ws.alloc<double>(cnt);
        L.v64.u = C.ws.alloc<double>(cnt);
        L.v64.w = C.ws.alloc<double>(cnt);
        L.v64.r = C.ws.alloc<double>(cnt);
        if (C.mixed) {
            L.v32.b = C.ws.alloc<float>(cnt);
            L.v32.u = C.ws.alloc<float>(cnt);
            L.v32.w = C.ws.alloc<float>(cnt);
            L.v32.r = C.ws.alloc<float>(cnt);
        }
    }
    C.cin = C.ws.alloc<double>(C.nN * m);
    C.cout = C.ws.alloc<double>(C.nN * m);
    C.ws_m = m;
    C.kr_m = 0;  // Krylov buffers lived in ws
    C.kr_restart = 0;
}

// ------------------------------------------------------------ V-cycle

template <typename T>
static VBuf<T>& vbuf(Level& L);
template <>
VBuf<double>& vbuf<double>(Level& L) { return L.v64; }
template <>
VBuf<float>& vbuf<float>(Level& L) { return L.v32; }


template <typename T>
static void coarse_solve(Ctx& C, const T* b, T* u, int m, hipStream_t st);
template <>
void coarse_solve<double>(Ctx& C, const double* b, double* u, int m, hipStream_t st) {
    HIPCHK(launch_gemv(C.Ainv, b, u, C.nN, m, st));
}
template <>
void coarse_solve<float>(Ctx& C, const float* b, float* u, int m, hipStream_t st) {
    HIPCHK((launch_convert<float, double>(b, C.cin, C.nN * m, st)));
    HIPCHK(launch_gemv(C.Ainv, C.cin, C.cout, C.nN, m, st));
    HIPCHK((launch_convert<double, float>(C.cout, u, C.nN * m, st)));
}

// z0 = V(b0), internal order, m columns (Algorithm 2, one pass from u = 0).
template <typename T>
static void vcycle_impl(Ctx& C, const T* b0, T* z0, int m, hipStream_t st) {
    const int N = C.N;
    const int tpre = C.prm.t_pre, tpost = C.prm.t_post;
    if (N == 0) {
        coarse_solve<T>(C, b0, z0, m, st);
        return;
    }
    for (int k = 0; k < N; ++k) {
        Level& L = C.lv[k];
        VBuf<T>& V = vbuf<T>(L);
        const T* bk = (k == 0) ? b0 : V.b;
        T* cur = V.u;
        T* oth = V.w;
        const T om = T(L.omega);
        if (tpre == 0) {
            HIPCHK(hipMemsetAsync(cur, 0, sizeof(T) * L.n * m, st));
        } else {
            mat_sweep<T>(SWEEP0, L, nullptr, bk, cur, om, m, nullptr, st);
            for (int t = 1; t < tpre; ++t) {
                mat_sweep<T>(SWEEP, L, cur, bk, oth, om, m, nullptr, st);
                std::swap(cur, oth);
            }
        }
        V.cur = cur;
        mat_spmv<T>(B_MINUS, L.A, cur, bk, V.r, m, st);
        Level& Ln = C.lv[k + 1];
        mat_spmv<T>(AX, L.R, V.r, nullptr, vbuf<T>(Ln).b, m, st);
    }
    {
        VBuf<T>& V = vbuf<T>(C.lv[N]);
        coarse_solve<T>(C, V.b, V.u, m, st);
        V.cur = V.u;
    }
    for (int k = N - 1; k >= 0; --k) {
        Level& L = C.lv[k];
        VBuf<T>& V = vbuf<T>(L);
        const T* bk = (k == 0) ? b0 : V.b;
        const T om = T(L.omega);
        T* cur = V.cur;
        auto other = [&](T* c) { return c == V.u ? V.w : V.u; };
        T* dst = (k == 0 && tpost == 0) ? z0 : other(cur);
        mat_spmv<T>(B_PLUS, L.T, vbuf<T>(C.lv[k + 1]).cur, cur, dst, m, st);
        cur = dst;
        for (int t = 0; t < tpost; ++t) {
            dst = (k == 0 && t == tpost - 1) ? z0 : other(cur);
            mat_sweep<T>(SWEEP, L, cur, bk, dst, om, m, nullptr, st);
            cur = dst;
        }
        V.cur = cur;
    }
}

// The V-cycle as a captured HIP graph: its ~40 launches (most of them small
// coarse-level kernels) are submitted as one graph launch, so the host no
// longer paces the coarse levels.  The graph is captured on a private stream
// the first time a (precision, m, input, output) combination is seen and
// replayed on the caller's stream; workspace reallocation drops the cache.  It
// holds only kernel nodes (no memset or copy nodes).
template <typename T>
static void vcycle_run(Ctx& C, const T* b0, T* z0, int m, hipStream_t st, bool allow_graph) {
    if (!allow_graph || C.prm.t_pre == 0 || C.N == 0) {
        vcycle_impl<T>(C, b0, z0, m, st);
        return;
    }
    const int prec = int(sizeof(T));
    for (auto& e : C.graphs)
        if (e.prec == prec && e.m == m && e.in == b0 && e.out == z0) {
            HIPCHK(hipGraphLaunch(e.e, st));
            return;
        }
    if (C.graphs.size() >= 8) {
        HIPCHK(hipStreamSynchronize(st));
        C.drop_graphs();
    }
    if (!C.cap) HIPCHK(hipStreamCreateWithFlags(&C.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(C.cap, hipStreamCaptureModeThreadLocal));
    try {
        vcycle_impl<T>(C, b0, z0, m, C.cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(C.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(C.cap, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        HIPCHK(err);
    }
    C.graphs.push_back({prec, m, b0, z0, g, ex});
    HIPCHK(hipGraphLaunch(ex, st));
}

// ------------------------------------------------------------ Krylov drivers

struct KrylovState {
    std::vector<int32_t> its;
    std::vector<double> rel;
    std::vector<double> bnorm;
};

static void ensure_krylov(Ctx& C, int m, int restart, int method, hipStream_t st) {
    const int64_t n = C.lv[0].n;
    if (C.kr_m >= m && (method != AMGDG_FGMRES || C.kr_restart >= restart) && C.kb) return;
    HIPCHK(hipStreamSynchronize(st));
    C.drop_graphs();
    for (void* p : {(void*)C.kb, (void*)C.kx, (void*)C.kr, (void*)C.kr2, (void*)C.kz, (void*)C.kp, (void*)C.kq,
                    (void*)C.kt, (void*)C.kr32, (void*)C.kz32, (void*)C.V, (void*)C.Z, (void*)C.active_d,
                    (void*)C.kgin, (void*)C.kgout})
        if (p) C.ws.free(p);
    C.kb = C.ws.alloc<double>(n * m);
    C.kx = C.ws.alloc<double>(n * m);
    C.kr = C.ws.alloc<double>(n * m);
    C.kr2 = C.ws.alloc<double>(n * m);
    C.kz = C.ws.alloc<double>(n * m);
    C.kp = C.ws.alloc<double>(n * m);
    C.kq = C.ws.alloc<double>(n * m);
    C.kt = C.ws.alloc<double>(n * m);
    C.kr32 = C.mixed ? C.ws.alloc<float>(n * m) : nullptr;
    C.kz32 = C.mixed ? C.ws.alloc<float>(n * m) : nullptr;
    C.kgin = C.ws.alloc<double>(n * m);
    C.kgout = C.ws.alloc<double>(n * m);
    C.active_d = C.ws.alloc<int32_t>(128);
    if (method == AMGDG_FGMRES) {
        C.V = C.ws.alloc<double>(n * (restart + 1));
        C.Z = C.ws.alloc<double>(n * restart);
        C.kr_restart = restart;
    } else {
        C.V = C.Z = nullptr;
        C.kr_restart = 0;
    }
    C.kr_m = m;
}

// z = V(r) in FP64 for arbitrary r, z: through the graph's fixed buffers.
static void precond_fp64(Ctx& C, const double* r, double* z, int m, hipStream_t st) {
    if (!C.use_graph) {
        vcycle_impl<double>(C, r, z, m, st);
        return;
    }
    const size_t bytes = sizeof(double) * size_t(C.lv[0].n) * m;
    if (r != C.kgin) HIPCHK(hipMemcpyAsync(C.kgin, r, bytes, hipMemcpyDeviceToDevice, st));
    vcycle_run<double>(C, C.kgin, C.kgout, m, st, true);
    if (z != C.kgout) HIPCHK(hipMemcpyAsync(z, C.kgout, bytes, hipMemcpyDeviceToDevice, st));
}

static void precond(Ctx& C, const double* r, double* z, int m, int precision, hipStream_t st) {
    const int64_t n = C.lv[0].n;
    if (precision == AMGDG_MIXED) {
        HIPCHK((launch_convert<double, float>(r, C.kr32, n * m, st)));
        vcycle_run<float>(C, C.kr32, C.kz32, m, st, C.use_graph);
        HIPCHK((launch_convert<float, double>(C.kz32, z, n * m, st)));
    } else {
        precond_fp64(C, r, z, m, st);
    }
}

// true residual t = b - A x and its per-column norms
static std::vector<double> true_res(Ctx& C, const double* b, const double* x, int m, hipStream_t st) {
    Level& L = C.lv[0];
    if (C.N == 0) {
        // level 0 is the coarsest level: it has no sliced copy; use the dense inverse path's operator
        throw Error(AMGDG_EUNSUPPORTED, "Krylov solve needs at least two levels");
    }
    mat_spmv<double>(B_MINUS, L.A, x, b, C.kt, m, st);
    return dotm(C, C.kt, C.kt, L.n, m, st);
}

static void check_nan(const std::vector<double>& v, const char* what) {
    for (double d : v)
        if (!std::isfinite(d)) throw Error(AMGDG_ENAN, std::string("NaN or Inf in ") + what);
}

// Preconditioned CG (flexible = false) or flexible CG with residual replacement
// (flexible = true): in the flexible variant, when the recursive residual of a
// column claims convergence or has dropped by kReplaceDrop since its last
// replacement and the true FP64 residual does not meet the tolerance, the true
// residual replaces the recursive one.  Per iteration: q = A p, p.q, the fused
// update of x and r (with ||r||^2 and, for the mixed V-cycle, the FP32 copy of
// r), the preconditioner, the fused r.z (and z.r_old), the new direction, and
// one readback of the status record (||r||^2 per column and the error flag).
static constexpr double kReplaceDrop = 1e-6;

static int solve_cg(Ctx& C, int m, int precision, double tol, int maxit, bool flexible, KrylovState& S,
                    hipStream_t st) {
    Level& L = C.lv[0];
    const int64_t n = L.n;
    const bool mixed = precision == AMGDG_MIXED;
    double *b = C.kb, *x = C.kx, *r = C.kr, *rn = C.kr2, *z = C.kz, *p = C.kp, *q = C.kq;
    double* sc = C.scal;
    double *d_pq = sc, *d_rz = sc + 64, *d_rz2 = sc + 128, *d_zro = sc + 192;
    int32_t* flag = reinterpret_cast<int32_t*>(C.stat + 64);
    float* r32 = mixed ? C.kr32 : nullptr;
    std::vector<int32_t> act(m, 1);
    std::vector<double> anchor(m, 1.0);
    std::vector<double> rr0 = true_res(C, b, x, m, st);
    HIPCHK(hipMemcpyAsync(r, C.kt, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
    S.its.assign(m, 0);
    S.rel.assign(m, 0.0);
    bool any = false;
    for (int c = 0; c < m; ++c) {
        S.rel[c] = std::sqrt(rr0[c]) / S.bnorm[c];
        anchor[c] = S.rel[c];
        if (S.rel[c] <= tol) act[c] = 0;
        any = any || act[c];
    }
    if (!any) return AMGDG_OK;
    auto upload_act = [&]() {
        HIPCHK(hipMemcpyAsync(C.active_d, act.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    };
    upload_act();
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
    auto apply_M = [&](double* rz_out, const double* r_old, double* zro) {
        if (mixed) vcycle_run<float>(C, C.kr32, C.kz32, m, st, C.use_graph);
        else if (!flexible) vcycle_run<double>(C, r, z, m, st, C.use_graph);  // r, z are fixed buffers here
        else precond_fp64(C, r, z, m, st);
        HIPCHK(launch_zdots(mixed ? C.kz32 : nullptr, z, r, r_old, n, m, C.kpart, C.counter, rz_out, zro, st));
    };
    if (mixed) HIPCHK((launch_convert<double, float>(r, r32, n * m, st)));
    apply_M(d_rz, nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(p, z, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
    mat_spmv<double>(AX, L.A, p, nullptr, q, m, st);
    HIPCHK(launch_dot_tail(p, q, n, m, C.kpart, C.counter, d_pq, st));
    if (!C.ev) HIPCHK(hipEventCreateWithFlags(&C.ev, hipEventDisableTiming));
    for (int it = 1; it <= maxit; ++it) {
        HIPCHK(launch_cg_update(x, r, flexible ? rn : r, p, q, r32, n, m, d_rz, d_pq, C.active_d, C.kpart, C.counter,
                                C.stat, flag, st));
        if (flexible) std::swap(r, rn);  // r: new residual, rn: previous
        HIPCHK(hipMemcpyAsync(C.stat_h, C.stat, sizeof(double) * 65, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(C.ev, st));
        // run ahead: the preconditioner of the new residual is queued before the
        // host looks at the status, so the GPU does not wait for the host; it
        // writes only z and the new dot products, so it is simply redone if the
        // residual gets replaced below
        apply_M(d_rz2, flexible ? rn : nullptr, flexible ? d_zro : nullptr);
        HIPCHK(hipEventSynchronize(C.ev));
        const int32_t f = *reinterpret_cast<const int32_t*>(C.stat_h + 64);
        if (f) {
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
            throw Error(f & 1 ? AMGDG_EBREAKDOWN : AMGDG_ENAN,
                        f & 1 ? "CG breakdown: p^T A p <= 0 (matrix or preconditioner not SPD)" : "NaN in CG");
        }
        bool need_true = false, changed = false;
        std::vector<int32_t> check(m, 0), repl(m, 0);
        for (int c = 0; c < m; ++c)
            if (act[c]) {
                S.its[c] = it;
                S.rel[c] = std::sqrt(C.stat_h[c]) / S.bnorm[c];
                if (S.rel[c] <= tol || (flexible && S.rel[c] <= anchor[c] * kReplaceDrop)) check[c] = 1;
                need_true = need_true || check[c];
            }
        if (need_true) {
            std::vector<double> tr = true_res(C, b, x, m, st);  // leaves b - A x in C.kt
            bool any_repl = false;
            for (int c = 0; c < m; ++c)
                if (check[c]) {
                    const double t = std::sqrt(tr[c]) / S.bnorm[c];
                    if (t <= tol) {
                        act[c] = 0;
                        S.rel[c] = t;
                        changed = true;
                    } else if (flexible) {
                        // residual replacement: the true residual takes the place of the recursive one
                        repl[c] = 1;
                        anchor[c] = t;
                        any_repl = true;
                    }
                }
            if (any_repl) {
                HIPCHK(hipMemcpyAsync(C.active_d + 64, repl.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
                HIPCHK(launch_copy_cols(C.kt, r, n, m, C.active_d + 64, st));
                if (mixed) HIPCHK((launch_convert<double, float>(r, r32, n * m, st)));
                apply_M(d_rz2, flexible ? rn : nullptr, flexible ? d_zro : nullptr);
                HIPCHK(hipStreamSynchronize(st));
            }
        }
        any = false;
        for (int c = 0; c < m; ++c) any = any || act[c];
        if (!any) {
            HIPCHK(hipStreamSynchronize(st));
            return AMGDG_OK;
        }
        if (changed) upload_act();
        HIPCHK(launch_cg_dir(p, z, n, m, d_rz2, flexible ? d_zro : nullptr, d_rz, C.active_d, st));
        std::swap(d_rz, d_rz2);
        mat_spmv<double>(AX, L.A, p, nullptr, q, m, st);
        HIPCHK(launch_dot_tail(p, q, n, m, C.kpart, C.counter, d_pq, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return AMGDG_ENOCONV;
}

static int solve_stationary(Ctx& C, int m, int precision, double tol, int maxit, KrylovState& S, hipStream_t st) {
    Level& L = C.lv[0];
    const int64_t n = L.n;
    std::vector<int32_t> act(m, 1);
    S.its.assign(m, 0);
    S.rel.assign(m, 0.0);
    std::vector<double> rr = true_res(C, C.kb, C.kx, m, st);
    for (int it = 1; it <= maxit; ++it) {
        HIPCHK(hipMemcpyAsync(C.kr, C.kt, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
        precond(C, C.kr, C.kz, m, precision, st);
        // x += z for active columns: alpha = active
        std::vector<double> a(m);
        for (int c = 0; c < m; ++c) a[c] = act[c] ? 1.0 : 0.0;
        HIPCHK(hipMemcpyAsync(C.scal + 1024, a.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        HIPCHK(launch_axpby_dev(C.kz, C.kx, n, m, C.scal + 1024, 1.0, 1.0, st));
        HIPCHK(hipStreamSynchronize(st));
        rr = true_res(C, C.kb, C.kx, m, st);
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

static int solve_fgmres(Ctx& C, int precision, double tol, int restart, int maxit, KrylovState& S,
                        hipStream_t st) {
    Level& L = C.lv[0];
    const int64_t n = L.n;
    double* x = C.kx;
    double* b = C.kb;
    S.its.assign(1, 0);
    S.rel.assign(1, 0.0);
    int total = 0;
    std::vector<double> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), y(restart);
    auto Hat = [&](int i, int j) -> double& { return H[size_t(i) * restart + j]; };
    while (true) {
        std::vector<double> rr = true_res(C, b, x, 1, st);
        const double beta = std::sqrt(rr[0]);
        check_nan(rr, "residual");
        S.rel[0] = beta / S.bnorm[0];
        S.its[0] = total;
        if (S.rel[0] <= tol) return AMGDG_OK;
        if (total >= maxit) return AMGDG_ENOCONV;
        // V_0 = r / beta
        HIPCHK(launch_axpby_dev(C.kt, C.V, n, 1, nullptr, 1.0 / beta, 0.0, st));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < restart; ++j) {
            double* vj = C.V + int64_t(j) * n;
            double* zj = C.Z + int64_t(j) * n;
            double* w = C.V + int64_t(j + 1) * n;
            precond(C, vj, zj, 1, precision, st);
            mat_spmv<double>(AX, L.A, zj, nullptr, w, 1, st);
            // CGS2
            std::vector<double> h(j + 2, 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                HIPCHK(launch_multidot(C.V, n, j + 1, w, n, C.scratch, C.scal, st));
                std::vector<double> hp(j + 1);
                HIPCHK(hipMemcpyAsync(hp.data(), C.scal, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                HIPCHK(hipMemcpyAsync(C.scal + 1024, hp.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
                HIPCHK(launch_multi_axpy(C.V, n, j + 1, C.scal + 1024, w, n, -1.0, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i <= j; ++i) h[i] += hp[i];
            }
            const double hn = std::sqrt(dot1(C, w, w, n, st));
            check_nan({hn}, "Arnoldi");
            if (hn > 0) HIPCHK(launch_axpby_dev(w, w, n, 1, nullptr, 1.0 / hn, 0.0, st));
            for (int i = 0; i <= j; ++i) Hat(i, j) = h[i];
            Hat(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
                Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
                Hat(i, j) = t;
            }
            const double den = std::hypot(Hat(j, j), Hat(j + 1, j));
            if (!(den > 0)) throw Error(AMGDG_EBREAKDOWN, "GMRES breakdown");
            cs[j] = Hat(j, j) / den;
            sn[j] = Hat(j + 1, j) / den;
            Hat(j, j) = den;
            Hat(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            jend = j + 1;
            if (std::fabs(g[j + 1]) <= tol * S.bnorm[0] || total >= maxit) break;
        }
        for (int i = jend - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < jend; ++l) s -= Hat(i, l) * y[l];
            y[i] = s / Hat(i, i);
        }
        HIPCHK(hipMemcpyAsync(C.scal + 1024, y.data(), sizeof(double) * jend, hipMemcpyHostToDevice, st));
        HIPCHK(launch_multi_axpy(C.Z, n, jend, C.scal + 1024, x, n, 1.0, st));
        HIPCHK(hipStreamSynchronize(st));
    }
}

static int solve_impl(Ctx& C, int m, const double* b_dev, double* x_dev, int method, int precision, double rtol,
                      int max_it, int restart, int flags, amgdg_solve_stats* stats, hipStream_t st) {
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    if (!b_dev || !x_dev) throw Error(AMGDG_EINVAL, "b or x is NULL");
    if (precision == AMGDG_MIXED && !C.mixed) throw Error(AMGDG_EINVAL, "mixed precision needs params.mixed = 1");
    if (precision != AMGDG_FP64 && precision != AMGDG_MIXED) throw Error(AMGDG_EINVAL, "bad precision");
    if (method == AMGDG_FGMRES && (m != 1 || restart < 1 || restart > 256))
        throw Error(AMGDG_EUNSUPPORTED, "FGMRES: m = 1 and 1 <= restart <= 256");
    if (method < AMGDG_STATIONARY || method > AMGDG_FGMRES) throw Error(AMGDG_EINVAL, "bad method");
    const auto t0 = std::chrono::steady_clock::now();
    C.use_graph = !(flags & AMGDG_EAGER);
    ensure_ws(C, m, st);
    ensure_krylov(C, m, restart, method, st);
    Level& L = C.lv[0];
    const int64_t n = L.n;
    const bool internal = flags & AMGDG_INTERNAL_ORDER;
    if (internal) HIPCHK(hipMemcpyAsync(C.kb, b_dev, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
    else HIPCHK((launch_permute<double, double>(b_dev, C.kb, C.perm_d, L.n_units, L.nb, m, 1, st)));
    if (flags & AMGDG_X0) {
        if (internal) HIPCHK(hipMemcpyAsync(C.kx, x_dev, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
        else HIPCHK((launch_permute<double, double>(x_dev, C.kx, C.perm_d, L.n_units, L.nb, m, 1, st)));
    } else {
        HIPCHK(hipMemsetAsync(C.kx, 0, sizeof(double) * n * m, st));
    }
    KrylovState S;
    S.bnorm = dotm(C, C.kb, C.kb, n, m, st);
    check_nan(S.bnorm, "b");
    for (double& v : S.bnorm) v = std::sqrt(v) > 0 ? std::sqrt(v) : 1.0;
    int rc;
    switch (method) {
        case AMGDG_STATIONARY: rc = solve_stationary(C, m, precision, rtol, max_it, S, st); break;
        case AMGDG_PCG: rc = solve_cg(C, m, precision, rtol, max_it, false, S, st); break;
        case AMGDG_FCG: rc = solve_cg(C, m, precision, rtol, max_it, true, S, st); break;
        default: rc = solve_fgmres(C, precision, rtol, restart, max_it, S, st); break;
    }
    // final true residuals
    std::vector<double> tr = true_res(C, C.kb, C.kx, m, st);
    if (internal) HIPCHK(hipMemcpyAsync(x_dev, C.kx, sizeof(double) * n * m, hipMemcpyDeviceToDevice, st));
    else HIPCHK((launch_permute<double, double>(C.kx, x_dev, C.perm_d, L.n_units, L.nb, m, 0, st)));
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        int all = 1, mx = 0;
        for (int c = 0; c < m; ++c) {
            const double rel = std::sqrt(tr[c]) / S.bnorm[c];
            if (c < 64) {
                stats->iterations[c] = S.its[c];
                stats->rel_residual[c] = rel;
            }
            mx = std::max(mx, S.its[c]);
            if (!(rel <= rtol)) all = 0;
        }
        stats->max_iterations = mx;
        stats->all_converged = all;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

// ------------------------------------------------------------ single steps

template <typename T>
static int apply_impl(Ctx& C, int k, int op, int m, const T* x, const T* b, T* y, int flags, hipStream_t st) {
    if (k < 0 || k > C.N) throw Error(AMGDG_EINVAL, "bad level");
    if (op != AMGDG_OP_COARSE && k == C.N) throw Error(AMGDG_EINVAL, "operation needs a non-coarsest level");
    if (op == AMGDG_OP_COARSE && k != C.N) throw Error(AMGDG_EINVAL, "AMGDG_OP_COARSE works on the coarsest level");
    if (m < 1 || m > 64) throw Error(AMGDG_EUNSUPPORTED, "m must be 1..64");
    ensure_ws(C, m, st);
    Level& L = C.lv[k];
    const bool perm = (k == 0) && !(flags & AMGDG_INTERNAL_ORDER);
    VBuf<T>& V = vbuf<T>(L);
    if (!V.b) throw Error(AMGDG_EINVAL, "FP32 operators not built (params.mixed = 0)");
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
                         op == AMGDG_OP_PROLONG);
    const bool uses_x = (op != AMGDG_OP_SWEEP0);
    if ((uses_b && !b) || (uses_x && !x)) throw Error(AMGDG_EINVAL, "missing input array");
    const bool fine_out = (op != AMGDG_OP_RESTRICT);
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
    if (what == AMGDG_A_ROWPTR || what == AMGDG_A_COLIDX || what == AMGDG_A_VALS) {
        const std::vector<int32_t>& rp = coarsest ? C.plan.AN_rp : C.plan.lv[k].A_rp;
        const std::vector<int32_t>& ci = coarsest ? C.plan.AN_ci : C.plan.lv[k].A_ci;
        const int64_t per = int64_t(L.nb) * L.nb;
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
        default: throw Error(AMGDG_EINVAL, "unknown export item");
    }
}

// ------------------------------------------------------------ plan queries

static void plan_item(const Plan& P, int k, int what, std::vector<int32_t>& out32, std::vector<int64_t>& out64) {
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
    } else {
        throw Error(AMGDG_EINVAL, "unknown plan item");
    }
    out32 = (what == AMGDG_A_ROWPTR || what == AMGDG_T_ROWPTR || what == AMGDG_R_ROWPTR) ? orp : oci;
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
    for (size_t i = 0; i < L.sweeps.size() && i < 16; ++i) out->sweeps[i] = L.sweeps[i];
    out->bytes_A = L.A.n_vals * 8;
    out->bytes_Dinv = (k < C.N) ? L.n_units * L.nb * L.nb * 8 : 0;
    out->bytes_T = L.T.n_vals * 8;
    out->bytes_R = L.R.n_vals * 8;
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
    ensure_ws(C, m, st);
    ensure_krylov(C, m, 0, AMGDG_PCG, st);
    Level& L = C.lv[0];
    const bool internal = flags & AMGDG_INTERNAL_ORDER;
    const bool graph = !(flags & AMGDG_EAGER);
    if (precision == AMGDG_FP64) {
        const double* r = static_cast<const double*>(r_dev);
        double* z = static_cast<double*>(z_dev);
        if (internal) {
            vcycle_run<double>(C, r, z, m, st, graph);
        } else {
            HIPCHK((launch_permute<double, double>(r, C.kr, C.perm_d, L.n_units, L.nb, m, 1, st)));
            vcycle_run<double>(C, C.kr, C.kz, m, st, graph);
            HIPCHK((launch_permute<double, double>(C.kz, z, C.perm_d, L.n_units, L.nb, m, 0, st)));
        }
    } else if (precision == AMGDG_MIXED) {
        if (!C.mixed) throw Error(AMGDG_EINVAL, "mixed precision needs params.mixed = 1");
        const float* r = static_cast<const float*>(r_dev);
        float* z = static_cast<float*>(z_dev);
        if (internal) {
            vcycle_run<float>(C, r, z, m, st, graph);
        } else {
            HIPCHK((launch_permute<float, float>(r, C.kr32, C.perm_d, L.n_units, L.nb, m, 1, st)));
            vcycle_run<float>(C, C.kr32, C.kz32, m, st, graph);
            HIPCHK((launch_permute<float, float>(C.kz32, z, C.perm_d, L.n_units, L.nb, m, 0, st)));
        }
    } else {
        throw Error(AMGDG_EINVAL, "bad precision");
    }
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

}  // extern "C"
