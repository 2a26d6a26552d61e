// Host side of the NLINV library: plans and workspace, the operator
// sequences of F, DF, DF^H and the normal operator (Eqs. 2-3 of Schaetz &
// Uecker), the IRGNM / CG driver with every scalar on the device, hipGraph
// capture of the Newton loop, the pass autotuner, kernel timing, and the
// C ABI declared in include/nlinv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "nlinv.h"
#include "aux_kernels.hpp"
#include "coil_pca.hpp"
#include "gn_vjp.hpp"
#include "gridding.hpp"
#include "launch.hpp"

using namespace nlinv;

namespace {

thread_local int g_last_hip = 0;

#define HIPCHK(expr)                                             \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) {                                  \
            g_last_hip = (int)e_;                                \
            return NLINV_EHIP;                                   \
        }                                                        \
    } while (0)

#define CHK(expr)                                                \
    do {                                                         \
        int st_ = (expr);                                        \
        if (st_ != NLINV_OK) return st_;                         \
    } while (0)

constexpr int kMaxNewton = 32;
constexpr int kMaxCG = 256;
constexpr int kStatsCap = 2 + kMaxNewton + kMaxNewton * kMaxCG;
constexpr int kSegLen = 4096;        // complex elements per reduction segment
constexpr int kCoilSeg = kThreads;   // Omega pixels per coil-sum workgroup (one per thread)
constexpr int kColModes = 9;         // ColMode values
constexpr int kRowModes = 4;         // RowMode values
constexpr int kTimingSlots = 8192;   // event pairs for kernel timing
constexpr int kMaxLanes = 8;          // streams for concurrent shape classes
constexpr int kMaxGraphs = 4;         // captured Newton loops kept per plan (by key)

bool size_supported(int n) {
    switch (n) {
#define X(N) case N:
        NLINV_FOR_EACH_SIZE(X)
#undef X
        return true;
        default: return false;
    }
}

hipError_t col_dispatch(int n, int mode, int variant, const ColArgs& a, int nplanes, hipStream_t s) {
    switch (n) {
#define X(N) case N: return launch_col<N>(mode, variant, a, nplanes, s);
        NLINV_FOR_EACH_SIZE(X)
#undef X
    }
    return hipErrorInvalidValue;
}

hipError_t row_dispatch(int n, int mode, int variant, const RowArgs& a, hipStream_t s) {
    switch (n) {
#define X(N) case N: return launch_row<N>(mode, variant, a, s);
        NLINV_FOR_EACH_SIZE(X)
#undef X
    }
    return hipErrorInvalidValue;
}

hipError_t plane_dispatch(int n, const PlaneArgs& a, hipStream_t s) {
    switch (n) {
#define X(N) case N: return launch_plane_normal<N>(a, s);
        NLINV_FOR_EACH_SIZE(X)
#undef X
    }
    return hipErrorInvalidValue;
}

hipError_t plane_cg_dispatch(int n, const PlaneCgArgs& a, hipStream_t s) {
    switch (n) {
#define X(N) case N: return launch_plane_cg<N>(a, s);
        NLINV_FOR_EACH_SIZE(X)
#undef X
    }
    return hipErrorInvalidValue;
}

bool col_ok(int n, int v) { return col_variant_ok(n, v); }
bool row_ok(int n, int v) { return row_variant_ok(n, v); }

// kernel classes for timing
enum KClass : int {
    KC_COL_WINV_IFFT = 0, KC_COL_P_IFFT, KC_COL_FFT_P, KC_COL_RESID_P_IFFT, KC_COL_PSF,
    KC_COL_FFT_WINV_ADD, KC_COL_FFT_GPROD, KC_COL_PUPD_WINV_IFFT, KC_COL_FFT_WINV_CG_UPD,
    KC_ROW_CACHE, KC_ROW_FWD, KC_ROW_DERIV, KC_ROW_ADJ,
    KC_COIL_SUM, KC_VEC_DOT, KC_VEC_OTHER, KC_SCALAR, KC_IMAGE,
    KC_CG_ITER,   // one whole CG iteration (its five launches), bracketed as one
    KC_PLANE_NORMAL, KC_PLANE_CG, KC_PLANE_CG_UPDATE,
    KC_NUM
};
const char* kKClassNames[KC_NUM] = {
    "col_winv_ifft", "col_p_ifft", "col_fft_p", "col_resid_p_ifft", "col_psf",
    "col_fft_winv_add", "col_fft_gprod", "col_pupd_winv_ifft", "col_fft_winv_cg_update",
    "row_cache", "row_fwd", "row_deriv", "row_adj",
    "coil_sum", "vec_dot", "vec_other", "scalar", "image", "cg_iteration", "plane_normal", "plane_cg",
    "plane_cg_update"};

int col_kclass(int mode) {
    switch (mode) {
        case COL_WINV_IFFT_CROP: return KC_COL_WINV_IFFT;
        case COL_P_IFFT_CROP: return KC_COL_P_IFFT;
        case COL_PAD_FFT_P: return KC_COL_FFT_P;
        case COL_RESID_P_IFFT: return KC_COL_RESID_P_IFFT;
        case COL_PAD_FFT_P2_IFFT: return KC_COL_PSF;
        case COL_PAD_FFT_WINV_ADD: return KC_COL_FFT_WINV_ADD;
        case COL_PUPD_WINV_IFFT_CROP: return KC_COL_PUPD_WINV_IFFT;
        case COL_PAD_FFT_WINV_CG_UPD: return KC_COL_FFT_WINV_CG_UPD;
        default: return KC_COL_FFT_GPROD;
    }
}
int row_kclass(int mode) {
    switch (mode) {
        case ROW_CACHE: return KC_ROW_CACHE;
        case ROW_FWD: return KC_ROW_FWD;
        case ROW_DERIV: return KC_ROW_DERIV;
        default: return KC_ROW_ADJ;
    }
}

// One shape class: frames of a plan that share n and n_om.  Every CG vector
// of the class is stored contiguously: chat parts [planes][kb*kb] (the band
// of k-space the solve keeps, column-tiled), rho parts [frames][m*m].
struct Class {
    int n = 0, m = 0, lo = 0;
    int kb = 0, kb_lo = 0;       // band [kb_lo, kb_lo + kb)^2 of the sensitivities the solve keeps
    int nframes = 0, nplanes = 0;
    std::vector<int> frames;     // plan frame index of each class frame
    std::vector<int> J, plane0;
    int colv[kColModes] = {};    // pass variant per column mode
    int rowv[kRowModes] = {};    // and per row mode
    // the normal operator entry point: 0 the axis passes, 1 the whole-plane
    // kernel (grids that have one); the same choice for the CG iteration of
    // the solves
    int normal_form = 0;
    int cg_form = 0;
    // the passes load the intermediates T and T2 non-temporally and the
    // column passes store them so (ColArgs::stream): where T exceeds what the
    // eight XCDs' L2s hold between two passes (stream_by_size)
    int stream = 0;

    int* plane_frame = nullptr;
    int* frame_plane0 = nullptr;
    int* frame_planes = nullptr;
    float2* tw = nullptr;
    float* winv = nullptr;       // [n][n] 1/w, row-major
    float* winv_t = nullptr;     // its band [kb][kb], column-tiled (solve layout)
    int tilew = 8;               // tile width of the solve layout
    float2 *x_c = nullptr, *x_r = nullptr, *dx_r = nullptr;   // the chat part of dx goes into x_c
    float2 *r_c = nullptr, *r_r = nullptr, *p_c = nullptr, *p_r = nullptr;
    float2 *q_c = nullptr, *q_r = nullptr, *xr_c = nullptr, *xr_r = nullptr;   // q_c: grid-sized scratch
    float2* y = nullptr;
    float* P = nullptr;
    float2 *c = nullptr, *T = nullptr, *aux = nullptr;
    float2* T2 = nullptr;        // band-side intermediate [planes][m][kb] (when kb < n)
    double* partial = nullptr;   // general partials; in CG: |DF p|^2 of the PSF pass
    double* partial2 = nullptr;  // CG: |r|^2 after the update
    double* part_p = nullptr;    // CG: |p|^2 of the direction update
    SegGeom geom{}, geomC{};
    Scalars sc{};
    bool chat_ref_zero = false;  // this solve's x_ref has chat = 0 in every frame (not read then)

    long long cplane() const { return (long long)n * n; }
    long long rplane() const { return (long long)m * m; }
    long long kplane() const { return (long long)kb * kb; }
};

struct GraphKey {
    int newton = -1, cg = -1;
    float a0 = 0, q = 0, amin = 0;
    std::vector<bool> zero_ref;  // per class: its chat reference is all zero (not read)
    bool operator==(const GraphKey& o) const {
        return newton == o.newton && cg == o.cg && a0 == o.a0 && q == o.q && amin == o.amin &&
               zero_ref == o.zero_ref;
    }
};

}  // namespace

struct nlinv_plan_s {
    int device = 0;
    std::vector<nlinv_dims> dims;
    std::vector<Class> classes;
    std::vector<std::pair<int, int>> loc;   // frame -> (class, class-local frame)
    float sob_a = 220.f, sob_hl = 16.f;
    std::vector<void*> allocs;
    hipStream_t cap_stream = nullptr;
    // shape classes are independent: with more than one, their Newton loops
    // run on up to kMaxLanes streams of their own (default priority; class i
    // on lane i mod lanes), forked from and joined back into the caller's
    // stream (as concurrent branches in a graph)
    std::vector<hipStream_t> lanes;
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    // Captured Newton loops, one per key (a temporal series alternates
    // between a cold first frame and warm-started ones), least recently used
    // dropped beyond kMaxGraphs.  Each has two instances launched in turn: a
    // launch of an instance whose previous launch is still running waits on
    // the host for it, which would leave the GPU idle while the next launch
    // is being submitted.
    struct GraphEntry {
        GraphKey key;
        hipGraphExec_t exec[2] = {nullptr, nullptr};
        int next = 0;
        long long used = 0;
        long long id = 0;             // owner id of its timing slots
    };
    std::vector<GraphEntry> graphs;
    long long graph_clock = 0;
    // kernel timing
    bool timing[KC_NUM] = {};
    int timing_stride[KC_NUM] = {};   // bracket every stride-th launch of the class
    long long timing_count[KC_NUM] = {};
    std::vector<hipEvent_t> ev;
    std::vector<unsigned char> ev_used;
    std::vector<int> ev_class;          // kernel class of each slot
    std::vector<long long> ev_owner;    // graph id of a slot owned by a captured graph
    long long capture_id = 0;
    int ev_next = 0;
    bool capturing = false;
    bool timing_failed = false;
    // dry run (nlinv_check_launch_args): launches only check their operands
    // and are counted; nothing reaches the GPU
    bool dry_run = false;
    long long dry_launches = 0;
    int dry_first_bad = -1;       // kernel class of the first launch with a missing operand
};

namespace {

template <class T>
int dalloc(nlinv_plan_s* p, T** out, size_t count) {
    void* q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return NLINV_ENOMEM;
    }
    p->allocs.push_back(q);
    e = hipMemset(q, 0, bytes);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return NLINV_EHIP;
    }
    *out = static_cast<T*>(q);
    return NLINV_OK;
}

void make_geom(SegGeom& g, int nplanes, int nframes, long long cn, long long rn, bool with_rho,
               const int* plane_frame) {
    g.nplanes = nplanes;
    g.nframes = nframes;
    g.cn = (int)cn;
    g.rn = (int)rn;
    g.cseg = (int)((cn + kSegLen - 1) / kSegLen);
    g.clen = (int)((cn + g.cseg - 1) / g.cseg);
    g.clen += g.clen & 1;
    g.rseg = with_rho ? (int)((rn + kSegLen - 1) / kSegLen) : 0;
    g.rlen = with_rho ? (int)((rn + g.rseg - 1) / g.rseg) : 2;
    g.rlen += g.rlen & 1;
    g.plane_frame = plane_frame;
}

int nseg(const SegGeom& g) { return g.nplanes * g.cseg + g.nframes * g.rseg; }

// ---- timing brackets --------------------------------------------------------

// Under stream capture an event record is added as an explicit event-record
// node after the stream's current capture dependencies, and becomes the new
// dependency set, so that it lands between the kernels it brackets.  A
// failure is cleared from HIP's last-error state (it must not fail the
// solve) and reported by nlinv_plan_timing_read.
hipError_t record_event(nlinv_plan_s* p, hipEvent_t e, hipStream_t s) {
    if (!p->capturing) return hipEventRecord(e, s);
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipError_t r = hipStreamGetCaptureInfo_v2(s, &st, nullptr, &g, &deps, &nd);
    if (r == hipSuccess && (st != hipStreamCaptureStatusActive || !g)) r = hipErrorIllegalState;
    if (r == hipSuccess) {
        std::vector<hipGraphNode_t> d(deps, deps + nd);
        hipGraphNode_t node = nullptr;
        r = hipGraphAddEventRecordNode(&node, g, d.empty() ? nullptr : d.data(), d.size(), e);
        if (r == hipSuccess) r = hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
    }
    if (r != hipSuccess) {
        (void)hipGetLastError();
        p->timing_failed = true;
    }
    return r;
}

// Slots: ev_used 0 = free, 1 = recorded by an eager launch (read once),
// 2 = owned by the captured graph (re-recorded by every replay).
int tbegin(nlinv_plan_s* p, int kc, hipStream_t s) {
    if (!p->timing[kc] || p->ev.empty()) return -1;
    if (p->timing_count[kc]++ % p->timing_stride[kc] != 0) return -1;
    for (int tries = 0; tries < kTimingSlots; ++tries) {
        const int slot = p->ev_next;
        p->ev_next = (p->ev_next + 1) % kTimingSlots;
        if (p->ev_used[slot] == 2) continue;
        if (record_event(p, p->ev[2 * slot], s) != hipSuccess) return -1;
        p->ev_class[slot] = kc;
        return slot;
    }
    return -1;
}
void tend(nlinv_plan_s* p, int slot, hipStream_t s) {
    if (slot < 0) return;
    if (record_event(p, p->ev[2 * slot + 1], s) == hipSuccess) {
        p->ev_used[slot] = p->capturing ? 2 : 1;
        p->ev_owner[slot] = p->capturing ? p->capture_id : 0;
    }
}
hipError_t destroy_entry(nlinv_plan_s::GraphEntry& g) {
    hipError_t e = hipSuccess;
    for (hipGraphExec_t& x : g.exec) {
        if (!x) continue;
        const hipError_t e2 = hipGraphExecDestroy(x);
        if (e == hipSuccess) e = e2;
        x = nullptr;
    }
    return e;
}
// Drop every captured graph (and free the timing slots they own).
int drop_graph(nlinv_plan_s* p) {
    if (p->graphs.empty()) return NLINV_OK;
    hipError_t e = hipSuccess;
    for (auto& g : p->graphs) {
        const hipError_t e2 = destroy_entry(g);
        if (e == hipSuccess) e = e2;
    }
    p->graphs.clear();
    for (auto& u : p->ev_used)
        if (u == 2) u = 0;
    HIPCHK(e);
    return NLINV_OK;
}

struct Frames {               // which planes / frames a sequence acts on
    int nplanes, nframes;
    const int* plane_frame;   // nullable
    const int* frame_plane0;  // nullable
    const int* frame_planes;  // nullable
    int tiled;                // planes in the column-tiled solve layout
    int kb, kb_lo;            // band of the sensitivity side (the whole grid for the operators)
};

// the operator entry points: one frame, caller's row-major arrays, whole grid
Frames single_frame(const Class& C, int J) { return Frames{J, 1, nullptr, nullptr, nullptr, 0, C.n, 0}; }
// inside a solve: every frame of the class, solve layout, the class's band
Frames class_frames(const Class& C) {
    return Frames{C.nplanes, C.nframes, C.plane_frame, C.frame_plane0, C.frame_planes, 1, C.kb, C.kb_lo};
}
// band-side intermediate: T itself when the band is the whole grid (the row
// passes then work in place), else the separate [planes][m][kb] buffer
float2* band_T(const Class& C, const Frames& fr) { return fr.kb < C.n ? C.T2 : C.T; }

// ---- launch helpers -----------------------------------------------------------

ColArgs col_args(const nlinv_plan_s* p, const Class& C, const Frames& fr) {
    ColArgs a{};
    a.tiled = fr.tiled;
    a.m = C.m;
    a.lo = C.lo;
    a.kb = fr.kb;
    a.kb_lo = fr.kb_lo;
    a.rs = (float)(1.0 / std::sqrt((double)C.n));
    a.tw2 = C.tw;
    a.winv = fr.tiled ? C.winv_t : C.winv;
    a.frame_plane0 = fr.frame_plane0;
    a.frame_planes = fr.frame_planes;
    a.stream = C.stream;
    a.fold.op = SC_NONE;
    (void)p;
    return a;
}

RowArgs row_args(const Class& C, const Frames& fr) {
    RowArgs a{};
    a.m = C.m;
    a.lo = C.lo;
    a.kb = fr.kb;
    a.kb_lo = fr.kb_lo;
    a.rs = (float)(1.0 / std::sqrt((double)C.n));
    a.tw2 = C.tw;
    a.stream = C.stream;
    a.fold.op = SC_NONE;
    return a;
}

bool col_mode_on_band(int mode) {
    return mode == COL_WINV_IFFT_CROP || mode == COL_PUPD_WINV_IFFT_CROP || mode == COL_PAD_FFT_WINV_ADD ||
           mode == COL_PAD_FFT_WINV_CG_UPD;
}
// column tiles per plane of a launch of `mode` with its class variant
int col_tiles(const Class& C, const Frames& fr, int mode) {
    return (col_mode_on_band(mode) ? fr.kb : C.n) / kColL[C.colv[mode]];
}

// Every operand a pass mode reads or writes unconditionally must be set: a
// launch with one missing is refused here instead of faulting on the GPU.
bool col_operands_ok(int mode, const ColArgs& a) {
    if (!a.in || !a.out || !a.tw2) return false;
    switch (mode) {
        case COL_WINV_IFFT_CROP: return a.winv;
        case COL_P_IFFT_CROP: case COL_PAD_FFT_P: case COL_PAD_FFT_P2_IFFT: return a.P;
        case COL_RESID_P_IFFT: return a.P && a.add1;
        case COL_PAD_FFT_WINV_ADD: return a.winv;
        case COL_PAD_FFT_GPROD: return a.add1;
        case COL_PUPD_WINV_IFFT_CROP: return a.winv && a.r_in && a.p_out && a.pr && a.rr;
        case COL_PAD_FFT_WINV_CG_UPD:
            return a.winv && a.add1 && a.dx && a.cg_a &&
                   (a.cs_blocks == 0 || (a.cs.aux && a.cs.add1 && a.cs.r_upd && a.cs.dx_upd && a.cs.cg_a));
        default: return false;
    }
}

bool row_operands_ok(int mode, const RowArgs& a) {
    if (!a.tw2 || (mode != ROW_FWD && !a.in) || (mode != ROW_CACHE && !a.out)) return false;
    switch (mode) {
        case ROW_CACHE: return a.c_out && (!a.out || a.rho);
        case ROW_FWD: return a.rho && a.c;
        case ROW_DERIV: return a.rho && a.c && a.drho;
        case ROW_ADJ: return a.rho && a.c && a.aux;
        default: return false;
    }
}

// dry run: count the launch, remember the first one that would be refused
int dry_launch(nlinv_plan_s* p, bool ok, int kc) {
    ++p->dry_launches;
    if (!ok && p->dry_first_bad < 0) p->dry_first_bad = kc;
    return ok ? NLINV_OK : NLINV_EINVAL;
}

int run_col(nlinv_plan_s* p, const Class& C, int mode, const ColArgs& a0, int nplanes, hipStream_t s) {
    if (p->dry_run) return dry_launch(p, col_operands_ok(mode, a0), col_kclass(mode));
    if (!col_operands_ok(mode, a0)) return NLINV_EINVAL;
    ColArgs a = a0;
    a.nplanes = nplanes;
    const int slot = tbegin(p, col_kclass(mode), s);
    hipError_t e = col_dispatch(C.n, mode, C.colv[mode], a, nplanes, s);
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

int run_row(nlinv_plan_s* p, const Class& C, int mode, const RowArgs& a, hipStream_t s) {
    if (p->dry_run) return dry_launch(p, row_operands_ok(mode, a), row_kclass(mode));
    if (!row_operands_ok(mode, a)) return NLINV_EINVAL;
    const int slot = tbegin(p, row_kclass(mode), s);
    hipError_t e = row_dispatch(C.n, mode, C.rowv[mode], a, s);
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

int grid_for(long long n, int per = kThreads) {
    long long g = (n + per - 1) / per;
    if (g > 65535) g = 65535;
    if (g < 1) g = 1;
    return (int)g;
}

int run_coil_sum(nlinv_plan_s* p, const CoilSumArgs& a, hipStream_t s) {
    const bool ok = a.aux && (a.r_upd ? (a.add1 && a.dx_upd && a.cg_a) : a.out != nullptr);
    if (p->dry_run) return dry_launch(p, ok, KC_COIL_SUM);
    if (!ok) return NLINV_EINVAL;
    const int slot = tbegin(p, KC_COIL_SUM, s);
    hipLaunchKernelGGL(k_coil_sum, dim3(a.nframes * a.segs), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

template <int OP>
int run_vec(nlinv_plan_s* p, const SegGeom& g, const VecPtrs& v, double* partial, hipStream_t s) {
    if (p->dry_run) return dry_launch(p, v.c0 && (OP != VEC_DOT || partial), OP == VEC_DOT ? KC_VEC_DOT : KC_VEC_OTHER);
    const int kc = OP == VEC_DOT ? KC_VEC_DOT : KC_VEC_OTHER;
    const int slot = tbegin(p, kc, s);
    hipLaunchKernelGGL((k_vec<OP>), dim3(nseg(g)), dim3(kThreads), 0, s, g, v, partial);
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

ScalarStep scalar_step(const Class& C, int op, const SegGeom& g, float scale_norm, int step, int it = 0,
                       int nsteps = 0, int ncg = 0, const double* partial = nullptr) {
    ScalarStep ss{};
    ss.op = op;
    ss.g = g;
    ss.partial = partial ? partial : C.partial;
    ss.frame_plane0 = C.frame_plane0;
    ss.frame_planes = C.frame_planes;
    ss.scale_norm = scale_norm;
    ss.step = step;
    ss.it = it;
    ss.nsteps = nsteps;
    ss.ncg = ncg;
    return ss;
}

int launch_scalar(nlinv_plan_s* p, Class& C, const ScalarStep& ss, hipStream_t s) {
    if (p->dry_run) return dry_launch(p, ss.partial != nullptr, KC_SCALAR);
    const int slot = tbegin(p, KC_SCALAR, s);
    hipLaunchKernelGGL(k_scalar, dim3(C.nframes), dim3(64), 0, s, ss, C.sc);
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

int run_scalar(nlinv_plan_s* p, Class& C, int op, const SegGeom& g, float scale_norm, int step,
               hipStream_t s, int it = 0, int nsteps = 0, int ncg = 0, const double* partial = nullptr) {
    return launch_scalar(p, C, scalar_step(C, op, g, scale_norm, step, it, nsteps, ncg, partial), s);
}

VecPtrs vptrs(float2* c0, float2* r0, float2* c1 = nullptr, float2* r1 = nullptr) {
    VecPtrs v{};
    v.c0 = c0; v.r0 = r0; v.c1 = c1; v.r1 = r1;
    return v;
}

// ---- operator sequences (shared by the single-frame calls and the solve) --





// one workgroup per (frame, segment of up to kCoilSeg Omega pixels)
CoilSumArgs coil_sum_args(const Class& C, const Frames& fr, float2* out, const float2* add1,
                          const float2* add2, const float* s1, const float* s2, float c1, float c2,
                          double* partial, long long poff) {
    CoilSumArgs cs{};
    cs.aux = C.aux;
    cs.out = out;
    cs.add1 = add1;
    cs.add2 = add2;
    cs.s1 = s1;
    cs.s2 = s2;
    cs.c1 = c1;
    cs.c2 = c2;
    cs.frame_plane0 = fr.frame_plane0;
    cs.frame_planes = fr.frame_planes;
    cs.nplanes = fr.nplanes;
    cs.nframes = fr.nframes;
    cs.E = C.m * C.m;
    cs.segs = (cs.E + kCoilSeg - 1) / kCoilSeg;
    cs.seg_len = (cs.E + cs.segs - 1) / cs.segs;
    cs.partial = partial;
    cs.poff = poff;
    return cs;
}

// Whether the coil-map row pass can go on into the forward model's first
// pass (RowArgs::c_out): Omega the centred half on compile-time slots.
bool coil_maps_fwd_ok(const Class& C) { return 2 * C.m == C.n && 4 * C.lo == C.n && half_slots_k2(C.n); }

// c = E^H W^{-1} chat
// (inside a solve, optionally with the previous Newton step's rho update
// and its last CG scalar step folded into the two passes; with fwd_out, the
// row pass also writes fwd_out = T of rho . c, the forward model's first
// pass, where coil_maps_fwd_ok)
int seq_coil_maps(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* chat, float2* c_out,
                  hipStream_t s, bool rho_update = false, const ScalarStep* fold = nullptr,
                  float2* fwd_out = nullptr, const float2* rho = nullptr) {
    ColArgs a = col_args(p, C, fr);
    a.in = chat;
    a.out = band_T(C, fr);
    a.plane_frame = fr.plane_frame;
    if (rho_update) {
        a.rho_acc = C.x_r;
        a.rho_step = C.dx_r;
    }
    CHK(run_col(p, C, COL_WINV_IFFT_CROP, a, fr.nplanes, s));
    RowArgs r = row_args(C, fr);
    r.in = band_T(C, fr);
    r.c_out = c_out;
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    if (fold) {
        r.fold = *fold;
        r.sc = C.sc;
    }
    if (fwd_out) {
        if (!coil_maps_fwd_ok(C)) return NLINV_EINVAL;
        r.out = fwd_out;
        r.rho = rho;
    }
    return run_row(p, C, ROW_CACHE, r, s);
}

// out = P . DFT(E(rho . c))
int seq_forward(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* rho, const float2* c,
                const float* P, long long p_stride, float2* out, hipStream_t s) {
    RowArgs r = row_args(C, fr);
    r.c = c;
    r.rho = rho;
    r.out = C.T;
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    CHK(run_row(p, C, ROW_FWD, r, s));
    ColArgs a = col_args(p, C, fr);
    a.in = C.T;
    a.out = out;
    a.P = P;
    a.p_stride = p_stride;
    a.plane_frame = fr.plane_frame;
    return run_col(p, C, COL_PAD_FFT_P, a, fr.nplanes, s);
}

// Newton step: T = crop_rows(IDFT_0(P . r0)) with the residual
// r0 = s y - P . DFT(E(rho . c)) never stored (the first step of DF^H r0);
// |r0|^2 partials into `partial`, `g` receives their geometry.  With
// row_done, the row pass of rho . c is already in T (seq_coil_maps).
int seq_residual_head(nlinv_plan_s* p, const Class& C, const Frames& fr, double* partial, SegGeom* g,
                      hipStream_t s, bool row_done = false) {
    if (!row_done) {
        RowArgs r = row_args(C, fr);
        r.c = C.c;
        r.rho = C.x_r;
        r.out = C.T;
        r.plane_frame = fr.plane_frame;
        r.nlines = fr.nplanes * C.m;
        CHK(run_row(p, C, ROW_FWD, r, s));
    }
    ColArgs a = col_args(p, C, fr);
    a.in = C.T;
    a.out = C.T;
    a.P = C.P;
    a.p_stride = C.cplane();
    a.plane_frame = fr.plane_frame;
    a.add1 = C.y;
    a.s1 = C.sc.s;
    a.c1 = 1.f;
    a.partial = partial;
    *g = C.geom;
    g->cseg = col_tiles(C, fr, COL_RESID_P_IFFT);
    g->rseg = 0;
    return run_col(p, C, COL_RESID_P_IFFT, a, fr.nplanes, s);
}

// T = row-DFT(E(drho . c + rho . E^H W^{-1} dchat))   (first half of DF)
int seq_deriv_head(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* rho, const float2* c,
                   const float2* drho, const float2* dchat, hipStream_t s) {
    ColArgs a = col_args(p, C, fr);
    a.in = dchat;
    a.out = band_T(C, fr);
    a.plane_frame = fr.plane_frame;
    CHK(run_col(p, C, COL_WINV_IFFT_CROP, a, fr.nplanes, s));
    RowArgs r = row_args(C, fr);
    r.in = band_T(C, fr);
    r.out = C.T;
    r.c = c;
    r.rho = rho;
    r.drho = drho;
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    return run_row(p, C, ROW_DERIV, r, s);
}

// Whether the adjoint row pass can sum the coil products over
// groups of 4 coils (RowArgs::cgroup): Omega the centred half with its
// output slots known at compile time for the pass's split, 4 lines of a row
// in one wavefront, whole groups of rows per workgroup and whole coil groups
// per frame.
bool coil_groups_ok(const Class& C, const Frames& fr) {
    // every frame's coil count known and a multiple of 4 (a class without
    // its frame list, as the allocation-free entry point builds, never groups)
    if (C.J.empty() || fr.nplanes % 4 != 0) return false;
    const int v = C.rowv[ROW_ADJ], L = row_lines(v), n = C.n;
    const int d1 = split_n1(n), n1 = row_swapped(v) ? n / d1 : d1, n2 = n / n1;
    const bool half = 2 * C.m == n && 4 * C.lo == n;
    const bool half_by_k2 = n1 % 2 == 0 && n2 % 2 == 0 && n2 % 4 == 0 && (n / 4) % n1 == 0;
    if (!half || !half_by_k2 || L % 4 != 0 || 64 % (4 * n1) != 0 || C.m % (L / 4) != 0) return false;
    for (int j : C.J)
        if (j % 4 != 0) return false;
    return true;
}

// from T = crop_rows(IDFT_0(...)): u = crop(IDFT_1(T)); aux = conj(c) u;
// dchat_out = W^{-H} E(conj(rho) u) + s1 add1 + s2 add2;
// drho_out = sum_j aux + s1 add1r + s2 add2r
// (with `partial` set: |(drho_out, dchat_out)|^2 partials into it, `g` their geometry)
int seq_adjoint_tail(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* rho, const float2* c,
                     float2* drho_out, float2* dchat_out, const float2* add1c, const float2* add1r,
                     const float2* add2c, const float2* add2r, const float* s1, const float* s2,
                     float c1, float c2, hipStream_t s, double* partial = nullptr, SegGeom* g = nullptr,
                     const ScalarStep* fold = nullptr) {
    RowArgs r = row_args(C, fr);
    r.in = C.T;
    r.out = band_T(C, fr);
    r.c = c;
    r.rho = rho;
    r.aux = C.aux;
    if (fold) {   // a scalar step on partials of earlier kernels, folded into the row pass
        r.fold = *fold;
        r.sc = C.sc;
    }
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    const bool groups = coil_groups_ok(C, fr);
    r.cgroup = groups ? 4 : 0;
    CHK(run_row(p, C, ROW_ADJ, r, s));
    ColArgs a = col_args(p, C, fr);
    a.in = band_T(C, fr);
    a.out = dchat_out;
    a.plane_frame = fr.plane_frame;
    a.add1 = add1c;
    a.add2 = add2c;
    a.s1 = s1;
    a.s2 = s2;
    a.c1 = c1;
    a.c2 = c2;
    a.partial = partial;
    CHK(run_col(p, C, COL_PAD_FFT_WINV_ADD, a, fr.nplanes, s));
    const int nt = col_tiles(C, fr, COL_PAD_FFT_WINV_ADD);
    CoilSumArgs cs = coil_sum_args(C, fr, drho_out, add1r, add2r, s1, s2, c1, c2, partial,
                                   (long long)fr.nplanes * nt);
    cs.self_dot = partial != nullptr;
    cs.group = groups ? 4 : 1;   // the adjoint row pass summed groups of 4 coils
    if (g) {
        *g = C.geom;
        g->cseg = nt;
        g->rseg = cs.segs;
    }
    return run_coil_sum(p, cs, s);
}

// One CG iteration on every frame of class C (Newton step `step`, CG
// iteration `it` of K).  The step length needs gamma = Re<p, N_alpha p>,
// which equals |DF p|^2 + alpha |p|^2: the direction update p = r + beta p,
// folded into the first column pass (beta == nullptr: p = r), writes the
// |p|^2 partials and the PSF pass the |DF p|^2 partials, so a = <r,r>/gamma
// is known before the adjoint half of N_alpha p is computed.  The last column
// pass and the coil sum then form q = N_alpha p in registers and apply
// r -= a q, dx += a p directly (q is never stored), writing the |r|^2
// partials from which beta follows.
// Geometry of the <b, b> partials of the Newton right-hand side: column tiles
// of the W^{-H} pass per plane, then the coil-sum segments per frame (as
// seq_adjoint_tail reports them).
SegGeom rhs_geom(const Class& C) {
    SegGeom g = C.geom;
    g.cseg = col_tiles(C, class_frames(C), COL_PAD_FFT_WINV_ADD);
    g.rseg = (int)((C.rplane() + kCoilSeg - 1) / kCoilSeg);
    return g;
}

// Geometry of the <r, r> partials a CG iteration leaves: column tiles of the
// CG-update pass per plane, then the segments of its fused coil sum per frame.
SegGeom plane_rr_geom(const Class& C);
SegGeom cg_rr_geom(const Class& C) {
    if (C.cg_form == 1) return plane_rr_geom(C);
    SegGeom g = C.geom;
    const int L = kColL[C.colv[COL_PAD_FFT_WINV_CG_UPD]];
    const int wg = pass_threads(C.n, L);
    g.cseg = col_tiles(C, class_frames(C), COL_PAD_FFT_WINV_CG_UPD);
    g.rseg = (int)((C.rplane() + wg - 1) / wg);
    return g;
}

// alpha: the Newton step's regularisation weight (a kernel argument of the
// passes that need it)
int seq_cg_iteration(nlinv_plan_s* p, Class& C, int step, int it, int nsteps, int ncg, float alpha,
                     hipStream_t s) {
    const Frames fr = class_frames(C);
    float2* TB = band_T(C, fr);
    const int iter_slot = tbegin(p, KC_CG_ITER, s);
    ColArgs a = col_args(p, C, fr);
    a.in = C.p_c;
    a.out = TB;
    a.plane_frame = fr.plane_frame;
    a.r_in = C.r_c;
    a.p_out = C.p_c;
    a.beta = nullptr;                 // it == 0: p = r
    a.pr = C.p_r;
    a.rr = C.r_r;
    a.partial = C.part_p;
    // it > 0: beta of the previous iteration, computed inside the pass;
    // it == 0: <b, b> of the right-hand side recorded by it
    a.fold = it > 0 ? scalar_step(C, SC_RR, cg_rr_geom(C), 0.f, step, it - 1, nsteps, ncg, C.partial2)
                    : scalar_step(C, SC_RR0, rhs_geom(C), 0.f, step, 0, nsteps, ncg, C.partial);
    a.fold.alpha = alpha;
    a.sc = C.sc;
    CHK(run_col(p, C, COL_PUPD_WINV_IFFT_CROP, a, fr.nplanes, s));
    RowArgs r = row_args(C, fr);
    r.in = TB;
    r.out = C.T;
    r.c = C.c;
    r.rho = C.x_r;
    r.drho = C.p_r;
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    CHK(run_row(p, C, ROW_DERIV, r, s));
    ColArgs b = col_args(p, C, fr);
    b.in = C.T;
    b.out = C.T;
    b.P = C.P;
    b.p_stride = C.cplane();
    b.plane_frame = fr.plane_frame;
    b.partial = C.partial;
    CHK(run_col(p, C, COL_PAD_FFT_P2_IFFT, b, fr.nplanes, s));
    // a = <r,r> / (|DF p|^2 + alpha |p|^2) per frame, folded into the adjoint row pass
    {
        const int tp = col_tiles(C, fr, COL_PUPD_WINV_IFFT_CROP);
        const int tg = col_tiles(C, fr, COL_PAD_FFT_P2_IFFT);
        ScalarStep ss = scalar_step(C, SC_GAMMA, C.geom, 0.f, step, it, nsteps, ncg, C.partial);
        ss.g.cseg = tg;
        ss.g.rseg = 0;
        ss.g2 = C.geom;            // per plane: |p_c|^2 tiles, then its share of |p_r|^2
        ss.g2.cseg = 2 * tp;
        ss.g2.rseg = 0;
        ss.partial2 = C.part_p;
        ss.alpha = alpha;
        r.fold = ss;
        r.sc = C.sc;
    }
    r.aux = C.aux;
    r.drho = nullptr;
    r.in = C.T;
    r.out = TB;
    const bool groups = coil_groups_ok(C, fr);
    r.cgroup = groups ? 4 : 0;
    CHK(run_row(p, C, ROW_ADJ, r, s));
    const int tu = col_tiles(C, fr, COL_PAD_FFT_WINV_CG_UPD);
    ColArgs e = col_args(p, C, fr);
    e.in = TB;
    e.out = C.r_c;
    // the step's chat part goes straight into x: x's chat part is not read
    // during CG (the linearisation uses the cached sensitivities c, and the
    // right-hand side is formed before it); its rho part is (rho in DF), so
    // that part collects in dx_r until CG ends
    e.dx = C.x_c;
    e.plane_frame = fr.plane_frame;
    e.add1 = C.p_c;
    e.s1 = nullptr;
    e.c1 = alpha;
    e.cg_a = C.sc.a;
    e.partial = C.partial2;
    // the rho parts: the coil sum in its CG form, as extra workgroups of the
    // same launch (segments of one workgroup's size)
    CoilSumArgs cs = coil_sum_args(C, fr, nullptr, C.p_r, nullptr, nullptr, nullptr, alpha, 0.f, C.partial2,
                                   (long long)C.nplanes * tu);
    cs.r_upd = C.r_r;
    cs.dx_upd = C.dx_r;
    cs.dx_zero = it == 0;            // dx = a p: no zero fill of dx beforehand
    cs.cg_a = C.sc.a;
    cs.group = groups ? 4 : 1;       // the adjoint row pass summed groups of 4 coils
    const SegGeom grr = cg_rr_geom(C);
    cs.segs = grr.rseg;
    cs.seg_len = (cs.E + cs.segs - 1) / cs.segs;
    e.cs = cs;
    e.cs_blocks = C.nframes * cs.segs;
    CHK(run_col(p, C, COL_PAD_FFT_WINV_CG_UPD, e, fr.nplanes, s));
    tend(p, iter_slot, s);
    // beta = <r,r>' / <r,r> from the |r|^2 partials: inside the next
    // iteration's first pass; after the last iteration (only its stats are
    // left) inside the next coil-map pass (the caller does that)
    return NLINV_OK;
}

// Geometry of the partials the whole-plane CG iteration leaves: <r, r> per
// plane's band, then the rho part in segments of kThreads elements per frame;
// |DF p|^2 per plane (cseg 1); |p_c|^2 and a share of |p_r|^2 per plane (cseg 2).
SegGeom plane_rr_geom(const Class& C) {
    SegGeom g = C.geom;
    g.cseg = 1;
    g.rseg = (int)((C.rplane() + kThreads - 1) / kThreads);
    return g;
}

// One CG iteration of class C with the whole-plane kernels (two launches;
// see plane_kernel.hpp): the same scalar steps as the five-pass iteration.
int seq_cg_iteration_plane(nlinv_plan_s* p, Class& C, int step, int it, int nsteps, int ncg, float alpha,
                           hipStream_t s) {
    const int iter_slot = tbegin(p, KC_CG_ITER, s);
    PlaneCgArgs a{};
    a.nplanes = C.nplanes;
    a.nframes = C.nframes;
    a.plane_frame = C.plane_frame;
    a.frame_plane0 = C.frame_plane0;
    a.frame_planes = C.frame_planes;
    a.m = C.m;
    a.lo = C.lo;
    a.kb = C.kb;
    a.klo = C.kb_lo;
    a.tw = C.tilew;
    a.rs = 1.0f / std::sqrt((float)C.n);
    a.alpha = alpha;
    a.tw2 = C.tw;
    a.P = C.P;
    a.p_stride = C.cplane();
    a.winv = C.winv_t;
    a.rho = C.x_r;
    a.c = C.c;
    a.r_c = C.r_c;
    a.p_c = C.p_c;
    a.q_c = C.q_c;
    a.x_c = C.x_c;
    a.r_r = C.r_r;
    a.p_r = C.p_r;
    a.dx_r = C.dx_r;
    a.aux = C.aux;
    a.part_g = C.part_p;
    a.part_r = C.partial2;
    a.rseg = plane_rr_geom(C).rseg;
    a.first_iter = it == 0;
    a.fold = it > 0 ? scalar_step(C, SC_RR, plane_rr_geom(C), 0.f, step, it - 1, nsteps, ncg, C.partial2)
                    : scalar_step(C, SC_RR0, rhs_geom(C), 0.f, step, 0, nsteps, ncg, C.partial);
    a.fold.alpha = alpha;
    a.sc = C.sc;
    const bool ok = a.r_c && a.p_c && a.q_c && a.x_c && a.r_r && a.p_r && a.dx_r && a.aux && a.part_g &&
                    a.part_r && a.P && a.winv && a.rho && a.c && a.tw2 && a.fold.partial;
    if (p->dry_run) {
        CHK(dry_launch(p, ok, KC_PLANE_CG));
    } else {
        if (!ok) return NLINV_EINVAL;
        const int slot = tbegin(p, KC_PLANE_CG, s);
        const hipError_t e = plane_cg_dispatch(C.n, a, s);
        tend(p, slot, s);
        HIPCHK(e);
    }
    // the update: a = <r, r> / (|DF p|^2 + alpha |p|^2) from the partials just written
    SegGeom g = C.geom;
    g.cseg = 1;
    g.rseg = 0;
    a.fold = scalar_step(C, SC_GAMMA, g, 0.f, step, it, nsteps, ncg, C.part_p);
    a.fold.g2 = C.geom;   // |p_c|^2 and the |p_r|^2 share of each plane
    a.fold.g2.cseg = 2;
    a.fold.g2.rseg = 0;
    a.fold.partial2 = C.part_p + C.nplanes;
    a.fold.alpha = alpha;
    if (p->dry_run) {
        CHK(dry_launch(p, ok, KC_PLANE_CG_UPDATE));
    } else {
        const int slot = tbegin(p, KC_PLANE_CG_UPDATE, s);
        hipLaunchKernelGGL(k_plane_cg_update<kThreads>, dim3(C.nplanes + C.nframes * a.rseg), dim3(kThreads), 0,
                           s, a);
        const hipError_t e = hipGetLastError();
        tend(p, slot, s);
        HIPCHK(e);
    }
    tend(p, iter_slot, s);
    return NLINV_OK;
}

// (drho_out, dchat_out) = (DF^H DF + alpha) (drho, dchat) of one frame in
// the operator layout (whole grid, row-major) with the whole-plane kernel:
// one workgroup per coil plane, then the coil sum for the rho part
int seq_normal_plane(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* rho, const float2* c,
                     const float* P, float alpha, const float2* drho, const float2* dchat, float2* drho_out,
                     float2* dchat_out, hipStream_t s) {
    if (fr.tiled || fr.kb != C.n || fr.nframes != 1 || !plane_kernel_size(C.n)) return NLINV_EINVAL;
    PlaneArgs a{};
    a.rho = rho;
    a.c = c;
    a.P = P;
    a.winv = C.winv;
    a.drho = drho;
    a.dchat = dchat;
    a.dchat_out = dchat_out;
    a.aux = C.aux;
    a.tw2 = C.tw;
    a.alpha = alpha;
    a.rs = 1.0f / std::sqrt((float)C.n);
    a.m = C.m;
    a.lo = C.lo;
    a.nplanes = fr.nplanes;
    if (p->dry_run) {
        CHK(dry_launch(p, rho && c && P && C.winv && drho && dchat && dchat_out && C.aux && C.tw,
                       KC_PLANE_NORMAL));
    } else {
        const int slot = tbegin(p, KC_PLANE_NORMAL, s);
        const hipError_t e = plane_dispatch(C.n, a, s);
        tend(p, slot, s);
        HIPCHK(e);
    }
    CoilSumArgs cs = coil_sum_args(C, fr, drho_out, drho, nullptr, nullptr, nullptr, alpha, 0.f, nullptr, 0);
    return run_coil_sum(p, cs, s);
}

// (drho_out, dchat_out) = (DF^H DF + alpha) (drho, dchat); with whole_plane
// (the operator entry point of a plan that chose it) by the whole-plane kernel
int seq_normal(nlinv_plan_s* p, const Class& C, const Frames& fr, const float2* rho, const float2* c,
               const float* P, long long p_stride, const float* alpha_f, float alpha_c,
               const float2* drho, const float2* dchat, float2* drho_out, float2* dchat_out,
               hipStream_t s, bool whole_plane = false) {
    if (whole_plane && C.normal_form == 1 && !alpha_f && p_stride == 0)
        return seq_normal_plane(p, C, fr, rho, c, P, alpha_c, drho, dchat, drho_out, dchat_out, s);
    CHK(seq_deriv_head(p, C, fr, rho, c, drho, dchat, s));
    ColArgs a = col_args(p, C, fr);
    a.in = C.T;
    a.out = C.T;
    a.P = P;
    a.p_stride = p_stride;
    a.plane_frame = fr.plane_frame;
    CHK(run_col(p, C, COL_PAD_FFT_P2_IFFT, a, fr.nplanes, s));
    return seq_adjoint_tail(p, C, fr, rho, c, drho_out, dchat_out, dchat, drho, nullptr, nullptr,
                            alpha_f, nullptr, alpha_c, 0.f, s);
}


// ---- the Newton loop of one solve (device-only work: capturable) ------------

float alpha_of(const nlinv_irgnm_params& prm, int step) {
    double a = (double)prm.alpha0 * std::pow((double)prm.alpha_q, step);
    if (a < prm.alpha_min) a = prm.alpha_min;
    return (float)a;
}

// The Newton loop of one shape class on stream s.
int enqueue_class_newton(nlinv_plan_s* p, Class& C, const nlinv_irgnm_params& prm, hipStream_t s) {
    const int N = prm.newton_steps, K = prm.cg_iters;
    for (int step = 0; step < N; ++step) {
        const float al = alpha_of(prm, step);
        {
            const Frames fr = class_frames(C);
            const long long ps = C.cplane();
            // linearisation cache c at x_n (with the previous step's rho
            // update and its last CG step's stats folded in)
            // (the coil-map row pass goes on into the forward model's row
            // pass where the geometry allows)
            const bool fused = coil_maps_fwd_ok(C);
            float2* fwd = fused ? C.T : nullptr;
            if (step > 0 && K > 0) {
                ScalarStep last = scalar_step(C, SC_RR, cg_rr_geom(C), 0.f, step - 1, K - 1, N, K, C.partial2);
                last.alpha = alpha_of(prm, step - 1);
                CHK(seq_coil_maps(p, C, fr, C.x_c, C.c, s, true, &last, fwd, C.x_r));
            } else {
                CHK(seq_coil_maps(p, C, fr, C.x_c, C.c, s, false, nullptr, fwd, C.x_r));
            }
            // r0 = s y - F(x_n) (its norm) and the first step of DF^H r0
            SegGeom g0{};
            CHK(seq_residual_head(p, C, fr, C.partial, &g0, s, fused));
            // b = DF^H r0 - alpha (x_n - x_ref) into r; ||r0|| recorded inside
            // its adjoint row pass, <b, b> inside the first CG pass
            {
                const ScalarStep r0 = scalar_step(C, SC_R0NORM, g0, 0.f, step);
                SegGeom gb{};
                CHK(seq_adjoint_tail(p, C, fr, C.x_r, C.c, C.r_r, C.r_c, C.x_c, C.x_r,
                                     C.chat_ref_zero ? nullptr : C.xr_c, C.xr_r, nullptr, nullptr, -al, al, s,
                                     C.partial, &gb, &r0));
                (void)gb;   // the geometry rhs_geom() gives the first CG pass
            }
        }
        for (int it = 0; it < K; ++it)
            CHK(C.cg_form == 1 ? seq_cg_iteration_plane(p, C, step, it, N, K, al, s)
                               : seq_cg_iteration(p, C, step, it, N, K, al, s));
        // the chat part of the step is already in x; rho += drho happens in
        // the next coil-map pass (dx_r is first written by CG iteration 0)
    }
    // sensitivities of the final x (for the image), with the last step's
    // rho update and last CG stats
    if (N > 0 && K > 0) {
        ScalarStep last = scalar_step(C, SC_RR, cg_rr_geom(C), 0.f, N - 1, K - 1, N, K, C.partial2);
        last.alpha = alpha_of(prm, N - 1);
        return seq_coil_maps(p, C, class_frames(C), C.x_c, C.c, s, true, &last);
    }
    return seq_coil_maps(p, C, class_frames(C), C.x_c, C.c, s);
}

int enqueue_newton(nlinv_plan_s* p, const nlinv_irgnm_params& prm, hipStream_t s) {
    const size_t nl = p->lanes.size();
    if (p->classes.size() == 1 || nl == 0) {
        for (Class& C : p->classes) CHK(enqueue_class_newton(p, C, prm, s));
        return NLINV_OK;
    }
    // class i on lane i mod nl (classes sharing a lane run one after another)
    HIPCHK(hipEventRecord(p->fork_ev, s));
    for (size_t l = 0; l < nl; ++l) HIPCHK(hipStreamWaitEvent(p->lanes[l], p->fork_ev, 0));
    for (size_t i = 0; i < p->classes.size(); ++i) CHK(enqueue_class_newton(p, p->classes[i], prm, p->lanes[i % nl]));
    for (size_t l = 0; l < nl; ++l) {
        HIPCHK(hipEventRecord(p->join_ev[l], p->lanes[l]));
        HIPCHK(hipStreamWaitEvent(s, p->join_ev[l], 0));
    }
    return NLINV_OK;
}

// row-major <-> column-tiled copies of `nplanes` planes of class C
template <class T>
int tile_copy(nlinv_plan_s* p, const Class& C, const T* src, T* dst, int nplanes, int to_tiled, hipStream_t s) {
    const int slot = tbegin(p, KC_VEC_OTHER, s);
    hipLaunchKernelGGL((k_tile<T>), dim3(grid_for((long long)nplanes * C.cplane())), dim3(kThreads), 0, s, src, dst,
                       nplanes, C.n, C.tilew, to_tiled);
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

// Several such copies, one launch per kTileBatch entries: entry i copies
// np[i] planes from src[i] to dst[i] (entries with np[i] <= 0 are skipped).
template <class T>
int tile_copy_batch(nlinv_plan_s* p, const Class& C, const std::vector<const T*>& src, const std::vector<T*>& dst,
                    const std::vector<int>& np, int to_tiled, hipStream_t s) {
    for (size_t i0 = 0; i0 < src.size(); i0 += kTileBatch) {
        TileBatch<T> b{};
        int cnt = 0, maxp = 0;
        for (size_t i = i0; i < src.size() && i < i0 + kTileBatch; ++i) {
            if (np[i] <= 0) continue;
            b.src[cnt] = src[i];
            b.dst[cnt] = dst[i];
            b.np[cnt] = np[i];
            maxp = std::max(maxp, np[i]);
            ++cnt;
        }
        if (cnt == 0) continue;
        const int slot = tbegin(p, KC_VEC_OTHER, s);
        hipLaunchKernelGGL((k_tile_batch<T>), dim3(grid_for((long long)maxp * C.cplane()), cnt), dim3(kThreads), 0, s,
                           b, C.n, C.tilew, to_tiled);
        hipError_t e = hipGetLastError();
        tend(p, slot, s);
        HIPCHK(e);
    }
    return NLINV_OK;
}

int check_params(const nlinv_irgnm_params* prm) {
    if (!prm) return NLINV_EINVAL;
    if (prm->newton_steps < 0 || prm->newton_steps > kMaxNewton) return NLINV_EINVAL;
    if (prm->cg_iters < 0 || prm->cg_iters > kMaxCG) return NLINV_EINVAL;
    if (!(prm->alpha0 >= 0.f) || !(prm->alpha_q >= 0.f) || !(prm->alpha_min >= 0.f) || !(prm->scale_norm >= 0.f))
        return NLINV_EINVAL;
    return NLINV_OK;
}

bool aligned(const void* q) { return ((uintptr_t)q & 15) == 0; }

// Where a warm start reads x0 (data units): the frame's own rho / chat
// arrays unless given here (a temporal series starts frame t from frame
// t - 1's results).
struct FrameSrc {
    const float2* rho0;
    const float2* chat0;
};

const float2* chat0_of(const nlinv_frame& F, const FrameSrc* src, int f) {
    return src && src[f].chat0 ? src[f].chat0 : (const float2*)F.chat;
}
const float2* rho0_of(const nlinv_frame& F, const FrameSrc* src, int f) {
    return src && src[f].rho0 ? src[f].rho0 : (const float2*)F.rho;
}

// Frames of class C in runs of at most kTileBatch: fn(first class frame, count)
template <class Fn>
int for_frame_batches(const Class& C, Fn&& fn) {
    for (int f0 = 0; f0 < C.nframes; f0 += kTileBatch) CHK(fn(f0, std::min(kTileBatch, C.nframes - f0)));
    return NLINV_OK;
}

// the band of caller planes into the solve layout, for every frame of C
// whose source is non-null
int band_in(nlinv_plan_s* p, const Class& C, const std::vector<const float2*>& src, float2* dst, hipStream_t s) {
    return for_frame_batches(C, [&](int f0, int cnt) -> int {
        BandBatch b{};
        int k = 0, maxp = 1;
        for (int i = 0; i < cnt; ++i) {
            const int lf = f0 + i;
            if (!src[lf]) continue;
            b.src[k] = src[lf];
            b.dst[k] = dst + (size_t)C.plane0[lf] * C.kplane();
            b.np[k] = C.J[lf];
            maxp = std::max(maxp, C.J[lf]);
            ++k;
        }
        if (k == 0) return NLINV_OK;
        const int slot = tbegin(p, KC_VEC_OTHER, s);
        hipLaunchKernelGGL(k_band_in, dim3(grid_for((long long)maxp * C.kplane()), k), dim3(kThreads), 0, s, b, C.n,
                           C.kb_lo, C.kb, C.tilew);
        hipError_t e = hipGetLastError();
        tend(p, slot, s);
        HIPCHK(e);
        return NLINV_OK;
    });
}

// Per-frame set-up: copy y and P into the class workspace, data scale, x0,
// x_ref (the band of the sensitivities), the record of the components
// outside the band.
int setup_frames(nlinv_plan_s* p, const nlinv_frame* frames, const nlinv_irgnm_params& prm, hipStream_t s,
                 const FrameSrc* src) {
    for (Class& C : p->classes) {
        {   // y and P of every frame into the solve layout, one launch each
            std::vector<const float2*> ys;
            std::vector<float2*> yd;
            std::vector<const float*> ps;
            std::vector<float*> pd;
            std::vector<int> nj, one;
            for (int lf = 0; lf < C.nframes; ++lf) {
                const nlinv_frame& F = frames[C.frames[lf]];
                ys.push_back((const float2*)F.y);
                yd.push_back(C.y + (size_t)C.plane0[lf] * C.cplane());
                nj.push_back(C.J[lf]);
                ps.push_back(F.P);
                pd.push_back(C.P + (size_t)lf * C.cplane());
                one.push_back(1);
            }
            CHK(tile_copy_batch(p, C, ys, yd, nj, 1, s));
            CHK(tile_copy_batch(p, C, ps, pd, one, 1, s));
        }
        CHK(run_vec<VEC_DOT>(p, C.geomC, vptrs(C.y, nullptr, C.y, nullptr), C.partial, s));
        CHK(run_scalar(p, C, SC_YNORM, C.geomC, prm.scale_norm, 0, s));
        // x0: warm start takes the caller's x (rho scaled below); else rho = 1 (scaled units), chat = 0
        const bool warm = (prm.flags & NLINV_WARM_START) != 0;
        if (warm) {
            std::vector<const float2*> c0(C.nframes);
            for (int lf = 0; lf < C.nframes; ++lf) {
                const nlinv_frame& F = frames[C.frames[lf]];
                c0[lf] = chat0_of(F, src, C.frames[lf]);
                HIPCHK(hipMemcpyAsync(C.x_r + (size_t)lf * C.rplane(), rho0_of(F, src, C.frames[lf]),
                                      C.rplane() * sizeof(float2), hipMemcpyDeviceToDevice, s));
            }
            CHK(band_in(p, C, c0, C.x_c, s));
            hipLaunchKernelGGL(k_scale_rho, dim3(grid_for((long long)C.nframes * C.rplane())), dim3(kThreads), 0, s,
                               C.x_r, (const float2*)C.x_r, (const float*)C.sc.s, C.nframes, (int)C.rplane(), 0);
        } else {   // the chat parts of all frames are contiguous: one fill
            HIPCHK(hipMemsetAsync(C.x_c, 0, (size_t)C.nplanes * C.kplane() * sizeof(float2), s));
            hipLaunchKernelGGL(k_fill, dim3(grid_for((long long)C.nframes * C.rplane())), dim3(kThreads), 0, s,
                               C.x_r, (long long)C.nframes * C.rplane(), make_float2(1.f, 0.f));
        }
        HIPCHK(hipGetLastError());
        bool any_ref = false;
        for (int lf = 0; lf < C.nframes; ++lf) any_ref = any_ref || frames[C.frames[lf]].chat_ref;
        C.chat_ref_zero = !warm && !any_ref;   // x_ref = x0, whose chat part is 0
        // x_ref (a zero chat part is not stored: the passes are not given it)
        if (!any_ref) {   // x_ref = x0 for every frame: one copy of each contiguous part
            HIPCHK(hipMemcpyAsync(C.xr_r, C.x_r, (size_t)C.nframes * C.rplane() * sizeof(float2),
                                  hipMemcpyDeviceToDevice, s));
            if (!C.chat_ref_zero)
                HIPCHK(hipMemcpyAsync(C.xr_c, C.x_c, (size_t)C.nplanes * C.kplane() * sizeof(float2),
                                      hipMemcpyDeviceToDevice, s));
        } else {
            std::vector<const float2*> cr(C.nframes, nullptr);
            for (int lf = 0; lf < C.nframes; ++lf) {
                const nlinv_frame& F = frames[C.frames[lf]];
                float2* rr = C.xr_r + (size_t)lf * C.rplane();
                if (F.rho_ref && F.chat_ref) {
                    cr[lf] = (const float2*)F.chat_ref;
                    HIPCHK(hipMemcpyAsync(rr, F.rho_ref, C.rplane() * sizeof(float2), hipMemcpyDeviceToDevice, s));
                    // a caller's x_ref is in data units: scale its rho part
                    hipLaunchKernelGGL(k_scale_rho, dim3(grid_for(C.rplane())), dim3(kThreads), 0, s, rr,
                                       (const float2*)rr, (const float*)(C.sc.s + lf), 1, (int)C.rplane(), 0);
                    HIPCHK(hipGetLastError());
                } else {
                    HIPCHK(hipMemcpyAsync(C.xr_c + (size_t)C.plane0[lf] * C.kplane(),
                                          C.x_c + (size_t)C.plane0[lf] * C.kplane(),
                                          (size_t)C.J[lf] * C.kplane() * sizeof(float2), hipMemcpyDeviceToDevice, s));
                    HIPCHK(hipMemcpyAsync(rr, C.x_r + (size_t)lf * C.rplane(), C.rplane() * sizeof(float2),
                                          hipMemcpyDeviceToDevice, s));
                }
            }
            CHK(band_in(p, C, cr, C.xr_c, s));
        }
        // components outside the band: D = |x0 - x_ref|^2 there (nonzero only
        // for a caller's x_ref), theta = 1
        const double* dpart = nullptr;
        const int dsegs = std::min(16, C.n / 4);   // row segments per plane (partials fit C.partial)
        if (any_ref && C.kb < C.n) {
            CHK(for_frame_batches(C, [&](int f0, int cnt) -> int {
                BandBatch b{};
                int maxp = 1;
                for (int i = 0; i < cnt; ++i) {
                    const int lf = f0 + i;
                    const nlinv_frame& F = frames[C.frames[lf]];
                    b.x0[i] = warm ? chat0_of(F, src, C.frames[lf]) : nullptr;
                    b.ref[i] = (F.rho_ref && F.chat_ref) ? (const float2*)F.chat_ref : nullptr;
                    b.np[i] = C.J[lf];
                    b.plane0[i] = C.plane0[lf];
                    maxp = std::max(maxp, C.J[lf]);
                }
                hipLaunchKernelGGL(k_inert_dist, dim3(maxp * dsegs, cnt), dim3(kThreads), 0, s, b, C.partial, C.n,
                                   C.kb_lo, C.kb, dsegs);
                HIPCHK(hipGetLastError());
                return NLINV_OK;
            }));
            dpart = C.partial;
        }
        hipLaunchKernelGGL(k_inert_init, dim3(grid_for(C.nframes)), dim3(kThreads), 0, s, C.sc.inert, dpart, dsegs,
                           (const int*)C.frame_plane0, (const int*)C.frame_planes, C.nplanes, C.nframes);
        HIPCHK(hipGetLastError());
    }
    return NLINV_OK;
}

int finish_frames(nlinv_plan_s* p, const nlinv_frame* frames, const nlinv_irgnm_params& prm, hipStream_t s,
                  const FrameSrc* src) {
    const int stats_len = 2 + prm.newton_steps + prm.newton_steps * prm.cg_iters;
    const bool warm = (prm.flags & NLINV_WARM_START) != 0;
    for (Class& C : p->classes) {
        // image (uses rho in scaled units times 1/s) into aux, rho / s into dx_r
        const int slot = tbegin(p, KC_IMAGE, s);
        hipLaunchKernelGGL(k_image, dim3(grid_for((long long)C.nframes * C.rplane())), dim3(kThreads), 0, s,
                           (const float2*)C.x_r, (const float2*)C.c, C.aux, (const int*)C.frame_plane0,
                           (const int*)C.frame_planes, C.nplanes, C.nframes, (int)C.rplane(),
                           (const float*)C.sc.inv_s);
        tend(p, slot, s);
        hipLaunchKernelGGL(k_scale_rho, dim3(grid_for((long long)C.nframes * C.rplane())), dim3(kThreads), 0, s,
                           C.dx_r, (const float2*)C.x_r, (const float*)C.sc.inv_s, C.nframes, (int)C.rplane(), 1);
        HIPCHK(hipGetLastError());
        // chat of every frame into the caller's planes: the band from the
        // solve layout, the rest x_ref + theta (x0 - x_ref)
        CHK(for_frame_batches(C, [&](int f0, int cnt) -> int {
            BandBatch b{};
            int maxp = 1;
            for (int i = 0; i < cnt; ++i) {
                const int lf = f0 + i;
                const nlinv_frame& F = frames[C.frames[lf]];
                b.band[i] = C.x_c + (size_t)C.plane0[lf] * C.kplane();
                b.x0[i] = warm ? chat0_of(F, src, C.frames[lf]) : nullptr;
                b.ref[i] = (F.rho_ref && F.chat_ref) ? (const float2*)F.chat_ref : nullptr;
                b.dst[i] = (float2*)F.chat;
                b.np[i] = C.J[lf];
                b.frame[i] = lf;
                maxp = std::max(maxp, C.J[lf]);
            }
            const int sl = tbegin(p, KC_VEC_OTHER, s);
            hipLaunchKernelGGL(k_chat_out, dim3(grid_for((long long)maxp * C.cplane()), cnt), dim3(kThreads), 0, s, b,
                               (const double*)C.sc.inert, C.n, C.kb_lo, C.kb, C.tilew);
            hipError_t e = hipGetLastError();
            tend(p, sl, s);
            HIPCHK(e);
            return NLINV_OK;
        }));
        // rho, image and stats of every frame: one launch per kCopyBatch copies
        CopyBatch b{};
        int cnt = 0;
        long long maxn = 0;
        auto add = [&](const void* src_, void* dst, long long words) {
            b.src[cnt] = (const uint64_t*)src_;
            b.dst[cnt] = (uint64_t*)dst;
            b.n[cnt] = words;
            maxn = std::max(maxn, words);
            ++cnt;
        };
        auto flush = [&]() -> hipError_t {
            if (cnt == 0) return hipSuccess;
            hipLaunchKernelGGL(k_copy_batch, dim3(grid_for(maxn), cnt), dim3(kThreads), 0, s, b);
            cnt = 0;
            maxn = 0;
            return hipGetLastError();
        };
        for (int lf = 0; lf < C.nframes; ++lf) {
            const nlinv_frame& F = frames[C.frames[lf]];
            if (cnt + 3 > kCopyBatch) HIPCHK(flush());
            add(C.dx_r + (size_t)lf * C.rplane(), F.rho, (long long)C.rplane());
            if (F.image) add(C.aux + (size_t)lf * C.rplane(), F.image, (long long)C.rplane());
            if (F.stats) add(C.sc.stats + (size_t)lf * kStatsCap, F.stats, stats_len);
        }
        HIPCHK(flush());
    }
    return NLINV_OK;
}

int validate_frames(nlinv_plan_s* p, const nlinv_frame* frames, int count) {
    if (!frames) return NLINV_EINVAL;
    for (int f = 0; f < count; ++f) {
        const nlinv_frame& F = frames[f];
        if (!F.y || !F.P || !F.rho || !F.chat) return NLINV_EINVAL;
        if (!aligned(F.y) || !aligned(F.P) || !aligned(F.rho) || !aligned(F.chat)) return NLINV_EINVAL;
        if ((F.rho_ref == nullptr) != (F.chat_ref == nullptr)) return NLINV_EINVAL;
        if (F.image && !aligned(F.image)) return NLINV_EINVAL;
        if (F.stats && ((uintptr_t)F.stats & 7)) return NLINV_EINVAL;
    }
    (void)p;
    return NLINV_OK;
}

int run_newton(nlinv_plan_s* p, const nlinv_irgnm_params& prm, hipStream_t s) {
    // stats_len must be known to the kernels that write stats
    for (Class& C : p->classes) C.sc.stats_len = kStatsCap;
    if (!(prm.flags & NLINV_USE_GRAPH)) return enqueue_newton(p, prm, s);
    GraphKey key{prm.newton_steps, prm.cg_iters, prm.alpha0, prm.alpha_q, prm.alpha_min, {}};
    for (const Class& C : p->classes) key.zero_ref.push_back(C.chat_ref_zero);
    nlinv_plan_s::GraphEntry* ent = nullptr;
    for (auto& g : p->graphs)
        if (g.key == key) ent = &g;
    if (!ent) {
        if ((int)p->graphs.size() >= kMaxGraphs) {   // drop the least recently used
            size_t lru = 0;
            for (size_t i = 1; i < p->graphs.size(); ++i)
                if (p->graphs[i].used < p->graphs[lru].used) lru = i;
            for (size_t k = 0; k < p->ev_used.size(); ++k)   // free the timing slots it owned
                if (p->ev_used[k] == 2 && p->ev_owner[k] == p->graphs[lru].id) p->ev_used[k] = 0;
            HIPCHK(destroy_entry(p->graphs[lru]));
            p->graphs.erase(p->graphs.begin() + lru);
        }
        nlinv_plan_s::GraphEntry fresh;
        fresh.id = ++p->capture_id;
        HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        p->capturing = true;
        for (long long& c : p->timing_count) c = 0;   // the graph's brackets start at launch 0
        const int st = enqueue_newton(p, prm, p->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        p->capturing = false;
        if (st != NLINV_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        HIPCHK(e);
        e = hipGraphInstantiate(&fresh.exec[0], g, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphInstantiate(&fresh.exec[1], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            (void)destroy_entry(fresh);
            HIPCHK(e);
        }
        fresh.key = key;
        p->graphs.push_back(fresh);
        ent = &p->graphs.back();
    }
    ent->used = ++p->graph_clock;
    HIPCHK(hipGraphLaunch(ent->exec[ent->next], s));
    ent->next ^= 1;
    return NLINV_OK;
}

int solve_all(nlinv_plan_s* p, const nlinv_frame* frames, const nlinv_irgnm_params& prm, hipStream_t s,
              const FrameSrc* src = nullptr) {
    CHK(setup_frames(p, frames, prm, s, src));
    CHK(run_newton(p, prm, s));
    return finish_frames(p, frames, prm, s, src);
}

// ---- twiddles -------------------------------------------------------------------

// tw2[k1][j2] = exp(-2 pi i k1 j2 / n) for the split n = N1 * N2 of the line FFTs
int make_twiddles(nlinv_plan_s* p, Class& C) {
    const int n1 = split_n1(C.n), n2 = C.n / n1;
    std::vector<float2> h(C.n);
    for (int k1 = 0; k1 < n1; ++k1)
        for (int j2 = 0; j2 < n2; ++j2) {
            const double ang = -2.0 * M_PI * (double)(k1 * j2) / (double)C.n;
            h[k1 * n2 + j2] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
    CHK(dalloc(p, &C.tw, C.n));
    HIPCHK(hipMemcpy(C.tw, h.data(), C.n * sizeof(float2), hipMemcpyHostToDevice));
    return NLINV_OK;
}

// a column variant valid for the grid and for `ncols` columns per plane
bool col_ok_cols(int n, int ncols, int v) { return col_ok(n, v) && ncols % kColL[v] == 0; }
int default_col_variant(int n, int ncols) {
    for (int v = 0; v < kNumColVariants; ++v)
        if (col_ok_cols(n, ncols, v)) return v;
    return -1;
}
int default_row_variant(int n) {
    for (int v = 0; v < kNumRowVariants; ++v)
        if (row_ok(n, v)) return v;
    return -1;
}

// 1/w[kappa] = (1 + a |k|^2)^(-l/2), k_d = (kappa_d - n/2)/n, in FP64 on the host
int make_weight_table(nlinv_plan_s* p, Class& C) {
    std::vector<float> h((size_t)C.n * C.n);
    for (int r = 0; r < C.n; ++r)
        for (int c = 0; c < C.n; ++c) {
            const double k0 = (double)(r - C.n / 2) / C.n, k1 = (double)(c - C.n / 2) / C.n;
            h[(size_t)r * C.n + c] = (float)std::pow(1.0 + (double)p->sob_a * (k0 * k0 + k1 * k1),
                                                     -(double)p->sob_hl);
        }
    CHK(dalloc(p, &C.winv, h.size()));
    HIPCHK(hipMemcpy(C.winv, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    // the band [kb_lo, kb_lo + kb)^2 in the solve layout [kb/tw][kb][tw]
    std::vector<float> t((size_t)C.kb * C.kb);
    for (int r = 0; r < C.kb; ++r)
        for (int c = 0; c < C.kb; ++c)
            t[((size_t)(c / C.tilew) * C.kb + r) * C.tilew + (c % C.tilew)] =
                h[(size_t)(C.kb_lo + r) * C.n + C.kb_lo + c];
    CHK(dalloc(p, &C.winv_t, t.size()));
    HIPCHK(hipMemcpy(C.winv_t, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    return NLINV_OK;
}

// Half-width h of the band of k-space the solve keeps of the sensitivities:
// outside [n/2 - h, n/2 + h)^2 every weight has 1/w <= 2^-40 (there
// |k|^2 >= (h/n)^2 and (1 + a (h/n)^2)^(l/2) >= 2^40), so those components
// of chat reach c = DTFT^{-1}(chat / w) only below 2^-40 of their size, far
// under single-precision rounding.  h is a multiple of 16 (the band side a
// multiple of 32: whole column tiles of every pass variant); h = n/2 (the
// whole grid) when the weight is too flat for a narrower band, or with
// NLINV_FULL_CHAT=1 set.
int band_half(int n, double a, double l) {
    const char* full = std::getenv("NLINV_FULL_CHAT");
    if ((full && full[0] == '1') || !(a > 0.0) || !(l > 0.0)) return n / 2;
    const double k = std::sqrt((std::pow(2.0, 80.0 / l) - 1.0) / a);   // |k| where 1/w = 2^-40
    int h = (int)std::ceil(k * n - 1e-9);
    h = (h + 15) / 16 * 16;
    return 2 * h >= n ? n / 2 : h;
}

// Whether the passes should stream their intermediates: T ([planes][m][n]
// complex) larger than 30 MiB, just under the 32 MB of the eight XCDs' L2s
// together.  Measured in graph-replayed solves: 32 planes of 256 x 512
// (32 MiB) 0.8 % faster streamed; 48 planes of 192 x 384 (27 MiB) 2.3 %
// slower.  (Timing whole CG iterations alone misjudges the first case.)
int stream_by_size(const Class& C) {
    return (double)C.nplanes * C.m * C.n * sizeof(float2) > 30.0 * 1024 * 1024 ? 1 : 0;
}

int build_class(nlinv_plan_s* p, Class& C) {
    C.tilew = plane_tile_width(C.n);
    C.stream = stream_by_size(C);
    {
        const int h = band_half(C.n, (double)p->sob_a, 2.0 * (double)p->sob_hl);
        C.kb = 2 * h;
        C.kb_lo = C.n / 2 - h;
    }
    CHK(make_twiddles(p, C));
    CHK(make_weight_table(p, C));
    const long long cn = C.cplane(), rn = C.rplane();
    const size_t cv = (size_t)C.nplanes * cn, rv = (size_t)C.nframes * rn, kv = (size_t)C.nplanes * C.kplane();
    std::vector<int> pf(C.nplanes), fp0(C.nframes), fpn(C.nframes);
    for (int lf = 0; lf < C.nframes; ++lf) {
        fp0[lf] = C.plane0[lf];
        fpn[lf] = C.J[lf];
        for (int j = 0; j < C.J[lf]; ++j) pf[C.plane0[lf] + j] = lf;
    }
    CHK(dalloc(p, &C.plane_frame, C.nplanes));
    CHK(dalloc(p, &C.frame_plane0, C.nframes));
    CHK(dalloc(p, &C.frame_planes, C.nframes));
    HIPCHK(hipMemcpy(C.plane_frame, pf.data(), pf.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C.frame_plane0, fp0.data(), fp0.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(C.frame_planes, fpn.data(), fpn.size() * sizeof(int), hipMemcpyHostToDevice));
    // CG vectors: the band of the sensitivities; q_c (grid-sized scratch) and y: whole planes
    float2** kvecs[] = {&C.x_c, &C.r_c, &C.p_c, &C.xr_c};
    for (float2** v : kvecs) CHK(dalloc(p, v, kv));
    CHK(dalloc(p, &C.q_c, cv));
    CHK(dalloc(p, &C.y, cv));
    float2** rvecs[] = {&C.x_r, &C.dx_r, &C.r_r, &C.p_r, &C.q_r, &C.xr_r};
    for (float2** v : rvecs) CHK(dalloc(p, v, rv));
    CHK(dalloc(p, &C.P, (size_t)C.nframes * cn));
    CHK(dalloc(p, &C.c, (size_t)C.nplanes * rn));
    CHK(dalloc(p, &C.aux, (size_t)C.nplanes * rn));
    CHK(dalloc(p, &C.T, (size_t)C.nplanes * C.m * C.n));
    if (C.kb < C.n) CHK(dalloc(p, &C.T2, (size_t)C.nplanes * C.m * C.kb));
    make_geom(C.geom, C.nplanes, C.nframes, cn, rn, true, C.plane_frame);
    make_geom(C.geomC, C.nplanes, C.nframes, cn, rn, false, C.plane_frame);
    // partials: the segment geometries, or (column tiles of the narrowest
    // variant per plane) + (coil-sum segments per frame)
    // (coil-sum segments are as small as one 64-thread workgroup when fused
    // into a column pass)
    const size_t tiles = (size_t)C.nplanes * (C.n / 4) + (size_t)C.nframes * ((rn + 63) / 64);
    CHK(dalloc(p, &C.partial, std::max<size_t>(tiles, (size_t)std::max(nseg(C.geom), nseg(C.geomC)))));
    CHK(dalloc(p, &C.partial2, std::max<size_t>(tiles, (size_t)nseg(C.geom))));
    // (also the whole-plane CG iteration's |DF p|^2 and |p|^2 partials: 3 per plane)
    // (the first CG pass's |p|^2 partials: 2 per plane and column tile)
    CHK(dalloc(p, &C.part_p, (size_t)(2 * C.nplanes + C.nframes) * (C.n / 4) + (size_t)3 * C.nplanes));
    CHK(dalloc(p, &C.sc.rr, (size_t)2 * C.nframes));
    CHK(dalloc(p, &C.sc.a, C.nframes));
    CHK(dalloc(p, &C.sc.beta, C.nframes));
    CHK(dalloc(p, &C.sc.brk, C.nframes));
    CHK(dalloc(p, &C.sc.s, C.nframes));
    CHK(dalloc(p, &C.sc.inv_s, C.nframes));
    CHK(dalloc(p, &C.sc.stats, (size_t)C.nframes * kStatsCap));
    CHK(dalloc(p, &C.sc.inert, (size_t)C.nframes * kInertLen));
    C.sc.nframes = C.nframes;
    C.sc.stats_len = kStatsCap;
    for (int m = 0; m < kColModes; ++m) C.colv[m] = default_col_variant(C.n, col_mode_on_band(m) ? C.kb : C.n);
    for (int& v : C.rowv) v = default_row_variant(C.n);
    for (int m = 0; m < kColModes; ++m)
        if (C.colv[m] < 0) return NLINV_EUNSUPPORTED;
    return NLINV_OK;
}

void free_plan(nlinv_plan_s* p) {
    if (!p) return;
    for (auto& g : p->graphs) (void)destroy_entry(g);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (hipStream_t q : p->lanes) (void)hipStreamDestroy(q);
    for (hipEvent_t e : p->join_ev) (void)hipEventDestroy(e);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (void* q : p->allocs) (void)hipFree(q);
    delete p;
}

int check_dims(const nlinv_dims& d) {
    if (d.n <= 0 || d.n_om <= 0 || d.ncoils <= 0) return NLINV_EINVAL;
    if (!size_supported(d.n) || !supported_len(d.n)) return NLINV_EUNSUPPORTED;
    if (default_col_variant(d.n, d.n) < 0 || default_row_variant(d.n) < 0) return NLINV_EUNSUPPORTED;
    if ((d.n_om & 1) || d.n_om > d.n) return NLINV_EUNSUPPORTED;
    if (d.ncoils > 64) return NLINV_EUNSUPPORTED;
    if (!(d.sobolev_a >= 0.f) || !(d.sobolev_l >= 0.f)) return NLINV_EINVAL;
    return NLINV_OK;
}

Class* class0(nlinv_plan_s* p) { return &p->classes[p->loc[0].first]; }

// Arguments of a representative launch of each pass mode on the class
// workspace (the contents are scratch at tuning time: a solve recomputes
// everything from its inputs).
ColArgs tune_col_args(nlinv_plan_s* p, Class& C, int mode) {
    const Frames fr = class_frames(C);
    float2* TB = band_T(C, fr);
    ColArgs a = col_args(p, C, fr);
    a.plane_frame = fr.plane_frame;
    a.P = C.P;
    a.p_stride = C.cplane();
    a.in = C.T;
    a.out = C.T;
    switch (mode) {
        case COL_WINV_IFFT_CROP: a.in = C.x_c; a.out = TB; break;
        case COL_PUPD_WINV_IFFT_CROP:
            a.in = C.p_c; a.out = TB; a.r_in = C.r_c; a.p_out = C.p_c; a.beta = C.sc.beta; a.pr = C.p_r;
            a.rr = C.r_r; a.partial = C.part_p;
            break;
        case COL_PAD_FFT_P2_IFFT: a.partial = C.partial; break;
        case COL_P_IFFT_CROP: a.in = C.q_c; break;
        case COL_PAD_FFT_P: a.out = C.q_c; break;
        case COL_RESID_P_IFFT: a.add1 = C.y; a.s1 = C.sc.s; break;   // in place on T
        case COL_PAD_FFT_WINV_ADD:
            a.in = TB; a.out = C.r_c; a.add1 = C.x_c; a.add2 = C.xr_c; a.c1 = -1.f; a.c2 = 1.f;
            break;
        case COL_PAD_FFT_WINV_CG_UPD:
            // q_c stands in for x (scratch: tuning must not touch the solution)
            a.in = TB; a.out = C.r_c; a.dx = C.q_c; a.add1 = C.p_c;
            a.c1 = 1.f; a.cg_a = C.sc.a; a.partial = C.partial2;
            break;
        default: break;
    }
    return a;
}

RowArgs tune_row_args(Class& C, int mode) {
    const Frames fr = class_frames(C);
    float2* TB = band_T(C, fr);
    RowArgs r = row_args(C, fr);
    r.in = C.T;
    r.out = C.T;
    if (mode == ROW_CACHE || mode == ROW_DERIV) r.in = TB;
    if (mode == ROW_ADJ) r.out = TB;
    r.c = C.c;
    r.rho = C.x_r;
    r.drho = C.p_r;
    r.aux = C.aux;
    r.c_out = C.c;
    r.plane_frame = fr.plane_frame;
    r.nlines = fr.nplanes * C.m;
    return r;
}

// Time `reps` launches of every valid variant of every pass mode the solve
// uses and keep the fastest per mode; NLINV_TUNE_VERBOSE prints the table.
int tune_class(nlinv_plan_s* p, Class& C, hipStream_t s) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const bool verbose = std::getenv("NLINV_TUNE_VERBOSE") != nullptr;
    const int reps = 10;
    const int nplanes = C.nplanes;
    auto timeit = [&](auto&& launch, float& ms) -> int {
        CHK(launch());
        HIPCHK(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) CHK(launch());
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        return NLINV_OK;
    };
    // ms per call of `launch` (a sequence that depends only on the plan's
    // state), `reps` calls captured as one graph and replayed, as the solves
    // replay theirs: the best of two replays after a warm-up one.  Kernel
    // timing brackets stay out of the capture.
    auto time_graph = [&](auto&& launch, float& best) -> int {
        bool saved[KC_NUM];
        for (int k = 0; k < KC_NUM; ++k) {
            saved[k] = p->timing[k];
            p->timing[k] = false;
        }
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
        int st = NLINV_OK;
        if (e == hipSuccess) {
            p->capturing = true;
            for (int r = 0; r < reps && st == NLINV_OK; ++r) st = launch(p->cap_stream);
            e = hipStreamEndCapture(p->cap_stream, &g);
            p->capturing = false;
        }
        for (int k = 0; k < KC_NUM; ++k) p->timing[k] = saved[k];
        hipGraphExec_t x = nullptr;
        if (st == NLINV_OK && e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        best = 1e30f;
        for (int k = 0; k < 3 && st == NLINV_OK && e == hipSuccess; ++k) {
            float ms = 0.f;
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = hipGraphLaunch(x, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (k > 0) best = std::min(best, ms / reps);
        }
        if (x) (void)hipGraphExecDestroy(x);
        CHK(st);
        HIPCHK(e);
        return NLINV_OK;
    };
    const int col_modes[] = {COL_WINV_IFFT_CROP, COL_PUPD_WINV_IFFT_CROP, COL_P_IFFT_CROP, COL_PAD_FFT_P,
                             COL_RESID_P_IFFT, COL_PAD_FFT_P2_IFFT, COL_PAD_FFT_WINV_ADD,
                             COL_PAD_FFT_WINV_CG_UPD};
    for (int mode : col_modes) {
        const ColArgs a = tune_col_args(p, C, mode);
        float best = 1e30f;
        int bestv = C.colv[mode];
        for (int v = 0; v < kNumColVariants; ++v) {
            // fewer lines than the tile width would split cache lines between
            // workgroups: cheap when timed warm here, not in a solve
            if (!col_ok_cols(C.n, col_mode_on_band(mode) ? C.kb : C.n, v) || kColL[v] < C.tilew) continue;
            C.colv[mode] = v;
            float ms = 0.f;
            CHK(timeit([&] { return run_col(p, C, mode, a, nplanes, s); }, ms));
            if (verbose)
                std::fprintf(stderr, "nlinv tune n=%d planes=%d %s L=%d: %.1f us\n", C.n, nplanes,
                             kKClassNames[col_kclass(mode)], kColL[v], 1e3 * ms);
            if (ms < best) { best = ms; bestv = v; }
        }
        C.colv[mode] = bestv;
    }
    const int row_modes[] = {ROW_CACHE, ROW_FWD, ROW_DERIV, ROW_ADJ};
    for (int mode : row_modes) {
        const RowArgs r = tune_row_args(C, mode);
        float best = 1e30f;
        int bestv = C.rowv[mode];
        for (int v = 0; v < kNumRowVariants; ++v) {
            if (!row_ok(C.n, v)) continue;
            // the transposed split exists for the CG loop's row passes only
            if (row_swapped(v) && mode != ROW_DERIV && mode != ROW_ADJ) continue;
            C.rowv[mode] = v;
            float ms = 0.f;
            CHK(timeit([&] { return run_row(p, C, mode, r, s); }, ms));
            if (verbose)
                std::fprintf(stderr, "nlinv tune n=%d planes=%d %s L=%d%s: %.1f us\n", C.n, nplanes,
                             kKClassNames[row_kclass(mode)], row_lines(v), row_swapped(v) ? " split swapped" : "",
                             1e3 * ms);
            if (ms < best) { best = ms; bestv = v; }
        }
        C.rowv[mode] = bestv;
    }
    // The CG loop's five passes, refined inside whole CG iterations captured
    // and replayed as in a solve: timed alone, a pass re-reads its own input
    // warm from the caches, while in the loop it reads what the pass before
    // it wrote, so the fastest variant alone is not always the fastest in the
    // loop (and eager launches, with their gaps, change what the caches hold
    // between passes).  One mode at a time, every valid variant (narrow ones
    // included: splitting cache lines between workgroups is priced here); a
    // change is kept only if the iteration gets at least 0.3 % faster.
    {
        {
            auto time_cg = [&](float& best) -> int {
                return time_graph([&](hipStream_t cs) { return seq_cg_iteration(p, C, 0, 1, 1, 2, 0.5f, cs); }, best);
            };
            float cur = 0.f;
            CHK(time_cg(cur));
            const int cm[] = {COL_PUPD_WINV_IFFT_CROP, COL_PAD_FFT_P2_IFFT, COL_PAD_FFT_WINV_CG_UPD};
            for (int mode : cm) {
                const int keep = C.colv[mode];
                int bestv = keep;
                for (int v = 0; v < kNumColVariants; ++v) {
                    if (v == keep || !col_ok_cols(C.n, col_mode_on_band(mode) ? C.kb : C.n, v)) continue;
                    C.colv[mode] = v;
                    float ms = 0.f;
                    CHK(time_cg(ms));
                    if (verbose)
                        std::fprintf(stderr, "nlinv tune n=%d planes=%d cg_iteration with %s L=%d: %.1f us (now %.1f)\n",
                                     C.n, nplanes, kKClassNames[col_kclass(mode)], kColL[v], 1e3 * ms, 1e3 * cur);
                    if (ms < 0.997f * cur) { cur = ms; bestv = v; }
                }
                C.colv[mode] = bestv;
            }
            const int rm[] = {ROW_DERIV, ROW_ADJ};
            for (int mode : rm) {
                const int keep = C.rowv[mode];
                int bestv = keep;
                for (int v = 0; v < kNumRowVariants; ++v) {
                    if (v == keep || !row_ok(C.n, v)) continue;
                    C.rowv[mode] = v;
                    float ms = 0.f;
                    CHK(time_cg(ms));
                    if (verbose)
                        std::fprintf(stderr, "nlinv tune n=%d planes=%d cg_iteration with %s L=%d%s: %.1f us (now %.1f)\n",
                                     C.n, nplanes, kKClassNames[row_kclass(mode)], row_lines(v),
                                     row_swapped(v) ? " split swapped" : "", 1e3 * ms, 1e3 * cur);
                    if (ms < 0.997f * cur) { cur = ms; bestv = v; }
                }
                C.rowv[mode] = bestv;
            }
        }
    }
    // the normal operator entry point: the axis passes against the
    // whole-plane kernel (grids that have one), on the plan's first frame
    // shape in the operator layout, with full-grid scratch standing in for
    // the operands
    C.normal_form = 0;
    if (plane_kernel_size(C.n) && C.frames.size() > 0 && C.frames[0] == 0) {
        const Frames fr = single_frame(C, C.J[0]);
        float ms[2] = {0.f, 0.f};
        for (int form = 0; form < 2; ++form) {
            C.normal_form = form;
            CHK(timeit([&] {
                return seq_normal(p, C, fr, C.x_r, C.c, C.P, 0, nullptr, 0.5f, C.p_r, C.y, C.q_r, C.q_c, s, true);
            }, ms[form]));
            if (verbose)
                std::fprintf(stderr, "nlinv tune n=%d planes=%d normal %s: %.1f us\n", C.n, C.J[0],
                             form ? "whole plane" : "axis passes", 1e3 * ms[form]);
        }
        C.normal_form = ms[1] < ms[0] ? 1 : 0;
    }
    // the solves' CG iteration: the five passes against the two whole-plane
    // launches (CG iteration 1 of 2, with its scalar folds, on scratch state;
    // captured and replayed, as in a solve)
    C.cg_form = 0;
    if (plane_kernel_size(C.n)) {
        float ms[2] = {0.f, 0.f};
        for (int form = 0; form < 2; ++form) {
            C.cg_form = form;
            CHK(time_graph([&](hipStream_t cs) {
                return form ? seq_cg_iteration_plane(p, C, 0, 1, 1, 2, 0.5f, cs)
                            : seq_cg_iteration(p, C, 0, 1, 1, 2, 0.5f, cs);
            }, ms[form]));
            if (verbose)
                std::fprintf(stderr, "nlinv tune n=%d planes=%d cg_iteration %s: %.1f us\n", C.n, nplanes,
                             form ? "whole plane" : "axis passes", 1e3 * ms[form]);
        }
        C.cg_form = ms[1] < ms[0] ? 1 : 0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return NLINV_OK;
}

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================

extern "C" {

const char* nlinv_status_string(int status) {
    switch (status) {
        case NLINV_OK: return "ok";
        case NLINV_EINVAL: return "invalid argument";
        case NLINV_EUNSUPPORTED: return "unsupported size";
        case NLINV_ENOMEM: return "out of device memory";
        case NLINV_EHIP: return "HIP error";
        case NLINV_ESCRATCH: return "frame too large for the static scratch of nlinv_normal_noalloc";
        default: return "unknown status";
    }
}

int nlinv_last_hip_error(void) { return g_last_hip; }

int nlinv_bandwidth_probe(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || !aligned(src) || !aligned(dst) || (bytes & 15)) return NLINV_EINVAL;
    const long long n16 = (long long)(bytes / 16);
    const long long per = (long long)kThreads * kProbeUnroll;
    const int blocks = (int)std::min<long long>((n16 + per - 1) / per, 8 * 256 * 16);
    if (n16 == 0) return NLINV_OK;
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream,
                       (const probe_v4*)src, (probe_v4*)dst, n16);
    HIPCHK(hipGetLastError());
    return NLINV_OK;
}

// ---- gridding of radial samples (Sec. 3.1-3.2) ------------------------------

static int grid_check(int32_t n, int32_t J, int32_t S, int32_t R, const float* angles, const float* dcf, float width,
                      float beta, const void* in, const void* out) {
    if (n < 1 || n > 65536 || J < 1 || J > 65535 * kGridCoilChunk || S < 1 || S > kMaxSpokes || R < 1) return NLINV_EINVAL;
    if ((long long)S * R > (1LL << 30)) return NLINV_EINVAL;
    if (!(width > 0.f) || !(width < (float)n) || !(beta >= 0.f) || !std::isfinite(beta)) return NLINV_EINVAL;
    if (!angles || !in || !out || ((uintptr_t)angles & 3) || (dcf && ((uintptr_t)dcf & 3)) ||
        ((uintptr_t)in & 7) || ((uintptr_t)out & 7))
        return NLINV_EINVAL;
    return NLINV_OK;
}

int nlinv_grid_radial(int32_t n, int32_t J, int32_t S, int32_t R, const float* angles, const float* dcf, float width,
                      float beta, const nlinv_c32* data, nlinv_c32* grid_out, void* stream) {
    CHK(grid_check(n, J, S, R, angles, dcf, width, beta, data, grid_out));
    GridArgs g{n, J, S, R, angles, dcf, (double)width, (double)beta, (const float2*)data, (float2*)grid_out,
               nullptr};
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_grid_radial, dim3((unsigned)((nn + kThreads - 1) / kThreads), (J + kGridCoilChunk - 1) / kGridCoilChunk),
                       dim3(kThreads), 0, (hipStream_t)stream, g);
    HIPCHK(hipGetLastError());
    return NLINV_OK;
}

int nlinv_degrid_radial(int32_t n, int32_t J, int32_t S, int32_t R, const float* angles, const float* dcf,
                        float width, float beta, const nlinv_c32* grid, nlinv_c32* data_out, void* stream) {
    CHK(grid_check(n, J, S, R, angles, dcf, width, beta, grid, data_out));
    GridArgs g{n, J, S, R, angles, dcf, (double)width, (double)beta, nullptr, (float2*)data_out, (const float2*)grid};
    const long long ns = (long long)S * R;
    hipLaunchKernelGGL(k_degrid_radial, dim3((unsigned)((ns + kThreads - 1) / kThreads), (J + kGridCoilChunk - 1) / kGridCoilChunk),
                       dim3(kThreads), 0, (hipStream_t)stream, g);
    HIPCHK(hipGetLastError());
    return NLINV_OK;
}

// ---- PCA channel compression (Sec. 3.2) ---------------------------------------

static void pca_layout(int32_t J, int64_t M, long long* chunk, int* G, size_t* off_A, size_t* off_l, size_t* off_V,
                       size_t* total) {
    long long c = std::max<long long>(kPcaChunk, (M + kPcaMaxPartials - 1) / kPcaMaxPartials);
    c = (c + kPcaTile - 1) / kPcaTile * kPcaTile;
    *chunk = c;
    *G = (int)((M + c - 1) / c);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t jj = (size_t)J * J;
    *off_A = up((size_t)*G * jj * sizeof(double2));
    *off_l = *off_A + up(jj * sizeof(double2));
    *off_V = *off_l + up((size_t)J * sizeof(double));
    *total = *off_V + up(jj * sizeof(float2));
}

size_t nlinv_coil_compress_workspace(int32_t J, int64_t M) {
    if (J < 1 || J > kPcaMaxJ || M < 1) return 0;
    long long chunk;
    int G;
    size_t a, l, v, t;
    pca_layout(J, M, &chunk, &G, &a, &l, &v, &t);
    return t;
}

int nlinv_coil_compress(int32_t J, int64_t M, int32_t K, const nlinv_c32* y, nlinv_c32* y_out, double* eigvals_out,
                        nlinv_c32* basis_out, void* workspace, size_t workspace_bytes, void* stream) {
    if (J < 1 || J > kPcaMaxJ || K < 1 || K > J || M < 1) return NLINV_EINVAL;
    if (!y || !y_out || !workspace || ((uintptr_t)y & 7) || ((uintptr_t)y_out & 7) || ((uintptr_t)workspace & 15) ||
        (eigvals_out && ((uintptr_t)eigvals_out & 7)) || (basis_out && ((uintptr_t)basis_out & 7)))
        return NLINV_EINVAL;
    long long chunk;
    int G;
    size_t oA, ol, oV, total;
    pca_layout(J, M, &chunk, &G, &oA, &ol, &oV, &total);
    if (workspace_bytes < total) return NLINV_EINVAL;
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    PcaArgs a{};
    a.J = J;
    a.K = K;
    a.M = M;
    a.G = G;
    a.chunk = chunk;
    a.y = (const float2*)y;
    a.partial = reinterpret_cast<double2*>(ws);
    a.A = reinterpret_cast<double2*>(ws + oA);
    a.lambda = eigvals_out ? eigvals_out : reinterpret_cast<double*>(ws + ol);
    a.V = basis_out ? (float2*)basis_out : reinterpret_cast<float2*>(ws + oV);
    a.y_out = (float2*)y_out;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pca_cov_partial, dim3(G), dim3(kThreads), 0, s, a);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_pca_cov_reduce, dim3((J * J + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_pca_eig, dim3(1), dim3(kThreads), 0, s, a);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_pca_compress, dim3((unsigned)((M + kThreads - 1) / kThreads), (K + kPcaCompressK - 1) / kPcaCompressK),
                       dim3(kThreads), 0, s, a);
    HIPCHK(hipGetLastError());
    return NLINV_OK;
}

const char* nlinv_kernel_class_name(int32_t kclass) {
    if (kclass < 0 || kclass >= KC_NUM) return nullptr;
    return kKClassNames[kclass];
}

int nlinv_plan_create(nlinv_plan* out, const nlinv_dims* dims, int32_t nframes) {
    return nlinv_plan_create_branched(out, dims, nframes, 0);
}

int nlinv_plan_create_branched(nlinv_plan* out, const nlinv_dims* dims, int32_t nframes, int32_t branch_frames) {
    if (!out || !dims || nframes <= 0 || nframes > 4096) return NLINV_EINVAL;
    *out = nullptr;
    for (int f = 0; f < nframes; ++f) CHK(check_dims(dims[f]));
    for (int f = 1; f < nframes; ++f)
        if (dims[f].sobolev_a != dims[0].sobolev_a || dims[f].sobolev_l != dims[0].sobolev_l) return NLINV_EINVAL;
    nlinv_plan_s* p = new (std::nothrow) nlinv_plan_s;
    if (!p) return NLINV_ENOMEM;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { g_last_hip = (int)e; delete p; return NLINV_EHIP; }
    p->dims.assign(dims, dims + nframes);
    p->sob_a = dims[0].sobolev_a;
    p->sob_hl = 0.5f * dims[0].sobolev_l;
    p->loc.resize(nframes);
    // frames of one shape share a class; with branch_frames > 0 a class
    // takes at most that many, and the next frames of the shape open another
    std::map<std::pair<int, int>, int> cls;
    for (int f = 0; f < nframes; ++f) {
        const auto key = std::make_pair(dims[f].n, dims[f].n_om);
        auto it = cls.find(key);
        int ci;
        if (it == cls.end() || (branch_frames > 0 && p->classes[it->second].nframes >= branch_frames)) {
            ci = (int)p->classes.size();
            cls[key] = ci;
            Class C;
            C.n = dims[f].n;
            C.m = dims[f].n_om;
            C.lo = C.n / 2 - C.m / 2;
            p->classes.push_back(C);
        } else {
            ci = it->second;
        }
        Class& C = p->classes[ci];
        p->loc[f] = {ci, C.nframes};
        C.frames.push_back(f);
        C.J.push_back(dims[f].ncoils);
        C.plane0.push_back(C.nplanes);
        C.nplanes += dims[f].ncoils;
        C.nframes += 1;
    }
    for (Class& C : p->classes) {
        if (C.nplanes > 65535) { free_plan(p); return NLINV_EUNSUPPORTED; }   // column-pass grid.y
        const int st = build_class(p, C);
        if (st != NLINV_OK) { free_plan(p); return st; }
    }
    e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { g_last_hip = (int)e; free_plan(p); return NLINV_EHIP; }
    if (p->classes.size() > 1) {   // a stream per shape class, up to kMaxLanes (default priority)
        e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
        const size_t nl = std::min(p->classes.size(), (size_t)kMaxLanes);
        for (size_t i = 0; e == hipSuccess && i < nl; ++i) {
            hipStream_t q = nullptr;
            hipEvent_t j = nullptr;
            e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
            if (e == hipSuccess) p->lanes.push_back(q);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
            if (e == hipSuccess) p->join_ev.push_back(j);
        }
        if (e != hipSuccess) { g_last_hip = (int)e; free_plan(p); return NLINV_EHIP; }
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) { g_last_hip = (int)e; free_plan(p); return NLINV_EHIP; }
    *out = p;
    return NLINV_OK;
}

int nlinv_plan_destroy(nlinv_plan plan) {
    if (!plan) return NLINV_OK;
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return NLINV_OK;
}

int nlinv_coil_maps(nlinv_plan p, const nlinv_c32* chat, nlinv_c32* c_out, void* stream) {
    if (!p || !chat || !c_out || !aligned(chat) || !aligned(c_out)) return NLINV_EINVAL;
    Class& C = *class0(p);
    return seq_coil_maps(p, C, single_frame(C, p->dims[0].ncoils), (const float2*)chat, (float2*)c_out,
                         (hipStream_t)stream);
}

int nlinv_forward(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* chat, const float* P,
                  nlinv_c32* y_out, nlinv_c32* c_out, void* stream) {
    if (!p || !rho || !chat || !P || !y_out) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(chat) || !aligned(P) || !aligned(y_out) || (c_out && !aligned(c_out)))
        return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const Frames fr = single_frame(C, p->dims[0].ncoils);
    float2* c = c_out ? (float2*)c_out : C.c;
    CHK(seq_coil_maps(p, C, fr, (const float2*)chat, c, s));
    return seq_forward(p, C, fr, (const float2*)rho, c, P, 0, (float2*)y_out, s);
}

int nlinv_deriv(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* chat, const nlinv_c32* c,
                const float* P, const nlinv_c32* drho, const nlinv_c32* dchat, nlinv_c32* dy_out,
                void* stream) {
    if (!p || !rho || !P || !drho || !dchat || !dy_out || (!c && !chat)) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(P) || !aligned(drho) || !aligned(dchat) || !aligned(dy_out) ||
        (c && !aligned(c)) || (chat && !aligned(chat)))
        return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const Frames fr = single_frame(C, p->dims[0].ncoils);
    const float2* cc = (const float2*)c;
    if (!cc) {
        CHK(seq_coil_maps(p, C, fr, (const float2*)chat, C.c, s));
        cc = C.c;
    }
    CHK(seq_deriv_head(p, C, fr, (const float2*)rho, cc, (const float2*)drho, (const float2*)dchat, s));
    ColArgs a = col_args(p, C, fr);
    a.in = C.T;
    a.out = (float2*)dy_out;
    a.P = P;
    return run_col(p, C, COL_PAD_FFT_P, a, fr.nplanes, s);
}

int nlinv_adjoint(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* chat, const nlinv_c32* c,
                  const float* P, const nlinv_c32* dy, nlinv_c32* drho_out, nlinv_c32* dchat_out,
                  void* stream) {
    if (!p || !rho || !P || !dy || !drho_out || !dchat_out || (!c && !chat)) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(P) || !aligned(dy) || !aligned(drho_out) || !aligned(dchat_out) ||
        (c && !aligned(c)) || (chat && !aligned(chat)))
        return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const Frames fr = single_frame(C, p->dims[0].ncoils);
    const float2* cc = (const float2*)c;
    if (!cc) {
        CHK(seq_coil_maps(p, C, fr, (const float2*)chat, C.c, s));
        cc = C.c;
    }
    ColArgs a = col_args(p, C, fr);
    a.in = (const float2*)dy;
    a.out = C.T;
    a.P = P;
    CHK(run_col(p, C, COL_P_IFFT_CROP, a, fr.nplanes, s));
    return seq_adjoint_tail(p, C, fr, (const float2*)rho, cc, (float2*)drho_out, (float2*)dchat_out, nullptr,
                            nullptr, nullptr, nullptr, nullptr, nullptr, 0.f, 0.f, s);
}

int nlinv_normal(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* chat, const nlinv_c32* c,
                 const float* P, float alpha, const nlinv_c32* drho, const nlinv_c32* dchat,
                 nlinv_c32* drho_out, nlinv_c32* dchat_out, void* stream) {
    if (!p || !rho || !P || !drho || !dchat || !drho_out || !dchat_out || (!c && !chat)) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(P) || !aligned(drho) || !aligned(dchat) || !aligned(drho_out) ||
        !aligned(dchat_out) || (c && !aligned(c)) || (chat && !aligned(chat)))
        return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const Frames fr = single_frame(C, p->dims[0].ncoils);
    const float2* cc = (const float2*)c;
    if (!cc) {
        CHK(seq_coil_maps(p, C, fr, (const float2*)chat, C.c, s));
        cc = C.c;
    }
    return seq_normal(p, C, fr, (const float2*)rho, cc, P, 0, nullptr, alpha, (const float2*)drho,
                      (const float2*)dchat, (float2*)drho_out, (float2*)dchat_out, s, true);
}

int nlinv_mask_gradient(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* chat, const nlinv_c32* c,
                        const nlinv_c32* g, float* gP_out, void* stream) {
    if (!p || !rho || !g || !gP_out || (!c && !chat)) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(g) || !aligned(gP_out) || (c && !aligned(c)) || (chat && !aligned(chat)))
        return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const int J = p->dims[0].ncoils;
    const Frames fr = single_frame(C, J);
    const float2* cc = (const float2*)c;
    if (!cc) {
        CHK(seq_coil_maps(p, C, fr, (const float2*)chat, C.c, s));
        cc = C.c;
    }
    RowArgs r = row_args(C, fr);
    r.c = cc;
    r.rho = (const float2*)rho;
    r.out = C.T;
    r.nlines = J * C.m;
    CHK(run_row(p, C, ROW_FWD, r, s));
    ColArgs a = col_args(p, C, fr);
    a.in = C.T;
    a.out = C.q_c;                  // real products Re(conj g . S) [J][n][n] as floats
    a.add1 = (const float2*)g;
    CHK(run_col(p, C, COL_PAD_FFT_GPROD, a, J, s));
    const int slot = tbegin(p, KC_COIL_SUM, s);
    hipLaunchKernelGGL(k_coil_sum_real, dim3(grid_for(C.cplane())), dim3(kThreads), 0, s,
                       (const float*)C.q_c, gP_out, J, (int)C.cplane());
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

int nlinv_image(nlinv_plan p, const nlinv_c32* rho, const nlinv_c32* c, nlinv_c32* image_out, void* stream) {
    if (!p || !rho || !c || !image_out || !aligned(rho) || !aligned(c) || !aligned(image_out)) return NLINV_EINVAL;
    Class& C = *class0(p);
    const hipStream_t s = (hipStream_t)stream;
    const int slot = tbegin(p, KC_IMAGE, s);
    hipLaunchKernelGGL(k_image, dim3(grid_for(C.rplane())), dim3(kThreads), 0, s, (const float2*)rho,
                       (const float2*)c, (float2*)image_out, (const int*)nullptr, (const int*)nullptr,
                       p->dims[0].ncoils, 1, (int)C.rplane(), (const float*)nullptr);
    hipError_t e = hipGetLastError();
    tend(p, slot, s);
    HIPCHK(e);
    return NLINV_OK;
}

int nlinv_irgnm_solve(nlinv_plan p, const nlinv_c32* y, const float* P, const nlinv_irgnm_params* prm,
                      nlinv_c32* rho_inout, nlinv_c32* chat_inout, const nlinv_c32* rho_ref,
                      const nlinv_c32* chat_ref, nlinv_c32* image_out, double* stats_out, void* stream) {
    if (!p) return NLINV_EINVAL;
    CHK(check_params(prm));
    if (p->dims.size() != 1) return NLINV_EINVAL;
    nlinv_frame f{};
    f.y = y;
    f.P = P;
    f.rho = rho_inout;
    f.chat = chat_inout;
    f.rho_ref = rho_ref;
    f.chat_ref = chat_ref;
    f.image = image_out;
    f.stats = stats_out;
    CHK(validate_frames(p, &f, 1));
    return solve_all(p, &f, *prm, (hipStream_t)stream);
}

int nlinv_irgnm_solve_batch(nlinv_plan p, const nlinv_frame* frames, const nlinv_irgnm_params* prm,
                            void* stream) {
    if (!p) return NLINV_EINVAL;
    CHK(check_params(prm));
    CHK(validate_frames(p, frames, (int)p->dims.size()));
    return solve_all(p, frames, *prm, (hipStream_t)stream);
}

int nlinv_irgnm_solve_series(nlinv_plan p, int32_t count, const nlinv_frame* frames,
                             const nlinv_irgnm_params* prm, void* stream) {
    if (!p || count < 0) return NLINV_EINVAL;
    CHK(check_params(prm));
    if (p->dims.size() != 1) return NLINV_EINVAL;
    CHK(validate_frames(p, frames, count));
    const hipStream_t s = (hipStream_t)stream;
    for (int t = 0; t < count; ++t) {
        nlinv_frame f = frames[t];
        nlinv_irgnm_params q = *prm;
        if (t == 0) {
            CHK(solve_all(p, &f, q, s));
            continue;
        }
        // x0 = x_ref = the previous frame's result, in data units: read from
        // its arrays (x_ref = x0 needs no arrays of its own)
        q.flags |= NLINV_WARM_START;
        f.rho_ref = nullptr;
        f.chat_ref = nullptr;
        const FrameSrc src{(const float2*)frames[t - 1].rho, (const float2*)frames[t - 1].chat};
        CHK(solve_all(p, &f, q, s, &src));
    }
    return NLINV_OK;
}

// ---- implicit derivative of a Gauss-Newton step (Eq. 3) ---------------------

namespace {
struct GnLayout {
    size_t lam_r, lam_c, ref_r, ref_c, yp, out_r, out_c, h_r, h_c, u, w, ones, part, total;
};
GnLayout gn_layout(const nlinv_dims& d) {
    const size_t cn = (size_t)d.ncoils * d.n * d.n * sizeof(float2), rn = (size_t)d.n_om * d.n_om * sizeof(float2);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    GnLayout L{};
    size_t o = 0;
    auto take = [&](size_t b) { const size_t at = o; o += up(b); return at; };
    L.lam_r = take(rn); L.lam_c = take(cn);
    L.ref_r = take(rn); L.ref_c = take(cn);
    L.yp = take(cn);
    L.out_r = take(rn); L.out_c = take(cn);
    L.h_r = take(rn); L.h_c = take(cn);
    L.u = take(cn); L.w = take(cn);
    L.ones = take((size_t)d.n * d.n * sizeof(float) + 8);
    L.part = take(2 * kDotBlocks * sizeof(double));
    L.total = o;
    return L;
}
int axpby(float2* z, float a, const float2* x, float b, const float2* y, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, s, z, a, x, b, y, n);
    HIPCHK(hipGetLastError());
    return NLINV_OK;
}
}  // namespace

size_t nlinv_gn_step_vjp_workspace(nlinv_plan p) {
    if (!p || p->dims.size() != 1) return 0;
    return gn_layout(p->dims[0]).total;
}

int nlinv_gn_step_vjp(nlinv_plan p, const nlinv_c32* rho_n, const nlinv_c32* chat_n, const nlinv_c32* y,
                      const float* P, float alpha, const nlinv_c32* rho_next, const nlinv_c32* chat_next,
                      const nlinv_c32* rho_ref, const nlinv_c32* chat_ref, const nlinv_c32* g_rho,
                      const nlinv_c32* g_chat, int32_t cg_iters, nlinv_c32* grad_y, nlinv_c32* grad_rho_ref,
                      nlinv_c32* grad_chat_ref, float* grad_P, double* grad_alpha, nlinv_c32* grad_rho_n,
                      nlinv_c32* grad_chat_n, void* workspace, size_t workspace_bytes, void* stream) {
    if (!p || p->dims.size() != 1 || !(alpha > 0.f) || cg_iters < 0 || cg_iters > kMaxCG) return NLINV_EINVAL;
    if ((grad_rho_n == nullptr) != (grad_chat_n == nullptr)) return NLINV_EINVAL;
    if (grad_rho_n && (!aligned(grad_rho_n) || !aligned(grad_chat_n))) return NLINV_EINVAL;
    const void* need[] = {rho_n, chat_n, y, P, rho_next, chat_next, rho_ref, chat_ref, g_rho, g_chat, workspace};
    for (const void* q : need)
        if (!q || !aligned(q)) return NLINV_EINVAL;
    const void* opt[] = {grad_y, grad_rho_ref, grad_chat_ref, grad_P, grad_alpha};
    for (const void* q : opt)
        if (q && !aligned(q) && q != (const void*)grad_alpha) return NLINV_EINVAL;
    if (grad_alpha && ((uintptr_t)grad_alpha & 7)) return NLINV_EINVAL;
    if ((grad_rho_ref == nullptr) != (grad_chat_ref == nullptr)) return NLINV_EINVAL;
    const nlinv_dims& d = p->dims[0];
    const GnLayout L = gn_layout(d);
    if (workspace_bytes < L.total) return NLINV_EINVAL;
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    auto W = [&](size_t off) { return reinterpret_cast<float2*>(ws + off); };
    const hipStream_t s = (hipStream_t)stream;
    const long long cn = (long long)d.ncoils * d.n * d.n, rn = (long long)d.n_om * d.n_om;
    const float2 *xr = (const float2*)rho_n, *xc = (const float2*)chat_n;
    // lambda = N_alpha^{-1} g by one Newton step of the solve on data whose
    // residual vanishes (y' = F(x_n), no scaling) towards x_ref' = x_n + g/alpha:
    // its right-hand side is -alpha (x_n - x_ref') = g, so it returns x_n + lambda
    CHK(nlinv_forward(p, rho_n, chat_n, P, (nlinv_c32*)W(L.yp), nullptr, stream));
    CHK(axpby(W(L.ref_r), 1.f, xr, 1.f / alpha, (const float2*)g_rho, rn, s));
    CHK(axpby(W(L.ref_c), 1.f, xc, 1.f / alpha, (const float2*)g_chat, cn, s));
    HIPCHK(hipMemcpyAsync(W(L.out_r), xr, rn * sizeof(float2), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(W(L.out_c), xc, cn * sizeof(float2), hipMemcpyDeviceToDevice, s));
    nlinv_irgnm_params prm{1, cg_iters, alpha, 1.f, 0.f, 0.f, NLINV_WARM_START};
    nlinv_frame f{};
    f.y = (const nlinv_c32*)W(L.yp);
    f.P = P;
    f.rho = (nlinv_c32*)W(L.out_r);
    f.chat = (nlinv_c32*)W(L.out_c);
    f.rho_ref = (const nlinv_c32*)W(L.ref_r);
    f.chat_ref = (const nlinv_c32*)W(L.ref_c);
    CHK(solve_all(p, &f, prm, s));
    CHK(axpby(W(L.lam_r), 1.f, W(L.out_r), -1.f, xr, rn, s));
    CHK(axpby(W(L.lam_c), 1.f, W(L.out_c), -1.f, xc, cn, s));
    const nlinv_c32 *lam_r = (const nlinv_c32*)W(L.lam_r), *lam_c = (const nlinv_c32*)W(L.lam_c);
    // dL/dy = DF lambda (kept in the data-sized scratch when grad_y is not wanted
    // but the linearisation point's gradient is)
    nlinv_c32* dfl = grad_y ? grad_y : (nlinv_c32*)W(L.yp);
    if (grad_y || grad_rho_n) CHK(nlinv_deriv(p, rho_n, chat_n, nullptr, P, lam_r, lam_c, dfl, stream));
    // dL/dx_ref = alpha lambda
    if (grad_rho_ref) {
        CHK(axpby((float2*)grad_rho_ref, alpha, W(L.lam_r), 0.f, nullptr, rn, s));
        CHK(axpby((float2*)grad_chat_ref, alpha, W(L.lam_c), 0.f, nullptr, cn, s));
    }
    // dL/dalpha = -Re<lambda, x_{n+1} - x_ref>
    if (grad_alpha) {
        CHK(axpby(W(L.h_r), 1.f, (const float2*)rho_next, -1.f, (const float2*)rho_ref, rn, s));
        CHK(axpby(W(L.h_c), 1.f, (const float2*)chat_next, -1.f, (const float2*)chat_ref, cn, s));
        double* part = reinterpret_cast<double*>(ws + L.part);
        hipLaunchKernelGGL(k_dot_re, dim3(kDotBlocks), dim3(kThreads), 0, s, (const float2*)W(L.lam_r),
                           (const float2*)W(L.h_r), rn, part);
        hipLaunchKernelGGL(k_dot_re, dim3(kDotBlocks), dim3(kThreads), 0, s, (const float2*)W(L.lam_c),
                           (const float2*)W(L.h_c), cn, part + kDotBlocks);
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, (const double*)part, 2 * kDotBlocks, -1.0,
                           grad_alpha);
        HIPCHK(hipGetLastError());
    }
    // dL/dP = Re sum_j conj(u_j) (y_j - 2 P w_j), u = A lambda, w = A (x_{n+1} - x_n / 2),
    // A = DF at x_n with P = 1
    if (grad_P) {
        float* ones = reinterpret_cast<float*>(ws + L.ones);
        const long long nn = (long long)d.n * d.n;
        hipLaunchKernelGGL(k_fill, dim3(grid_for((nn + 1) / 2)), dim3(kThreads), 0, s, reinterpret_cast<float2*>(ones),
                           (nn + 1) / 2, make_float2(1.f, 1.f));
        HIPCHK(hipGetLastError());
        CHK(axpby(W(L.h_r), 1.f, (const float2*)rho_next, -0.5f, xr, rn, s));
        CHK(axpby(W(L.h_c), 1.f, (const float2*)chat_next, -0.5f, xc, cn, s));
        CHK(nlinv_deriv(p, rho_n, chat_n, nullptr, ones, lam_r, lam_c, (nlinv_c32*)W(L.u), stream));
        CHK(nlinv_deriv(p, rho_n, chat_n, nullptr, ones, (const nlinv_c32*)W(L.h_r), (const nlinv_c32*)W(L.h_c),
                        (nlinv_c32*)W(L.w), stream));
        hipLaunchKernelGGL(k_gn_grad_P, dim3(grid_for(nn)), dim3(kThreads), 0, s, (const float2*)W(L.u),
                           (const float2*)y, (const float2*)W(L.w), P, grad_P, d.ncoils, nn);
        HIPCHK(hipGetLastError());
    }
    // dL/dx_n = DF_lambda^H (y - F(x_n) - DF dx) - DF_dx^H (DF lambda): the step's
    // dependence on its linearisation point (F bilinear: DF_h k = DF_k h, and
    // the normal equations' N lambda = g cancel the direct terms);
    // y - F(x_n) - DF dx = y - DF (x_{n+1} - x_n / 2)
    if (grad_rho_n) {
        CHK(axpby(W(L.ref_r), 1.f, (const float2*)rho_next, -0.5f, xr, rn, s));
        CHK(axpby(W(L.ref_c), 1.f, (const float2*)chat_next, -0.5f, xc, cn, s));
        CHK(nlinv_deriv(p, rho_n, chat_n, nullptr, P, (const nlinv_c32*)W(L.ref_r), (const nlinv_c32*)W(L.ref_c),
                        (nlinv_c32*)W(L.u), stream));
        CHK(axpby(W(L.u), 1.f, (const float2*)y, -1.f, W(L.u), cn, s));              // linearised residual
        CHK(nlinv_adjoint(p, lam_r, lam_c, nullptr, P, (const nlinv_c32*)W(L.u), (nlinv_c32*)W(L.ref_r),
                          (nlinv_c32*)W(L.ref_c), stream));                          // DF_lambda^H (...)
        CHK(axpby(W(L.h_r), 1.f, (const float2*)rho_next, -1.f, xr, rn, s));        // dx
        CHK(axpby(W(L.h_c), 1.f, (const float2*)chat_next, -1.f, xc, cn, s));
        CHK(nlinv_adjoint(p, (const nlinv_c32*)W(L.h_r), (const nlinv_c32*)W(L.h_c), nullptr, P, dfl,
                          (nlinv_c32*)W(L.out_r), (nlinv_c32*)W(L.out_c), stream));  // DF_dx^H (DF lambda)
        CHK(axpby((float2*)grad_rho_n, 1.f, W(L.ref_r), -1.f, W(L.out_r), rn, s));
        CHK(axpby((float2*)grad_chat_n, 1.f, W(L.ref_c), -1.f, W(L.out_c), cn, s));
    }
    return NLINV_OK;
}

// ---- host-side check of the launch arguments ----------------------------------

int nlinv_check_launch_args(int32_t n, int32_t n_om, int32_t ncoils, int32_t nframes, int32_t newton, int32_t cg,
                            int32_t drop_mode, int64_t* launches, int32_t* first_bad) {
    if (!launches || !first_bad || nframes < 1 || nframes > 64 || newton < 0 || newton > kMaxNewton || cg < 0 ||
        cg > kMaxCG)
        return NLINV_EINVAL;
    nlinv_dims d{n, n_om, ncoils, 220.f, 32.f};
    CHK(check_dims(d));
    // a plan whose device pointers are placeholders: in a dry run they are
    // never dereferenced and no HIP call is made
    nlinv_plan_s pl;
    pl.dry_run = true;
    pl.dims.assign((size_t)nframes, d);
    Class C;
    C.n = n;
    C.m = n_om;
    C.lo = n / 2 - n_om / 2;
    {
        const int h = band_half(n, 220.0, 32.0);
        C.kb = 2 * h;
        C.kb_lo = n / 2 - h;
    }
    C.tilew = plane_tile_width(n);
    for (int f = 0; f < nframes; ++f) {
        C.frames.push_back(f);
        C.J.push_back(ncoils);
        C.plane0.push_back(C.nplanes);
        C.nplanes += ncoils;
        C.nframes += 1;
    }
    uintptr_t fake = 0x10000;
    auto ptr = [&](auto*& q) { q = reinterpret_cast<std::remove_reference_t<decltype(q)>>(fake += 0x10000); };
    ptr(C.plane_frame); ptr(C.frame_plane0); ptr(C.frame_planes); ptr(C.tw); ptr(C.winv); ptr(C.winv_t);
    ptr(C.x_c); ptr(C.x_r); ptr(C.dx_r); ptr(C.r_c); ptr(C.r_r); ptr(C.p_c); ptr(C.p_r); ptr(C.q_c); ptr(C.q_r);
    ptr(C.xr_c); ptr(C.xr_r); ptr(C.y); ptr(C.P); ptr(C.c); ptr(C.T); ptr(C.aux); ptr(C.partial); ptr(C.partial2);
    ptr(C.part_p);
    if (C.kb < C.n) ptr(C.T2);
    ptr(C.sc.rr); ptr(C.sc.a); ptr(C.sc.beta); ptr(C.sc.brk); ptr(C.sc.s); ptr(C.sc.inv_s); ptr(C.sc.stats);
    ptr(C.sc.inert);
    C.sc.nframes = C.nframes;
    C.sc.stats_len = kStatsCap;
    const long long cn = C.cplane(), rn = C.rplane();
    make_geom(C.geom, C.nplanes, C.nframes, cn, rn, true, C.plane_frame);
    make_geom(C.geomC, C.nplanes, C.nframes, cn, rn, false, C.plane_frame);
    for (int m = 0; m < kColModes; ++m) C.colv[m] = default_col_variant(n, col_mode_on_band(m) ? C.kb : n);
    for (int& v : C.rowv) v = default_row_variant(n);
    // a planted omission (tests): the tuner's launch of column mode drop_mode
    // loses its last operand set, as a dropped argument line would
    pl.classes.push_back(C);
    Class& K = pl.classes[0];
    pl.loc.assign((size_t)nframes, {0, 0});
    nlinv_irgnm_params prm{newton, cg, 1.f, 0.5f, 0.f, 100.f, NLINV_USE_GRAPH};
    int st = enqueue_newton(&pl, prm, nullptr);
    // the tuner's representative launch of every mode
    const int col_modes[] = {COL_WINV_IFFT_CROP, COL_PUPD_WINV_IFFT_CROP, COL_P_IFFT_CROP, COL_PAD_FFT_P,
                             COL_RESID_P_IFFT, COL_PAD_FFT_P2_IFFT, COL_PAD_FFT_WINV_ADD, COL_PAD_FFT_WINV_CG_UPD};
    for (int mode : col_modes) {
        ColArgs a = tune_col_args(&pl, K, mode);
        if (mode == drop_mode) {   // what a swallowed argument line leaves
            a.cg_a = nullptr;
            a.r_in = nullptr;
            a.add1 = nullptr;
            a.winv = nullptr;
            a.P = nullptr;
        }
        const int s2 = run_col(&pl, K, mode, a, K.nplanes, nullptr);
        if (st == NLINV_OK) st = s2;
    }
    for (int mode : {ROW_CACHE, ROW_FWD, ROW_DERIV, ROW_ADJ}) {
        const int s2 = run_row(&pl, K, mode, tune_row_args(K, mode), nullptr);
        if (st == NLINV_OK) st = s2;
    }
    // the tuner's whole-plane normal operator and its coil sum, and a
    // whole-plane CG iteration (grids that have them)
    if (plane_kernel_size(n)) {
        int s2 = seq_normal_plane(&pl, K, single_frame(K, K.J[0]), K.x_r, K.c, K.P, 0.5f, K.p_r, K.y, K.q_r,
                                  K.q_c, nullptr);
        if (st == NLINV_OK) st = s2;
        s2 = seq_cg_iteration_plane(&pl, K, 0, 1, 1, 2, 0.5f, nullptr);
        if (st == NLINV_OK) st = s2;
    }
    *launches = pl.dry_launches;
    *first_bad = pl.dry_first_bad;
    return st;
}

int nlinv_plan_autotune(nlinv_plan p, void* stream) {
    if (!p) return NLINV_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    const std::string arch = arch_name(p->device);
    const char* path = std::getenv("NLINV_TUNE_CACHE");
    // cache lines: arch n planes kb <kColModes column variants> <kRowModes row variants>
    // <normal operator form> <CG iteration form> <streaming intermediates>
    std::map<std::string, std::vector<int>> cache;
    if (path) {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string a;
            int n, np, kb;
            if (!(ls >> a >> n >> np >> kb)) continue;
            std::vector<int> v;
            int x;
            while (ls >> x) v.push_back(x);
            if ((int)v.size() != kColModes + kRowModes + 3) continue;
            std::ostringstream k;
            k << a << ' ' << n << ' ' << np << ' ' << kb;
            cache[k.str()] = v;
        }
    }
    bool changed = false;
    for (Class& C : p->classes) {
        std::ostringstream k;
        k << arch << ' ' << C.n << ' ' << C.nplanes << ' ' << C.kb;
        auto it = cache.find(k.str());
        bool ok = it != cache.end();
        if (ok) {
            for (int i = 0; i < kColModes + kRowModes; ++i)
                ok = ok && (i < kColModes ? col_ok_cols(C.n, col_mode_on_band(i) ? C.kb : C.n, it->second[i])
                                          : row_ok(C.n, it->second[i]));
            for (int i = 0; i < 2; ++i) {
                const int nf = it->second[kColModes + kRowModes + i];
                ok = ok && (nf == 0 || (nf == 1 && plane_kernel_size(C.n)));
            }
            const int st = it->second[kColModes + kRowModes + 2];
            ok = ok && (st == 0 || st == 1);
        }
        if (ok) {
            for (int i = 0; i < kColModes; ++i) C.colv[i] = it->second[i];
            for (int i = 0; i < kRowModes; ++i) C.rowv[i] = it->second[kColModes + i];
            C.normal_form = it->second[kColModes + kRowModes];
            C.cg_form = it->second[kColModes + kRowModes + 1];
            C.stream = it->second[kColModes + kRowModes + 2];
            continue;
        }
        CHK(tune_class(p, C, s));
        std::vector<int> v(C.colv, C.colv + kColModes);
        v.insert(v.end(), C.rowv, C.rowv + kRowModes);
        v.push_back(C.normal_form);
        v.push_back(C.cg_form);
        v.push_back(C.stream);
        cache[k.str()] = v;
        changed = true;
    }
    CHK(drop_graph(p));   // variants are baked into a captured graph
    if (path && changed) {
        std::ofstream o(path);
        for (auto& kv : cache) {
            o << kv.first;
            for (int x : kv.second) o << ' ' << x;
            o << '\n';
        }
    }
    return NLINV_OK;
}

int nlinv_plan_variant(nlinv_plan p, int32_t n, int32_t* col_variant, int32_t* row_variant) {
    if (!p || !col_variant || !row_variant) return NLINV_EINVAL;
    for (Class& C : p->classes)
        if (C.n == n) {
            *col_variant = C.colv[COL_PAD_FFT_P2_IFFT];
            *row_variant = C.rowv[ROW_DERIV];
            return NLINV_OK;
        }
    *col_variant = *row_variant = -1;
    return NLINV_EINVAL;
}

int nlinv_plan_normal_form(nlinv_plan p, int32_t n, int32_t* form) {
    if (!p || !form) return NLINV_EINVAL;
    for (Class& C : p->classes)
        if (C.n == n) {
            *form = C.normal_form;
            return NLINV_OK;
        }
    *form = -1;
    return NLINV_EINVAL;
}

int nlinv_plan_set_normal_form(nlinv_plan p, int32_t n, int32_t form) {
    if (!p || form < 0 || form > 1 || (form == 1 && !plane_kernel_size(n))) return NLINV_EINVAL;
    bool found = false;
    for (Class& C : p->classes)
        if (C.n == n) {
            C.normal_form = form;
            found = true;
        }
    return found ? NLINV_OK : NLINV_EINVAL;
}

int nlinv_plan_cg_form(nlinv_plan p, int32_t n, int32_t* form) {
    if (!p || !form) return NLINV_EINVAL;
    for (Class& C : p->classes)
        if (C.n == n) {
            *form = C.cg_form;
            return NLINV_OK;
        }
    *form = -1;
    return NLINV_EINVAL;
}

int nlinv_plan_set_cg_form(nlinv_plan p, int32_t n, int32_t form) {
    if (!p || form < 0 || form > 1 || (form == 1 && !plane_kernel_size(n))) return NLINV_EINVAL;
    bool found = false;
    for (Class& C : p->classes)
        if (C.n == n) {
            C.cg_form = form;
            found = true;
        }
    if (!found) return NLINV_EINVAL;
    CHK(drop_graph(p));   // the form is baked into a captured graph
    return NLINV_OK;
}

int nlinv_plan_streaming(nlinv_plan p, int32_t n, int32_t* on) {
    if (!p || !on) return NLINV_EINVAL;
    for (Class& C : p->classes)
        if (C.n == n) {
            *on = C.stream;
            return NLINV_OK;
        }
    *on = -1;
    return NLINV_EINVAL;
}

int nlinv_plan_set_streaming(nlinv_plan p, int32_t n, int32_t on) {
    if (!p || on < 0 || on > 1) return NLINV_EINVAL;
    bool found = false;
    for (Class& C : p->classes)
        if (C.n == n) {
            C.stream = on;
            found = true;
        }
    if (!found) return NLINV_EINVAL;
    CHK(drop_graph(p));   // the launch arguments are baked into a captured graph
    return NLINV_OK;
}

int nlinv_plan_band(nlinv_plan p, int32_t n, int32_t* kb, int32_t* kb_lo) {
    if (!p || !kb || !kb_lo) return NLINV_EINVAL;
    for (Class& C : p->classes)
        if (C.n == n) {
            *kb = C.kb;
            *kb_lo = C.kb_lo;
            return NLINV_OK;
        }
    *kb = *kb_lo = -1;
    return NLINV_EINVAL;
}

int nlinv_plan_set_variant(nlinv_plan p, int32_t n, int32_t col_variant, int32_t row_variant) {
    if (!p) return NLINV_EINVAL;
    if (!col_ok(n, col_variant) || !row_ok(n, row_variant)) return NLINV_EINVAL;
    bool found = false;
    for (Class& C : p->classes)
        if (C.n == n) {
            for (int& v : C.colv) v = col_variant;
            for (int& v : C.rowv) v = row_variant;
            found = true;
        }
    if (!found) return NLINV_EINVAL;
    CHK(drop_graph(p));
    return NLINV_OK;
}

int nlinv_plan_timing_enable(nlinv_plan p, int32_t kclass, int32_t enable) {
    if (!p || kclass < 0 || kclass >= KC_NUM || enable < 0) return NLINV_EINVAL;
    if (enable && p->ev.empty()) {
        p->ev.resize(2 * kTimingSlots);
        p->ev_used.assign(kTimingSlots, 0);
        p->ev_class.assign(kTimingSlots, -1);
        p->ev_owner.assign(kTimingSlots, 0);
        // timing-only events: no system-scope fence (cache writeback) at
        // each record, which would stall the kernels around the bracket;
        // their times are read after the stream has been synchronised
        for (auto& e : p->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    p->timing[kclass] = enable != 0;
    p->timing_stride[kclass] = enable > 0 ? enable : 1;
    p->timing_count[kclass] = 0;
    CHK(drop_graph(p));   // a captured graph holds the old brackets
    return NLINV_OK;
}

int nlinv_plan_timing_read(nlinv_plan p, int32_t* launches, double* total_ms) {
    return nlinv_plan_timing_read_class(p, -1, launches, total_ms);
}

int nlinv_plan_timing_read_class(nlinv_plan p, int32_t kclass, int32_t* launches, double* total_ms) {
    if (!p || !launches || !total_ms || kclass < -1 || kclass >= KC_NUM) return NLINV_EINVAL;
    if (p->timing_failed) {
        p->timing_failed = false;
        return NLINV_EHIP;
    }
    int cnt = 0;
    double tot = 0.0;
    for (int k = 0; k < (int)p->ev_used.size(); ++k) {
        if (!p->ev_used[k] || (kclass >= 0 && p->ev_class[k] != kclass)) continue;
        HIPCHK(hipEventSynchronize(p->ev[2 * k + 1]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]));
        tot += ms;
        ++cnt;
        if (p->ev_used[k] == 1) p->ev_used[k] = 0;
    }
    *launches = cnt;
    *total_ms = tot;
    return NLINV_OK;
}

}  // extern "C"

// =============================================================================
// The normal operator without a plan and without allocation
// =============================================================================
//
// nlinv_normal_noalloc runs the kernels of nlinv_normal on workspace taken
// from `scratch`, a static device array of kNoallocScratchBytes: the line-FFT
// twiddles, the inverse Sobolev weight table, the sensitivities (when the
// caller passes none), the coil products and the pass intermediate T.  The
// tables are rebuilt by a kernel at every call (they depend on the frame's
// n, a and l), so a call depends on nothing an earlier call left.  Each GPU
// holds its own copy of the array; calls that overlap on one GPU race on it.

static __device__ __align__(256) unsigned char scratch[NLINV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNoallocScratchBytes = NLINV_NOALLOC_SCRATCH_BYTES;

// Device address of `scratch` on each device, looked up once per device
// with that device current (in host code the array's name is only a
// host-side stand-in and must never be handed to a kernel).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(unsigned char** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return NLINV_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* q = nullptr;
        HIPCHK(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        if (!q) return NLINV_EHIP;
        g_scratch_ptr[dev] = q;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return NLINV_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// tw2[k1][j2] = exp(-2 pi i k1 j2 / n) and 1/w = (1 + a |k|^2)^(-hl) on the
// row-major grid, both evaluated in FP64 and rounded once to FP32 (the
// plan's host tables are made the same way)
__global__ __launch_bounds__(kThreads) void k_noalloc_tables(float2* tw, float* winv, int n, int n1, double a,
                                                             double hl) {
    const int n2 = n / n1;
    const long long tot = (long long)n * n;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const int r = (int)(g / n), c = (int)(g % n);
        const double k0 = (double)(r - n / 2) / n, k1 = (double)(c - n / 2) / n;
        winv[g] = (float)pow(1.0 + a * (k0 * k0 + k1 * k1), -hl);
        if (g < n) {
            const int kk1 = (int)g / n2, j2 = (int)g % n2;
            const double ang = -2.0 * 3.14159265358979323846 * (double)(kk1 * j2) / (double)n;
            tw[g] = make_float2((float)cos(ang), (float)sin(ang));
        }
    }
}

}  // namespace

extern "C" int nlinv_normal_noalloc(const nlinv_dims* dims, const nlinv_c32* rho, const nlinv_c32* chat,
                                    const nlinv_c32* c, const float* P, float alpha, const nlinv_c32* drho,
                                    const nlinv_c32* dchat, nlinv_c32* drho_out, nlinv_c32* dchat_out,
                                    void* stream) {
    if (!dims || !rho || !P || !drho || !dchat || !drho_out || !dchat_out || (!c && !chat)) return NLINV_EINVAL;
    if (!aligned(rho) || !aligned(P) || !aligned(drho) || !aligned(dchat) || !aligned(drho_out) ||
        !aligned(dchat_out) || (c && !aligned(c)) || (chat && !aligned(chat)))
        return NLINV_EINVAL;
    CHK(check_dims(*dims));
    const int n = dims->n, m = dims->n_om, J = dims->ncoils;
    // scratch layout: tw | winv | aux | T | c (c only when the caller gives none)
    const size_t b_tw = round256((size_t)n * sizeof(float2));
    const size_t b_w = round256((size_t)n * n * sizeof(float));
    const size_t b_om = round256((size_t)J * m * m * sizeof(float2));
    const size_t b_T = round256((size_t)J * m * n * sizeof(float2));
    const size_t need = b_tw + b_w + b_om + b_T + (c ? 0 : b_om);
    if (need > kNoallocScratchBytes) return NLINV_ESCRATCH;
    unsigned char* base = nullptr;
    CHK(scratch_ptr(&base));
    const hipStream_t s = (hipStream_t)stream;

    // a plan-shaped description of the frame on the scratch (no allocation:
    // the plan's containers stay empty and timing stays off)
    nlinv_plan_s pl;
    pl.sob_a = dims->sobolev_a;
    pl.sob_hl = 0.5f * dims->sobolev_l;
    Class C;
    C.n = n;
    C.m = m;
    C.lo = n / 2 - m / 2;
    C.kb = n;
    C.kb_lo = 0;
    C.nframes = 1;
    C.nplanes = J;
    C.tilew = plane_tile_width(n);
    C.tw = reinterpret_cast<float2*>(base);
    C.winv = reinterpret_cast<float*>(base + b_tw);
    C.aux = reinterpret_cast<float2*>(base + b_tw + b_w);
    C.T = reinterpret_cast<float2*>(base + b_tw + b_w + b_om);
    C.c = c ? nullptr : reinterpret_cast<float2*>(base + b_tw + b_w + b_om + b_T);
    for (int& v : C.colv) v = default_col_variant(n, n);
    for (int& v : C.rowv) v = default_row_variant(n);

    hipLaunchKernelGGL(k_noalloc_tables, dim3(grid_for((long long)n * n)), dim3(kThreads), 0, s, C.tw, C.winv, n,
                       split_n1(n), (double)pl.sob_a, (double)pl.sob_hl);
    HIPCHK(hipGetLastError());
    const Frames fr = single_frame(C, J);
    const float2* cc = (const float2*)c;
    if (!cc) {
        CHK(seq_coil_maps(&pl, C, fr, (const float2*)chat, C.c, s));
        cc = C.c;
    }
    return seq_normal(&pl, C, fr, (const float2*)rho, cc, P, 0, nullptr, alpha, (const float2*)drho,
                      (const float2*)dchat, (float2*)drho_out, (float2*)dchat_out, s);
}
