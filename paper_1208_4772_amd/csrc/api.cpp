// C ABI of the solver: argument validation, device tables, and the
// per-step launch sequence (CFL reduction, then five stages, each optionally
// preceded by the sensor and the viscous-gradient kernels).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dg.h"
#include "common.hpp"
#include "launch.hpp"
#include "refelem.hpp"

using namespace dg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(DG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// ---- tuning table: the workgroup shape (waves per workgroup) of the FP32
// matrix-core stage kernel per (device architecture, order, precision,
// viscosity), filled by dg_autotune or from a file, applied to new handles
// and to batch groups.  Process-wide, guarded by a mutex.
using TuneKey = std::tuple<std::string, int, int, int>;   // arch, P, precision, av
struct TuneEntry {
    int waves = 0;
    double stage_us = 0.0;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

bool tunable_waves(int w) { return w == 2 || w == 4 || w == 8; }

// "gfx950" from "gfx950:sramecc+:xnack-"
std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a(p.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int tuned_waves(const std::string &arch, int P, int precision, int av) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey(arch, P, precision, av ? 1 : 0));
    return it == g_tune.end() ? 0 : it->second.waves;
}

}  // namespace

int dg::report_error(int code, const std::string &msg) { return fail(code, msg); }

struct dg_mesh {
    DevMesh dm;
    // unique per handle over the process's life (an address can be reused
    // by a later handle; this number is not)
    unsigned long long serial = 0;
    int precision = DG_FP64_PLAIN;
    size_t elem_bytes = 8;
    std::vector<void *> allocs;
    // viscous handles: scratch of a pure rhs evaluation (viscosity [K] then
    // sigma grad U, 2x state) and of dg_viscosity ([K]), separate so that
    // the two calls may run on different streams; allocated at setup
    char *rhs_scratch = nullptr;
    void *visc_scratch = nullptr;
    // recorded at the end of every call that enqueues work on a stream that
    // is not being captured; dg_mesh_destroy waits for it
    hipEvent_t done = nullptr;

    template <typename T>
    int alloc(T **p, size_t count) {
        void *q = nullptr;
        if (count == 0) count = 1;
        const hipError_t e = hipMalloc(&q, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            size_t fr = 0, tot = 0;
            (void)hipMemGetInfo(&fr, &tot);
            return fail(DG_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed (" +
                                       hipGetErrorString(e) + "; device free " + std::to_string(fr) + " of " +
                                       std::to_string(tot) + " bytes)");
        }
        allocs.push_back(q);
        owned_bytes += count * sizeof(T);
        *p = static_cast<T *>(q);
        return DG_OK;
    }
    size_t owned_bytes = 0;
    ~dg_mesh() {
        if (done) (void)hipEventDestroy(done);
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
    // hipGraph of two fused steps (parity 0 then 1), replayed by dg_run
    bool graphs = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    void *graph_U = nullptr, *graph_work = nullptr;

    // per-launch stage-kernel timing (event pairs, reused across calls)
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    double stage_ms = 0.0;
    long stage_launches = 0;

    hipError_t time_begin(hipStream_t st) {
        if (!timing) return hipSuccess;
        if (events_used + 2 > events.size()) {
            for (int n = 0; n < 64; ++n) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                events.push_back(e);
            }
        }
        return hipEventRecord(events[events_used], st);
    }
    hipError_t time_end(hipStream_t st) {
        if (!timing) return hipSuccess;
        hipError_t r = hipEventRecord(events[events_used + 1], st);
        events_used += 2;
        return r;
    }
    // after the stream has synchronised
    hipError_t time_collect() {
        for (size_t n = 0; n + 1 < events_used; n += 2) {
            float ms = 0.f;
            hipError_t r = hipEventElapsedTime(&ms, events[n], events[n + 1]);
            if (r != hipSuccess) return r;
            stage_ms += ms;
            stage_launches += 1;
        }
        events_used = 0;
        return hipSuccess;
    }

    size_t state_count() const { return size_t(dm.K) * kFields * dm.Np; }
    size_t state_bytes() const { return state_count() * elem_bytes; }
    // work layout: R | A | B | Q (2x state, AV) | eps [K] (AV)
    size_t off_R() const { return 0; }
    size_t off_A() const { return align256(state_bytes()); }
    size_t off_B() const { return 2 * align256(state_bytes()); }
    size_t off_Q() const { return 3 * align256(state_bytes()); }
    size_t off_eps() const { return off_Q() + (dm.av ? align256(2 * state_bytes()) : 0); }
    size_t work_bytes() const { return off_eps() + (dm.av ? align256(size_t(dm.K) * elem_bytes) : 0); }
    // mark the end of this call's work on st (not while st is capturing:
    // the event would become a graph node)
    void mark(hipStream_t st) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
            (void)hipEventRecord(done, st);
    }
};

extern "C" {

const char *dg_last_error(void) { return g_err.c_str(); }

int dg_version(void) { return 100; }

int dg_reference_nodes(int P, double *r, double *s) {
    RefOps o;
    if (!build_reference(P, o)) return fail(DG_EINVAL, "order P must be 1..5");
    if (!r || !s) return fail(DG_EINVAL, "null output");
    std::memcpy(r, o.r.data(), sizeof(double) * o.Np);
    std::memcpy(s, o.s.data(), sizeof(double) * o.Np);
    return DG_OK;
}

int dg_face_nodes(int P, int *fmask) {
    RefOps o;
    if (!build_reference(P, o)) return fail(DG_EINVAL, "order P must be 1..5");
    if (!fmask) return fail(DG_EINVAL, "null output");
    std::memcpy(fmask, o.fmask.data(), sizeof(int) * 3 * o.Nfp);
    return DG_OK;
}

int dg_reference_operators(int P, double *Dr, double *Ds, double *LIFT, double *Vinv) {
    RefOps o;
    if (!build_reference(P, o)) return fail(DG_EINVAL, "order P must be 1..5");
    if (Dr) std::memcpy(Dr, o.Dr.data(), sizeof(double) * o.Dr.size());
    if (Ds) std::memcpy(Ds, o.Ds.data(), sizeof(double) * o.Ds.size());
    if (LIFT) std::memcpy(LIFT, o.LIFT.data(), sizeof(double) * o.LIFT.size());
    if (Vinv) std::memcpy(Vinv, o.Vinv.data(), sizeof(double) * o.Vinv.size());
    return DG_OK;
}

int dg_weak_operators(int P, int *ncub, int *ng, double *wq, double *Icub, double *Drc, double *Dsc, double *wg,
                      double *If) {
    WeakOps W;
    if (P < 1 || P > 5 || !build_weak(P, W)) return fail(DG_EINVAL, "order P must be 1..5");
    if (ncub) *ncub = W.ncub;
    if (ng) *ng = W.ng;
    auto put = [](double *dst, const std::vector<double> &v) {
        if (dst) std::memcpy(dst, v.data(), sizeof(double) * v.size());
    };
    put(wq, W.wq);
    put(Icub, W.Icub);
    put(Drc, W.Drc);
    put(Dsc, W.Dsc);
    put(wg, W.wg);
    put(If, W.If);
    return DG_OK;
}

int dg_mesh_setup(const dg_mesh_desc *d, void *stream, dg_mesh **out) {
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(DG_EINVAL, "desc is NULL");
    if (d->P < 1 || d->P > 5) return fail(DG_EINVAL, "order P must be 1..5");
    if (d->K < 1) return fail(DG_EINVAL, "K must be >= 1");
    if (d->precision != DG_FP64_PLAIN && d->precision != DG_FP32 && d->precision != DG_FP32_BF16X3)
        return fail(DG_EINVAL, "precision must be DG_FP64_PLAIN, DG_FP32 or DG_FP32_BF16X3");
    if (!(d->gamma > 1.0)) return fail(DG_EINVAL, "gamma must be > 1");
    if (!(d->cfl > 0.0)) return fail(DG_EINVAL, "cfl must be > 0");
    if (!d->EToE || !d->EToF || !d->bc || !d->x || !d->y) return fail(DG_EINVAL, "null mesh array");
    if (d->av_enable && (!(d->av_kappa > 0.0) || !(d->av_eps0 >= 0.0)))
        return fail(DG_EINVAL, "av_kappa must be > 0 and av_eps0 >= 0");
    if (d->riemann != DG_RIEMANN_LF && d->riemann != DG_RIEMANN_HLLC)
        return fail(DG_EINVAL, "riemann must be DG_RIEMANN_LF or DG_RIEMANN_HLLC");
    if (d->form != DG_FORM_NODAL && d->form != DG_FORM_WEAK)
        return fail(DG_EINVAL, "form must be DG_FORM_NODAL or DG_FORM_WEAK");
    if (d->form == DG_FORM_WEAK && d->av_enable)
        return fail(DG_EINVAL, "the weak form is inviscid: av_enable must be 0");
    if (d->form == DG_FORM_WEAK && d->precision == DG_FP32_BF16X3)
        return fail(DG_EINVAL, "the weak form runs in DG_FP64_PLAIN or DG_FP32");
    const int K = d->K, P = d->P;
    RefOps ref;
    if (!build_reference(P, ref)) return fail(DG_EINVAL, "reference element construction failed");
    const int Np = ref.Np, Nfp = ref.Nfp;
    // the kernels' compile-time face table must agree with the nodes
    for (int f = 0; f < 3; ++f)
        for (int j = 0; j < Nfp; ++j)
            if (ref.fmask[f * Nfp + j] != face_node(P, f, j))
                return fail(DG_EINVAL, "internal: face node table mismatch");
    // connectivity checks (host)
    std::vector<int> nbr(size_t(K) * 3), finfo(K, 0);
    for (long k = 0; k < K; ++k) {
        int info = 0;
        for (int f = 0; f < 3; ++f) {
            const int kn = d->EToE[k * 3 + f], fn = d->EToF[k * 3 + f];
            const int code = d->bc[k * 3 + f];
            if (code < 0 || code > 2)
                return fail(DG_EINVAL, "bc code must be 0, 1 or 2 (element " + std::to_string(k) + ")");
            if (kn < 0 || kn >= K || fn < 0 || fn > 2)
                return fail(DG_EINVAL, "EToE/EToF out of range at element " + std::to_string(k));
            if (code == 0) {
                if (kn == k && fn == f)
                    return fail(DG_EINVAL, "interior face glued to itself at element " + std::to_string(k));
                if (d->EToE[kn * 3 + fn] != k || d->EToF[kn * 3 + fn] != f)
                    return fail(DG_EINVAL, "non-reciprocal connectivity at element " + std::to_string(k));
                if (d->bc[kn * 3 + fn] != 0)
                    return fail(DG_EINVAL, "interior face matched to a boundary face at element " +
                                               std::to_string(k));
            } else if (kn != k || fn != f) {
                return fail(DG_EINVAL, "boundary face must have EToE=k, EToF=f (element " +
                                           std::to_string(k) + ")");
            }
            nbr[k * 3 + f] = kn;
            info |= (fn & 3) << (4 * f);
            info |= (code & 3) << (4 * f + 2);
        }
        finfo[k] = info;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    dg_mesh *m = new dg_mesh();
    {
        static std::atomic<unsigned long long> next_serial{1};
        m->serial = next_serial.fetch_add(1);
    }
    DevMesh &dm = m->dm;
    dm.K = K;
    dm.P = P;
    dm.Np = Np;
    dm.Nfp = Nfp;
    dm.fp32 = d->precision == DG_FP32 || d->precision == DG_FP32_BF16X3;
    dm.bf3 = d->precision == DG_FP32_BF16X3;
    dm.av = d->av_enable != 0;
    dm.riemann = d->riemann;
    dm.weak = d->form == DG_FORM_WEAK;
    dm.gamma = d->gamma;
    dm.cfl = d->cfl;
    for (int c = 0; c < 4; ++c) dm.qinf[c] = d->freestream[c];
    dm.av_s0 = std::isnan(d->av_s0) ? -4.0 * std::log10(double(P)) : d->av_s0;
    dm.av_kappa = d->av_kappa;
    m->precision = d->precision;
    m->elem_bytes = dm.fp32 ? 4 : 8;

    auto cleanup = [&](int code) {
        delete m;
        return code;
    };
    int *nbr_d, *finfo_d, *flag_d, *count_d;
    double *x_d, *y_d, *geo64, *fgeo64, *wmass, *emax64, *ops64, *scal, *partial;
    const size_t nops = ops_size(Np, Nfp);
    int rc = DG_OK;
    if ((rc = m->alloc(&nbr_d, size_t(K) * 3)) || (rc = m->alloc(&finfo_d, size_t(K))) ||
        (rc = m->alloc(&flag_d, 1)) || (rc = m->alloc(&count_d, 4)) ||
        (rc = m->alloc(&x_d, size_t(K) * Np)) || (rc = m->alloc(&y_d, size_t(K) * Np)) ||
        (rc = m->alloc(&geo64, size_t(K) * 4 * Np)) || (rc = m->alloc(&fgeo64, size_t(K) * 9 * Nfp)) ||
        (rc = m->alloc(&wmass, size_t(K) * Np)) || (rc = m->alloc(&emax64, size_t(K))) ||
        (rc = m->alloc(&ops64, nops + size_t(Np) * Np)) || (rc = m->alloc(&scal, S_NSCAL)) ||
        (rc = m->alloc(&partial, size_t(partial_slots(K, P)) * 4 + 4)))
        return cleanup(rc);
    dm.nbr = nbr_d;
    dm.finfo = finfo_d;
    dm.flag = flag_d;
    dm.count = count_d;
    dm.geo64 = geo64;
    dm.fgeo64 = fgeo64;
    dm.wmass = wmass;
    dm.emax64 = emax64;
    dm.ops64 = ops64;
    dm.scal = scal;
    dm.partial = partial;
    dm.npartial = partial_slots(K, P);

    std::vector<double> ops(nops + size_t(Np) * Np);
    std::memcpy(ops.data() + off_Dr(Np, Nfp), ref.Dr.data(), sizeof(double) * Np * Np);
    std::memcpy(ops.data() + off_Ds(Np, Nfp), ref.Ds.data(), sizeof(double) * Np * Np);
    std::memcpy(ops.data() + off_LIFT(Np, Nfp), ref.LIFT.data(), sizeof(double) * Np * 3 * Nfp);
    std::memcpy(ops.data() + off_Vinv(Np, Nfp), ref.Vinv.data(), sizeof(double) * Np * Np);
    std::memcpy(ops.data() + nops, ref.M.data(), sizeof(double) * Np * Np);

#define SETUP_TRY(expr)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            fail(DG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
            return cleanup(DG_EDEVICE);                                                     \
        }                                                                                   \
    } while (0)

    SETUP_TRY(hipMemcpyAsync(nbr_d, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(finfo_d, finfo.data(), sizeof(int) * finfo.size(), hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(x_d, d->x, sizeof(double) * size_t(K) * Np, hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(y_d, d->y, sizeof(double) * size_t(K) * Np, hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemcpyAsync(ops64, ops.data(), sizeof(double) * ops.size(), hipMemcpyHostToDevice, st));
    SETUP_TRY(hipMemsetAsync(count_d, 0, sizeof(int) * 4, st));
    SETUP_TRY(hipMemsetAsync(flag_d, 0, sizeof(int), st));
    SETUP_TRY(launch_reset_scalars(dm, st));
    SETUP_TRY(launch_geometry(dm, x_d, y_d, geo64, fgeo64, wmass, emax64, d->av_eps0, st));
    SETUP_TRY(launch_check_normals(dm, st));
    int counts[4] = {0, 0, 0, 0};
    SETUP_TRY(hipMemcpyAsync(counts, count_d, sizeof(counts), hipMemcpyDeviceToHost, st));
    SETUP_TRY(hipStreamSynchronize(st));
    if (counts[0] > 0) {
        fail(DG_EGEOM, std::to_string(counts[0]) + " nodes with J <= 0 (clockwise or folded elements)");
        return cleanup(DG_EGEOM);
    }
    if (counts[1] > 0) {
        fail(DG_EGEOM, std::to_string(counts[1]) +
                           " interior face nodes whose normal is not minus the neighbour's");
        return cleanup(DG_EGEOM);
    }
    if (!dm.fp32 && !dm.weak && !dm.av) {
        // an FP64 handle whose elements are all straight runs the stage's
        // product on the FP64 matrix cores (k_stage_mfma64)
        int *flags_d;
        if ((rc = m->alloc(&flags_d, size_t(K)))) return cleanup(rc);
        SETUP_TRY(launch_affine_flags(dm, flags_d, st));
        std::vector<int> flags(K);
        SETUP_TRY(hipMemcpyAsync(flags.data(), flags_d, sizeof(int) * K, hipMemcpyDeviceToHost, st));
        SETUP_TRY(hipStreamSynchronize(st));
        if (std::all_of(flags.begin(), flags.end(), [](int f) { return f != 0; })) {
            const size_t nA = mfma64_opsA_values(P);
            double *opsA64_d, *geoA64_d;
            if ((rc = m->alloc(&opsA64_d, nA)) || (rc = m->alloc(&geoA64_d, size_t(K) * 16))) return cleanup(rc);
            SETUP_TRY(launch_pack_affine64(dm, geoA64_d, st));
            std::vector<double> opsA64(nA);
            mfma64_fill_opsA(P, ref.Dr.data(), ref.Ds.data(), ref.LIFT.data(), opsA64.data());
            SETUP_TRY(hipMemcpyAsync(opsA64_d, opsA64.data(), sizeof(double) * nA, hipMemcpyHostToDevice, st));
            // slots of the time-step bound that a run's step-closing stage reduces
            unsigned long long *vmax64_d;
            if ((rc = m->alloc(&vmax64_d, 2 * kVmaxSlots))) return cleanup(rc);
            SETUP_TRY(hipStreamSynchronize(st));
            dm.opsA64 = opsA64_d;
            dm.geoA64 = geoA64_d;
            dm.vmax = vmax64_d;
        }
    }
    if (dm.fp32) {
        float *geo32, *fgeo32, *emax32, *ops32;
        if ((rc = m->alloc(&geo32, size_t(K) * 4 * Np)) || (rc = m->alloc(&fgeo32, size_t(K) * 9 * Nfp)) ||
            (rc = m->alloc(&emax32, size_t(K))) || (rc = m->alloc(&ops32, nops)))
            return cleanup(rc);
        SETUP_TRY(launch_cast(geo64, geo32, size_t(K) * 4 * Np, st));
        SETUP_TRY(launch_cast(fgeo64, fgeo32, size_t(K) * 9 * Nfp, st));
        SETUP_TRY(launch_cast(emax64, emax32, size_t(K), st));
        SETUP_TRY(launch_cast(ops64, ops32, nops, st));
        dm.geo32 = geo32;
        dm.fgeo32 = fgeo32;
        dm.emax32 = emax32;
        dm.ops32 = ops32;
        // matrix-core kernel tables: packed connectivity, affine records for
        // every element, per-node records for curved ones, A operand
        int *conn4_d, *cidx_d, *cpre_d, *flags_d;
        float *geoA_d, *opsA_d;
        const size_t nA = mfma_opsA_floats(P);
        if ((rc = m->alloc(&conn4_d, size_t(K) * 4)) || (rc = m->alloc(&cidx_d, size_t(K))) ||
            (rc = m->alloc(&cpre_d, size_t(K) + 1)) ||
            (rc = m->alloc(&flags_d, size_t(K))) || (rc = m->alloc(&geoA_d, size_t(K) * 16)) ||
            (rc = m->alloc(&opsA_d, nA)))
            return cleanup(rc);
        std::vector<float> opsA(nA);
        mfma_fill_opsA(P, ref.Dr.data(), ref.Ds.data(), ref.LIFT.data(), opsA.data());
        SETUP_TRY(hipMemcpyAsync(opsA_d, opsA.data(), sizeof(float) * nA, hipMemcpyHostToDevice, st));
        if (dm.bf3) {
            const size_t nB = mfma_opsB_words(P);
            unsigned *opsB_d;
            if ((rc = m->alloc(&opsB_d, nB))) return cleanup(rc);
            std::vector<unsigned> opsB(nB);
            mfma_fill_opsB(P, ref.Dr.data(), ref.Ds.data(), ref.LIFT.data(), opsB.data());
            SETUP_TRY(hipMemcpyAsync(opsB_d, opsB.data(), sizeof(unsigned) * nB, hipMemcpyHostToDevice, st));
            SETUP_TRY(hipStreamSynchronize(st));
            dm.opsB = opsB_d;
        }
        SETUP_TRY(launch_affine_flags(dm, flags_d, st));
        std::vector<int> flags(K), cidx(K), cpre(size_t(K) + 1);
        SETUP_TRY(hipMemcpyAsync(flags.data(), flags_d, sizeof(int) * K, hipMemcpyDeviceToHost, st));
        SETUP_TRY(hipStreamSynchronize(st));
        int Kc = 0;
        for (long k = 0; k < K; ++k) {
            cpre[k] = Kc;
            cidx[k] = flags[k] ? -1 : Kc++;
        }
        cpre[K] = Kc;
        std::vector<int> conn4(size_t(K) * 4);
        for (long k = 0; k < K; ++k) {
            conn4[k * 4 + 0] = nbr[k * 3 + 0];
            conn4[k * 4 + 1] = nbr[k * 3 + 1];
            conn4[k * 4 + 2] = nbr[k * 3 + 2];
            conn4[k * 4 + 3] = finfo[k] | (cidx[k] >= 0 ? mfma_curved_bit() : 0);
        }
        SETUP_TRY(hipMemcpyAsync(conn4_d, conn4.data(), sizeof(int) * conn4.size(), hipMemcpyHostToDevice, st));
        float *geoC_d;
        if ((rc = m->alloc(&geoC_d, size_t(Kc) * (4 * Np + 9 * Nfp)))) return cleanup(rc);
        SETUP_TRY(hipMemcpyAsync(cidx_d, cidx.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
        SETUP_TRY(hipMemcpyAsync(cpre_d, cpre.data(), sizeof(int) * (size_t(K) + 1), hipMemcpyHostToDevice, st));
        SETUP_TRY(launch_pack_geometry(dm, cidx_d, geoA_d, geoC_d, st));
        dm.conn4 = conn4_d;
        dm.cidx = cidx_d;
        dm.cpre = cpre_d;
        dm.geoA = geoA_d;
        dm.geoC = geoC_d;
        dm.opsA = opsA_d;
        dm.Kc = Kc;
        unsigned long long *vmax_d;
        if ((rc = m->alloc(&vmax_d, 2 * kVmaxSlots))) return cleanup(rc);
        dm.vmax = vmax_d;
        int dev = 0, ncu = 0;
        SETUP_TRY(hipGetDevice(&dev));
        SETUP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        dm.ncu = ncu > 0 ? ncu : 256;
        // workgroup shape: DG_WAVES_PER_BLOCK if set, else the tuning
        // table's choice for this kind of handle, else the default
        if (const char *e = std::getenv("DG_WAVES_PER_BLOCK")) {
            const int w = std::atoi(e);
            if (tunable_waves(w)) dm.waves_per_block = w;
        }
        if (!dm.waves_per_block && !dm.weak)
            dm.waves_per_block = tuned_waves(device_arch(), dm.P, d->precision, dm.av);
        SETUP_TRY(hipStreamSynchronize(st));
    }
    if (dm.weak) {
        // over-integrated weak form: cubature operators and the per-element
        // tables, computed in FP64 on the device; curved elements are those
        // whose nodal metric terms are not constant
        WeakOps W;
        if (!build_weak(P, W)) {
            fail(DG_EINVAL, "weak-form operator construction failed");
            return cleanup(DG_EINVAL);
        }
        const int NQ = W.ncub, NG = W.ng;
        std::vector<double> wops;
        wops.insert(wops.end(), W.Icub.begin(), W.Icub.end());
        wops.insert(wops.end(), W.Drc.begin(), W.Drc.end());
        wops.insert(wops.end(), W.Dsc.begin(), W.Dsc.end());
        wops.insert(wops.end(), W.wq.begin(), W.wq.end());
        wops.insert(wops.end(), W.If.begin(), W.If.end());
        wops.insert(wops.end(), W.Minv.begin(), W.Minv.end());
        if (wops.size() != weak_ops_size(P)) {
            fail(DG_EINVAL, "internal: weak-form operator table size");
            return cleanup(DG_EINVAL);
        }
        std::vector<double> dsg;
        dsg.insert(dsg.end(), W.Drg.begin(), W.Drg.end());
        dsg.insert(dsg.end(), W.Dsg.begin(), W.Dsg.end());
        dsg.insert(dsg.end(), W.wg.begin(), W.wg.end());
        double *wops_d, *dsg_d, *geoA_d, *geoF_d;
        int *wflags_d, *widx_d;
        if ((rc = m->alloc(&wops_d, wops.size())) || (rc = m->alloc(&dsg_d, dsg.size())) ||
            (rc = m->alloc(&geoA_d, size_t(K) * 5)) || (rc = m->alloc(&geoF_d, size_t(K) * 3 * NG * 3)) ||
            (rc = m->alloc(&wflags_d, size_t(K))) || (rc = m->alloc(&widx_d, size_t(K))))
            return cleanup(rc);
        SETUP_TRY(hipMemcpyAsync(wops_d, wops.data(), sizeof(double) * wops.size(), hipMemcpyHostToDevice, st));
        SETUP_TRY(hipMemcpyAsync(dsg_d, dsg.data(), sizeof(double) * dsg.size(), hipMemcpyHostToDevice, st));
        dm.wops64 = wops_d;
        SETUP_TRY(launch_affine_flags(dm, wflags_d, st));
        std::vector<int> wflags(K), widx(K);
        SETUP_TRY(hipMemcpyAsync(wflags.data(), wflags_d, sizeof(int) * K, hipMemcpyDeviceToHost, st));
        SETUP_TRY(hipStreamSynchronize(st));
        int Kc = 0;
        for (long k = 0; k < K; ++k) widx[k] = wflags[k] ? -1 : Kc++;
        SETUP_TRY(hipMemcpyAsync(widx_d, widx.data(), sizeof(int) * K, hipMemcpyHostToDevice, st));
        dm.widx = widx_d;
        dm.wKc = Kc;
        double *geoC_d, *minv_d, *work_d;
        if ((rc = m->alloc(&geoC_d, size_t(Kc) * NQ * 4 + 1)) || (rc = m->alloc(&minv_d, size_t(Kc) * Np * Np + 1)) ||
            (rc = m->alloc(&work_d, size_t(Kc) * Np * Np + 1)))
            return cleanup(rc);
        SETUP_TRY(hipMemsetAsync(count_d, 0, sizeof(int) * 4, st));
        SETUP_TRY(launch_weak_geometry(dm, x_d, y_d, dsg_d, dsg_d + W.Drg.size(), dsg_d + 2 * W.Drg.size(), geoA_d,
                                       geoF_d, geoC_d, minv_d, work_d, st));
        int wc[4] = {0, 0, 0, 0};
        SETUP_TRY(hipMemcpyAsync(wc, count_d, sizeof(wc), hipMemcpyDeviceToHost, st));
        SETUP_TRY(hipStreamSynchronize(st));
        if (wc[0] > 0 || wc[2] > 0) {
            fail(DG_EGEOM, std::to_string(wc[0]) + " cubature points with J <= 0, " + std::to_string(wc[2]) +
                               " mass matrices not positive definite");
            return cleanup(DG_EGEOM);
        }
        dm.wgeoA64 = geoA_d;
        dm.wgeoF64 = geoF_d;
        dm.wgeoC64 = geoC_d;
        dm.wminv64 = minv_d;
        if (dm.fp32) {
            float *o32, *a32, *f32, *c32, *m32;
            const size_t nC = size_t(Kc) * NQ * 4, nM = size_t(Kc) * Np * Np;
            if ((rc = m->alloc(&o32, wops.size())) || (rc = m->alloc(&a32, size_t(K) * 5)) ||
                (rc = m->alloc(&f32, size_t(K) * 3 * NG * 3)) || (rc = m->alloc(&c32, nC + 1)) ||
                (rc = m->alloc(&m32, nM + 1)))
                return cleanup(rc);
            SETUP_TRY(launch_cast(wops_d, o32, wops.size(), st));
            SETUP_TRY(launch_cast(geoA_d, a32, size_t(K) * 5, st));
            SETUP_TRY(launch_cast(geoF_d, f32, size_t(K) * 3 * NG * 3, st));
            SETUP_TRY(launch_cast(geoC_d, c32, nC, st));
            SETUP_TRY(launch_cast(minv_d, m32, nM, st));
            dm.wops32 = o32;
            dm.wgeoA32 = a32;
            dm.wgeoF32 = f32;
            dm.wgeoC32 = c32;
            dm.wminv32 = m32;
            if (Kc == 0) {
                // every element straight: the stage runs on the matrix cores
                std::vector<float> fr(weak_mfma_opsA_values(P));
                weak_mfma_fill_opsA(P, W.Icub.data(), W.Drc.data(), W.Dsc.data(), W.If.data(), W.Minv.data(),
                                    fr.data());
                float *fa;
                if ((rc = m->alloc(&fa, fr.size()))) return cleanup(rc);
                SETUP_TRY(hipMemcpyAsync(fa, fr.data(), sizeof(float) * fr.size(), hipMemcpyHostToDevice, st));
                SETUP_TRY(hipStreamSynchronize(st));
                dm.wopsA = fa;
            }
        }
        SETUP_TRY(hipStreamSynchronize(st));
    }
    if (dm.av) {
        char *rs;
        const size_t rbytes = align256(size_t(K) * m->elem_bytes) + 2 * m->state_bytes();
        if ((rc = m->alloc(&rs, rbytes))) return cleanup(rc);
        m->rhs_scratch = rs;
        if (dm.fp32) {
            float *vs;
            if ((rc = m->alloc(&vs, size_t(K)))) return cleanup(rc);
            m->visc_scratch = vs;
        }
    }
    SETUP_TRY(hipEventCreateWithFlags(&m->done, hipEventDisableTiming));
    *out = m;
    g_err.clear();
    return DG_OK;
#undef SETUP_TRY
}

int dg_mesh_destroy(dg_mesh *m) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    // the handle's last enqueued work (other streams are not waited for)
    if (m->done) (void)hipEventSynchronize(m->done);
    delete m;
    return DG_OK;
}

int dg_buffer_bytes(const dg_mesh *m, size_t *state_bytes, size_t *work_bytes) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (state_bytes) *state_bytes = m->state_bytes();
    if (work_bytes) *work_bytes = m->work_bytes();
    return DG_OK;
}

static int check_ptr(const void *p, const char *what) {
    if (!p) return fail(DG_EINVAL, std::string(what) + " is NULL");
    return DG_OK;
}

// sensor + viscous gradient of state U into the work buffer
static int av_prepare(dg_mesh *m, const void *U, char *work, hipStream_t st) {
    void *eps = work + m->off_eps();
    void *Q = work + m->off_Q();
    HIP_TRY(launch_sensor(m->dm, U, eps, st));
    HIP_TRY(launch_avgrad(m->dm, U, eps, Q, st));
    return DG_OK;
}

int dg_rhs(dg_mesh *m, const void *U, void *rhs, double t, void *stream) {
    (void)t;
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(rhs, "rhs")) return rc;
    if (U == rhs) return fail(DG_EINVAL, "U and rhs must not alias");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m->dm.av) {
        // the handle's own scratch for the viscosity and sigma grad U
        char *base = m->rhs_scratch;
        void *eps = base;
        void *Q = base + align256(size_t(m->dm.K) * m->elem_bytes);
        HIP_TRY(launch_sensor(m->dm, U, eps, st));
        HIP_TRY(launch_avgrad(m->dm, U, eps, Q, st));
        HIP_TRY(launch_stage(m->dm, U, nullptr, nullptr, rhs, 0, eps, Q, st));
    } else {
        HIP_TRY(launch_stage(m->dm, U, nullptr, nullptr, rhs, 0, nullptr, nullptr, st));
    }
    m->mark(st);
    return DG_OK;
}

// One step: dt reduction on the device, then five stages ping-ponging
// U -> A -> B -> A -> B -> U so that no stage writes the buffer whose face
// traces other workgroups are still reading.
// One step of a run of an FP64 handle on the FP64 matrix cores: dt from
// the bound the previous step's last stage (or the run's first bound) left
// in the slots, then the five stages, the last of which reduces the next
// bound.  The same sums as launch_cfl and the stages, so the same bits.
static int step_fused64(dg_mesh *m, void *U, void *work, double dt, hipStream_t st) {
    char *w = static_cast<char *>(work);
    void *R = w + m->off_R();
    void *A = w + m->off_A();
    void *B = w + m->off_B();
    void *in[5] = {U, A, B, A, B};
    void *out[5] = {A, B, A, B, U};
    HIP_TRY(launch_dt_slots64(m->dm, dt, st));
    for (int s = 0; s < 5; ++s) {
        HIP_TRY(m->time_begin(st));
        HIP_TRY(launch_stage_mfma64(m->dm, in[s], out[s], R, nullptr, s, s == 4, st));
        HIP_TRY(m->time_end(st));
    }
    return DG_OK;
}

static int step_impl(dg_mesh *m, void *U, void *work, double dt, hipStream_t st, int fused_parity = -1) {
    if (fused_parity >= 0 && !m->dm.fp32) return step_fused64(m, U, work, dt, st);
    char *w = static_cast<char *>(work);
    void *R = w + m->off_R();
    void *A = w + m->off_A();
    void *B = w + m->off_B();
    void *Q = m->dm.av ? w + m->off_Q() : nullptr;
    void *eps = m->dm.av ? w + m->off_eps() : nullptr;
    void *in[5] = {U, A, B, A, B};
    void *out[5] = {A, B, A, B, U};
    if (fused_parity >= 0) {
        // matrix-core path: the first stage turns the CFL bound in
        // vmax[parity] into dt and clears vmax[1 - parity]; without
        // viscosity the previous step's last stage left the bound (of this
        // step's state), with viscosity this step's first sensor does (it
        // needs the viscosity of this state)
        unsigned long long *vin = m->dm.vmax + fused_parity * kVmaxSlots;
        unsigned long long *vout = m->dm.vmax + (1 - fused_parity) * kVmaxSlots;
        for (int s = 0; s < 5; ++s) {
            MfmaStep ms;
            ms.dt_fixed = dt;
            if (s == 0) {
                ms.cfl_mode = 1;
                ms.vmax_in = vin;
                ms.vmax_out = vout;
            }
            if (s == 4 && !m->dm.av) {
                ms.cfl_accum = 1;
                ms.vmax_out = vout;
            }
            if (m->dm.av) {
                if (s == 0)
                    HIP_TRY(launch_sensor_cfl(m->dm, in[0], eps, vin, st));
                else
                    HIP_TRY(launch_sensor(m->dm, in[s], eps, st));
                HIP_TRY(launch_avgrad(m->dm, in[s], eps, Q, st));
            }
            HIP_TRY(m->time_begin(st));
            HIP_TRY(launch_stage_mfma(m->dm, in[s], out[s], R, nullptr, s, ms, st, eps, Q));
            HIP_TRY(m->time_end(st));
        }
        return DG_OK;
    }
    if (m->dm.av) {
        if (int rc = av_prepare(m, U, w, st)) return rc;
    }
    HIP_TRY(launch_cfl(m->dm, U, eps, dt, st));
    for (int s = 0; s < 5; ++s) {
        if (m->dm.av && s > 0) {
            if (int rc = av_prepare(m, in[s], w, st)) return rc;
        }
        HIP_TRY(m->time_begin(st));
        HIP_TRY(launch_stage(m->dm, in[s], out[s], R, nullptr, s, eps, Q, st));
        HIP_TRY(m->time_end(st));
    }
    return DG_OK;
}

// Capture two fused steps (parities 0 and 1) of this U/work pair into a
// graph on a private stream; replays then run on the caller's stream.  The
// kernels read dt and the CFL bound from device memory, so the graph stays
// valid from step to step; it is rebuilt when the buffers change.
static int ensure_step_graph(dg_mesh *m, void *U, void *work) {
    if (m->graph_exec && m->graph_U == U && m->graph_work == work) return DG_OK;
    if (m->graph_exec) {
        HIP_TRY(hipGraphExecDestroy(m->graph_exec));
        m->graph_exec = nullptr;
    }
    if (!m->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed));
    int rc0 = step_impl(m, U, work, 0.0, m->cap_stream, 0);
    int rc1 = rc0 ? rc0 : step_impl(m, U, work, 0.0, m->cap_stream, 1);
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(m->cap_stream, &g);
    if (rc1) {
        if (g) (void)hipGraphDestroy(g);
        return rc1;
    }
    if (ec != hipSuccess) return fail(DG_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipError_t ei = hipGraphInstantiate(&m->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(DG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    m->graph_U = U;
    m->graph_work = work;
    return DG_OK;
}

// ---------------------------------------------------------------------------
// step without a caller work buffer: the work lives in a file-scope device
// array of fixed size (one copy per GPU, held until the process ends)
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[DG_STATIC_WORK_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).  The array's name is only a host-side
// stand-in; every use from the host goes through this address.
int scratch_address(void **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DG_EDEVICE, "device id out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(DG_EDEVICE, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DG_OK;
}
}  // namespace

int dg_step_static(dg_mesh *m, void *U, double dt, void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (m->work_bytes() > size_t(DG_STATIC_WORK_BYTES))
        return fail(DG_EINVAL, "work buffer of " + std::to_string(m->work_bytes()) + " bytes exceeds the " +
                                   std::to_string(size_t(DG_STATIC_WORK_BYTES)) + "-byte static work area");
    void *work = nullptr;
    if (int rc = scratch_address(&work)) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = step_impl(m, U, work, dt, st)) return rc;
    m->mark(st);
    return DG_OK;
}

int dg_prolong_operator(int P, int Q, double *I) {
    if (P < 1 || Q > 5 || Q < P) return fail(DG_EINVAL, "need 1 <= P <= Q <= 5");
    if (!I) return fail(DG_EINVAL, "I is NULL");
    RefOps a, b;
    if (!build_reference(P, a) || !build_reference(Q, b)) return fail(DG_EINVAL, "reference element construction failed");
    for (int i = 0; i < b.Np; ++i)
        for (int j = 0; j < a.Np; ++j) {
            double v = 0.0;
            for (int n = 0; n < a.Np; ++n) v += b.V[i * b.Np + n] * a.Vinv[n * a.Np + j];
            I[i * a.Np + j] = v;
        }
    return DG_OK;
}

int dg_prolong(const dg_mesh *from, const void *U_from, const dg_mesh *to, void *U_to, void *stream) {
    if (!from || !to) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U_from, "U_from")) return rc;
    if (int rc = check_ptr(U_to, "U_to")) return rc;
    if (from->dm.K != to->dm.K) return fail(DG_EINVAL, "the two handles have different element counts");
    if (to->dm.P < from->dm.P) return fail(DG_EINVAL, "the target order is lower than the source order");
    if (from->elem_bytes != to->elem_bytes) return fail(DG_EINVAL, "the two handles differ in state precision");
    if (U_from == U_to) return fail(DG_EINVAL, "U_from and U_to must not alias");
    const int np = from->dm.Np, nq = to->dm.Np;
    std::vector<double> I(size_t(np) * nq);
    if (int rc = dg_prolong_operator(from->dm.P, to->dm.P, I.data())) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_prolong(from->dm.K, np, nq, I.data(), to->dm.fp32, U_from, U_to, st));
    const_cast<dg_mesh *>(to)->mark(st);
    return DG_OK;
}

int dg_set_graphs(dg_mesh *m, int enable) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    m->graphs = enable != 0;
    return DG_OK;
}

int dg_step(dg_mesh *m, void *U, void *work, double dt, void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(work, "work")) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (int rc = step_impl(m, U, work, dt, st)) return rc;
    m->mark(st);
    return DG_OK;
}

int dg_run(dg_mesh *m, void *U, void *work, int nsteps, dg_run_stats *stats, void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(work, "work")) return rc;
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(launch_reset_scalars(m->dm, st));
    HIP_TRY(hipMemsetAsync(m->dm.flag, 0, sizeof(int), st));
    HIP_TRY(hipEventRecord(e0, st));
    // fused runs: the bound of each step's state comes from the previous
    // step's last stage (FP32 matrix-core handles; FP64 handles on the FP64
    // matrix cores, which have no viscosity)
    const bool fused64 = !m->dm.fp32 && m->dm.opsA64 && !m->dm.av && !m->dm.weak;
    const bool fused = (m->dm.fp32 && !m->dm.weak) || fused64;
    if (fused && nsteps > 0) {
        if (m->dm.av)
            HIP_TRY(hipMemsetAsync(m->dm.vmax, 0, 2 * kVmaxSlots * sizeof(unsigned long long), st));
        else
            HIP_TRY(launch_cfl_vmax(m->dm, U, m->dm.vmax, st));
    }
    int done = 0;
    if (fused && m->graphs && !m->timing && nsteps >= 2) {
        if (int rc = ensure_step_graph(m, U, work)) return rc;
        for (; done + 2 <= nsteps; done += 2) HIP_TRY(hipGraphLaunch(m->graph_exec, st));
    }
    for (int n = done; n < nsteps; ++n) {
        if (int rc = step_impl(m, U, work, 0.0, st, fused ? (n & 1) : -1)) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
    }
    HIP_TRY(hipEventRecord(e1, st));
    // a fused viscous run checks each step's state in its first sensor: the
    // final state still needs the check
    if (fused && m->dm.av && nsteps > 0) HIP_TRY(launch_cfl_vmax(m->dm, U, m->dm.vmax, st));
    // diagnostics at the end: totals and the residual ||rhs(U)||_inf
    char *w = static_cast<char *>(work);
    void *scratch = w + m->off_A();
    HIP_TRY(launch_totals(m->dm, U, st));
    if (m->dm.av) {
        if (int rc = av_prepare(m, U, w, st)) return rc;
    }
    HIP_TRY(launch_stage(m->dm, U, nullptr, nullptr, scratch, 0, m->dm.av ? w + m->off_eps() : nullptr,
                         m->dm.av ? w + m->off_Q() : nullptr, st));
    HIP_TRY(launch_residual(m->dm, scratch, st));
    double scal[S_NSCAL];
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(scal, m->dm.scal, sizeof(scal), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&flag, m->dm.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    m->mark(st);
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(m->time_collect());
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        stats->steps = nsteps;
        stats->status = flag ? DG_ENONFINITE : DG_OK;
        stats->t = scal[S_T];
        stats->dt_min = nsteps ? scal[S_DTMIN] : 0.0;
        stats->dt_max = scal[S_DTMAX];
        for (int c = 0; c < 4; ++c) {
            stats->totals[c] = scal[S_TOT + c];
            stats->residual[c] = scal[S_RES + c];
        }
        stats->wall_s = ms * 1e-3;
        stats->dof_updates_per_s =
            ms > 0 ? double(m->state_count()) * 5.0 * nsteps / (ms * 1e-3) : 0.0;
    }
    if (flag) return fail(DG_ENONFINITE, "state became non-finite or non-positive (rho or p)");
    return DG_OK;
}

int dg_totals(dg_mesh *m, const void *U, double out[4], void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (!out) return fail(DG_EINVAL, "out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_totals(m->dm, U, st));
    HIP_TRY(hipMemcpyAsync(out, m->dm.scal + S_TOT, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DG_OK;
}

int dg_residual(dg_mesh *m, const void *U, void *work, double out[4], void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(work, "work")) return rc;
    if (!out) return fail(DG_EINVAL, "out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(work);
    void *scratch = w + m->off_A();
    if (m->dm.av) {
        if (int rc = av_prepare(m, U, w, st)) return rc;
    }
    HIP_TRY(launch_stage(m->dm, U, nullptr, nullptr, scratch, 0, m->dm.av ? w + m->off_eps() : nullptr,
                         m->dm.av ? w + m->off_Q() : nullptr, st));
    HIP_TRY(launch_residual(m->dm, scratch, st));
    HIP_TRY(hipMemcpyAsync(out, m->dm.scal + S_RES, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DG_OK;
}

int dg_viscosity(dg_mesh *m, const void *U, double *eps, void *stream) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (!m->dm.av) return fail(DG_EINVAL, "mesh was set up without artificial viscosity");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(eps, "eps")) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (m->dm.fp32) {
        // state-precision scratch, then widen into the caller's doubles
        HIP_TRY(launch_sensor(m->dm, U, m->visc_scratch, st));
        HIP_TRY(launch_eps_to_double(m->dm, m->visc_scratch, eps, st));
    } else {
        HIP_TRY(launch_sensor(m->dm, U, eps, st));
    }
    m->mark(st);
    return DG_OK;
}

int dg_set_kernel_timing(dg_mesh *m, int enable) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    m->timing = enable != 0;
    return DG_OK;
}

int dg_autotune(dg_mesh *m, const void *U, void *work, void *stream, int *waves_per_block, double *stage_us) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (int rc = check_ptr(U, "U")) return rc;
    if (int rc = check_ptr(work, "work")) return rc;
    if (waves_per_block) *waves_per_block = 0;
    if (stage_us) *stage_us = 0.0;
    if (!m->dm.fp32 || m->dm.weak) return DG_OK;   // only the matrix-core kernel has a launch shape to tune
    hipStream_t st = static_cast<hipStream_t>(stream);
    const std::string arch = device_arch();
    // drop captured step graphs, which hold the old launch shape
    auto set_shape = [&](int w) {
        if (m->dm.waves_per_block != w && m->graph_exec) {
            (void)hipGraphExecDestroy(m->graph_exec);
            m->graph_exec = nullptr;
            m->graph_U = m->graph_work = nullptr;
        }
        m->dm.waves_per_block = w;
    };
    if (const int cached = tuned_waves(arch, m->dm.P, m->precision, m->dm.av)) {
        set_shape(cached);
        if (waves_per_block) *waves_per_block = cached;
        return DG_OK;
    }
    // candidates: workgroups of 2, 4 and 8 wavefronts (2, 4 or 8 times the
    // elements one wavefront holds), each timed over the five Runge-Kutta
    // stages of a step as a run executes them (ping-pong buffers), reading
    // U and writing only the work buffer's A, B and R slots (scratch between
    // steps: a step's first stage overwrites them without reading them);
    // a viscous handle's stage kernel reads the viscosity and sigma grad U
    // of U, computed once here into the work buffer
    static const int kCand[3] = {2, 4, 8};
    char *w = static_cast<char *>(work);
    void *A = w + m->off_A(), *B = w + m->off_B(), *R = w + m->off_R();
    void *eps = m->dm.av ? w + m->off_eps() : nullptr;
    void *Q = m->dm.av ? w + m->off_Q() : nullptr;
    const void *in5[5] = {U, A, B, A, B};
    void *out5[5] = {A, B, A, B, A};
    if (m->dm.av) {
        HIP_TRY(launch_sensor(m->dm, U, eps, st));
        HIP_TRY(launch_avgrad(m->dm, U, eps, Q, st));
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int saved = m->dm.waves_per_block;
    int rc = DG_OK;
    // time `reps` launches of candidate c, cycling through the five stages
    // (ms per launch)
    auto time_one = [&](int c, int reps, float *ms_per) -> hipError_t {
        m->dm.waves_per_block = c;
        hipError_t e = launch_stage_mfma(m->dm, in5[0], out5[0], R, nullptr, 0, MfmaStep(), st, eps, Q);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_stage_mfma(m->dm, in5[r % 5], out5[r % 5], R, nullptr, r % 5, MfmaStep(), st, eps, Q);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        *ms_per = ms / reps;
        return e;
    };
    // size the sample to about 2 ms per candidate and round, then take the
    // best of two interleaved rounds so that a hiccup does not decide
    float probe = 0.f;
    hipError_t e = time_one(4, 2, &probe);
    int reps = probe > 0.f ? int(2.0f / probe) : 50;
    reps = reps < 5 ? 5 : (reps > 200 ? 200 : reps);
    reps = (reps + 4) / 5 * 5;   // whole steps
    float best_of[3] = {0.f, 0.f, 0.f};
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
        for (int ci = 0; ci < 3 && e == hipSuccess; ++ci) {
            float ms = 0.f;
            e = time_one(kCand[ci], reps, &ms);
            if (round == 0 || ms < best_of[ci]) best_of[ci] = ms;
        }
    if (e != hipSuccess) rc = fail(DG_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    int best = 0;
    float best_ms = 0.f;
    for (int ci = 0; ci < 3; ++ci)
        if (best == 0 || best_of[ci] < best_ms) {
            best = kCand[ci];
            best_ms = best_of[ci];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    m->dm.waves_per_block = saved;
    if (rc != DG_OK) return rc;
    set_shape(best);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey(arch, m->dm.P, m->precision, m->dm.av ? 1 : 0)] = TuneEntry{best, 1e3 * best_ms};
    }
    if (waves_per_block) *waves_per_block = best;
    if (stage_us) *stage_us = 1e3 * best_ms;
    return DG_OK;
}

int dg_tuning_set(const char *arch, int P, int precision, int av_enable, int waves_per_block) {
    if (!arch || !*arch) return fail(DG_EINVAL, "arch is empty");
    if (P < 1 || P > 5) return fail(DG_EINVAL, "P must be in 1..5");
    if (precision != DG_FP32 && precision != DG_FP32_BF16X3)
        return fail(DG_EINVAL, "only the FP32 matrix-core precisions have a workgroup shape");
    if (!tunable_waves(waves_per_block)) return fail(DG_EINVAL, "waves_per_block must be 2, 4 or 8");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey(arch, P, precision, av_enable ? 1 : 0)] = TuneEntry{waves_per_block, 0.0};
    return DG_OK;
}

int dg_tuning_lookup(const char *arch, int P, int precision, int av_enable, int *waves_per_block) {
    if (!arch || !waves_per_block) return fail(DG_EINVAL, "null argument");
    *waves_per_block = tuned_waves(arch, P, precision, av_enable);
    return DG_OK;
}

int dg_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return DG_OK;
}

int dg_device_arch(char *buf, size_t size) {
    if (!buf || size == 0) return fail(DG_EINVAL, "null buffer");
    const std::string a = device_arch();
    if (a.size() + 1 > size) return fail(DG_EINVAL, "buffer too small");
    std::memcpy(buf, a.c_str(), a.size() + 1);
    return DG_OK;
}

// File format: one entry per line, "arch P precision av waves stage_us",
// '#' starts a comment line.
int dg_tuning_save(const char *path, int *entries) {
    if (!path) return fail(DG_EINVAL, "path is NULL");
    std::ostringstream os;
    os << "# arch P precision av waves_per_block stage_us\n";
    int n = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : g_tune) {
            char line[256];
            std::snprintf(line, sizeof(line), "%s %d %d %d %d %.3f\n", std::get<0>(kv.first).c_str(),
                          std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), kv.second.waves,
                          kv.second.stage_us);
            os << line;
            ++n;
        }
    }
    std::ofstream f(path, std::ios::trunc);
    if (!f) return fail(DG_EINVAL, std::string("cannot open ") + path + " for writing");
    f << os.str();
    if (!f) return fail(DG_EINVAL, std::string("write to ") + path + " failed");
    if (entries) *entries = n;
    return DG_OK;
}

int dg_tuning_load(const char *path, int *entries) {
    if (!path) return fail(DG_EINVAL, "path is NULL");
    std::ifstream f(path);
    if (!f) return fail(DG_EINVAL, std::string("cannot open ") + path);
    std::vector<std::pair<TuneKey, TuneEntry>> got;
    std::string line;
    int lineno = 0;
    while (std::getline(f, line)) {
        ++lineno;
        const size_t b = line.find_first_not_of(" \t\r");
        if (b == std::string::npos || line[b] == '#') continue;
        std::istringstream is(line);
        std::string arch, extra;
        int P = 0, prec = -1, av = -1, w = 0;
        double us = 0.0;
        if (!(is >> arch >> P >> prec >> av >> w >> us) || (is >> extra) || P < 1 || P > 5 ||
            (prec != DG_FP32 && prec != DG_FP32_BF16X3) || (av != 0 && av != 1) || !tunable_waves(w))
            return fail(DG_EINVAL, std::string(path) + ":" + std::to_string(lineno) + ": bad tuning entry");
        got.emplace_back(TuneKey(arch, P, prec, av), TuneEntry{w, us});
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
    if (entries) *entries = int(got.size());
    return DG_OK;
}

int dg_kernel_time(dg_mesh *m, void *stream, double *stage_ms_total, long *stage_launches) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(m->time_collect());
    if (stage_ms_total) *stage_ms_total = m->stage_ms;
    if (stage_launches) *stage_launches = m->stage_launches;
    m->stage_ms = 0.0;
    m->stage_launches = 0;
    return DG_OK;
}

int dg_status(dg_mesh *m, void *stream, int *device_flag) {
    if (!m) return fail(DG_EINVAL, "mesh is NULL");
    if (!device_flag) return fail(DG_EINVAL, "device_flag is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(device_flag, m->dm.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DG_OK;
}

// ---------------------------------------------------------------------------
// footprints and batching
// ---------------------------------------------------------------------------

int dg_mesh_footprint(const dg_mesh *m, size_t *bytes) {
    if (!m || !bytes) return fail(DG_EINVAL, "null argument");
    *bytes = m->owned_bytes + m->state_bytes() + m->work_bytes();
    return DG_OK;
}

int dg_mesh_curved(const dg_mesh *m, int *curved) {
    if (!m || !curved) return fail(DG_EINVAL, "null argument");
    *curved = m->dm.weak ? m->dm.wKc : (m->dm.fp32 ? m->dm.Kc : -1);
    return DG_OK;
}

int dg_estimate_footprint(int K, int P, int precision, int av_enable, size_t *bytes) {
    if (!bytes || K < 1 || P < 1 || P > 5) return fail(DG_EINVAL, "bad arguments");
    const size_t Np = size_t(n_nodes(P)), Nfp = size_t(P + 1), k = size_t(K);
    const bool f32 = precision == DG_FP32 || precision == DG_FP32_BF16X3;
    const size_t s = f32 ? 4 : 8;
    size_t b = k * (3 + 1) * 4;                                   // nbr, finfo
    b += k * Np * 2 * 8;                                          // node coordinates
    b += k * (4 * Np + 9 * Nfp + Np + 1) * 8;                     // FP64 geometry, mass weights, eps_max
    if (f32)
        b += k * (4 * Np + 9 * Nfp + 1) * 4 + k * (4 + 1 + 1 + 1) * 4 + k * 16 * 4  // FP32 copies, conn, flags
             + k * (4 * Np + 9 * Nfp) * 4;                        // curved records (upper bound)
    const size_t state = k * 4 * Np * s;
    size_t work = 3 * align256(state);
    if (av_enable) work += align256(2 * state) + align256(k * s);
    *bytes = b + state + work + (1u << 20);                       // operators, scalars, scratch
    return DG_OK;
}

}  // extern "C"

namespace {

struct Slot {
    bool used = false, finished = false;
    dg_mesh *mesh = nullptr;
    void *U = nullptr, *work = nullptr;
    int total = 0, remaining = 0, parity = 0;
    size_t footprint = 0;
};

// Device tables of one order P: argument records [parity][stage][job] and
// the work list of (job, tile) items.
// Device tables of one kind of solve (order P, BF16x3 product, viscosity):
// argument records [parity][stage][job] (job stride: the batch's slot
// count) and the work lists of (job, tile) items, with their lengths in
// device memory.  A group, once it has appeared, stays until the batch is
// destroyed (an empty group's launches find an empty list), so a captured
// step stays valid while solves of known kinds join and leave.
struct Group {
    int P = 0;
    bool bf3 = false;
    bool av = false;               // viscous handles: sensor and gradient records too
    int waves = 4;                 // stage kernel workgroup shape (tuning table or default)
    std::vector<int> slots;
    void *jobs = nullptr;          // [2][5][max_slots] stage records
    void *avjobs = nullptr;        // [2][5][max_slots] sensor/gradient records
    void *items = nullptr;         // (job, tile) of the stage kernel
    size_t items_cap = 0;          // entries (int2)
    void *eitems = nullptr;        // viscous: (job, block of 256 elements) for the per-element sensor
    size_t eitems_cap = 0;
    void *aitems = nullptr;        // viscous: (job, tile) of the gradient and per-node sensor
    size_t aitems_cap = 0;
    int *counts = nullptr;         // device [3]: items, eitems, aitems
    int nitems = 0, neitems = 0, naitems = 0;
};

}  // namespace

struct dg_batch {
    size_t budget = 0, used = 0;
    std::vector<Slot> slots;
    std::vector<Group> groups;
    std::vector<int> singles;      // slots stepped one by one (FP64 handles)
    // what the captured graph's one-by-one launches were made for: slot,
    // handle serial, state and work buffer of each (the handle's tables and
    // the buffers' addresses are baked into the graph, so a new solve in a
    // reused slot needs a new graph, even where the allocator hands out the
    // same addresses again)
    std::vector<std::tuple<int, unsigned long long, const void *, const void *>> graph_singles;
    bool dirty = true;
    long epoch_steps = 0;          // steps since the tables were last built
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    hipEvent_t done = nullptr;     // end of the last advance's work; destroy waits for it
    int captures = 0;              // step graphs captured so far
    ~dg_batch() {
        if (done) (void)hipEventDestroy(done);
        if (graph) (void)hipGraphExecDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (Group &g : groups) {
            if (g.jobs) (void)hipFree(g.jobs);
            if (g.avjobs) (void)hipFree(g.avjobs);
            if (g.items) (void)hipFree(g.items);
            if (g.eitems) (void)hipFree(g.eitems);
            if (g.aitems) (void)hipFree(g.aitems);
            if (g.counts) (void)hipFree(g.counts);
        }
    }
};

namespace {

bool batched_path(const dg_mesh *m) { return m->dm.fp32 && !m->dm.weak; }

// Rebuild the per-kind tables for the active, unfinished slots.  Groups are
// kept once created; the step graph is captured again only when a new group
// appears or a work list outgrows its table.
int rebuild(dg_batch *b, hipStream_t st) {
    b->singles.clear();
    const size_t max_jobs = b->slots.size();
    bool stale_graph = false;
    for (int key = 0; key < 20; ++key) {
        const int P = 1 + key % 5;
        const bool bf3 = (key / 5) & 1, av = key >= 10;
        std::vector<int> members;
        for (size_t i = 0; i < b->slots.size(); ++i) {
            const Slot &s = b->slots[i];
            if (s.used && !s.finished && batched_path(s.mesh) && s.mesh->dm.P == P && s.mesh->dm.bf3 == bf3 &&
                s.mesh->dm.av == av)
                members.push_back(int(i));
        }
        Group *g = nullptr;
        for (Group &o : b->groups)
            if (o.P == P && o.bf3 == bf3 && o.av == av) g = &o;
        if (!g) {
            if (members.empty()) continue;
            Group ng;
            ng.P = P;
            ng.bf3 = bf3;
            ng.av = av;
            // the shape the tuning table holds for this kind now; the group
            // keeps it for its lifetime
            const int tw = tuned_waves(device_arch(), P, bf3 ? DG_FP32_BF16X3 : DG_FP32, av);
            ng.waves = tw ? tw : mfma_default_waves();
            if (hipMalloc(&ng.jobs, 2 * 5 * max_jobs * mfma_args_bytes()) != hipSuccess ||
                (av && hipMalloc(&ng.avjobs, 2 * 5 * max_jobs * av_args_bytes()) != hipSuccess) ||
                hipMalloc(reinterpret_cast<void **>(&ng.counts), 3 * sizeof(int)) != hipSuccess) {
                if (ng.jobs) (void)hipFree(ng.jobs);
                if (ng.avjobs) (void)hipFree(ng.avjobs);
                return fail(DG_ENOMEM, "batch table allocation failed");
            }
            b->groups.push_back(ng);
            g = &b->groups.back();
            stale_graph = true;
        }
        g->slots = members;
    }
    for (size_t i = 0; i < b->slots.size(); ++i) {
        const Slot &s = b->slots[i];
        if (s.used && !s.finished && !batched_path(s.mesh)) b->singles.push_back(int(i));
    }
    for (Group &g : b->groups) {
        const size_t nj = g.slots.size();
        const size_t rec = mfma_args_bytes(), arec = av_args_bytes();
        std::vector<char> jobs(2 * 5 * max_jobs * rec, 0), avjobs(g.av ? 2 * 5 * max_jobs * arec : 0, 0);
        std::vector<int> items, eitems, aitems;
        for (size_t j = 0; j < nj; ++j) {
            Slot &s = b->slots[g.slots[j]];
            dg_mesh *m = s.mesh;
            char *w = static_cast<char *>(s.work);
            void *R = w + m->off_R(), *A = w + m->off_A(), *B = w + m->off_B();
            void *Q = g.av ? w + m->off_Q() : nullptr;
            void *eps = g.av ? w + m->off_eps() : nullptr;
            void *in[5] = {s.U, A, B, A, B};
            void *out[5] = {A, B, A, B, s.U};
            for (int ps = 0; ps < 2; ++ps) {
                const int par = (s.parity + ps) & 1;
                unsigned long long *vin = m->dm.vmax + par * kVmaxSlots;
                unsigned long long *vout = m->dm.vmax + (1 - par) * kVmaxSlots;
                for (int st5 = 0; st5 < 5; ++st5) {
                    // the same time-step handling as a fused single-mesh step
                    MfmaStep ms;
                    if (st5 == 0) {
                        ms.cfl_mode = 1;
                        ms.vmax_in = vin;
                        ms.vmax_out = vout;
                    }
                    if (st5 == 4 && !g.av) {
                        ms.cfl_accum = 1;
                        ms.vmax_out = vout;
                    }
                    mfma_fill_args(m->dm, in[st5], out[st5], R, st5, ms, g.waves,
                                   jobs.data() + ((ps * 5 + st5) * max_jobs + j) * rec, eps, Q);
                    if (g.av)
                        av_fill_args(m->dm, in[st5], eps, Q, st5 == 0 ? vin : nullptr,
                                     avjobs.data() + ((ps * 5 + st5) * max_jobs + j) * arec);
                }
            }
            const int nt = mfma_tiles(m->dm, g.waves);
            for (int tt = 0; tt < nt; ++tt) {
                items.push_back(int(j));
                items.push_back(tt);
            }
            if (g.av) {
                const int ne = sensor_elem_blocks(m->dm);
                for (int tt = 0; tt < ne; ++tt) {
                    eitems.push_back(int(j));
                    eitems.push_back(tt);
                }
                const int na = av_tiles(m->dm);
                for (int tt = 0; tt < na; ++tt) {
                    aitems.push_back(int(j));
                    aitems.push_back(tt);
                }
            }
        }
        g.nitems = int(items.size() / 2);
        g.neitems = int(eitems.size() / 2);
        g.naitems = int(aitems.size() / 2);
        // work lists grow by doubling; a new table means a new address, so
        // the captured graph is stale
        auto grow = [&](void **p, size_t *cap, size_t need) -> int {
            if (*cap >= need && *p) return DG_OK;
            size_t nc = *cap ? *cap : 4096;
            while (nc < need) nc *= 2;
            if (*p) (void)hipFree(*p);
            *p = nullptr;
            *cap = 0;
            if (hipMalloc(p, nc * 2 * sizeof(int)) != hipSuccess) return fail(DG_ENOMEM, "batch table allocation failed");
            *cap = nc;
            stale_graph = true;
            return DG_OK;
        };
        if (int rc = grow(&g.items, &g.items_cap, size_t(g.nitems))) return rc;
        if (g.av) {
            if (int rc = grow(&g.eitems, &g.eitems_cap, size_t(g.neitems))) return rc;
            if (int rc = grow(&g.aitems, &g.aitems_cap, size_t(g.naitems))) return rc;
        }
        HIP_TRY(hipMemcpyAsync(g.jobs, jobs.data(), jobs.size(), hipMemcpyHostToDevice, st));
        if (g.av) HIP_TRY(hipMemcpyAsync(g.avjobs, avjobs.data(), avjobs.size(), hipMemcpyHostToDevice, st));
        if (!items.empty())
            HIP_TRY(hipMemcpyAsync(g.items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, st));
        if (!eitems.empty())
            HIP_TRY(hipMemcpyAsync(g.eitems, eitems.data(), eitems.size() * sizeof(int), hipMemcpyHostToDevice, st));
        if (!aitems.empty())
            HIP_TRY(hipMemcpyAsync(g.aitems, aitems.data(), aitems.size() * sizeof(int), hipMemcpyHostToDevice, st));
        const int counts[3] = {g.nitems, g.neitems, g.naitems};
        HIP_TRY(hipMemcpyAsync(g.counts, counts, sizeof(counts), hipMemcpyHostToDevice, st));
        // the host buffers go out of scope: wait for the copies
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (stale_graph && b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    // FP64 slots step inside the graph too, their launches carrying their
    // handles' and buffers' addresses: any change of those needs a new graph
    std::vector<std::tuple<int, unsigned long long, const void *, const void *>> sig;
    for (int i : b->singles) {
        const Slot &s = b->slots[i];
        sig.emplace_back(i, s.mesh->serial, s.U, s.work);
    }
    if (sig != b->graph_singles && b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    b->graph_singles = sig;
    b->epoch_steps = 0;
    b->dirty = false;
    return DG_OK;
}

// One lockstep step of every active slot; ps = parity of the epoch step.
int batch_step(dg_batch *b, int ps, hipStream_t st) {
    const size_t rec = mfma_args_bytes(), arec = av_args_bytes(), nj = b->slots.size();
    for (int s5 = 0; s5 < 5; ++s5)
        for (const Group &g : b->groups) {
            if (g.av) {
                const char *avjobs = static_cast<const char *>(g.avjobs) + (ps * 5 + s5) * nj * arec;
                HIP_TRY(launch_av_batch(g.P, s5 == 0, avjobs, g.aitems, g.counts + 2, int(g.aitems_cap), g.eitems,
                                        g.counts + 1, int(g.eitems_cap), st));
            }
            const char *jobs = static_cast<const char *>(g.jobs) + (ps * 5 + s5) * nj * rec;
            HIP_TRY(launch_stage_mfma_batch(g.P, g.bf3, g.av, g.waves, jobs, g.items, g.counts, int(g.items_cap),
                                            st));
        }
    for (int i : b->singles) {
        Slot &s = b->slots[i];
        if (int rc = step_impl(s.mesh, s.U, s.work, 0.0, st)) return rc;
    }
    return DG_OK;
}

}  // namespace

extern "C" {

int dg_batch_create(size_t hbm_budget_bytes, int max_slots, dg_batch **out) {
    if (!out) return fail(DG_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1) return fail(DG_EINVAL, "max_slots must be >= 1");
    dg_batch *b = new dg_batch();
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(DG_EDEVICE, "hipEventCreateWithFlags failed");
    }
    b->budget = hbm_budget_bytes;
    b->slots.resize(max_slots);
    *out = b;
    return DG_OK;
}

int dg_batch_destroy(dg_batch *b) {
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    // the batch's tables may still be read by its last advance
    if (b->done) (void)hipEventSynchronize(b->done);
    delete b;
    return DG_OK;
}

int dg_batch_admit(dg_batch *b, dg_mesh *m, void *U, void *work, int nsteps, void *stream, int *slot) {
    if (!b || !m || !U || !work || !slot) return fail(DG_EINVAL, "null argument");
    if (nsteps < 1) return fail(DG_EINVAL, "nsteps must be >= 1");
    *slot = -1;
    size_t fp = 0;
    dg_mesh_footprint(m, &fp);
    if (b->used + fp > b->budget)
        return fail(DG_EBUSY, "HBM budget: " + std::to_string(b->used) + " + " + std::to_string(fp) +
                                  " bytes exceeds " + std::to_string(b->budget));
    int free_slot = -1;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (!b->slots[i].used) {
            free_slot = int(i);
            break;
        }
    if (free_slot < 0) return fail(DG_EBUSY, "no free slot");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_reset_scalars(m->dm, st));
    HIP_TRY(hipMemsetAsync(m->dm.flag, 0, sizeof(int), st));
    if (batched_path(m)) {
        if (m->dm.av)
            HIP_TRY(hipMemsetAsync(m->dm.vmax, 0, 2 * kVmaxSlots * sizeof(unsigned long long), st));
        else
            HIP_TRY(launch_cfl_vmax(m->dm, U, m->dm.vmax, st));
    }
    Slot &s = b->slots[free_slot];
    s = Slot();
    s.used = true;
    s.mesh = m;
    s.U = U;
    s.work = work;
    s.total = s.remaining = nsteps;
    s.parity = 0;
    s.footprint = fp;
    b->used += fp;
    b->dirty = true;
    *slot = free_slot;
    return DG_OK;
}

int dg_batch_advance(dg_batch *b, int max_steps, void *stream, int *steps_run) {
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    if (steps_run) *steps_run = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int n = max_steps;
    bool any = false;
    for (const Slot &s : b->slots)
        if (s.used && !s.finished) {
            any = true;
            n = s.remaining < n ? s.remaining : n;
        }
    if (!any || n <= 0) return DG_OK;
    if (b->dirty)
        if (int rc = rebuild(b, st)) return rc;
    int done = 0;
    // an odd epoch position first takes one eager step
    if ((b->epoch_steps & 1) && done < n) {
        if (int rc = batch_step(b, 1, st)) return rc;
        ++done;
        ++b->epoch_steps;
    }
    if (n - done >= 2) {
        if (!b->graph) {
            if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
            int rc0 = batch_step(b, 0, b->cap_stream);
            int rc1 = rc0 ? rc0 : batch_step(b, 1, b->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
            if (rc1) {
                if (g) (void)hipGraphDestroy(g);
                return rc1;
            }
            if (ec != hipSuccess) return fail(DG_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
            hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) return fail(DG_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
            ++b->captures;
        }
        for (; done + 2 <= n; done += 2) {
            HIP_TRY(hipGraphLaunch(b->graph, st));
            b->epoch_steps += 2;
        }
    }
    for (; done < n; ++done) {
        if (int rc = batch_step(b, int(b->epoch_steps & 1), st)) return rc;
        ++b->epoch_steps;
    }
    for (Slot &s : b->slots)
        if (s.used && !s.finished) {
            s.remaining -= n;
            s.parity = (s.parity + n) & 1;
            if (s.remaining == 0) {
                s.finished = true;
                b->dirty = true;
                // a batched viscous slot checks each step's state in that
                // step's first sensor: check the final state as dg_run does
                if (batched_path(s.mesh) && s.mesh->dm.av)
                    HIP_TRY(launch_cfl_vmax(s.mesh->dm, s.U, s.mesh->dm.vmax, st));
            }
        }
    for (Slot &s : b->slots)
        if (s.used) s.mesh->mark(st);
    (void)hipEventRecord(b->done, st);
    if (steps_run) *steps_run = n;
    return DG_OK;
}

int dg_batch_poll(dg_batch *b, void *stream, int *done_slots, int max_done, int *ndone) {
    if (!b || !ndone) return fail(DG_EINVAL, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // state checks of the running slots: a slot whose state went non-finite
    // (or rho <= 0, p <= 0) retires now instead of running out its steps
    std::vector<int> flags(b->slots.size(), 0);
    for (size_t i = 0; i < b->slots.size(); ++i) {
        const Slot &s = b->slots[i];
        if (s.used && !s.finished)
            HIP_TRY(hipMemcpyAsync(&flags[i], s.mesh->dm.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < b->slots.size(); ++i) {
        Slot &s = b->slots[i];
        if (s.used && !s.finished && flags[i]) {
            s.finished = true;
            b->dirty = true;
        }
    }
    int n = 0;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (b->slots[i].used && b->slots[i].finished) {
            if (done_slots && n < max_done) done_slots[n] = int(i);
            ++n;
        }
    *ndone = n;
    return DG_OK;
}

int dg_batch_slot_stats(dg_batch *b, int slot, void *stream, dg_run_stats *stats) {
    if (!b || !stats || slot < 0 || slot >= int(b->slots.size()) || !b->slots[slot].used)
        return fail(DG_EINVAL, "bad slot");
    const Slot &s = b->slots[slot];
    hipStream_t st = static_cast<hipStream_t>(stream);
    double scal[S_NSCAL];
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(scal, s.mesh->dm.scal, sizeof(scal), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&flag, s.mesh->dm.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memset(stats, 0, sizeof(*stats));
    stats->steps = s.total - s.remaining;
    stats->status = flag ? DG_ENONFINITE : DG_OK;
    stats->t = scal[S_T];
    stats->dt_min = stats->steps ? scal[S_DTMIN] : 0.0;
    stats->dt_max = scal[S_DTMAX];
    return DG_OK;
}

int dg_batch_info(dg_batch *b, int *captures, int *groups) {
    if (!b) return fail(DG_EINVAL, "batch is NULL");
    if (captures) *captures = b->captures;
    if (groups) *groups = int(b->groups.size());
    return DG_OK;
}

int dg_batch_release(dg_batch *b, int slot) {
    if (!b || slot < 0 || slot >= int(b->slots.size()) || !b->slots[slot].used)
        return fail(DG_EINVAL, "bad slot");
    b->used -= b->slots[slot].footprint;
    b->slots[slot] = Slot();
    b->dirty = true;
    return DG_OK;
}

}  // extern "C"
