// C ABI of libmadlens_amd.so: parameter validation, the device arena,
// float64 host tables, and the orchestration of the PM step, initial
// conditions and lens projection on one HIP stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <algorithm>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/madlens.h"
#include "cosmo_host.h"
#include "adjoint.h"
#include "batch.h"
#include "fft.h"
#include "particles.h"

using namespace ml;

namespace {

constexpr double PI = 3.14159265358979323846;

bool only_2_3(int n) {
    if (n <= 0) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

struct Layout {
    size_t bytes = 0;
    size_t take(size_t n) {
        size_t off = (bytes + 255) & ~size_t(255);
        bytes = off + n;
        return off;
    }
};

// Offsets of every device array inside the arena.
struct ArenaPlan {
    size_t disp[2], mom[2], id[2], acc, key, count, start, scan_sum, status;
    size_t mesh[3], nyq[3], halo, tw_nm, tw_hm, twp_nm, tw_np, tw_hp, twp_np, g_ic, atab, dtab, pmax;
    size_t xbc, fbc, dots, fmax, noise, g_ic_dom, adom, ddom, cacc;
    // PM_MODE_PGD: filtered Green's function, shift, its bound, spare mesh
    size_t pgd_g, pgd_s, pgd_bits, pgd_m, pgd_nyq;
    // PM_MODE_TANGENT: x_dot, p_dot (each with the sort's second buffer), f_dot
    size_t tan;
    size_t total;
};

constexpr int ATAB_N = 8192;
constexpr double ATAB_AMIN = 0.004;

ArenaPlan plan_arena(const pm_params& p, const lens_params& l, size_t es) {
    (void)l;
    ArenaPlan a{};
    Layout L;
    size_t n = (size_t)p.np * p.np * p.np;
    size_t nm = (size_t)p.nm;
    size_t nt = nm / TILE;
    for (int b = 0; b < 2; ++b) {
        a.disp[b] = L.take(3 * n * es);
        a.mom[b] = L.take(3 * n * es);
        a.id[b] = L.take(n * 4);
    }
    a.acc = L.take(3 * n * es);
    a.key = L.take(n * 4);
    const size_t nkeys = nt * nt * nt * BPT;  // sort blocks
    a.count = L.take(nkeys * 4);
    a.start = L.take((nkeys + 1) * 4);
    a.scan_sum = L.take((nkeys + 1023) / 1024 * 4);
    a.status = L.take(256);
    for (int j = 0; j < 3; ++j) {
        a.mesh[j] = L.take(nm * nm * nm * es);
        a.nyq[j] = L.take(nm * nm * 2 * es);
    }
    a.halo = L.take((size_t)paint_halo_elems((int)nt, (int)es) * es);
    a.tw_nm = L.take(nm * 2 * es);
    a.tw_hm = L.take(nm / 2 * 2 * es);
    a.twp_nm = L.take((nm / 2 + 1) * 2 * es);
    size_t np_ = (size_t)p.np;
    a.tw_np = L.take(np_ * 2 * es);
    a.tw_hp = L.take(np_ / 2 * 2 * es);
    a.twp_np = L.take((np_ / 2 + 1) * 2 * es);
    a.g_ic = L.take((3 * (np_ / 2) * (np_ / 2) + 1) * es);
    a.atab = L.take(2 * ATAB_N * es);
    a.dtab = L.take(2 * ATAB_N * es);
    a.pmax = L.take(256);
    // reverse pass: sorted-order cotangent scratch, reductions, the noise of
    // the last initial conditions, Omega_m derivative tables
    a.xbc = L.take(3 * n * es);
    a.fbc = L.take(3 * n * es);
    a.dots = L.take(64 * sizeof(double));
    a.fmax = L.take(256);
    a.noise = L.take(n * es);
    a.g_ic_dom = L.take((3 * (np_ / 2) * (np_ / 2) + 1) * es);
    a.adom = L.take(ATAB_N * es);
    a.ddom = L.take(ATAB_N * es);
    a.cacc = L.take(256);
    a.pgd_g = a.pgd_s = a.pgd_bits = a.pgd_m = a.pgd_nyq = a.tan = 0;
    if (p.modes & PM_MODE_PGD) {
        a.pgd_g = L.take((3 * (nm / 2) * (nm / 2) + 1) * es);
        a.pgd_s = L.take(3 * n * es);
        a.pgd_bits = L.take(256);
        a.pgd_m = L.take(nm * nm * nm * es);
        a.pgd_nyq = L.take(nm * nm * 2 * es);
    }
    if (p.modes & PM_MODE_TANGENT) a.tan = L.take(15 * n * es);
    a.total = L.bytes;
    return a;
}

int validate(const pm_params* p, const lens_params* l) {
    if (!p || !l) return PM_EINVAL;
    if (p->dtype != PM_F32 && p->dtype != PM_F64) return PM_EINVAL;
    if (p->modes & ~(PM_MODE_PGD | PM_MODE_TANGENT | PM_MODE_CKPT_FORCE)) return PM_EINVAL;
    if (p->np < 16 || p->nm < 16 || p->np % 16 || p->nm % 16) return PM_EINVAL;
    if (p->nm != p->np && p->nm != 2 * p->np) return PM_EINVAL;
    if (!only_2_3(p->np) || !only_2_3(p->nm) || p->nm > 1024) return PM_EINVAL;
    bool fft_ok = p->dtype == PM_F32 ? fft_supported<float>(p->nm) && fft_supported<float>(p->np)
                                     : fft_supported<double>(p->nm) && fft_supported<double>(p->np);
    if (!fft_ok) return PM_EINVAL;
    if (!(p->box > 0) || !(p->omega_m > 0 && p->omega_m < 1) || !(p->h > 0) || !(p->sigma8 > 0))
        return PM_EINVAL;
    if (!(p->omega_b > 0 && p->omega_b < p->omega_m) || !(p->t_cmb > 0)) return PM_EINVAL;
    if (l->npix < 16 || l->npix > 8192) return PM_EINVAL;
    if (!(l->fov_deg > 0 && l->fov_deg <= 22.0)) return PM_EINVAL;
    if (l->nsrc < 1 || l->nsrc > MAX_SRC || !l->z_src) return PM_EINVAL;
    for (int s = 0; s < l->nsrc; ++s)
        if (!(l->z_src[s] > 0 && l->z_src[s] < 20)) return PM_EINVAL;
    return PM_OK;
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return PM_EDEVICE;  \
    } while (0)

// Optional per-kernel timing with HIP events on the simulation's stream.
// Events come from a pool created when profiling is switched on, so the
// timed loop creates nothing.
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int name; hipEvent_t a, b; hipStream_t s; };
    std::vector<Rec> recs;
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<long> cnt;
    hipStream_t st = nullptr;
    int cur = -1;
    std::string only;  // when set, only launches of this name are recorded

    int name_id(const char* n) {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == n) return (int)i;
        names.emplace_back(n);
        ms.push_back(0.0);
        cnt.push_back(0);
        return (int)names.size() - 1;
    }
    // s: the stream the timed launch goes to (NULL: the simulation's)
    void begin(const char* n, hipStream_t s = nullptr) {
        cur = -1;
        if (!on || used + 2 > pool.size()) return;
        if (!only.empty() && only != n) return;
        cur = (int)recs.size();
        recs.push_back({name_id(n), pool[used], pool[used + 1], s ? s : st});
        used += 2;
        (void)hipEventRecord(recs.back().a, recs.back().s);
    }
    void end() {
        if (cur < 0) return;
        (void)hipEventRecord(recs[cur].b, recs[cur].s);
        cur = -1;
    }
    int enable(bool e, hipStream_t s) {
        st = s;
        if (e && pool.empty()) {
            pool.resize(16384);  // 8192 launches
            for (auto& ev : pool)
                if (hipEventCreate(&ev) != hipSuccess) return PM_EDEVICE;
        }
        on = e;
        return PM_OK;
    }
    int resolve() {
        if (recs.empty()) return PM_OK;
        for (auto& r : recs)
            if (hipEventSynchronize(r.b) != hipSuccess) return PM_EDEVICE;
        for (auto& r : recs) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return PM_EDEVICE;
            ms[r.name] += t;
            cnt[r.name] += 1;
        }
        recs.clear();
        used = 0;
        return PM_OK;
    }
    ~Prof() {
        for (auto& ev : pool) (void)hipEventDestroy(ev);
    }
};

struct ProfScope {
    Prof& p;
    ProfScope(Prof& pr, const char* n, hipStream_t s = nullptr) : p(pr) { p.begin(n, s); }
    ~ProfScope() { p.end(); }
};

// The arguments of every pass of one slot's fused step (the device
// parameter block of a batch holds one array per pass).
template <class T> struct BatchSlotArgs {
    FillArgs fill;
    ScanArgs scan;
    ScatterArgs<T> scatter;
    PaintArgs<T> paint;
    LensGatherArgs<T> lens;
    R2cArgs<T> r2c;
    C2cArgs<T> fwd;
    GradArgs<T> grad;
    C2cArgs<T> inv;
    DualArgs<T> dual;
    C2rArgs<T> c2r[3];
    ReadoutArgs<T> readout;
};

struct SimBase {
    Prof prof;
    virtual ~SimBase() {}
    virtual int init_ic(const void* noise, double a0) = 0;
    virtual int init_ic_seed(uint64_t seed, double a0) = 0;
    virtual int noise(uint64_t seed, void* out) = 0;
    virtual int reconfigure(const pm_params* p, const lens_params* l) = 0;
    virtual int step(double a0, double a1) = 0;
    virtual int lens(double a0, double a1, void* kappa) = 0;
    virtual int set_interpolation(int on) = 0;
    virtual int set_replica_rotation(int on, uint64_t seed) = 0;
    virtual int set_pgd(int on, double alpha0, double mu, double k_l, double k_s) = 0;
    virtual int run(const double* agrid, int nsteps, void* kappa) = 0;
    virtual int get_state(void* x, void* p, double* a) = 0;
    virtual int set_state(const void* x, const void* p, double a) = 0;
    virtual int get_force(void* rho, void* fm, void* acc) = 0;
    virtual int sync() = 0;
    virtual int background(double a, double out[3]) const = 0;
    virtual hipStream_t stream() const = 0;
    virtual int lens_vjp(double a0, double a1, const void* kbar, void* xbar, void* phbar,
                         double* cb) = 0;
    virtual int step_vjp(double a0, double a1, double a2, void* xbar, void* pbar,
                         const void* phbar, double* cb) = 0;
    virtual int init_ic_vjp(double a1, const void* xbar, const void* pbar, void* nbar,
                            double* cb) = 0;
    virtual int vjp_cosmo_read(double* cb) = 0;
    virtual size_t checkpoint_bytes() const = 0;
    virtual int checkpoint_save(void* buf) = 0;
    virtual int checkpoint_load(const void* buf, double a) = 0;
    virtual int init_ic_jvp(const void* nd, double om_dot, double s8_dot) = 0;
    virtual int set_tangent(const void* xd, const void* pd, double om_dot) = 0;
    virtual int get_tangent(void* xd, void* pd, void* fd) = 0;
    virtual int step_jvp(double a0, double a1) = 0;
    virtual int lens_jvp(double a0, double a1, void* kd) = 0;
};

template <class T> struct Sim final : SimBase {
    pm_params P{};
    int npix = 0, nsrc = 0;
    double fov = 0;
    std::vector<double> zsrc, chisrc;
    HostCosmo cosmo;
    Geo geo{};
    hipStream_t st = nullptr;
    char* arena = nullptr;
    ArenaPlan ap{};
    Parts<T> cur{}, alt{};
    SortBufs sb{};
    uint32_t* status = nullptr;
    uint32_t* scan_sum = nullptr;
    T* mesh[3]{};
    cx<T>* nyq[3]{};
    T* halo = nullptr;
    cx<T>*tw_nm, *tw_hm, *twp_nm, *tw_np, *tw_hp, *twp_np;
    T *g_ic, *atab, *dtab;
    uint32_t* pmax_bits = nullptr;
    T *xbc, *fbc, *noise_copy, *g_ic_dom, *adom, *ddom;
    double* dots = nullptr;
    double* cacc = nullptr;  // device accumulator of (dL/dOmega_m, dL/dsigma_8)
    uint32_t* fmax_bits = nullptr;
    HostCosmo cosmo_p, cosmo_m;  // Omega_m +- DOM for the finite-difference factors
    static constexpr double DOM = 1e-5;
    std::vector<double> chisrc_p, chisrc_m;
    bool meshes_valid = false;  // mesh[0..2] hold the force meshes of the current state
    double dchi_tab = 0;
    double a_cur = -1.0;
    bool ic_fresh = false;  // the state is the initial conditions of noise_copy
    // sub-evolution projection (the lens moves each image along its step's
    // drift to the scale factor of its own distance)
    bool interp = false;
    // the current state is the end of the KDK step kdk_a0 -> kdk_a1, whose
    // last kick was kdk_k2 times the force now in acc (else kdk_a1 < 0)
    double kdk_a0 = -1.0, kdk_a1 = -1.0;
    T kdk_k2 = T(0);
    // replica rotation: replica (nx, ny, nz) is the box under one of the 48
    // cube symmetries, hashed from its offsets and rot_seed
    bool rot = false;
    uint64_t rot_seed = 0;
    // PGD correction of the projected positions: S = alpha0 a^mu times the
    // force of the density filtered by exp(-k_l^2/k^2) exp(-(k/k_s)^4)
    bool pgd = false;
    double pgd_alpha0 = 0, pgd_mu = 0, pgd_kl = 0, pgd_ks = 1;
    T* pgd_g = nullptr;            // [3 (Nm/2)^2 + 1] filtered Green's function
    T* pgd_s = nullptr;            // [3][Np^3] filtered force at the particles
    T* pgd_m = nullptr;            // [Nm^3] + Nyquist plane: the filtered force's
    T* pgd_nyq = nullptr;          // first component (the others use mesh 1, 2)
    uint32_t* pgd_bits = nullptr;  // max |pgd_s| (float bits)
    // forward-mode tangent of (x, p, f) along (noise, Omega_m, sigma_8), in
    // tile order and Mpc/h (PM_MODE_TANGENT): x_dot and p_dot (each with a
    // second buffer the sort's scatter permutes into) and f_dot
    T* tan_mem = nullptr;
    T *tx = nullptr, *tx_alt = nullptr, *tp = nullptr, *tp_alt = nullptr, *tf = nullptr;
    bool tan_valid = false;  // the tangent belongs to the current state
    bool tan_carry = false;  // the next sort permutes the tangent too
    bool tan_gather = false;  // the next force readout computes the tangent's share too
    double tan_om = 0;       // its Omega_m component
    double cell = 0;  // mesh cell, Mpc/h
    int ntiles = 0;

    bool own_arena = true;  // false: the arena is the static scratch array
    // pm_run projects each shell on a second stream, beside the paint and the
    // force transform (the projection reads only the sorted particles; the
    // readout, which moves them, waits for it)
    hipStream_t st_lens = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    ~Sim() override {
        if (st_lens) {
            (void)hipStreamSynchronize(st_lens);
            (void)hipStreamDestroy(st_lens);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (arena && own_arena) (void)hipFree(arena);
    }

    template <class U> U* at(size_t off) { return reinterpret_cast<U*>(arena + off); }

    // Cosmology, box and map geometry: everything of the parameters that does
    // not change the arena.
    void set_physics(const pm_params* p, const lens_params* l) {
        P = *p;
        npix = l->npix;
        nsrc = l->nsrc;
        fov = l->fov_deg;
        zsrc.assign(l->z_src, l->z_src + l->nsrc);
        cosmo.init(p->omega_m, p->h, p->n_s, p->sigma8, p->omega_b, p->t_cmb);
        cosmo_p.init(p->omega_m + DOM, p->h, p->n_s, p->sigma8, p->omega_b, p->t_cmb);
        cosmo_m.init(p->omega_m - DOM, p->h, p->n_s, p->sigma8, p->omega_b, p->t_cmb);
        chisrc.clear();
        chisrc_p.clear();
        chisrc_m.clear();
        for (double z : zsrc) {
            chisrc.push_back(cosmo.chi_of_z(z));
            chisrc_p.push_back(cosmo_p.chi_of_z(z));
            chisrc_m.push_back(cosmo_m.chi_of_z(z));
        }
        cell = p->box / p->nm;
        a_cur = -1.0;
        ic_fresh = false;
        tan_valid = false;
        kdk_a0 = kdk_a1 = -1.0;
        meshes_valid = false;
    }

    // mem: device memory of at least plan_arena's size to hold the arena
    // (not owned); NULL allocates it.
    int create(const pm_params* p, const lens_params* l, void* stream, void* mem = nullptr) {
        st = reinterpret_cast<hipStream_t>(stream);
        set_physics(p, l);
        geo.np = p->np;
        geo.nm = p->nm;
        geo.B = p->nm / p->np;
        geo.nt = p->nm / TILE;
        geo.ncb = geo.nt * BPT;
        geo.npart = (long)p->np * p->np * p->np;
        ntiles = geo.nt * geo.nt * geo.ncb;  // sort blocks (keys)
        ap = plan_arena(*p, *l, sizeof(T));
        // (a handle in the static scratch creates nothing: it projects in line)
        if (!mem && (hipStreamCreateWithFlags(&st_lens, hipStreamNonBlocking) != hipSuccess ||
                     hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
                     hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess)) {
            (void)hipGetLastError();
            return PM_EDEVICE;
        }
        if (mem) {
            arena = static_cast<char*>(mem);
            own_arena = false;
        } else if (hipMalloc(&arena, ap.total) != hipSuccess) {
            arena = nullptr;
            (void)hipGetLastError();
            return PM_ENOMEM;
        }
        for (int b = 0; b < 2; ++b) {
            Parts<T>& q = b ? alt : cur;
            q.disp = at<T>(ap.disp[b]);
            q.mom = at<T>(ap.mom[b]);
            q.id = at<uint32_t>(ap.id[b]);
            q.acc = at<T>(ap.acc);
        }
        sb.key = at<uint32_t>(ap.key);
        sb.count = at<uint32_t>(ap.count);
        sb.start = at<uint32_t>(ap.start);
        scan_sum = at<uint32_t>(ap.scan_sum);
        status = at<uint32_t>(ap.status);
        for (int j = 0; j < 3; ++j) {
            mesh[j] = at<T>(ap.mesh[j]);
            nyq[j] = at<cx<T>>(ap.nyq[j]);
        }
        halo = at<T>(ap.halo);
        tw_nm = at<cx<T>>(ap.tw_nm);
        tw_hm = at<cx<T>>(ap.tw_hm);
        twp_nm = at<cx<T>>(ap.twp_nm);
        tw_np = at<cx<T>>(ap.tw_np);
        tw_hp = at<cx<T>>(ap.tw_hp);
        twp_np = at<cx<T>>(ap.twp_np);
        g_ic = at<T>(ap.g_ic);
        atab = at<T>(ap.atab);
        dtab = at<T>(ap.dtab);
        pmax_bits = at<uint32_t>(ap.pmax);
        xbc = at<T>(ap.xbc);
        fbc = at<T>(ap.fbc);
        dots = at<double>(ap.dots);
        fmax_bits = at<uint32_t>(ap.fmax);
        noise_copy = at<T>(ap.noise);
        g_ic_dom = at<T>(ap.g_ic_dom);
        adom = at<T>(ap.adom);
        ddom = at<T>(ap.ddom);
        cacc = at<double>(ap.cacc);
        if (p->modes & PM_MODE_PGD) {
            pgd_g = at<T>(ap.pgd_g);
            pgd_s = at<T>(ap.pgd_s);
            pgd_bits = at<uint32_t>(ap.pgd_bits);
            pgd_m = at<T>(ap.pgd_m);
            pgd_nyq = at<T>(ap.pgd_nyq);
        }
        if (p->modes & PM_MODE_TANGENT) {
            const size_t n3 = 3 * (size_t)geo.npart;
            tan_mem = at<T>(ap.tan);
            tx = tan_mem;
            tx_alt = tan_mem + n3;
            tp = tan_mem + 2 * n3;
            tp_alt = tan_mem + 3 * n3;
            tf = tan_mem + 4 * n3;
        }
        return upload_tables();
    }

    int reconfigure(const pm_params* p, const lens_params* l) override {
        if (p->np != P.np || p->nm != P.nm || p->dtype != P.dtype || p->modes != P.modes ||
            l->npix != npix || l->nsrc != nsrc)
            return PM_EINVAL;
        HIPCHK(hipStreamSynchronize(st));
        set_physics(p, l);
        return upload_tables();
    }

    static void twiddles(std::vector<T>& v, int n, int count) {
        // exp(-2 pi i t / n), t < count
        v.resize(2 * count);
        for (int t = 0; t < count; ++t) {
            double ang = -2.0 * PI * (double)t / (double)n;
            v[2 * t] = (T)std::cos(ang);
            v[2 * t + 1] = (T)std::sin(ang);
        }
    }

    int upload(size_t off, const std::vector<T>& v) {
        HIPCHK(hipMemcpy(arena + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return PM_OK;
    }

    int upload_tables() {
        std::vector<T> v;
        int rc;
        const int nm = P.nm, np = P.np;
        twiddles(v, nm, nm);
        if ((rc = upload(ap.tw_nm, v))) return rc;
        twiddles(v, nm / 2, nm / 2);
        if ((rc = upload(ap.tw_hm, v))) return rc;
        twiddles(v, nm, nm / 2 + 1);
        if ((rc = upload(ap.twp_nm, v))) return rc;
        twiddles(v, np, np);
        if ((rc = upload(ap.tw_np, v))) return rc;
        twiddles(v, np / 2, np / 2);
        if ((rc = upload(ap.tw_hp, v))) return rc;
        twiddles(v, np, np / 2 + 1);
        if ((rc = upload(ap.twp_np, v))) return rc;
        // Zel'dovich: s_hat_j (mesh cells) = i n_j G delta-per-noise with
        // G = Nm sqrt(P(k) Np^3 / L^3) / (2 pi n^2 Np^3), k = 2 pi |n| / L
        {
            int nmax = 3 * (np / 2) * (np / 2);
            v.assign(nmax + 1, T(0));
            double L = P.box, np3 = (double)np * np * np;
            for (int q = 1; q <= nmax; ++q) {
                double k = 2.0 * PI * std::sqrt((double)q) / L;
                double amp = std::sqrt(cosmo.pk(k) * np3 / (L * L * L));
                v[q] = (T)((double)nm * amp / (2.0 * PI * q * np3));
            }
            if ((rc = upload(ap.g_ic, v))) return rc;
            // d G / d Omega_m by central differences (sigma8 held fixed)
            for (int q = 1; q <= nmax; ++q) {
                double k = 2.0 * PI * std::sqrt((double)q) / L;
                double ap_ = std::sqrt(cosmo_p.pk(k) * np3 / (L * L * L));
                double am_ = std::sqrt(cosmo_m.pk(k) * np3 / (L * L * L));
                v[q] = (T)((double)nm * (ap_ - am_) / (2.0 * DOM) / (2.0 * PI * q * np3));
            }
            v[0] = T(0);
            if ((rc = upload(ap.g_ic_dom, v))) return rc;
        }
        // a(chi) and da/dchi on a uniform chi grid for the lens weights
        {
            double chimax = cosmo.chi(ATAB_AMIN);
            dchi_tab = chimax / (ATAB_N - 2);
            std::vector<double> a0(ATAB_N), ap_(ATAB_N), am_(ATAB_N);
            cosmo.a_of_chi_grid(dchi_tab, ATAB_N, a0.data());
            cosmo_p.a_of_chi_grid(dchi_tab, ATAB_N, ap_.data());
            cosmo_m.a_of_chi_grid(dchi_tab, ATAB_N, am_.data());
            v.resize(2 * ATAB_N);
            for (int k = 0; k < ATAB_N; ++k) {
                v[2 * k] = (T)a0[k];
                v[2 * k + 1] = (T)cosmo.dadchi(a0[k]);
            }
            if ((rc = upload(ap.atab, v))) return rc;
            // D(a(chi_k)) and dD/dchi on the same grid, for sub-evolution
            std::vector<double> dk(ATAB_N), ddk(ATAB_N);
            cosmo.growth_grid(a0.data(), ATAB_N, dk.data(), ddk.data());
            for (int k = 0; k < ATAB_N; ++k) {
                v[2 * k] = (T)dk[k];
                v[2 * k + 1] = (T)(ddk[k] * cosmo.dadchi(a0[k]));
            }
            if ((rc = upload(ap.dtab, v))) return rc;
            std::vector<T> w(ATAB_N);
            for (int k = 0; k < ATAB_N; ++k) w[k] = (T)((ap_[k] - am_[k]) / (2.0 * DOM));
            if ((rc = upload(ap.adom, w))) return rc;
            // d D(a(chi)) / d Omega_m on the same grid (the sub-evolution
            // move's cosmology derivative), each side on its own a(chi)
            std::vector<double> dp(ATAB_N), dm(ATAB_N), tmp(ATAB_N);
            cosmo_p.growth_grid(ap_.data(), ATAB_N, dp.data(), tmp.data());
            cosmo_m.growth_grid(am_.data(), ATAB_N, dm.data(), tmp.data());
            for (int k = 0; k < ATAB_N; ++k) w[k] = (T)((dp[k] - dm[k]) / (2.0 * DOM));
            if ((rc = upload(ap.ddom, w))) return rc;
        }
        // the PGD filter lives on the box's wave numbers
        if (pgd && (rc = upload_pgd_table())) return rc;
        launch_fill_u32(status, 0u, 1, st);
        launch_fill<double>(cacc, 0.0, 2, st);
        HIPCHK(hipStreamSynchronize(st));
        return PM_OK;
    }

    // G(q) = 1 / (2 pi q Nm^2) of the Poisson solve (mesh-cell units), times
    // the PGD filter exp(-k_l^2 / k^2) exp(-(k / k_s)^4) at k = 2 pi sqrt(q) / L
    int upload_pgd_table() {
        const int h = P.nm / 2;
        const size_t ng = 3 * (size_t)h * h + 1;
        std::vector<T> g(ng);
        const double gscale = 1.0 / (2.0 * PI * (double)P.nm * (double)P.nm);
        g[0] = T(0);
        for (size_t q = 1; q < ng; ++q) {
            const double k = 2.0 * PI * std::sqrt((double)q) / P.box;
            const double kq = k / pgd_ks;
            g[q] = (T)(gscale / (double)q * std::exp(-(pgd_kl * pgd_kl) / (k * k)) *
                       std::exp(-(kq * kq) * (kq * kq)));
        }
        HIPCHK(hipMemcpyAsync(pgd_g, g.data(), ng * sizeof(T), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return PM_OK;
    }

    // ---- pipeline pieces ---------------------------------------------------
    void sort(T kick, T drift, int mode) {
        launch_fill_u32(sb.count, 0u, ntiles, st);
        { ProfScope ps(prof, "kick_drift_key"); launch_kick_drift_key<T>(cur, sb, geo, kick, drift, mode, status, st); }
        { ProfScope ps(prof, "scan"); launch_scan(sb.count, sb.start, scan_sum, ntiles, st); }
        if (tan_carry) {
            TanCarry<T> tc;
            tc.x_src = tx;
            tc.x_dst = tx_alt;
            tc.p_src = tp;
            tc.p_dst = tp_alt;
            { ProfScope ps(prof, "scatter_tangent"); launch_scatter<T>(cur, alt, sb, geo, st, tc); }
            std::swap(tx, tx_alt);
            std::swap(tp, tp_alt);
        } else {
            ProfScope ps(prof, "scatter");
            launch_scatter<T>(cur, alt, sb, geo, st);
        }
        std::swap(cur.disp, alt.disp);
        std::swap(cur.mom, alt.mom);
        std::swap(cur.id, alt.id);
    }

    void fft_forward_grad(int n, const T* G, const cx<T>* tw, const cx<T>* twh, const cx<T>* twp,
                          HaloMerge<T> hm = HaloMerge<T>(),
                          const std::function<void()>& after_fwd = nullptr) {
        // Poisson: G(q) = 1 / (2 pi q Nm^2) computed in the kernel (G == NULL)
        const T gscale = (T)(1.0 / (2.0 * PI * (double)n * (double)n));
        { ProfScope ps(prof, "fft_r2c_axis2"); fft_r2c_rows<T>(n, mesh[0], nyq[0], twh, twp, st, hm); }
        { ProfScope ps(prof, "fft_c2c_axis1_fwd");
          fft_c2c_axis1<T>(n, 1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw, st); }
        if (after_fwd) after_fwd();  // work to overlap with the rest of the transform
        PtrTriple om{{mesh[0], mesh[1], mesh[2]}}, on{{nyq[0], nyq[1], nyq[2]}};
        // axis 0: IFFT0(n0 h) -> mesh 0, IFFT0(h) -> mesh 1 (h = i G X)
        { ProfScope ps(prof, "fft_grad_axis0");
          fft_grad_axis0<T>(n, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], om, on, tw, G, gscale, st); }
        { ProfScope ps(prof, "fft_c2c_axis1_inv");
          fft_c2c_axis1<T>(n, -1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw, st); }
        // axis 1: n1 times mesh 1 in place, the plain transform into mesh 2
        { ProfScope ps(prof, "fft_c2c_axis1_dual");
          fft_c2c_axis1_dual<T>(n, reinterpret_cast<cx<T>*>(mesh[1]), nyq[1],
                                reinterpret_cast<cx<T>*>(mesh[2]), nyq[2], tw, st); }
        // axis 2, the last component times n2
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "fft_c2r_axis2");
            fft_c2r_rows<T>(n, mesh[j], nyq[j], twh, twp, st, j == 2);
        }
    }

    // CIC density into mesh[0].  With defer_merge the paint boxes' shells are
    // left in `halo` for the r2c pass to merge (force path).
    void paint(bool defer_merge = false) {
        T mass = (T)std::pow((double)geo.B, 3);
        ProfScope ps(prof, "paint");
        launch_paint<T>(cur, sb, geo, mass, mesh[0], halo, st, !defer_merge);
    }

    void force(T kick2, int do_kick) {
        paint(true);
        fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm, paint_halo_merge<T>(geo, halo));
        meshes_valid = true;
        if (tan_gather) {  // the first part of force_jvp_cur, on the same force boxes
            launch_fill_u32(fmax_bits, 0u, 1, st);
            TanGather<T> tg;
            tg.xdot = tx;
            tg.fbc = fbc;
            tg.vmax_bits = fmax_bits;
            tg.inv_h = T(1) / (T)cell;
            tg.mass = (T)std::pow((double)geo.B, 3);
            ProfScope ps(prof, "readout_kick_jvp_gather");
            launch_readout_tangent<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], kick2, do_kick, status,
                                      tg, st);
            return;
        }
        ProfScope ps(prof, "readout_kick");
        launch_readout<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], kick2, do_kick, status, st);
    }

    int check_launch() {
        return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
    }

    // ---- API ------------------------------------------------------------
    int check_a0(double a0) {
        if (!(a0 > 0 && a0 <= 1)) return PM_EINVAL;
        double chi0 = cosmo.chi(a0);
        for (double c : chisrc)
            if (c > chi0) return PM_EINVAL;
        return PM_OK;
    }

    int init_ic(const void* noise, double a0) override {
        if (!noise) return PM_EINVAL;
        int rc = check_a0(a0);
        if (rc) return rc;
        const size_t n = (size_t)P.np * P.np * P.np;
        HIPCHK(hipMemcpyAsync(noise_copy, noise, n * sizeof(T), hipMemcpyDeviceToDevice, st));
        return init_from_noise_copy(a0);
    }

    int init_ic_seed(uint64_t seed, double a0) override {
        int rc = check_a0(a0);
        if (rc) return rc;
        launch_noise<T>(noise_copy, (long)P.np * P.np * P.np, seed, st);
        return init_from_noise_copy(a0);
    }

    int noise(uint64_t seed, void* out) override {
        if (!out) return PM_EINVAL;
        launch_noise<T>(reinterpret_cast<T*>(out), (long)P.np * P.np * P.np, seed, st);
        return check_launch();
    }

    // Zel'dovich initial conditions from the noise held in noise_copy.
    int init_from_noise_copy(double a0) {
        const int np = P.np;
        size_t n = (size_t)np * np * np;
        HIPCHK(hipMemcpyAsync(mesh[0], noise_copy, n * sizeof(T), hipMemcpyDeviceToDevice, st));
        meshes_valid = false;
        fft_forward_grad(np, g_ic, tw_np, tw_hp, twp_np);
        launch_init_ic<T>(cur, geo, mesh[0], mesh[1], mesh[2], (T)cosmo.D(a0), (T)cosmo.gp(a0), st);
        sort(T(0), T(0), 0);
        force(T(0), 0);
        a_cur = a0;
        ic_fresh = true;
        tan_valid = false;
        kdk_a0 = kdk_a1 = -1.0;
        return check_launch();
    }

    int step(double a0, double a1) override {
        if (a_cur < 0 || std::fabs(a0 - a_cur) > 1e-12 * std::fabs(a_cur) + 1e-15) return PM_ESTATE;
        if (!(a1 > 0 && a1 <= 1.5)) return PM_EINVAL;
        double ah = 0.5 * (a0 + a1);
        T k1 = (T)cosmo.kick(a0, ah, a0);
        T dr = (T)cosmo.drift(a0, a1, ah);
        T k2 = (T)cosmo.kick(ah, a1, a1);
        sort(k1, dr, MODE_KICK | MODE_DRIFT);
        force(k2, 1);
        a_cur = a1;
        ic_fresh = false;
        tan_valid = false;  // a tangent step sets it again
        kdk_a0 = a0;
        kdk_a1 = a1;
        kdk_k2 = k2;
        return check_launch();
    }

    int lens(double a0, double a1, void* kappa) override {
        if (!kappa) return PM_EINVAL;
        if (a_cur < 0 || std::fabs(a1 - a_cur) > 1e-12 * std::fabs(a_cur) + 1e-15) return PM_ESTATE;
        // sub-evolution needs the drift momentum of the step a0 -> a1:
        // p - K2 f of the state that pm_step(a0, a1) left
        if (interp && (kdk_a1 < 0 || std::fabs(a0 - kdk_a0) > 1e-12 * std::fabs(a0) + 1e-15 ||
                       std::fabs(a1 - kdk_a1) > 1e-12 * std::fabs(a1) + 1e-15))
            return PM_ESTATE;
        if (pgd) pgd_shift(a1);
        int rc = project_shell(a0, a1, reinterpret_cast<T*>(kappa), interp ? kdk_k2 : T(0));
        return rc ? rc : check_launch();
    }

    int set_interpolation(int on) override {
        interp = on != 0;
        return PM_OK;
    }

    int set_replica_rotation(int on, uint64_t seed) override {
        rot = on != 0;
        rot_seed = seed;
        return PM_OK;
    }

    int set_pgd(int on, double alpha0, double mu, double k_l, double k_s) override {
        if (!on) {
            pgd = false;
            return PM_OK;
        }
        if (!(P.modes & PM_MODE_PGD)) return PM_EINVAL;  // no buffers in the arena
        if (!std::isfinite(alpha0) || !std::isfinite(mu) || !std::isfinite(k_l) ||
            !(k_l >= 0) || !(k_s > 0))
            return PM_EINVAL;
        pgd_kl = k_l;
        pgd_ks = k_s;
        int rc = upload_pgd_table();
        if (rc) return rc;
        pgd_alpha0 = alpha0;
        pgd_mu = mu;
        pgd = true;
        return PM_OK;
    }

    // PGD: the filtered force of the current (tile-sorted) state into pgd_s
    // (cells) and max |pgd_s| into pgd_bits; the lens adds alpha0 a^mu times
    // it to every image.  Uses the meshes (the force meshes are no longer
    // valid).
    //
    // The density's spectrum after the axis-2 and axis-1 passes stays in
    // mesh 0 (and its Nyquist plane): the force of the same positions starts
    // from it (force_from_spectrum), so a run pays for one paint and one
    // forward transform per step.  The filtered force's components go to
    // pgd_m, mesh 1 and mesh 2.
    void pgd_shift(double a) {
        const int nm = P.nm;
        paint(true);
        { ProfScope ps(prof, "fft_r2c_axis2");
          fft_r2c_rows<T>(nm, mesh[0], nyq[0], tw_hm, twp_nm, st, paint_halo_merge<T>(geo, halo)); }
        { ProfScope ps(prof, "fft_c2c_axis1_fwd");
          fft_c2c_axis1<T>(nm, 1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm, st); }
        cx<T>* pm_ = reinterpret_cast<cx<T>*>(pgd_m);
        cx<T>* pn_ = reinterpret_cast<cx<T>*>(pgd_nyq);
        PtrTriple om{{pgd_m, mesh[1], mesh[2]}}, on{{pgd_nyq, nyq[1], nyq[2]}};
        { ProfScope ps(prof, "fft_grad_axis0");
          fft_grad_axis0<T>(nm, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], om, on, tw_nm, pgd_g,
                            T(0), st); }
        { ProfScope ps(prof, "fft_c2c_axis1_inv"); fft_c2c_axis1<T>(nm, -1, pm_, pn_, tw_nm, st); }
        { ProfScope ps(prof, "fft_c2c_axis1_dual");
          fft_c2c_axis1_dual<T>(nm, reinterpret_cast<cx<T>*>(mesh[1]), nyq[1],
                                reinterpret_cast<cx<T>*>(mesh[2]), nyq[2], tw_nm, st); }
        T* comp[3] = {pgd_m, mesh[1], mesh[2]};
        const cx<T>* cn[3] = {pn_, nyq[1], nyq[2]};
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "fft_c2r_axis2");
            fft_c2r_rows<T>(nm, comp[j], cn[j], tw_hm, twp_nm, st, j == 2);
        }
        Parts<T> q = cur;
        q.acc = pgd_s;
        { ProfScope ps(prof, "pgd_readout");
          launch_readout<T>(q, sb, geo, pgd_m, mesh[1], mesh[2], T(0), 0, status, st); }
        (void)a;
        Parts<T> m = cur;
        m.mom = pgd_s;
        launch_fill_u32(pgd_bits, 0u, 1, st);
        launch_drift_momentum_max<T>(m, geo.npart, T(0), pgd_bits, st);
        meshes_valid = false;
    }

    // The force meshes from the spectrum that pgd_shift left in mesh 0: the
    // passes of fft_forward_grad after the axis-2 and axis-1 forward passes.
    void force_from_spectrum() {
        const int n = P.nm;
        const T gscale = (T)(1.0 / (2.0 * PI * (double)n * (double)n));
        PtrTriple om{{mesh[0], mesh[1], mesh[2]}}, on{{nyq[0], nyq[1], nyq[2]}};
        { ProfScope ps(prof, "fft_grad_axis0");
          fft_grad_axis0<T>(n, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], om, on, tw_nm, nullptr,
                            gscale, st); }
        { ProfScope ps(prof, "fft_c2c_axis1_inv");
          fft_c2c_axis1<T>(n, -1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm, st); }
        { ProfScope ps(prof, "fft_c2c_axis1_dual");
          fft_c2c_axis1_dual<T>(n, reinterpret_cast<cx<T>*>(mesh[1]), nyq[1],
                                reinterpret_cast<cx<T>*>(mesh[2]), nyq[2], tw_nm, st); }
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "fft_c2r_axis2");
            fft_c2r_rows<T>(n, mesh[j], nyq[j], tw_hm, twp_nm, st, j == 2);
        }
    }

    // The plain projection's arguments and mean terms of the shell
    // (chi(a1), chi(a0)]; false when the shell lies wholly behind the
    // farthest source plane (its images and its mean term both need
    // chi < chi_s, so it adds nothing).
    bool plain_lens_args(double a0, double a1, LensArgs<T>& la, MapAdd<T>& mv) const {
        la = LensArgs<T>{};
        mv = MapAdd<T>{};
        la.npix = npix;
        la.nsrc = nsrc;
        la.cell = (T)cell;
        double chi_far = cosmo.chi(a0), chi_near = cosmo.chi(a1);
        double chis_max = 0;
        for (double c : chisrc) chis_max = std::max(chis_max, c);
        if (chi_near >= chis_max) return false;
        la.chi_near = (T)chi_near;
        la.chi_far = (T)chi_far;
        la.cnear_d = chi_near / cell;
        la.cfar_d = chi_far / cell;
        double dth = fov * PI / 180.0 / npix;
        la.inv_dtheta = (T)(1.0 / dth);
        double vp = std::pow(P.box / P.np, 3);
        la.wbase = (T)(1.5 * P.omega_m / (C_H0 * C_H0) * vp / (dth * dth));
        for (int s = 0; s < nsrc; ++s) la.chi_src[s] = (T)chisrc[s];
        la.atab = atab;
        la.ntab = ATAB_N;
        la.dchi = (T)dchi_tab;
        plan_sources(la, chi_near, chi_far, true);
        for (int s = 0; s < nsrc; ++s) mv.v[s] = (T)cosmo.shell_mean(chi_near, chi_far, chisrc[s]);
        return true;
    }

    // Which maps take which images of the shell (chi_near, chi_far]: a
    // source beyond the far bound takes every image, one inside the shell
    // those in front of it, one in front of the shell none (a relative margin
    // of 1e-6 keeps images whose float distance rounds across a source on the
    // per-image test).  With moved images allowed (sub-evolution, the PGD
    // shift: images can leave the shell's bounds) every source takes the
    // per-image test.  The sources beyond the shell can share the
    // accumulators A and B, their maps A - ratio B with ratio = 1 / (cs
    // inv_chi_ref), inv_chi_ref being the factor the kernel applies in T,
    // and the sources in front of it then take no accumulator.  That is
    // done when it lets the region grow against one accumulator per source
    // (the region side follows from the accumulator count): at the same
    // region side it measured slower.  A shell with no source beyond it
    // keeps A and B unused.
    void plan_sources(LensArgs<T>& la, double chi_near, double chi_far, bool fixed_bounds) const {
        int nbeyond = 0, nnone = 0;
        for (int s = 0; s < nsrc; ++s) {
            if (chisrc[s] > chi_far * (1.0 + 1e-6)) ++nbeyond;
            if (fixed_bounds && chisrc[s] < chi_near * (1.0 - 1e-6)) ++nnone;
        }
        const int n_dec = 2 + (nsrc - nnone - nbeyond);
        la.dec = (fixed_bounds && region_side(n_dec, npix) > region_side(nsrc, npix)) ? 1 : 0;
        la.inv_chi_ref = (T)(1.0 / chi_far);
        la.ndirect = 0;
        for (int s = 0; s < nsrc; ++s) {
            la.ratio[s] = 0.0;
            if (la.dec && chisrc[s] > chi_far * (1.0 + 1e-6)) {
                la.slot[s] = -1;
                la.ratio[s] = 1.0 / ((double)la.inv_chi_ref * chisrc[s]);
            } else if (fixed_bounds && chisrc[s] < chi_near * (1.0 - 1e-6)) {
                la.slot[s] = -2;
            } else {
                la.slot[s] = 2 * la.dec + la.ndirect;
                la.direct_src[la.ndirect++] = s;
            }
        }
        la.nacc = 2 * la.dec + la.ndirect;
        la.rs = region_side(la.dec ? la.nacc : nsrc, npix);
    }

    // 64 x 64-pixel regions when their fixed-point accumulators fit in 128 KB
    // of LDS: each region's frustum is then twice as wide, and the tile
    // columns it reads hold fewer particles outside it
    static int region_side(int ns, int np_) {
        return ((size_t)ns * 64 * 64 * 8 <= 131072 && np_ >= 256) ? 64 : 32;
    }

    // Born projection of the shell (chi(a1), chi(a0)] of the current,
    // tile-sorted positions (which must be those at a1) into kappa.  With
    // sub-evolution the step's drift momentum is mom - sub_k2 * acc.
    // With PGD on, pgd_shift must have run for the current state.
    int project_shell(double a0, double a1, T* kappa, T sub_k2 = T(0), hipStream_t ls = nullptr) {
        if (!ls) ls = st;
        LensArgs<T> la;
        MapAdd<T> mv;
        if (!plain_lens_args(a0, a1, la, mv)) return PM_OK;
        la.rot = rot ? 1 : 0;
        la.rot_seed = (unsigned long long)rot_seed;
        if (interp) {
            const double ah = 0.5 * (a0 + a1);
            la.sub = 1;
            la.dtab = dtab;
            la.d_end = (T)cosmo.D(a1);
            la.sub_scale = (T)(1.0 / cosmo.gp(ah));
            la.sub_dr = (T)cosmo.drift(a0, a1, ah);
            la.sub_k2 = sub_k2;
            la.pmax_bits = pmax_bits;
            launch_fill_u32(pmax_bits, 0u, 1, ls);
            { ProfScope ps(prof, "drift_momentum_max", ls);
              launch_drift_momentum_max<T>(cur, geo.npart, sub_k2, pmax_bits, ls); }
        }
        if (pgd) {  // images shifted by alpha0 a1^mu times the filtered force
            la.shift = pgd_s;
            la.shift_scale = (T)(pgd_alpha0 * std::pow(a1, pgd_mu));
            la.shift_bits = pgd_bits;
        }
        if (interp || pgd) plan_sources(la, cosmo.chi(a1), cosmo.chi(a0), false);
        { ProfScope ps(prof, "lens_gather", ls);
          launch_lens_gather<T>(cur, sb, geo, la, mv, kappa, ls); }
        return PM_OK;
    }

    // nsteps KDK steps along agrid with the projection of every shell: the
    // same operations as pm_step and lens_project in turn, but each step's
    // readout also applies the next step's first half-kick and drift and
    // computes its sort keys (no separate kick/drift pass, no force array
    // in between), and each shell is projected right after the paint, while
    // the particles are at the end of their step.
    int run(const double* agrid, int nsteps, void* kappa) override {
        if (!agrid || !kappa || nsteps < 1) return PM_EINVAL;
        if (a_cur < 0 || std::fabs(agrid[0] - a_cur) > 1e-12 * std::fabs(a_cur) + 1e-15)
            return PM_ESTATE;
        for (int i = 0; i < nsteps; ++i)
            if (!(agrid[i + 1] > 0 && agrid[i + 1] <= 1.5)) return PM_EINVAL;
        T* kap = reinterpret_cast<T*>(kappa);
        for (int i = 0; i < nsteps; ++i) {
            const double a0 = agrid[i], a1 = agrid[i + 1], ah = 0.5 * (a0 + a1);
            if (i == 0) {
                sort((T)cosmo.kick(a0, ah, a0), (T)cosmo.drift(a0, a1, ah), MODE_KICK | MODE_DRIFT);
            } else {  // keys and histogram come from the previous readout
                { ProfScope ps(prof, "scan"); launch_scan(sb.count, sb.start, scan_sum, ntiles, st); }
                { ProfScope ps(prof, "scatter"); launch_scatter<T>(cur, alt, sb, geo, st); }
                std::swap(cur.disp, alt.disp);
                std::swap(cur.mom, alt.mom);
                std::swap(cur.id, alt.id);
            }
            // with PGD the shift's paint and forward passes are the force's
            // (and the projection needs the shift); without, the projection
            // runs on the second stream beside the transform
            if (pgd || !st_lens) {
                if (pgd) pgd_shift(a1);
                else paint(true);
                int rc = project_shell(a0, a1, kap, T(0));  // mom is the drift momentum here
                if (rc) return rc;
                if (pgd) force_from_spectrum();
                else fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm,
                                      paint_halo_merge<T>(geo, halo));
            } else {
                // The shell's projection, started after the forward axis-1
                // pass, shares the GPU with the fused axis-0 pass and the
                // inverse passes: it costs the step less there than beside
                // the paint, the axis-2 or the forward axis-1 pass.
                int rc = 0;
                paint(true);
                fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm, paint_halo_merge<T>(geo, halo), [&] {
                    if (hipEventRecord(ev_fork, st) != hipSuccess ||
                        hipStreamWaitEvent(st_lens, ev_fork, 0) != hipSuccess) {
                        rc = PM_EDEVICE;
                        return;
                    }
                    rc = project_shell(a0, a1, kap, T(0), st_lens);
                    if (hipEventRecord(ev_join, st_lens) != hipSuccess && !rc) rc = PM_EDEVICE;
                });
                if (rc) return rc;
                HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
            }
            const T k2 = (T)cosmo.kick(ah, a1, a1);
            ReadoutNext<T> nx;
            if (i + 1 < nsteps) {
                const double a2 = agrid[i + 2], ah2 = 0.5 * (a1 + a2);
                nx.on = 1;
                nx.kick = (T)cosmo.kick(a1, ah2, a1);
                nx.drift = (T)cosmo.drift(a1, a2, ah2);
                launch_fill_u32(sb.count, 0u, ntiles, st);
            }
            ProfScope ps(prof, nx.on ? "readout_kick_drift_key" : "readout_kick");
            launch_readout<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], k2, 1, status, st, nx);
        }
        meshes_valid = true;
        a_cur = agrid[nsteps];
        ic_fresh = false;
        tan_valid = false;
        kdk_a0 = agrid[nsteps - 1];
        kdk_a1 = agrid[nsteps];
        kdk_k2 = (T)cosmo.kick(0.5 * (kdk_a0 + kdk_a1), kdk_a1, kdk_a1);
        return check_launch();
    }

    int get_state(void* x, void* p, double* a) override {
        if (a) *a = a_cur;
        if (a_cur < 0) return PM_ESTATE;
        if (x || p)
            launch_get_state<T>(cur, geo, (T)cell, reinterpret_cast<T*>(x), reinterpret_cast<T*>(p),
                                nullptr, st);
        return check_launch();
    }

    int set_state(const void* x, const void* p, double a) override {
        if (!x || !p || !(a > 0)) return PM_EINVAL;
        launch_set_state<T>(cur, geo, (T)cell, reinterpret_cast<const T*>(x),
                            reinterpret_cast<const T*>(p), st);
        sort(T(0), T(0), 0);
        force(T(0), 0);
        a_cur = a;
        ic_fresh = false;
        tan_valid = false;
        kdk_a0 = kdk_a1 = -1.0;
        return check_launch();
    }

    // Checkpoints in the library's own particle order: displacements,
    // momenta, ids and the sort's block offsets, each 256-byte aligned; with
    // PM_MODE_CKPT_FORCE then the three force meshes and the accelerations.
    bool ckpt_force() const { return (P.modes & PM_MODE_CKPT_FORCE) != 0; }
    size_t checkpoint_bytes() const override {
        const size_t n = (size_t)geo.npart, es = sizeof(T);
        const size_t nkeys = (size_t)ntiles;
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        size_t b = 2 * al(3 * n * es) + al(n * 4) + al((nkeys + 1) * 4);
        if (ckpt_force()) {
            const size_t n3 = (size_t)P.nm * P.nm * P.nm;
            b += 3 * al(n3 * es) + al(3 * n * es);
        }
        return b;
    }

    int checkpoint_save(void* buf) override {
        if (!buf) return PM_EINVAL;
        if (a_cur < 0) return PM_ESTATE;
        const size_t n = (size_t)geo.npart, es = sizeof(T);
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        char* b = reinterpret_cast<char*>(buf);
        HIPCHK(hipMemcpyAsync(b, cur.disp, 3 * n * es, hipMemcpyDeviceToDevice, st));
        b += al(3 * n * es);
        HIPCHK(hipMemcpyAsync(b, cur.mom, 3 * n * es, hipMemcpyDeviceToDevice, st));
        b += al(3 * n * es);
        HIPCHK(hipMemcpyAsync(b, cur.id, n * 4, hipMemcpyDeviceToDevice, st));
        b += al(n * 4);
        HIPCHK(hipMemcpyAsync(b, sb.start, ((size_t)ntiles + 1) * 4, hipMemcpyDeviceToDevice, st));
        if (ckpt_force()) {
            b += al(((size_t)ntiles + 1) * 4);
            // every path that leaves the meshes valid has also left the
            // accelerations of the current state (its readout wrote them)
            if (!meshes_valid) force(T(0), 0);
            const size_t n3 = (size_t)P.nm * P.nm * P.nm;
            for (int j = 0; j < 3; ++j) {
                HIPCHK(hipMemcpyAsync(b, mesh[j], n3 * es, hipMemcpyDeviceToDevice, st));
                b += al(n3 * es);
            }
            HIPCHK(hipMemcpyAsync(b, cur.acc, 3 * n * es, hipMemcpyDeviceToDevice, st));
        }
        return check_launch();
    }

    // Restore a checkpoint of this handle's shape at scale factor a: the
    // particles come back in the order they were saved in, so no sort is
    // needed; the force there is copied back (PM_MODE_CKPT_FORCE) or
    // recomputed, as pm_set_state does.
    int checkpoint_load(const void* buf, double a) override {
        if (!buf || !(a > 0)) return PM_EINVAL;
        const size_t n = (size_t)geo.npart, es = sizeof(T);
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        const char* b = reinterpret_cast<const char*>(buf);
        HIPCHK(hipMemcpyAsync(cur.disp, b, 3 * n * es, hipMemcpyDeviceToDevice, st));
        b += al(3 * n * es);
        HIPCHK(hipMemcpyAsync(cur.mom, b, 3 * n * es, hipMemcpyDeviceToDevice, st));
        b += al(3 * n * es);
        HIPCHK(hipMemcpyAsync(cur.id, b, n * 4, hipMemcpyDeviceToDevice, st));
        b += al(n * 4);
        HIPCHK(hipMemcpyAsync(sb.start, b, ((size_t)ntiles + 1) * 4, hipMemcpyDeviceToDevice, st));
        if (ckpt_force()) {
            b += al(((size_t)ntiles + 1) * 4);
            const size_t n3 = (size_t)P.nm * P.nm * P.nm;
            for (int j = 0; j < 3; ++j) {
                HIPCHK(hipMemcpyAsync(mesh[j], b, n3 * es, hipMemcpyDeviceToDevice, st));
                b += al(n3 * es);
            }
            HIPCHK(hipMemcpyAsync(cur.acc, b, 3 * n * es, hipMemcpyDeviceToDevice, st));
            meshes_valid = true;
        } else {
            force(T(0), 0);
        }
        a_cur = a;
        ic_fresh = false;
        tan_valid = false;
        kdk_a0 = kdk_a1 = -1.0;
        return check_launch();
    }

    int get_force(void* rho, void* fm, void* acc) override {
        if (a_cur < 0) return PM_ESTATE;
        size_t n3 = (size_t)P.nm * P.nm * P.nm;
        paint();
        if (rho) HIPCHK(hipMemcpyAsync(rho, mesh[0], n3 * sizeof(T), hipMemcpyDeviceToDevice, st));
        fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm);
        meshes_valid = true;
        launch_readout<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], T(0), 0, status, st);
        if (fm) {
            // force meshes are in cell units; scale to Mpc/h into the caller's buffer
            for (int j = 0; j < 3; ++j)
                launch_scale_copy<T>(reinterpret_cast<T*>(fm) + j * n3, mesh[j], (T)cell, (long)n3, st);
        }
        if (acc)
            launch_get_state<T>(cur, geo, (T)cell, nullptr, nullptr, reinterpret_cast<T*>(acc), st);
        return check_launch();
    }

    int sync() override {
        HIPCHK(hipStreamSynchronize(st));
        uint32_t s = 0;
        HIPCHK(hipMemcpy(&s, status, 4, hipMemcpyDeviceToHost));
        return s ? PM_ENONFINITE : PM_OK;
    }


    // ---- reverse pass ------------------------------------------------------
    bool at_a(double a) const { return a_cur >= 0 && std::fabs(a - a_cur) <= 1e-12 * std::fabs(a_cur) + 1e-15; }

    int read_dots(double* out, int nread) {
        HIPCHK(hipMemcpyAsync(out, dots, nread * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return PM_OK;
    }

    // Force-node VJP at the current state: xbar += (df/dx)^T (ckick pbar), then
    // mode 0: drift reverse (pbar += dr xbar, dots[1] = sum xbar . p_half);
    // mode 1: initial-condition cotangent sbar = d0 xbar + gp0 pbar into fbc.
    void force_vjp(T ckick, const T* xbar_in, const T* pbar_in, int mode, T dr, T k2, T d0,
                   T gp0, T* xbar_out, T* pbar_out, const T* phbar = nullptr) {
        const long n = geo.npart;
        const T H = (T)cell;
        if (!meshes_valid) {
            paint();
            fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm);
            meshes_valid = true;
        }
        launch_fill_u32(fmax_bits, 0u, 1, st);
        { ProfScope ps(prof, "vjp_readout");
          launch_fvjp_readout<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], xbar_in, pbar_in, H, ckick,
                                 xbc, fbc, dots, fmax_bits, st); }
        meshes_valid = false;
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "vjp_paint_values");
            launch_paint_values<T>(cur, sb, geo, T(1), mesh[j], halo, fbc + j * n, fmax_bits, st);
        }
        const int nm = P.nm;
        const T gscale = (T)(1.0 / (2.0 * PI * (double)nm * (double)nm));
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "fft_r2c_axis2");
            fft_r2c_rows<T>(nm, mesh[j], nyq[j], tw_hm, twp_nm, st);
        }
        for (int j = 0; j < 3; ++j) {
            ProfScope ps(prof, "fft_c2c_axis1_fwd");
            fft_c2c_axis1<T>(nm, 1, reinterpret_cast<cx<T>*>(mesh[j]), nyq[j], tw_nm, st);
        }
        PtrTriple im{{mesh[0], mesh[1], mesh[2]}}, in_{{nyq[0], nyq[1], nyq[2]}};
        { ProfScope ps(prof, "fft_div_axis0");
          fft_div_axis0<T>(nm, im, in_, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm, nullptr,
                           gscale, st); }
        { ProfScope ps(prof, "fft_c2c_axis1_inv");
          fft_c2c_axis1<T>(nm, -1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm, st); }
        { ProfScope ps(prof, "fft_c2r_axis2"); fft_c2r_rows<T>(nm, mesh[0], nyq[0], tw_hm, twp_nm, st); }
        T mass = (T)std::pow((double)geo.B, 3);
        ProfScope ps(prof, "vjp_paintgrad");
        launch_fvjp_paintgrad<T>(cur, sb, geo, mesh[0], mass, xbc, H, mode, dr, k2, d0, gp0, xbar_out,
                                 pbar_in, pbar_out, phbar, fbc, fbc + n, fbc + 2 * n, dots, st);
    }

    int step_vjp(double a0, double a1, double a2, void* xbar, void* pbar, const void* phbar,
                 double* cb) override {
        if (!xbar || !pbar) return PM_EINVAL;
        if (!at_a(a1)) return PM_ESTATE;
        double ah = 0.5 * (a0 + a1);
        double k2 = cosmo.kick(ah, a1, a1), dr = cosmo.drift(a0, a1, ah);
        double dk2 = (cosmo_p.kick(ah, a1, a1) - cosmo_m.kick(ah, a1, a1)) / (2 * DOM);
        double ddr = (cosmo_p.drift(a0, a1, ah) - cosmo_m.drift(a0, a1, ah)) / (2 * DOM);
        double k1n = 0.0, dk1n = 0.0;
        if (a2 > a1) {
            double ah2 = 0.5 * (a1 + a2);
            k1n = cosmo.kick(a1, ah2, a1);
            dk1n = (cosmo_p.kick(a1, ah2, a1) - cosmo_m.kick(a1, ah2, a1)) / (2 * DOM);
        }
        launch_fill<double>(dots, 0.0, 64, st);
        T* xb = reinterpret_cast<T*>(xbar);
        T* pb = reinterpret_cast<T*>(pbar);
        force_vjp((T)(k2 + k1n), xb, pb, 0, (T)dr, (T)k2, T(0), T(1), xb, pb,
                  reinterpret_cast<const T*>(phbar));
        int rc = check_launch();
        if (rc) return rc;
        if (!cb) {
            CosmoCoef c;
            c.add(0, dk2 + dk1n, 0.0);
            c.add(1, ddr, 0.0);
            launch_cosmo_acc(dots, cacc, c, st);
            return check_launch();
        }
        double d[2];
        if ((rc = read_dots(d, 2))) return rc;
        cb[0] += d[0] * (dk2 + dk1n) + d[1] * ddr;
        return PM_OK;
    }

    int init_ic_vjp(double a1, const void* xbar, const void* pbar, void* nbar, double* cb) override {
        if (!xbar || !pbar || !nbar) return PM_EINVAL;
        if (a_cur < 0 || !(a1 > a_cur)) return PM_ESTATE;
        const double a0 = a_cur, ah = 0.5 * (a0 + a1);
        const double k1 = cosmo.kick(a0, ah, a0);
        const double dk1 = (cosmo_p.kick(a0, ah, a0) - cosmo_m.kick(a0, ah, a0)) / (2 * DOM);
        const double d0 = cosmo.D(a0), gp0 = cosmo.gp(a0);
        const double dd0 = (cosmo_p.D(a0) - cosmo_m.D(a0)) / (2 * DOM);
        const double dgp0 = (cosmo_p.gp(a0) - cosmo_m.gp(a0)) / (2 * DOM);
        launch_fill<double>(dots, 0.0, 64, st);
        // the kick at a0 uses the initial force: xbar += (df/dx)^T (K1 pbar); sbar -> fbc
        force_vjp((T)k1, reinterpret_cast<const T*>(xbar), reinterpret_cast<const T*>(pbar), 1, T(0),
                  T(0), (T)d0, (T)gp0, nullptr, nullptr);
        const int np = P.np;
        const long n = geo.npart;
        // ds/dOmega_m on the lattice from the stored noise, dotted with sbar
        HIPCHK(hipMemcpyAsync(mesh[0], noise_copy, n * sizeof(T), hipMemcpyDeviceToDevice, st));
        fft_forward_grad(np, g_ic_dom, tw_np, tw_hp, twp_np);
        launch_dot_sorted_lattice<T>(cur, geo, fbc, mesh[0], mesh[1], mesh[2], dots + 5, st);
        // noise_bar = S^T sbar
        launch_sorted_to_lattice<T>(cur, geo, fbc, mesh[0], mesh[1], mesh[2], st);
        for (int j = 0; j < 3; ++j) fft_r2c_rows<T>(np, mesh[j], nyq[j], tw_hp, twp_np, st);
        for (int j = 0; j < 3; ++j)
            fft_c2c_axis1<T>(np, 1, reinterpret_cast<cx<T>*>(mesh[j]), nyq[j], tw_np, st);
        PtrTriple im{{mesh[0], mesh[1], mesh[2]}}, in_{{nyq[0], nyq[1], nyq[2]}};
        fft_div_axis0<T>(np, im, in_, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_np, g_ic, T(0), st);
        fft_c2c_axis1<T>(np, -1, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_np, st);
        fft_c2r_rows<T>(np, mesh[0], nyq[0], tw_hp, twp_np, st);
        HIPCHK(hipMemcpyAsync(nbar, mesh[0], n * sizeof(T), hipMemcpyDeviceToDevice, st));
        meshes_valid = false;
        int rc = check_launch();
        if (rc) return rc;
        if (!cb) {
            CosmoCoef c;
            c.add(0, dk1, 0.0);
            c.add(1, dd0, 0.0);
            c.add(2, dgp0, 0.0);
            c.add(5, 1.0, 0.0);
            c.add(3, 0.0, 1.0 / P.sigma8);
            launch_cosmo_acc(dots, cacc, c, st);
            return check_launch();
        }
        double d[6];
        if ((rc = read_dots(d, 6))) return rc;
        cb[0] += d[0] * dk1 + d[1] * dd0 + d[2] * dgp0 + d[5];
        cb[1] += d[3] / P.sigma8;
        return PM_OK;
    }

    // Projection arguments and the weights' Omega_m derivative for the
    // derivative passes of the shell (chi(a1), chi(a0)]; false when the shell
    // lies wholly behind the farthest source plane (its images and its mean
    // term both need chi < chi_s, so it adds nothing).
    bool derivative_lens_args(double a0, double a1, LensArgs<T>& la, LensVjpArgs<T>& lv,
                              double& chi_near, double& chi_far) {
        la = LensArgs<T>{};
        lv = LensVjpArgs<T>{};
        la.npix = npix;
        la.nsrc = nsrc;
        la.cell = (T)cell;
        chi_far = cosmo.chi(a0);
        chi_near = cosmo.chi(a1);
        double chis_max = 0;
        for (double c : chisrc) chis_max = std::max(chis_max, c);
        if (chi_near >= chis_max) return false;
        la.chi_near = (T)chi_near;
        la.chi_far = (T)chi_far;
        la.cnear_d = chi_near / cell;
        la.cfar_d = chi_far / cell;
        double dth = fov * PI / 180.0 / npix;
        la.inv_dtheta = (T)(1.0 / dth);
        double vp = std::pow(P.box / P.np, 3);
        la.wbase = (T)(1.5 * P.omega_m / (C_H0 * C_H0) * vp / (dth * dth));
        for (int s = 0; s < nsrc; ++s) la.chi_src[s] = (T)chisrc[s];
        la.atab = atab;
        la.ntab = ATAB_N;
        la.dchi = (T)dchi_tab;
        la.rot = rot ? 1 : 0;
        la.rot_seed = (unsigned long long)rot_seed;
        lv.omega_m = (T)P.omega_m;
        for (int s = 0; s < nsrc; ++s) lv.dchis_dom[s] = (T)((chisrc_p[s] - chisrc_m[s]) / (2 * DOM));
        lv.dadom = adom;
        lv.ntab = ATAB_N;
        lv.dchi = (T)dchi_tab;
        return true;
    }

    int lens_vjp(double a0, double a1, const void* kbar, void* xbar, void* phbar,
                 double* cb) override {
        if (!kbar || !xbar) return PM_EINVAL;
        if (pgd) return PM_EINVAL;  // no reverse pass for the PGD correction
        if (interp && !phbar) return PM_EINVAL;
        if (!at_a(a1)) return PM_ESTATE;
        LensArgs<T> la;
        LensVjpArgs<T> lv;
        double chi_near, chi_far;
        if (!derivative_lens_args(a0, a1, la, lv, chi_near, chi_far)) return PM_OK;
        if (interp) {
            // the step's drift momentum is p - K2 f of the state at a1 (the
            // force there is recomputed by pm_set_state or left by pm_step)
            sub_lens_args(a0, a1, la, lv);
            lv.phbar = reinterpret_cast<T*>(phbar);
        }
        launch_fill<double>(dots, 0.0, 64, st);
        const T* kb = reinterpret_cast<const T*>(kbar);
        { ProfScope ps(prof, "lens_vjp");
          launch_lens_vjp<T>(cur, geo, la, lv, kb, reinterpret_cast<T*>(xbar), dots, st); }
        launch_map_sums<T>(kb, npix, nsrc, dots + 8, st);
        int rc = check_launch();
        if (rc) return rc;
        // the mean term of each map at a fixed shell partition
        double dmean[MAX_SRC];
        for (int s = 0; s < nsrc; ++s) {
            double mp = cosmo_p.shell_mean(chi_near, chi_far, chisrc_p[s]);
            double mm = cosmo_m.shell_mean(chi_near, chi_far, chisrc_m[s]);
            dmean[s] = (mp - mm) / (2 * DOM);
        }
        if (!cb) {
            CosmoCoef c;
            c.add(4, 1.0, 0.0);
            for (int s = 0; s < nsrc; ++s) c.add(8 + s, dmean[s], 0.0);
            launch_cosmo_acc(dots, cacc, c, st);
            return check_launch();
        }
        double d[8 + MAX_SRC];
        if ((rc = read_dots(d, 8 + nsrc))) return rc;
        double g = d[4];
        for (int s = 0; s < nsrc; ++s) g += d[8 + s] * dmean[s];
        cb[0] += g;
        return PM_OK;
    }

    int vjp_cosmo_read(double* cb) override {
        if (!cb) return PM_EINVAL;
        double acc[2];
        HIPCHK(hipMemcpyAsync(acc, cacc, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        launch_fill<double>(cacc, 0.0, 2, st);
        cb[0] += acc[0];
        cb[1] += acc[1];
        return check_launch();
    }

    // ---- forward mode (tangents) ---------------------------------------------
    // The tangent's buffers are part of the arena of a PM_MODE_TANGENT handle.
    int ensure_tangent() const { return tan_mem ? PM_OK : PM_EINVAL; }

    // Force tangent at the current state along tx into tf; with pd set, also
    // the second half-kick p_dot += K2 f_dot + ck2 f.  Leaves the meshes
    // holding the tangent's force meshes.  gathered: the step's readout has
    // already computed fbc and the paint's bound (tan_gather).
    void force_jvp_cur(T* pd, T k2, T ck2, bool gathered = false) {
        const T H = (T)cell;
        const T mass = (T)std::pow((double)geo.B, 3);
        if (!gathered) {
            if (!meshes_valid) {
                paint();
                fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm);
                meshes_valid = true;
            }
            launch_fill_u32(fmax_bits, 0u, 1, st);
            ProfScope ps(prof, "jvp_gather");
            launch_fjvp_gather<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], tx, T(1) / H, mass, fbc,
                                  fmax_bits, st);
        }
        meshes_valid = false;
        // the tangent paint reads x_dot (Mpc/h): mass / H turns it into cells
        { ProfScope ps(prof, "jvp_paint");
          launch_paint_tangent<T>(cur, sb, geo, mass / H, mesh[0], halo, tx, fmax_bits, st, false); }
        fft_forward_grad(P.nm, nullptr, tw_nm, tw_hm, twp_nm, paint_halo_merge<T>(geo, halo));
        { ProfScope ps(prof, "jvp_readout_kick");
          launch_fjvp_readout_kick<T>(cur, sb, geo, mesh[0], mesh[1], mesh[2], fbc, H, k2, ck2, pd, tf,
                                      st); }
    }

    int init_ic_jvp(const void* nd, double om_dot, double s8_dot) override {
        if (ensure_tangent()) return PM_EINVAL;
        if (!nd || !std::isfinite(om_dot) || !std::isfinite(s8_dot)) return PM_EINVAL;
        if (!ic_fresh) return PM_ESTATE;
        const int np = P.np;
        const long n = geo.npart;
        const double a0 = a_cur;
        const T H = (T)cell;
        // lattice-order tangents go to the spare buffers first
        T* xl = tx_alt;
        T* pl = tp_alt;
        meshes_valid = false;
        // displacement tangent of the noise direction; sigma_8 scales the
        // noise, so its tangent adds (s8_dot / s8) noise
        HIPCHK(hipMemcpyAsync(mesh[0], nd, n * sizeof(T), hipMemcpyDeviceToDevice, st));
        if (s8_dot != 0.0) launch_lin<T>(mesh[0], noise_copy, T(1), (T)(s8_dot / P.sigma8), n, st);
        fft_forward_grad(np, g_ic, tw_np, tw_hp, twp_np);
        if (om_dot != 0.0) {
            // + Om_dot dS/dOm (the amplitude table's Omega_m difference), then
            // the growth factors' difference times the displacement itself
            for (int j = 0; j < 3; ++j) launch_lin<T>(xl + j * n, mesh[j], T(0), T(1), n, st);
            HIPCHK(hipMemcpyAsync(mesh[0], noise_copy, n * sizeof(T), hipMemcpyDeviceToDevice, st));
            fft_forward_grad(np, g_ic_dom, tw_np, tw_hp, twp_np);
            for (int j = 0; j < 3; ++j) launch_lin<T>(xl + j * n, mesh[j], T(1), (T)om_dot, n, st);
            HIPCHK(hipMemcpyAsync(mesh[0], noise_copy, n * sizeof(T), hipMemcpyDeviceToDevice, st));
            fft_forward_grad(np, g_ic, tw_np, tw_hp, twp_np);
            const double dd0 = (cosmo_p.D(a0) - cosmo_m.D(a0)) / (2 * DOM);
            const double dgp0 = (cosmo_p.gp(a0) - cosmo_m.gp(a0)) / (2 * DOM);
            launch_ic_tangent<T>(xl, xl + n, xl + 2 * n, mesh[0], mesh[1], mesh[2], xl, pl,
                                 (T)cosmo.D(a0), (T)cosmo.gp(a0), (T)(om_dot * dd0),
                                 (T)(om_dot * dgp0), H, n, st);
        } else {
            launch_ic_tangent<T>(mesh[0], mesh[1], mesh[2], mesh[0], mesh[1], mesh[2], xl, pl,
                                 (T)cosmo.D(a0), (T)cosmo.gp(a0), T(0), T(0), H, n, st);
        }
        launch_lattice_to_sorted<T>(cur, geo, xl, tx, st);
        launch_lattice_to_sorted<T>(cur, geo, pl, tp, st);
        force_jvp_cur(nullptr, T(0), T(0));
        tan_om = om_dot;
        tan_valid = true;
        return check_launch();
    }

    int set_tangent(const void* xd, const void* pd, double om_dot) override {
        if (ensure_tangent()) return PM_EINVAL;
        if (!xd || !pd || !std::isfinite(om_dot)) return PM_EINVAL;
        if (a_cur < 0) return PM_ESTATE;
        launch_lattice_to_sorted<T>(cur, geo, reinterpret_cast<const T*>(xd), tx, st);
        launch_lattice_to_sorted<T>(cur, geo, reinterpret_cast<const T*>(pd), tp, st);
        force_jvp_cur(nullptr, T(0), T(0));
        tan_om = om_dot;
        tan_valid = true;
        return check_launch();
    }

    int get_tangent(void* xd, void* pd, void* fd) override {
        if (ensure_tangent()) return PM_EINVAL;
        if (!tan_valid) return PM_ESTATE;
        const long n = geo.npart;
        T* out[3] = {reinterpret_cast<T*>(xd), reinterpret_cast<T*>(pd), reinterpret_cast<T*>(fd)};
        const T* src[3] = {tx, tp, tf};
        for (int i = 0; i < 3; ++i)
            if (out[i])
                launch_sorted_to_lattice<T>(cur, geo, src[i], out[i], out[i] + n, out[i] + 2 * n, st);
        return check_launch();
    }

    int step_jvp(double a0, double a1) override {
        if (ensure_tangent()) return PM_EINVAL;
        if (!tan_valid) return PM_ESTATE;
        if (!at_a(a0)) return PM_ESTATE;
        if (!(a1 > 0 && a1 <= 1.5)) return PM_EINVAL;
        const double om_dot = tan_om;
        const double ah = 0.5 * (a0 + a1);
        const double k1 = cosmo.kick(a0, ah, a0), dr = cosmo.drift(a0, a1, ah);
        const double k2 = cosmo.kick(ah, a1, a1);
        const double dk1 = (cosmo_p.kick(a0, ah, a0) - cosmo_m.kick(a0, ah, a0)) / (2 * DOM);
        const double ddr = (cosmo_p.drift(a0, a1, ah) - cosmo_m.drift(a0, a1, ah)) / (2 * DOM);
        const double dk2 = (cosmo_p.kick(ah, a1, a1) - cosmo_m.kick(ah, a1, a1)) / (2 * DOM);
        { ProfScope ps(prof, "jvp_kick_drift");
          launch_jvp_pre<T>(cur, geo, tx, tp, tf, (T)cell, (T)k1, (T)dr, (T)(om_dot * dk1),
                            (T)(om_dot * ddr), st); }
        // the forward step with the kernels of pm_step; its sort carries the
        // tangent, and its readout computes the tangent's share of the force
        tan_carry = true;
        tan_gather = true;
        int rc = step(a0, a1);
        tan_carry = false;
        tan_gather = false;
        if (rc) return rc;
        force_jvp_cur(tp, (T)k2, (T)(om_dot * dk2), true);
        tan_valid = true;
        return check_launch();
    }

    // Sub-evolution fields of the derivative passes' lens arguments for the
    // step a0 -> a1: the drift momentum is p - K2 f of the state at a1.
    void sub_lens_args(double a0, double a1, LensArgs<T>& la, LensVjpArgs<T>& lv) {
        const double ah = 0.5 * (a0 + a1);
        la.sub = 1;
        la.dtab = dtab;
        la.d_end = (T)cosmo.D(a1);
        la.sub_scale = (T)(1.0 / cosmo.gp(ah));
        la.sub_dr = (T)std::fabs(cosmo.drift(a0, a1, ah));
        la.sub_k2 = (T)cosmo.kick(ah, a1, a1);
        lv.ddom = ddom;
        lv.dd_end_dom = (T)((cosmo_p.D(a1) - cosmo_m.D(a1)) / (2 * DOM));
        lv.dscale_dom = (T)((1.0 / cosmo_p.gp(ah) - 1.0 / cosmo_m.gp(ah)) / (2 * DOM));
    }

    int lens_jvp(double a0, double a1, void* kd) override {
        if (ensure_tangent() || !kd) return PM_EINVAL;
        if (pgd) return PM_EINVAL;  // no tangent pass for the PGD correction
        if (!tan_valid || !at_a(a1)) return PM_ESTATE;
        LensArgs<T> la;
        LensVjpArgs<T> lv;
        double chi_near, chi_far;
        if (!derivative_lens_args(a0, a1, la, lv, chi_near, chi_far)) return PM_OK;
        const double om_dot = tan_om;
        T ck2 = T(0);
        if (interp) {
            sub_lens_args(a0, a1, la, lv);
            const double ah = 0.5 * (a0 + a1);
            ck2 = (T)(om_dot * (cosmo_p.kick(ah, a1, a1) - cosmo_m.kick(ah, a1, a1)) / (2 * DOM));
        }
        T* kdot = reinterpret_cast<T*>(kd);
        { ProfScope ps(prof, "lens_jvp");
          launch_lens_jvp<T>(cur, geo, la, lv, tx, tp, tf, ck2, (T)om_dot, kdot, st); }
        if (om_dot != 0.0) {
            // the mean term's Omega_m derivative at a fixed shell partition
            MapAdd<T> mv{};
            for (int s = 0; s < nsrc; ++s) {
                const double mp = cosmo_p.shell_mean(chi_near, chi_far, chisrc_p[s]);
                const double mm = cosmo_m.shell_mean(chi_near, chi_far, chisrc_m[s]);
                mv.v[s] = (T)(om_dot * (mp - mm) / (2 * DOM));
            }
            launch_map_add<T>(kdot, npix, nsrc, mv, st);
        }
        return check_launch();
    }

    // ---- batched stepping (pm_batch_*) ----------------------------------------
    // A handle joins a batch at a_grid[0] after its initial conditions: the
    // batch enqueues this step's first half-kick, drift and sort keys on its
    // own stream; each batched step then runs pm_run's fused step (sort,
    // paint, shell, force, readout that starts the next step).
    bool batch_compatible(const pm_params& shape, int npx, int ns) const {
        return P.np == shape.np && P.nm == shape.nm && P.dtype == shape.dtype && npix == npx &&
               nsrc == ns && !interp && !pgd && !rot;
    }

    // bst must already wait for the handle's own stream (its initial conditions).
    int batch_begin(hipStream_t bst, double a0, double a1) {
        if (a_cur < 0 || std::fabs(a0 - a_cur) > 1e-12 * std::fabs(a_cur) + 1e-15) return PM_ESTATE;
        const double ah = 0.5 * (a0 + a1);
        launch_fill_u32(sb.count, 0u, ntiles, bst);
        launch_kick_drift_key<T>(cur, sb, geo, (T)cosmo.kick(a0, ah, a0),
                                 (T)cosmo.drift(a0, a1, ah), MODE_KICK | MODE_DRIFT, status, bst);
        a_cur = -1.0;  // between steps until the batch leaves it at a step's end
        ic_fresh = false;
        tan_valid = false;
        kdk_a0 = kdk_a1 = -1.0;
        meshes_valid = false;
        return check_launch();
    }

    // The arguments of every pass of the fused step a0 -> a1 (a2 > a1: the
    // next step's end, whose first half-kick and drift the readout applies;
    // a2 <= 0: the last step), and the host's bookkeeping of the sort's
    // buffer swap.  kappa NULL: no projection.
    void batch_step_args(double a0, double a1, double a2, T* kappa, BatchSlotArgs<T>& o) {
        const int nm = P.nm;
        o.scan = ScanArgs{sb.count, sb.start, scan_sum, ntiles, 1};
        o.scatter = ScatterArgs<T>{cur, alt, sb, geo, 1};
        std::swap(cur.disp, alt.disp);
        std::swap(cur.mom, alt.mom);
        std::swap(cur.id, alt.id);
        o.paint = PaintArgs<T>{cur, sb, geo, (T)std::pow((double)geo.B, 3), mesh[0], halo, 1};
        o.lens = LensGatherArgs<T>{};
        if (kappa && plain_lens_args(a0, a1, o.lens.la, o.lens.mean)) {
            // the batch's grid has one region side for every shell: one
            // accumulator per source
            o.lens.la.dec = 0;
            o.lens.la.rs = region_side(nsrc, npix);
            o.lens.p = cur;
            o.lens.sb = sb;
            o.lens.g = geo;
            o.lens.kappa = kappa;
            o.lens.on = 1;
        }
        o.r2c = R2cArgs<T>{mesh[0], nyq[0], tw_hm, twp_nm, paint_halo_merge<T>(geo, halo), 1};
        o.fwd = fft_c2c_axis1_args<T>(nm, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm);
        const T gscale = (T)(1.0 / (2.0 * PI * (double)nm * (double)nm));
        PtrTriple om{{mesh[0], mesh[1], mesh[2]}}, on{{nyq[0], nyq[1], nyq[2]}};
        o.grad = fft_grad_axis0_args<T>(nm, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], om, on,
                                        tw_nm, nullptr, gscale);
        C2cArgs<T> inv = fft_c2c_axis1_args<T>(nm, reinterpret_cast<cx<T>*>(mesh[0]), nyq[0], tw_nm);
        o.inv = inv;
        o.dual = fft_c2c_axis1_dual_args<T>(nm, reinterpret_cast<cx<T>*>(mesh[1]), nyq[1],
                                            reinterpret_cast<cx<T>*>(mesh[2]), nyq[2], tw_nm);
        for (int j = 0; j < 3; ++j)
            o.c2r[j] = C2rArgs<T>{mesh[j], nyq[j], tw_hm, twp_nm, j == 2 ? 1 : 0, 1};
        const double ah = 0.5 * (a0 + a1);
        ReadoutNext<T> nx;
        o.fill = FillArgs{sb.count, (long)ntiles, 0};
        if (a2 > a1) {
            const double ah2 = 0.5 * (a1 + a2);
            nx.on = 1;
            nx.kick = (T)cosmo.kick(a1, ah2, a1);
            nx.drift = (T)cosmo.drift(a1, a2, ah2);
            o.fill.on = 1;
        }
        o.readout = ReadoutArgs<T>{cur, sb, geo, mesh[0], mesh[1], mesh[2],
                                   (T)cosmo.kick(ah, a1, a1), 1, status, nx, 1};
        if (a2 <= a1) {  // the step ends the handle's run: the state is at a1
            meshes_valid = true;
            a_cur = a1;
            kdk_a0 = a0;
            kdk_a1 = a1;
            kdk_k2 = (T)cosmo.kick(ah, a1, a1);
        }
    }

    // Leaving a batch before its last step: the state is between two steps
    // (drifted, keys written) and no call can continue it.
    void batch_abandon() {
        a_cur = -1.0;
        kdk_a0 = kdk_a1 = -1.0;
        meshes_valid = false;
    }

    hipStream_t stream() const override { return st; }

    int background(double a, double out[3]) const override {
        out[0] = cosmo.D(a);
        out[1] = cosmo.gp(a);
        out[2] = cosmo.chi(a);
        return PM_OK;
    }
};

}  // namespace

struct pm_sim {
    std::unique_ptr<SimBase> impl;
    int dtype;
};

namespace {

// ---- batches: one launch per pass over same-shape simulations ---------------
// The device parameter block holds one array of argument structs per pass
// (capacity entries; three per slot for the c2r pass).  A step fills a
// pinned host copy, copies it to the device on the batch's stream and
// replays the launches (a HIP graph of kernel nodes only, captured at the
// first step, or the launches themselves), so nothing in the launches
// changes from step to step.
struct BatchBase {
    virtual ~BatchBase() {}
    virtual int attach(pm_sim* sim, const double* a_grid, int nsteps, int* slot_out) = 0;
    virtual int lens(pm_sim* sim, void* kappa) = 0;
    virtual int detach(pm_sim* sim) = 0;
    virtual int step(int* running_out) = 0;
};

template <class T> struct Batch final : BatchBase {
    pm_params shape{};
    int npix = 0, nsrc = 0, cap = 0;
    bool use_graph = true;
    hipStream_t st = nullptr;
    bool own_stream = false;
    Geo geo{};
    LensArgs<T> lshape{};
    struct Slot {
        pm_sim* h = nullptr;
        Sim<T>* sim = nullptr;
        std::vector<double> agrid;
        int next = 0;
        T* kappa = nullptr;
    };
    std::vector<Slot> slots;
    // parameter block: offsets of the per-pass arrays
    size_t o_fill, o_scan, o_scatter, o_paint, o_lens, o_r2c, o_fwd, o_grad, o_inv, o_dual, o_c2r,
        o_readout, bytes;
    char* dev = nullptr;
    char* host[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t handoff = nullptr;  // orders a handle's stream with the batch's
    int ring = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~Batch() override {
        if (st) (void)hipStreamSynchronize(st);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int i = 0; i < 2; ++i) {
            if (copied[i]) (void)hipEventDestroy(copied[i]);
            if (host[i]) (void)hipHostFree(host[i]);
        }
        if (handoff) (void)hipEventDestroy(handoff);
        if (dev) (void)hipFree(dev);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }

    int create(const pm_params* p, const lens_params* l, int capacity, int graph_on,
               void* stream) {
        shape = *p;
        npix = l->npix;
        nsrc = l->nsrc;
        cap = capacity;
        use_graph = graph_on != 0;
        geo.np = p->np;
        geo.nm = p->nm;
        geo.B = p->nm / p->np;
        geo.nt = p->nm / TILE;
        geo.ncb = geo.nt * BPT;
        geo.npart = (long)p->np * p->np * p->np;
        lshape.npix = npix;
        lshape.nsrc = nsrc;
        lshape.rs = Sim<T>::region_side(nsrc, npix);
        slots.resize(cap);
        size_t b = 0;
        auto take = [&](size_t n) {
            size_t off = (b + 255) & ~size_t(255);
            b = off + n;
            return off;
        };
        o_fill = take(cap * sizeof(FillArgs));
        o_scan = take(cap * sizeof(ScanArgs));
        o_scatter = take(cap * sizeof(ScatterArgs<T>));
        o_paint = take(cap * sizeof(PaintArgs<T>));
        o_lens = take(cap * sizeof(LensGatherArgs<T>));
        o_r2c = take(cap * sizeof(R2cArgs<T>));
        o_fwd = take(cap * sizeof(C2cArgs<T>));
        o_grad = take(cap * sizeof(GradArgs<T>));
        o_inv = take(cap * sizeof(C2cArgs<T>));
        o_dual = take(cap * sizeof(DualArgs<T>));
        o_c2r = take(3 * cap * sizeof(C2rArgs<T>));
        o_readout = take(cap * sizeof(ReadoutArgs<T>));
        bytes = b;
        if (stream) {
            st = reinterpret_cast<hipStream_t>(stream);
        } else {
            // graph capture needs a stream other than the legacy default one
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return PM_EDEVICE;
            own_stream = true;
        }
        prepare_lens_gather_batch<T>();
        if (hipMalloc(&dev, bytes) != hipSuccess) {
            dev = nullptr;
            (void)hipGetLastError();
            return PM_ENOMEM;
        }
        for (int i = 0; i < 2; ++i) {
            if (hipHostMalloc(&host[i], bytes, hipHostMallocDefault) != hipSuccess) {
                host[i] = nullptr;
                (void)hipGetLastError();
                return PM_ENOMEM;
            }
            std::memset(host[i], 0, bytes);
            HIPCHK(hipEventCreateWithFlags(&copied[i], hipEventDisableTiming));
        }
        HIPCHK(hipEventCreateWithFlags(&handoff, hipEventDisableTiming));
        return PM_OK;
    }

    // Later work on `to` waits for everything enqueued on `from` so far.
    int order(hipStream_t from, hipStream_t to) {
        HIPCHK(hipEventRecord(handoff, from));
        HIPCHK(hipStreamWaitEvent(to, handoff, 0));
        return PM_OK;
    }

    int find(pm_sim* h) const {
        for (int i = 0; i < cap; ++i)
            if (slots[i].h == h) return i;
        return -1;
    }

    int attach(pm_sim* h, const double* a_grid, int nsteps, int* slot_out) override {
        if (!h || !a_grid || nsteps < 1 || h->dtype != shape.dtype) return PM_EINVAL;
        if (find(h) >= 0) return PM_EINVAL;
        auto* sim = dynamic_cast<Sim<T>*>(h->impl.get());
        if (!sim || !sim->batch_compatible(shape, npix, nsrc)) return PM_EINVAL;
        for (int i = 0; i < nsteps; ++i)
            if (!(a_grid[i + 1] > 0 && a_grid[i + 1] <= 1.5)) return PM_EINVAL;
        int k = find(nullptr);
        if (k < 0) return PM_EFULL;
        if (sim->a_cur < 0 ||
            std::fabs(a_grid[0] - sim->a_cur) > 1e-12 * std::fabs(sim->a_cur) + 1e-15)
            return PM_ESTATE;
        int rc = order(sim->st, st);  // the handle's initial conditions first
        if (rc) return rc;
        if ((rc = sim->batch_begin(st, a_grid[0], a_grid[1]))) return rc;
        Slot& s = slots[k];
        s.h = h;
        s.sim = sim;
        s.agrid.assign(a_grid, a_grid + nsteps + 1);
        s.next = 0;
        s.kappa = nullptr;
        if (slot_out) *slot_out = k;
        return PM_OK;
    }

    int lens(pm_sim* h, void* kappa) override {
        int k = find(h);
        if (k < 0) return PM_EINVAL;
        slots[k].kappa = reinterpret_cast<T*>(kappa);
        return PM_OK;
    }

    int detach(pm_sim* h) override {
        int k = find(h);
        if (k < 0) return PM_EINVAL;
        Slot& s = slots[k];
        // the handle's later work waits for the batch's steps enqueued so far
        int rc = order(st, s.sim->st);
        if (rc) return rc;
        if (s.next < (int)s.agrid.size() - 1) s.sim->batch_abandon();
        s = Slot{};
        return PM_OK;
    }

    template <class A> A* arr(char* base, size_t off) { return reinterpret_cast<A*>(base + off); }

    void launch_all(char* base) {
        const int nm = shape.nm;
        const int ntiles = geo.nt * geo.nt * geo.ncb;
        launch_scan_batch(arr<ScanArgs>(base, o_scan), ntiles, cap, st);
        launch_scatter_batch<T>(arr<ScatterArgs<T>>(base, o_scatter), geo, cap, st);
        launch_paint_batch<T>(arr<PaintArgs<T>>(base, o_paint), geo, cap, st);
        launch_lens_gather_batch<T>(arr<LensGatherArgs<T>>(base, o_lens), lshape, cap, st);
        fft_r2c_rows_batch<T>(nm, arr<R2cArgs<T>>(base, o_r2c), cap, st);
        fft_c2c_axis1_batch<T>(nm, 1, arr<C2cArgs<T>>(base, o_fwd), cap, st);
        fft_grad_axis0_batch<T>(nm, arr<GradArgs<T>>(base, o_grad), cap, st);
        fft_c2c_axis1_batch<T>(nm, -1, arr<C2cArgs<T>>(base, o_inv), cap, st);
        fft_c2c_axis1_dual_batch<T>(nm, arr<DualArgs<T>>(base, o_dual), cap, st);
        fft_c2r_rows_batch<T>(nm, arr<C2rArgs<T>>(base, o_c2r), 3 * cap, st);
        launch_fill_batch(arr<FillArgs>(base, o_fill), ntiles, cap, st);
        launch_readout_batch<T>(arr<ReadoutArgs<T>>(base, o_readout), geo, cap, st);
    }

    int step(int* running_out) override {
        char* h = host[ring];
        HIPCHK(hipEventSynchronize(copied[ring]));  // its last copy has been read
        std::memset(h, 0, bytes);  // every pass of an idle slot: on = 0
        int running = 0;
        for (int k = 0; k < cap; ++k) {
            Slot& s = slots[k];
            const int n = (int)s.agrid.size() - 1;
            if (!s.sim || s.next >= n) continue;
            const int i = s.next;
            BatchSlotArgs<T> a;
            s.sim->batch_step_args(s.agrid[i], s.agrid[i + 1], i + 1 < n ? s.agrid[i + 2] : -1.0,
                                   s.kappa, a);
            arr<FillArgs>(h, o_fill)[k] = a.fill;
            arr<ScanArgs>(h, o_scan)[k] = a.scan;
            arr<ScatterArgs<T>>(h, o_scatter)[k] = a.scatter;
            arr<PaintArgs<T>>(h, o_paint)[k] = a.paint;
            arr<LensGatherArgs<T>>(h, o_lens)[k] = a.lens;
            arr<R2cArgs<T>>(h, o_r2c)[k] = a.r2c;
            arr<C2cArgs<T>>(h, o_fwd)[k] = a.fwd;
            arr<GradArgs<T>>(h, o_grad)[k] = a.grad;
            arr<C2cArgs<T>>(h, o_inv)[k] = a.inv;
            arr<DualArgs<T>>(h, o_dual)[k] = a.dual;
            for (int j = 0; j < 3; ++j) arr<C2rArgs<T>>(h, o_c2r)[3 * k + j] = a.c2r[j];
            arr<ReadoutArgs<T>>(h, o_readout)[k] = a.readout;
            ++s.next;
            if (s.next < n) ++running;
        }
        if (running_out) *running_out = running;
        HIPCHK(hipMemcpyAsync(dev, h, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(hipEventRecord(copied[ring], st));
        ring ^= 1;
        if (!use_graph) {
            launch_all(dev);
            return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
        }
        if (!exec) {
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            launch_all(dev);
            hipError_t e = hipStreamEndCapture(st, &graph);
            if (e != hipSuccess || !graph) {
                (void)hipGetLastError();
                return PM_EDEVICE;
            }
            HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(exec, st));
        return PM_OK;
    }
};

}  // namespace

struct pm_batch {
    std::unique_ptr<BatchBase> impl;
};

namespace {

// The arena of pm_run_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  In host code its name
// is a host-side stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device (with that device current) on
// the entry point's first call there, and only that address is passed on.
__device__ __align__(256) unsigned char scratch[PM_NOALLOC_MAX_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

int scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return PM_EDEVICE;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return PM_EDEVICE;
        }
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return PM_OK;
}

template <class T>
int run_noalloc_t(const pm_params* p, const lens_params* l, void* stream, const void* noise,
                  const double* a_grid, int32_t nsteps, void* kappa) {
    void* mem = nullptr;
    int rc = scratch_for_current_device(&mem);
    if (rc) return rc;
    // the previous call on this stream may still read the array: the table
    // uploads below are ordered with the host, not with the stream
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return PM_EDEVICE;
    Sim<T> sim;
    if ((rc = sim.create(p, l, stream, mem))) return rc;
    if ((rc = sim.init_ic(noise, a_grid[0]))) return rc;
    return sim.run(a_grid, nsteps, kappa);
}

}  // namespace

extern "C" {

int pm_batch_create(const pm_params* shape, const lens_params* lens_shape, int32_t capacity,
                    int32_t use_graph, void* hip_stream, pm_batch** out) {
    if (!out) return PM_EINVAL;
    *out = nullptr;
    int rc = validate(shape, lens_shape);
    if (rc) return rc;
    if (capacity < 1 || capacity > 1024) return PM_EINVAL;
    pm_batch* b = new (std::nothrow) pm_batch;
    if (!b) return PM_ENOMEM;
    if (shape->dtype == PM_F32) {
        auto* impl = new (std::nothrow) Batch<float>;
        b->impl.reset(impl);
        rc = impl ? impl->create(shape, lens_shape, capacity, use_graph, hip_stream) : PM_ENOMEM;
    } else {
        auto* impl = new (std::nothrow) Batch<double>;
        b->impl.reset(impl);
        rc = impl ? impl->create(shape, lens_shape, capacity, use_graph, hip_stream) : PM_ENOMEM;
    }
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return PM_OK;
}

int pm_batch_destroy(pm_batch* b) {
    if (!b) return PM_EINVAL;
    delete b;
    return PM_OK;
}

int pm_batch_attach(pm_batch* b, pm_sim* sim, const double* a_grid, int32_t nsteps,
                    int32_t* slot_out) {
    if (!b) return PM_EINVAL;
    int k = -1;
    int rc = b->impl->attach(sim, a_grid, nsteps, &k);
    if (rc == PM_OK && slot_out) *slot_out = k;
    return rc;
}

int pm_batch_lens(pm_batch* b, pm_sim* sim, void* kappa) {
    return b ? b->impl->lens(sim, kappa) : PM_EINVAL;
}

int pm_batch_detach(pm_batch* b, pm_sim* sim) { return b ? b->impl->detach(sim) : PM_EINVAL; }

int pm_batch_step(pm_batch* b, int32_t* running_out) {
    if (!b) return PM_EINVAL;
    int r = 0;
    int rc = b->impl->step(&r);
    if (running_out) *running_out = r;
    return rc;
}

int pm_run_noalloc(const pm_params* p, const lens_params* l, void* hip_stream, const void* noise,
                   const double* a_grid, int32_t nsteps, void* kappa) {
    int rc = validate(p, l);
    if (rc) return rc;
    if (p->modes != 0 || !noise || !a_grid || !kappa || nsteps < 1) return PM_EINVAL;
    if (plan_arena(*p, *l, p->dtype == PM_F64 ? 8 : 4).total > PM_NOALLOC_MAX_BYTES)
        return PM_ETOOBIG;
    return p->dtype == PM_F32
               ? run_noalloc_t<float>(p, l, hip_stream, noise, a_grid, nsteps, kappa)
               : run_noalloc_t<double>(p, l, hip_stream, noise, a_grid, nsteps, kappa);
}

size_t pm_footprint(const pm_params* p, const lens_params* l) {
    if (validate(p, l) != PM_OK) return 0;
    return plan_arena(*p, *l, p->dtype == PM_F64 ? 8 : 4).total;
}

int pm_create(const pm_params* p, const lens_params* l, void* hip_stream, pm_sim** out) {
    if (!out) return PM_EINVAL;
    *out = nullptr;
    int rc = validate(p, l);
    if (rc) return rc;
    pm_sim* s = new (std::nothrow) pm_sim;
    if (!s) return PM_ENOMEM;
    s->dtype = p->dtype;
    if (p->dtype == PM_F32) {
        auto* impl = new (std::nothrow) Sim<float>;
        if (!impl) { delete s; return PM_ENOMEM; }
        s->impl.reset(impl);
        rc = impl->create(p, l, hip_stream);
    } else {
        auto* impl = new (std::nothrow) Sim<double>;
        if (!impl) { delete s; return PM_ENOMEM; }
        s->impl.reset(impl);
        rc = impl->create(p, l, hip_stream);
    }
    if (rc) {
        delete s;
        return rc;
    }
    *out = s;
    return PM_OK;
}

int pm_destroy(pm_sim* sim) {
    if (!sim) return PM_EINVAL;
    delete sim;
    return PM_OK;
}

int pm_init_ic(pm_sim* sim, const void* noise, double a0) {
    return sim ? sim->impl->init_ic(noise, a0) : PM_EINVAL;
}
int pm_init_ic_seed(pm_sim* sim, uint64_t seed, double a0) {
    return sim ? sim->impl->init_ic_seed(seed, a0) : PM_EINVAL;
}
int pm_noise(pm_sim* sim, uint64_t seed, void* noise_out) {
    return sim ? sim->impl->noise(seed, noise_out) : PM_EINVAL;
}
int pm_reconfigure(pm_sim* sim, const pm_params* p, const lens_params* l) {
    if (!sim) return PM_EINVAL;
    int rc = validate(p, l);
    return rc ? rc : sim->impl->reconfigure(p, l);
}
int pm_step(pm_sim* sim, double a0, double a1) { return sim ? sim->impl->step(a0, a1) : PM_EINVAL; }
int pm_run(pm_sim* sim, const double* a_grid, int32_t nsteps, void* kappa) {
    return sim ? sim->impl->run(a_grid, nsteps, kappa) : PM_EINVAL;
}
int pm_set_interpolation(pm_sim* sim, int32_t on) {
    return sim ? sim->impl->set_interpolation(on) : PM_EINVAL;
}
int pm_set_replica_rotation(pm_sim* sim, int32_t on, uint64_t seed) {
    return sim ? sim->impl->set_replica_rotation(on, seed) : PM_EINVAL;
}
int pm_set_pgd(pm_sim* sim, int32_t on, double alpha0, double mu, double k_l, double k_s) {
    return sim ? sim->impl->set_pgd(on, alpha0, mu, k_l, k_s) : PM_EINVAL;
}
int lens_project(pm_sim* sim, double a0, double a1, void* kappa) {
    return sim ? sim->impl->lens(a0, a1, kappa) : PM_EINVAL;
}
int pm_get_state(pm_sim* sim, void* x, void* p, double* a) {
    return sim ? sim->impl->get_state(x, p, a) : PM_EINVAL;
}
int pm_set_state(pm_sim* sim, const void* x, const void* p, double a) {
    return sim ? sim->impl->set_state(x, p, a) : PM_EINVAL;
}
int pm_get_force(pm_sim* sim, void* rho, void* fm, void* acc) {
    return sim ? sim->impl->get_force(rho, fm, acc) : PM_EINVAL;
}
int pm_sync(pm_sim* sim) { return sim ? sim->impl->sync() : PM_EINVAL; }
int lens_project_vjp(pm_sim* sim, double a0, double a1, const void* kappa_bar, void* x_bar,
                     void* ph_bar, double cosmo_bar[2]) {
    return sim ? sim->impl->lens_vjp(a0, a1, kappa_bar, x_bar, ph_bar, cosmo_bar) : PM_EINVAL;
}
int pm_step_vjp(pm_sim* sim, double a0, double a1, double a2, void* x_bar, void* p_bar,
                const void* ph_bar, double cosmo_bar[2]) {
    return sim ? sim->impl->step_vjp(a0, a1, a2, x_bar, p_bar, ph_bar, cosmo_bar) : PM_EINVAL;
}
int pm_init_ic_vjp(pm_sim* sim, double a1, const void* x_bar, const void* p_bar, void* noise_bar,
                   double cosmo_bar[2]) {
    return sim ? sim->impl->init_ic_vjp(a1, x_bar, p_bar, noise_bar, cosmo_bar) : PM_EINVAL;
}
size_t pm_checkpoint_bytes(const pm_sim* sim) { return sim ? sim->impl->checkpoint_bytes() : 0; }
int pm_checkpoint_save(pm_sim* sim, void* buf) {
    return sim ? sim->impl->checkpoint_save(buf) : PM_EINVAL;
}
int pm_checkpoint_load(pm_sim* sim, const void* buf, double a) {
    return sim ? sim->impl->checkpoint_load(buf, a) : PM_EINVAL;
}
int pm_vjp_cosmo_read(pm_sim* sim, double cosmo_bar[2]) {
    return sim ? sim->impl->vjp_cosmo_read(cosmo_bar) : PM_EINVAL;
}
int pm_init_ic_jvp(pm_sim* sim, const void* noise_dot, double omega_m_dot, double sigma8_dot) {
    return sim ? sim->impl->init_ic_jvp(noise_dot, omega_m_dot, sigma8_dot) : PM_EINVAL;
}
int pm_set_tangent(pm_sim* sim, const void* x_dot, const void* p_dot, double omega_m_dot) {
    return sim ? sim->impl->set_tangent(x_dot, p_dot, omega_m_dot) : PM_EINVAL;
}
int pm_get_tangent(pm_sim* sim, void* x_dot, void* p_dot, void* f_dot) {
    return sim ? sim->impl->get_tangent(x_dot, p_dot, f_dot) : PM_EINVAL;
}
int pm_step_jvp(pm_sim* sim, double a0, double a1) {
    return sim ? sim->impl->step_jvp(a0, a1) : PM_EINVAL;
}
int lens_project_jvp(pm_sim* sim, double a0, double a1, void* kappa_dot) {
    return sim ? sim->impl->lens_jvp(a0, a1, kappa_dot) : PM_EINVAL;
}
int pm_background(const pm_sim* sim, double a, double out[3]) {
    return sim && out ? sim->impl->background(a, out) : PM_EINVAL;
}

int pm_profile(pm_sim* sim, int enable) {
    if (!sim) return PM_EINVAL;
    return sim->impl->prof.enable(enable != 0, sim->impl->stream());
}

int pm_profile_only(pm_sim* sim, const char* name) {
    if (!sim) return PM_EINVAL;
    sim->impl->prof.only = name ? name : "";
    return PM_OK;
}

int pm_profile_read(pm_sim* sim, int max_kernels, char* names, double* ms_total, long* counts,
                    int* n_out) {
    if (!sim || !n_out || max_kernels < 0) return PM_EINVAL;
    Prof& p = sim->impl->prof;
    int rc = p.resolve();
    if (rc) return rc;
    int n = (int)p.names.size();
    *n_out = n;
    for (int i = 0; i < n && i < max_kernels; ++i) {
        if (names) {
            std::strncpy(names + 32 * i, p.names[i].c_str(), 31);
            names[32 * i + 31] = 0;
        }
        if (ms_total) ms_total[i] = p.ms[i];
        if (counts) counts[i] = p.cnt[i];
        p.ms[i] = 0.0;
        p.cnt[i] = 0;
    }
    return PM_OK;
}

const char* pm_strerror(int code) {
    switch (code) {
        case PM_OK: return "ok";
        case PM_EINVAL: return "invalid argument or unsupported size";
        case PM_ENOMEM: return "device arena could not be allocated";
        case PM_EDEVICE: return "HIP runtime error";
        case PM_ESTATE: return "simulation is not in the required state";
        case PM_ENONFINITE: return "non-finite particle position";
        case PM_EAGAIN: return "not finished yet";
        case PM_EFULL: return "every slot of the batch is taken";
        case PM_ETOOBIG:
            return "arena larger than the static scratch of the non-allocating entry point";
        default: return "unknown error";
    }
}

}  // extern "C"
