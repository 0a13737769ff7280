// C ABI of the barotropic subcycle library: argument validation, mesh and
// plan management, and the launch sequences of the forward paths.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "consumers.h"
#include "ensemble.h"
#include "kernels.h"
#include "se_internal.h"

namespace sesub {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }

DevBuf::~DevBuf() {
    if (p) (void)hipFree(p);
}

se_status DevBuf::alloc(size_t bytes) {
    if (p) {
        (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    if (bytes == 0) return SE_OK;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
        return SE_ERR_OOM;
    }
    n = bytes;
    return SE_OK;
}

se_status DevBuf::upload(const void *src, size_t bytes) {
    se_status s = alloc(bytes);
    if (s != SE_OK || bytes == 0) return s;
    if (hipMemcpy(p, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("host to device copy failed");
        return SE_ERR_HIP;
    }
    return SE_OK;
}

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

se_status hip_fail(hipError_t e, const char *where) {
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return SE_ERR_HIP;
}

#define SE_TRY(x)                         \
    do {                                  \
        se_status _s = (x);               \
        if (_s != SE_OK) return _s;       \
    } while (0)

#define HIP_TRY(x, where)                         \
    do {                                          \
        hipError_t _e = (x);                      \
        if (_e != hipSuccess) return hip_fail(_e, where); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

constexpr int kEpts[] = {1, 2, 3, 4, 6, 8};

int pick_ept(int need) {
    for (int e : kEpts)
        if (e >= need) return e;
    return -1;
}

// Geometry of a triangle set as 5 SoA arrays (gbx gby gcx gcy Ae).
template <typename T>
std::vector<T> pack_geom(const HostMesh &m, const std::vector<int32_t> *sel, int64_t off) {
    const int64_t n = sel ? static_cast<int64_t>(sel->size()) : m.ne;
    std::vector<T> g(5 * n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t e = sel ? (*sel)[i] - off : i;
        const double *gn = &m.gN[6 * e];
        g[i] = static_cast<T>(gn[2]);
        g[n + i] = static_cast<T>(gn[3]);
        g[2 * n + i] = static_cast<T>(gn[4]);
        g[3 * n + i] = static_cast<T>(gn[5]);
        g[4 * n + i] = static_cast<T>(m.Ae[e]);
    }
    return g;
}

// Register tiers that compile without scratch spills (triangles per thread).
bool ept_ok(bool f32, int ept, int block, bool sm = false) {
    if (ept < 0) return false;
    if (block == 256) return f32 ? ept <= 8 : ept <= 6;
    if (block == 512) return f32 ? ept <= 8 : ept <= 4;
    // 1024 threads: at most 128 VGPRs (the AB3-AM4 form holds two more transports)
    return f32 ? ept <= (sm ? 3 : 4) : ept <= (sm ? 1 : 3);
}

// Host-side construction and statistics of a plan (no device memory).
se_status plan_host(const std::vector<const HostMesh *> &members, const std::vector<int64_t> &voff,
                    const std::vector<int64_t> &eoff, int32_t T, int32_t K, int32_t block,
                    HostTiles &ht, se_plan_stats_t &st) {
    if (T < 64 || T > 8192 || K < 1 || K > 8 || (block != 256 && block != 512 && block != 1024)) {
        set_error("se_set_plan: tile in [64, 8192], k_fused in [1, 8], block 256, 512 or 1024");
        return SE_ERR_ARG;
    }
    SE_TRY(build_tiles(members, voff, eoff, T, K, ht));
    // a few tiles with more local triangles than the rest (a long coast, a fold of the
    // curve) set the register tier of all: when at most one tile in 50 exceeds the tier
    // below, those tiles are halved instead
    {
        const int e0 = pick_ept((ht.max_ne + block - 1) / block);
        int lower = 0;
        for (int e : kEpts)
            if (e < e0) lower = e;
        if (e0 > 0 && lower > 0) {
            const int32_t cap = lower * block;
            const size_t nt = ht.hdr.size();
            size_t over = 0;
            for (size_t t = 0; t < nt; ++t) over += ht.nE[t * (K + 1) + K] > cap;
            if (over > 0 && over * 50 <= nt) {
                HostTiles hs;
                SE_TRY(build_tiles(members, voff, eoff, T, K, hs, cap));
                if (hs.max_ne <= cap) ht = std::move(hs);
            }
        }
    }
    st = se_plan_stats_t{};
    const int ept = pick_ept((ht.max_ne + block - 1) / block);
    st.ntiles = static_cast<int32_t>(ht.hdr.size());
    st.max_tri = ht.max_ne;
    st.max_vtx = ht.max_nv;
    st.tri_per_thread = ept;
    st.lds_f32 = tile_lds_bytes(true, false, block, K, ht.max_nv, ht.max_ne, ht.max_nvu, ht.max_cs);
    st.lds_f64 = tile_lds_bytes(false, false, block, K, ht.max_nv, ht.max_ne, ht.max_nvu, ht.max_cs);
    // owned triangles must fit the slots that carry running sums
    const bool own_ok = ept > 0 && ht.max_nown <= own_slots(ept) * block;
    st.ok_f32 = own_ok && ept_ok(true, ept, block) && st.lds_f32 <= 160 * 1024;
    st.ok_f64 = own_ok && ept_ok(false, ept, block) && st.lds_f64 <= 160 * 1024;
    st.lds_sesm_f32 = tile_lds_bytes(true, true, block, K, ht.max_nv, ht.max_ne, ht.max_nvu,
                                     ht.max_cs);
    st.lds_sesm_f64 = tile_lds_bytes(false, true, block, K, ht.max_nv, ht.max_ne, ht.max_nvu,
                                     ht.max_cs);
    st.ok_sesm_f32 = own_ok && ept_ok(true, ept, block, true) && st.lds_sesm_f32 <= 160 * 1024;
    st.ok_sesm_f64 = own_ok && ept_ok(false, ept, block, true) && st.lds_sesm_f64 <= 160 * 1024;
    int64_t nv = 0, ne = 0;
    for (const HostMesh *m : members) {
        nv += m->nv;
        ne += m->ne;
    }
    // compulsory bytes of one launch (all tiles), per precision s
    int64_t sumV = 0, sumVu = 0, sumE = 0, sumC = 0;
    for (size_t t = 0; t < ht.hdr.size(); ++t) {
        sumV += ht.nV[t * (K + 1) + K];
        sumVu += ht.nV[t * (K + 1) + K - 1];
        sumE += ht.nE[t * (K + 1) + K];
    }
    sumC = ht.n_ent;
    st.tri_overhead = static_cast<double>(sumE) / ne;
    st.vtx_overhead = static_cast<double>(sumV) / nv;
    for (int f = 0; f < 2; ++f) {
        const double s = f == 0 ? 4.0 : 8.0;
        const double bytes = sumV * (4 + 2 * s) + sumVu * (s + 2) + sumC * 0.0 +
                             sumE * (4 + 12 + 5 * s + 2 * s + 2 * s + s) +
                             ne * (32.0 + 2 * s) + nv * (s + 8.0);
        (f == 0 ? st.bytes_per_vs_f32 : st.bytes_per_vs_f64) = bytes / (static_cast<double>(nv) * K);
    }
    return SE_OK;
}

// Build and upload a tile plan for a set of meshes forming a disjoint union.
se_status make_plan(const std::vector<const HostMesh *> &members, const std::vector<int64_t> &voff,
                    const std::vector<int64_t> &eoff, int32_t T, int32_t K, int32_t block,
                    std::unique_ptr<DevTiles> &out) {
    HostTiles ht;
    se_plan_stats_t st;
    SE_TRY(plan_host(members, voff, eoff, T, K, block, ht, st));
    const int ept = st.tri_per_thread;
    if (!st.ok_f32 && !st.ok_f64) {
        set_error("se_set_plan: tile too large for the register or LDS budget (reduce tile or "
                  "k_fused)");
        return SE_ERR_ARG;
    }
    auto p = std::make_unique<DevTiles>();
    p->T = T;
    p->K = K;
    p->block = block;
    p->ept = ept;
    p->ntiles = static_cast<int32_t>(ht.hdr.size());
    p->max_nv = ht.max_nv;
    p->max_ne = ht.max_ne;
    p->max_nvu = ht.max_nvu;
    p->max_cs = ht.max_cs;
    p->ell = ht.ell;
    p->lds_bytes64 = st.lds_f64;
    p->lds_bytes32 = st.lds_f32;
    p->ok32 = st.ok_f32;
    p->ok64 = st.ok_f64;
    p->lds_sm32 = st.lds_sesm_f32;
    p->lds_sm64 = st.lds_sesm_f64;
    p->ok_sm32 = st.ok_sesm_f32;
    p->ok_sm64 = st.ok_sesm_f64;
    p->hdr_host = ht.hdr;
    p->le_gid_host = ht.le_gid;
    p->nE_host = ht.nE;
    static_assert(sizeof(TileHdr) == sizeof(TileHdrK), "tile header layouts differ");
    SE_TRY(p->hdr.upload(ht.hdr.data(), ht.hdr.size() * sizeof(TileHdr)));
    SE_TRY(p->nV.upload(ht.nV.data(), ht.nV.size() * 4));
    SE_TRY(p->nE.upload(ht.nE.data(), ht.nE.size() * 4));
    SE_TRY(p->lv_gid.upload(ht.lv_gid.data(), ht.lv_gid.size() * 4));
    const int64_t nle = static_cast<int64_t>(ht.le_gid.size());
    {
        std::vector<uint32_t> rec(4 * nle);
        for (int64_t i = 0; i < nle; ++i) {
            rec[4 * i] = static_cast<uint32_t>(ht.le_gid[i]);
            for (int k = 0; k < 3; ++k) rec[4 * i + 1 + k] = ht.le_tri[3 * i + k];
        }
        SE_TRY(p->le_rec.upload(rec.data(), rec.size() * 4));
    }
    SE_TRY(p->cs_row.upload(ht.cs_row.data(), ht.cs_row.size() * 2));
    // local geometry per tile, gathered member by member
    std::vector<double> g64(4 * nle), a64e(nle);
    std::vector<float> g32(4 * nle), a32e(nle);
    for (int64_t i = 0; i < nle; ++i) {
        const int64_t ge = ht.le_gid[i];
        size_t mi = std::upper_bound(eoff.begin(), eoff.end(), ge) - eoff.begin() - 1;
        const HostMesh &m = *members[mi];
        const int64_t e = ge - eoff[mi];
        const double *gn = &m.gN[6 * e];
        for (int q = 0; q < 4; ++q) {
            g64[4 * i + q] = gn[2 + q];
            g32[4 * i + q] = static_cast<float>(gn[2 + q]);
        }
        a64e[i] = m.Ae[e];
        a32e[i] = static_cast<float>(m.Ae[e]);
    }
    SE_TRY(p->geo64.upload(g64.data(), g64.size() * 8));
    SE_TRY(p->geo32.upload(g32.data(), g32.size() * 4));
    SE_TRY(p->ae64.upload(a64e.data(), a64e.size() * 8));
    SE_TRY(p->ae32.upload(a32e.data(), a32e.size() * 4));
    // reciprocal dual-cell areas per local vertex (contiguous per tile: no index round
    // trip); FP32: of the FP32-rounded area, rounded once
    const int64_t nlv = static_cast<int64_t>(ht.lv_gid.size());
    std::vector<double> a64(nlv);
    std::vector<float> a32(nlv);
    for (int64_t i = 0; i < nlv; ++i) {
        const int64_t gv = ht.lv_gid[i];
        size_t mi = std::upper_bound(voff.begin(), voff.end(), gv) - voff.begin() - 1;
        const double av = members[mi]->Av[gv - voff[mi]];
        a64[i] = 1.0 / av;
        a32[i] = 1.0f / static_cast<float>(av);
    }
    SE_TRY(p->lav64.upload(a64.data(), nlv * 8));
    SE_TRY(p->lav32.upload(a32.data(), nlv * 4));
    // raise the LDS limit of the forward-backward tile kernels this plan runs now, so
    // that a later launch needs no attribute call (the adjoint may be graph-captured)
    for (int f = 0; f < 2; ++f)
        p->prepared[f] = p->ok(f == 1, false) && prepare_tile(f == 1, 0, p->ept, p->block) == hipSuccess;
    // the adjoint on the plan: recompute with trajectory output (mode 3) and the reverse
    // tile kernel (up to four triangles per thread, with 1024-thread workgroups three in
    // FP32 and two in FP64; a tile's owned vertices within two per thread, its LDS within
    // 160 KiB)
    for (int f = 0; f < 2; ++f) {
        const bool f32 = f == 1;
        p->lds_adj[f] = static_cast<size_t>(adj_tile_lds_bytes(f32, block, K, p->max_nv,
                                                               p->max_nvu, p->max_cs));
        p->adj_ready[f] = p->prepared[f] && ept <= 4 &&
                          T <= 2 * block && p->lds_adj[f] <= 160 * 1024 &&
                          prepare_tile(f32, 3, ept, block) == hipSuccess &&
                          prepare_adj_tile(f32, ept, block) == hipSuccess;
    }
    out = std::move(p);
    return SE_OK;
}

struct Layout {
    size_t eta_alt, U_alt, sum, U0c, phi, vol, total;
    size_t vub, vRb, vRe;  // viscous term: U / H_e, R - V^0, R - V^0 + V^m
    size_t sv[8], se[7];   // AB3-AM4 only: 8 vertex arrays, 7 triangle (transport) arrays
};

Layout fwd_layout(int64_t nv, int64_t ne, bool f32, int32_t nsub, int64_t width,
                  bool sesm = false, bool visc = false) {
    const size_t s = f32 ? 4 : 8;
    Layout L{};
    size_t o = 0;
    if (sesm) {
        for (int k = 0; k < 8; ++k) {
            L.sv[k] = o;
            o += al(nv * s);
        }
        for (int k = 0; k < 7; ++k) {
            L.se[k] = o;
            o += al(2 * ne * s);
        }
    }
    L.eta_alt = o;
    o += al(nv * s);
    L.U_alt = o;
    o += al(2 * ne * s);
    L.sum = o;
    o += al(16 * ne);
    L.U0c = o;
    o += al(2 * ne * s);
    L.phi = o;
    o += al(3 * ne * s);
    L.vol = o;
    o += al(static_cast<size_t>(nsub + 1) * width * 8);
    if (visc) {
        L.vub = o;
        o += al(2 * ne * s);
        L.vRb = o;
        o += al(2 * ne * s);
        L.vRe = o;
        o += al(2 * ne * s);
    }
    L.total = o;
    return L;
}

struct AdjLayout {
    size_t ckpt, traj[2], lam_eta, lam_U, psi, gR, gH0, total;
    size_t etraj, lam_eta2, lam_U2;   // tile reverse sweep: forward elevations (two
                                      // segments), second adjoint state
    int32_t nseg, k;
};

AdjLayout adj_layout(int64_t nv, int64_t ne, bool f32, int32_t nsub, int32_t k, size_t base) {
    const size_t s = f32 ? 4 : 8;
    const size_t st = al((nv + 2 * ne) * s);   // one state (eta then U)
    AdjLayout L{};
    L.k = k;
    L.nseg = (nsub + k - 1) / k;
    size_t o = base;
    L.ckpt = o;
    o += st * L.nseg;
    // two segment buffers: the reverse sweep of one segment reads one while the
    // recompute of the previous segment writes the other
    L.traj[0] = o;
    o += st * k;
    L.traj[1] = o;
    o += st * k;
    L.lam_eta = o;
    o += al(nv * s);
    L.lam_U = o;
    o += al(2 * ne * s);
    L.psi = o;
    o += al(4 * ne * s);
    L.gR = o;
    o += al(2 * ne * s);
    L.gH0 = o;
    o += al(nv * s);
    // the tile reverse sweep: elevations of one segment's substeps (slot m at m nv), the
    // second buffer of the adjoint state (launches alternate between the two)
    L.etraj = o;
    o += 2 * al(static_cast<size_t>(k) * nv * s);
    L.lam_eta2 = o;
    o += al(nv * s);
    L.lam_U2 = o;
    o += al(2 * ne * s);
    L.total = o;
    return L;
}

int64_t vol_width(int64_t nv) { return std::max<int64_t>((nv + 63) / 64, (nv + 255) / 256); }

// Largest |lambda| among the roots of the SESM characteristic polynomial of
// eq. (eqdp_1) at CFL number c (Durand-Kerner iteration on the monic degree-6
// polynomial; the printed '+-' of its lambda^2 term read as '-').
double sesm_max_root(double c, double b, double d, double g, double z) {
    const double c2 = c * c;
    const double co[7] = {
        b * z * c2,
        c2 * (b * (g - 2 * z) - z / 2),
        -c2 * ((d + 3 * g - 1) * b + g / 2 - 1.5 * z),
        c2 / 2 * (b * (6 * d + 6 * g + 4 * z - 4) + d + 4 * g + z - 1),
        1 + c2 / 2 * (b * (-6 * d - 2 * g - 2 * z + 2) - 4 * d - 3 * g - 3 * z + 3),
        -2 + c2 * d / 2 * (2 * b + 3),
        1.0};
    using cd = std::complex<double>;
    auto P = [&](cd x) {
        cd r = co[6];
        for (int k = 5; k >= 0; --k) r = r * x + co[k];
        return r;
    };
    cd rt[6];
    for (int k = 0; k < 6; ++k) rt[k] = std::pow(cd(0.4, 0.9), k);
    for (int it = 0; it < 500; ++it) {
        double delta = 0.0;
        for (int k = 0; k < 6; ++k) {
            cd den = 1.0;
            for (int j = 0; j < 6; ++j)
                if (j != k) den *= rt[k] - rt[j];
            const cd step = P(rt[k]) / den;
            rt[k] -= step;
            delta = std::max(delta, std::abs(step));
        }
        if (delta < 1e-14) break;
    }
    double mx = 0.0;
    for (int k = 0; k < 6; ++k) mx = std::max(mx, std::abs(rt[k]));
    return mx;
}

// Whether every CFL number in (0, c] is stable for the SESM coefficients.
bool sesm_stable_upto(double c, double b, double d, double g, double z) {
    const int n = 400;
    for (int i = 1; i <= n; ++i)
        if (sesm_max_root(c * i / n, b, d, g, z) > 1.0 + 1e-9) return false;
    return true;
}

inline bool visc_on(const se_params *p) { return p->visc_A0 > 0.0 || p->visc_Cv > 0.0; }

se_status check_params(const se_mesh *m, const se_params *p, int32_t nsub, double dt) {
    if (!m || !p) {
        set_error("null mesh or params");
        return SE_ERR_ARG;
    }
    if (p->precision != SE_F64 && p->precision != SE_F32_MIXED) {
        set_error("unknown precision");
        return SE_ERR_ARG;
    }
    if (nsub < 1 || !(dt > 0.0) || !std::isfinite(dt)) {
        set_error("need nsub >= 1 and a finite dt > 0");
        return SE_ERR_ARG;
    }
    if (!(p->g > 0.0) || !std::isfinite(p->g) || !(p->theta >= 0.0) || !std::isfinite(p->theta) ||
        !std::isfinite(p->eta_ref)) {
        set_error("need g > 0, theta >= 0 and a finite eta_ref");
        return SE_ERR_ARG;
    }
    if (p->scheme != SE_SCHEME_SE && p->scheme != SE_SCHEME_SESM) {
        set_error("unknown scheme");
        return SE_ERR_ARG;
    }
    if (p->reserved != 0) {
        set_error("se_params.reserved must be 0");
        return SE_ERR_ARG;
    }
    if (!(p->visc_A0 >= 0.0) || !std::isfinite(p->visc_A0) || !(p->visc_Cv >= 0.0) ||
        !std::isfinite(p->visc_Cv)) {
        set_error("visc_A0 and visc_Cv must be finite and >= 0");
        return SE_ERR_ARG;
    }
    const bool sesm = p->scheme == SE_SCHEME_SESM;
    if (sesm && !(std::isfinite(p->beta) && std::isfinite(p->delta) && std::isfinite(p->gamma) &&
                  std::isfinite(p->zeta))) {
        set_error("SESM coefficients must be finite");
        return SE_ERR_ARG;
    }
    if (p->flags & SE_CHECK_CFL) {
        if (!(p->h_max > 0.0)) {
            set_error("SE_CHECK_CFL needs h_max > 0");
            return SE_ERR_ARG;
        }
        const double dts = dt / nsub;
        const double c = dts * std::sqrt(p->g * p->h_max * m->h.mu_max);
        if (sesm) {
            if (!sesm_stable_upto(c, p->beta, p->delta, p->gamma, p->zeta)) {
                set_error("CFL: dt_s sqrt(g h_max mu_max) = " + std::to_string(c) +
                          " is beyond the stability range of the SESM coefficients");
                return SE_ERR_CFL;
            }
        } else {
            const double lim = 2.0 / std::sqrt(1.0 + 2.0 * p->theta);
            if (c > lim) {
                set_error("CFL: dt_s sqrt(g h_max mu_max) = " + std::to_string(c) +
                          " exceeds the stability bound " + std::to_string(lim));
                return SE_ERR_CFL;
            }
        }
    }
    return SE_OK;
}

StepC make_step(const se_params *p, int32_t nsub, double dt) {
    StepC c{};
    c.dts = dt / nsub;
    c.g = p->g;
    c.theta = p->theta;
    c.opt = 1.0 + p->theta;
    c.thM = p->theta / static_cast<double>(nsub);
    c.Mdbl = static_cast<double>(nsub);
    c.eta_ref = p->eta_ref;
    c.dts_f = static_cast<float>(c.dts);
    c.g_f = static_cast<float>(c.g);
    c.theta_f = static_cast<float>(c.theta);
    c.opt_f = static_cast<float>(c.opt);
    c.eta_ref_f = static_cast<float>(c.eta_ref);
    c.nsub = nsub;
    c.flags = ((p->flags & SE_LINEAR_H) ? KF_LINEAR_H : 0) |
              ((p->flags & SE_TRACK_VOLUME) ? KF_TRACK_VOLUME : 0);
    if (p->scheme == SE_SCHEME_SESM) {   // eq. (eq4_7)
        c.ab0 = 1.5 + p->beta;
        c.ab1 = 0.5 + 2.0 * p->beta;
        c.ab2 = p->beta;
        c.am0 = p->delta;
        c.am1 = 1.0 - p->delta - p->gamma - p->zeta;
        c.am2 = p->gamma;
        c.am3 = p->zeta;
        c.ab0_f = static_cast<float>(c.ab0);
        c.ab1_f = static_cast<float>(c.ab1);
        c.ab2_f = static_cast<float>(c.ab2);
        c.am0_f = static_cast<float>(c.am0);
        c.am1_f = static_cast<float>(c.am1);
        c.am2_f = static_cast<float>(c.am2);
        c.am3_f = static_cast<float>(c.am3);
    }
    return c;
}

se_status check_device(const se_mesh *m) {
    if (m->device < 0) {
        set_error("host-only mesh (created with device < 0) cannot run kernels");
        return SE_ERR_ARG;
    }
    return SE_OK;
}

// Default plan when the caller set none: the first candidate that runs in
// both precisions without spills.
se_status ensure_plan(se_mesh *m) {
    if (m->plan) return SE_OK;
    std::vector<const HostMesh *> mem{&m->h};
    static const int32_t cand[][3] = {{1024, 4, 512}, {512, 4, 512}, {512, 4, 256}, {512, 2, 256},
                                      {256, 4, 256}, {256, 2, 256}, {128, 2, 256}, {64, 1, 256}};
    for (const auto &c : cand) {
        HostTiles ht;
        se_plan_stats_t st;
        if (plan_host(mem, {0, m->h.nv}, {0, m->h.ne}, c[0], c[1], c[2], ht, st) != SE_OK) continue;
        if (!st.ok_f32 || !st.ok_f64 || !st.ok_sesm_f32 || !st.ok_sesm_f64) continue;
        SE_TRY(make_plan(mem, {0, m->h.nv}, {0, m->h.ne}, c[0], c[1], c[2], m->plan));
        m->plan_T = c[0];
        m->plan_K = c[1];
        m->plan_block = c[2];
        return SE_OK;
    }
    set_error("no default plan fits this mesh");
    return SE_ERR_ARG;
}

}  // namespace
}  // namespace sesub

using namespace sesub;

static se_status ensure_visc(se_mesh *m);
static se_status ensure_tile_visc(se_mesh *m);
static ViscArgs visc_args(const se_mesh *m, bool f32, const se_params *p, const void *H0,
                          const void *eta, const void *U, void *ubar);

extern "C" {

const char *se_last_error(void) { return g_err.c_str(); }

se_status se_sesm_coefficients(double theta, double beta, double *out) {
    if (!out || !std::isfinite(theta) || !std::isfinite(beta)) {
        set_error("se_sesm_coefficients: bad argument");
        return SE_ERR_ARG;
    }
    const double chi = 0.5 * theta;            // SE dissipation 2 chi = theta
    const double zeta = 0.010 - 0.135 * chi;    // eq. (eqdp_6), second line
    const double gamma = 0.083 - 0.514 * chi;
    out[0] = beta > 0.0 ? beta : 0.281105;      // largest stability range (Sec. 3.2)
    out[1] = 2.0 * chi + gamma + 2.0 * zeta + 0.5;   // eq. (eqdp_4)
    out[2] = gamma;
    out[3] = zeta;
    return SE_OK;
}

se_status se_mesh_create(const se_mesh_desc *desc, int device, se_mesh **out) {
    if (!desc || !out) {
        set_error("se_mesh_create: null argument");
        return SE_ERR_ARG;
    }
    *out = nullptr;
    auto m = std::make_unique<se_mesh>();
    m->device = device;
    SE_TRY(build_host_mesh(*desc, m->h));
    for (double v : m->h.Av) m->h.Av_total += v;
    if (device < 0) {   // host-only mesh: reordering and geometry, no device arrays
        *out = m.release();
        return SE_OK;
    }
    DeviceGuard dg(device);
    if (!dg.ok) {
        set_error("se_mesh_create: cannot select device " + std::to_string(device));
        return SE_ERR_HIP;
    }
    const HostMesh &h = m->h;
    DevMesh &d = m->d;
    d.nv = h.nv;
    d.ne = h.ne;
    SE_TRY(d.tri.upload(h.tri.data(), h.tri.size() * 4));
    SE_TRY(d.row_ptr.upload(h.row_ptr.data(), h.row_ptr.size() * 4));
    std::vector<int32_t> pcol(h.col.size());
    for (size_t j = 0; j < h.col.size(); ++j) pcol[j] = 3 * (h.col[j] >> 2) + (h.col[j] & 3);
    SE_TRY(d.pcol.upload(pcol.data(), pcol.size() * 4));
    auto g64 = pack_geom<double>(h, nullptr, 0);
    auto g32 = pack_geom<float>(h, nullptr, 0);
    SE_TRY(d.geom64.upload(g64.data(), g64.size() * 8));
    SE_TRY(d.geom32.upload(g32.data(), g32.size() * 4));
    SE_TRY(d.Av64.upload(h.Av.data(), h.Av.size() * 8));
    std::vector<float> av32(h.Av.begin(), h.Av.end());
    SE_TRY(d.Av32.upload(av32.data(), av32.size() * 4));
    const uint32_t zero = 0;
    SE_TRY(d.faults.upload(&zero, 4));
    *out = m.release();
    return SE_OK;
}

void se_mesh_destroy(se_mesh *mesh) {
    if (!mesh) return;
    if (mesh->device < 0) {
        delete mesh;
        return;
    }
    DeviceGuard dg(mesh->device);
    delete mesh;
}

se_status se_mesh_info(const se_mesh *m, int64_t *nv, int64_t *ne, int64_t *nnz, double *mu_max) {
    if (!m) {
        set_error("se_mesh_info: null mesh");
        return SE_ERR_ARG;
    }
    if (nv) *nv = m->h.nv;
    if (ne) *ne = m->h.ne;
    if (nnz) *nnz = 3 * m->h.ne;
    if (mu_max) *mu_max = m->h.mu_max;
    return SE_OK;
}

se_status se_mesh_perm(const se_mesh *m, int32_t *vperm, int32_t *eperm) {
    if (!m) {
        set_error("se_mesh_perm: null mesh");
        return SE_ERR_ARG;
    }
    if (vperm) std::memcpy(vperm, m->h.vperm.data(), m->h.nv * 4);
    if (eperm) std::memcpy(eperm, m->h.eperm.data(), m->h.ne * 4);
    return SE_OK;
}

se_status se_mesh_csr(const se_mesh *m, int32_t *tri, int32_t *row_ptr, int32_t *col) {
    if (!m) {
        set_error("se_mesh_csr: null mesh");
        return SE_ERR_ARG;
    }
    if (tri) std::memcpy(tri, m->h.tri.data(), m->h.tri.size() * 4);
    if (row_ptr) std::memcpy(row_ptr, m->h.row_ptr.data(), m->h.row_ptr.size() * 4);
    if (col) std::memcpy(col, m->h.col.data(), m->h.col.size() * 4);
    return SE_OK;
}

se_status se_mesh_neighbours(const se_mesh *m, int32_t *nb, double *l, double *lod) {
    if (!m) {
        set_error("se_mesh_neighbours: null mesh");
        return SE_ERR_ARG;
    }
    std::vector<int32_t> nb4;
    std::vector<double> vg;
    SE_TRY(build_visc_tables(m->h, nb4, vg));
    for (int64_t e = 0; e < m->h.ne; ++e)
        for (int j = 0; j < 3; ++j) {
            if (nb) nb[3 * e + j] = nb4[4 * e + j];
            if (l) l[3 * e + j] = vg[6 * e + 2 * j];
            if (lod) lod[3 * e + j] = vg[6 * e + 2 * j + 1];
        }
    return SE_OK;
}

se_status se_mesh_geometry(const se_mesh *m, double *Av, double *Ae, double *gN) {
    if (!m) {
        set_error("se_mesh_geometry: null mesh");
        return SE_ERR_ARG;
    }
    if (Av) std::memcpy(Av, m->h.Av.data(), m->h.nv * 8);
    if (Ae) std::memcpy(Ae, m->h.Ae.data(), m->h.ne * 8);
    if (gN) std::memcpy(gN, m->h.gN.data(), m->h.ne * 48);
    return SE_OK;
}

se_status se_batch_set_plan_impl(se_batch *b, int32_t tile, int32_t k_fused, int32_t block);
se_status se_batch_get_plan_impl(const se_batch *b, int32_t *tile, int32_t *k_fused, int32_t *block);
se_status se_batch_plan_stats_impl(const se_batch *b, int32_t tile, int32_t k_fused, int32_t block,
                                   se_plan_stats_t *stats);
se_status se_batch_faults_impl(se_batch *b, void *stream, uint32_t *bits);

se_status se_set_plan(void *obj, int32_t kind, int32_t tile, int32_t k_fused, int32_t block) {
    if (obj && kind == 1) return se_batch_set_plan_impl(static_cast<se_batch *>(obj), tile, k_fused, block);
    if (!obj || kind != 0) {
        set_error("se_set_plan: null object or unknown kind (0 mesh, 1 batch)");
        return SE_ERR_ARG;
    }
    se_mesh *m = static_cast<se_mesh *>(obj);
    if (m->device < 0) {   // host-only mesh: validate and remember the plan
        HostTiles ht;
        se_plan_stats_t st;
        std::vector<const HostMesh *> mem{&m->h};
        SE_TRY(plan_host(mem, {0, m->h.nv}, {0, m->h.ne}, tile, k_fused, block, ht, st));
        m->plan_T = tile;
        m->plan_K = k_fused;
        m->plan_block = block;
        return SE_OK;
    }
    DeviceGuard dg(m->device);
    std::unique_ptr<DevTiles> p;
    std::vector<const HostMesh *> mem{&m->h};
    SE_TRY(make_plan(mem, {0, m->h.nv}, {0, m->h.ne}, tile, k_fused, block, p));
    m->plan = std::move(p);
    m->plan_T = tile;
    m->plan_K = k_fused;
    m->plan_block = block;
    return SE_OK;
}

se_status se_get_plan(const void *obj, int32_t kind, int32_t *tile, int32_t *k_fused,
                      int32_t *block) {
    if (obj && kind == 1)
        return se_batch_get_plan_impl(static_cast<const se_batch *>(obj), tile, k_fused, block);
    if (!obj || kind != 0) {
        set_error("se_get_plan: null object or unsupported kind");
        return SE_ERR_ARG;
    }
    const se_mesh *m = static_cast<const se_mesh *>(obj);
    if (tile) *tile = m->plan_T;
    if (k_fused) *k_fused = m->plan_K;
    if (block) *block = m->plan_block;
    return SE_OK;
}

se_status se_plan_stats(const void *obj, int32_t kind, int32_t tile, int32_t k_fused,
                        int32_t block, se_plan_stats_t *stats) {
    if (obj && stats && kind == 1)
        return se_batch_plan_stats_impl(static_cast<const se_batch *>(obj), tile, k_fused, block,
                                        stats);
    if (!obj || !stats || kind != 0) {
        set_error("se_plan_stats: bad argument");
        return SE_ERR_ARG;
    }
    const se_mesh *m = static_cast<const se_mesh *>(obj);
    HostTiles ht;
    std::vector<const HostMesh *> mem{&m->h};
    return plan_host(mem, {0, m->h.nv}, {0, m->h.ne}, tile, k_fused, block, ht, *stats);
}

se_status se_workspace_bytes(const se_mesh *m, const se_params *p, int32_t nsub,
                             int32_t ckpt_every, size_t *bytes) {
    if (!m || !p || !bytes || nsub < 1) {
        set_error("se_workspace_bytes: bad argument");
        return SE_ERR_ARG;
    }
    const bool f32 = p->precision == SE_F32_MIXED;
    const Layout L = fwd_layout(m->h.nv, m->h.ne, f32, nsub, vol_width(m->h.nv),
                                p->scheme == SE_SCHEME_SESM, visc_on(p));
    *bytes = L.total;
    if (ckpt_every > 0) {
        const int32_t k = std::min(ckpt_every, nsub);
        *bytes = adj_layout(m->h.nv, m->h.ne, f32, nsub, k, L.total).total;
    }
    return SE_OK;
}

static se_status check_state(const se_state *st, const se_forcing *fo, const void *ws) {
    if (!st || !fo || !st->eta || !st->U || !fo->R || !fo->f || !fo->H0 || !ws) {
        set_error("null state, forcing or workspace array");
        return SE_ERR_ARG;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return SE_ERR_ARG;
    }
    return SE_OK;
}

// Access policy of the tile kernels for nv vertices: stream each tile's own tables and
// the write-back past the caches when one launch moves more than half of the 256 MiB
// last-level cache (about 236 B per vertex in FP32, 356 in FP64); smaller working sets
// stay cached from launch to launch and keep ordinary accesses (lat-lon workload, 2.2M
// vertices: 150 -> 136 us per launch with it; the 65k-vertex adjoint basin 10% slower).
static int32_t stream_policy(int64_t nv, bool f32) {
    return (f32 ? 236.0 : 356.0) * static_cast<double>(nv) > 128.0 * 1024 * 1024 ? 1 : 0;
}

// Launch arguments of the tile kernel on one mesh: plan tables, forcing, workspace
// (running sum, U^0 copy, volume partials); K substeps per launch, no average output.
static TileArgs tile_args(const se_mesh *m, const DevTiles &P, bool f32, const se_forcing *fo,
                          char *w, const Layout &L, const StepC &c) {
    TileArgs a{};
    a.nt = stream_policy(m->h.nv, f32);
    a.hdr = P.hdr.as<const TileHdrK>();
    a.nV = P.nV.as<const int32_t>();
    a.nE = P.nE.as<const int32_t>();
    a.lv_gid = P.lv_gid.as<const int32_t>();
    a.le_rec = P.le_rec.as<const uint32_t>();
    a.cs_row = P.cs_row.as<const uint16_t>();
    a.lgeo = f32 ? P.geo32.p : P.geo64.p;
    a.lae = f32 ? P.ae32.p : P.ae64.p;
    a.lv_av = f32 ? P.lav32.p : P.lav64.p;
    a.mem = nullptr;
    a.c0 = c;
    a.R = fo->R;
    a.f = fo->f;
    a.H0 = fo->H0;
    a.W = fo->W;
    a.Av = f32 ? m->d.Av32.p : m->d.Av64.p;
    a.Av64 = m->d.Av64.as<const double>();
    a.sum = w + L.sum;
    a.U0c = w + L.U0c;
    a.Uavg = nullptr;
    a.vol_part = reinterpret_cast<double *>(w + L.vol);
    a.faults = m->d.faults.as<uint32_t>();
    a.K = P.K;
    a.ksub = P.K;
    a.ntiles = P.ntiles;
    a.xcd = 1;
    a.cap_nv = P.max_nv;
    a.cap_ne = P.max_ne;
    a.cap_nvu = P.max_nvu;
    a.cap_cs = P.max_cs;
    a.ell = P.ell ? 1 : 0;
    return a;
}

se_status se_subcycle(se_mesh *m, const se_params *p, se_state *st, const se_forcing *fo,
                      int32_t nsub, double dt, void *ws, void *stream) {
    return sesub::subcycle_tile(m, p, st, fo, nsub, dt, ws, stream, true);
}

}  // extern "C"

// The tile-kernel subcycle behind se_subcycle and se_subcycle_noalloc.  With
// may_alloc false nothing is allocated: a missing plan or missing viscous tables are
// errors instead of being built here.
se_status sesub::subcycle_tile(se_mesh *m, const se_params *p, se_state *st,
                               const se_forcing *fo, int32_t nsub, double dt, void *ws,
                               void *stream, bool may_alloc) {
    SE_TRY(check_params(m, p, nsub, dt));
    const bool visc = visc_on(p);
    if (visc && p->scheme != SE_SCHEME_SE) {
        set_error("se_subcycle: the viscous term is implemented for SE_SCHEME_SE only");
        return SE_ERR_UNSUPPORTED;
    }
    SE_TRY(check_state(st, fo, ws));
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    if (may_alloc) {
        SE_TRY(ensure_plan(m));
    } else if (!m->plan) {
        set_error("se_subcycle_noalloc: the mesh has no tile plan yet (se_set_plan, or one "
                  "se_subcycle call, makes one)");
        return SE_ERR_ARG;
    }
    const DevTiles &P = *m->plan;
    const bool f32 = p->precision == SE_F32_MIXED;
    const bool sm = p->scheme == SE_SCHEME_SESM;
    if (!P.ok(f32, sm)) {
        set_error("se_subcycle: the current plan does not fit the register/LDS budget of this "
                  "precision and scheme (see se_plan_stats)");
        return SE_ERR_ARG;
    }
    const size_t es = f32 ? 4 : 8;
    size_t lds = P.lds(f32, sm);
    if (visc) {
        // two rings per substep; the velocities u = U / H_e of the tile's triangles and
        // their edge-neighbour ids in LDS
        lds = ((lds + 2 * es * static_cast<size_t>(P.max_ne) + 15) & ~static_cast<size_t>(15)) +
              8 * static_cast<size_t>(P.max_ne);
        // register budget of the viscous form (no spills): 1024-thread workgroups up to
        // three triangles per thread (FP32; FP64 one), 512-thread ones up to six (FP32)
        // or four (FP64)
        const bool regs_ok = P.block == 1024 ? P.ept <= (f32 ? 3 : 1)
                             : P.block == 512 ? P.ept <= (f32 ? 6 : 4) : true;
        if (P.K < 2 || lds > 160 * 1024 || !regs_ok) {
            set_error("se_subcycle: with the viscous term the plan needs k_fused >= 2, " +
                      std::to_string(lds) + " bytes of LDS within 160 KiB and at most " +
                      "3 / 1 (1024 threads) or 6 / 4 (512 threads) triangles per thread "
                      "(FP32 / FP64)");
            return SE_ERR_ARG;
        }
        if (!may_alloc && (!m->d.vnb.p || !m->plan->vnb.p)) {
            set_error("se_subcycle_noalloc: the viscous tables of this mesh and plan are not "
                      "built yet (one se_subcycle call with the viscous term builds them)");
            return SE_ERR_ARG;
        }
        SE_TRY(ensure_visc(m));
        SE_TRY(ensure_tile_visc(m));
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nv = m->h.nv, ne = m->h.ne;
    const Layout L = fwd_layout(nv, ne, f32, nsub, vol_width(nv), sm, visc);
    char *w = static_cast<char *>(ws);
    StepC c = make_step(p, nsub, dt);
    c.ntiles = P.ntiles;
    c.vol_off = 0;

    TileArgs a = tile_args(m, P, f32, fo, w, L, c);
    a.Uavg = st->Uavg;
    a.ksub = visc ? P.K / 2 : P.K;
    void *eta_u = st->eta, *U_u = st->U;
    void *eta_w = w + L.eta_alt, *U_w = w + L.U_alt;
    const int nlaunch = (nsub + a.ksub - 1) / a.ksub;
    const int mode = sm ? 1 : (visc ? 2 : 0);
    if (visc) {
        // R - V(eta^0, U^0), read by every launch in place of R
        ViscArgs va = visc_args(m, f32, p, fo->H0, st->eta, st->U, w + L.vub);
        va.base = fo->R;
        va.sign = -1;
        va.out = w + L.vRb;
        HIP_TRY(launch_visc(f32, va, s), "se_subcycle viscous term");
        a.R = w + L.vRb;
        a.vnb = P.vnb.as<const uint32_t>();
        a.vgeo = f32 ? P.vgeo32.p : P.vgeo64.p;
        a.vA0 = p->visc_A0;
        a.vCv = p->visc_Cv;
    }
    HIP_TRY(prepare_tile(f32, mode, P.ept, P.block), "se_subcycle prepare");
    a.eta_u = eta_u;
    a.eta_w = eta_w;
    a.U_u = U_u;
    a.U_w = U_w;
    if (sm)
        for (int k = 0; k < 2; ++k) {
            for (int q = 0; q < 4; ++q) a.sm_v[k][q] = w + L.sv[4 * k + q];
            for (int q = 0; q < 3; ++q) a.sm_e[k][q] = w + L.se[3 * k + q];
        }
    for (int ch = 0; ch < nlaunch; ++ch) {
        a.chunk = ch;
        HIP_TRY(launch_tile(f32, mode, P.ept, P.block, a, P.ntiles, lds, s), "se_subcycle launch");
    }
    if (sm) {
        // the last substep's transport update (pending) and the final elevation
        const int lw = (nlaunch - 1) & 1;
        PlainArgs fa{};
        fa.nv = nv;
        fa.ne = ne;
        fa.tri = m->d.tri.as<const int32_t>();
        fa.geom = f32 ? m->d.geom32.p : m->d.geom64.p;
        fa.H0 = fo->H0;
        fa.R = fo->R;
        fa.f = fo->f;
        fa.eta = st->eta;
        fa.U = st->U;
        fa.eta1 = a.sm_v[lw][0];
        fa.etaA = a.sm_v[lw][3];
        fa.U1 = a.sm_e[lw][0];
        fa.Uab = a.sm_e[lw][2];
        fa.faults = m->d.faults.as<uint32_t>();
        fa.c = c;
        HIP_TRY(launch_sesm_fin(f32, fa, s), "se_subcycle final update");
    } else if (nlaunch % 2 == 1) {
        HIP_TRY(hipMemcpyAsync(eta_u, eta_w, nv * es, hipMemcpyDeviceToDevice, s), "copy eta");
        HIP_TRY(hipMemcpyAsync(U_u, U_w, 2 * ne * es, hipMemcpyDeviceToDevice, s), "copy U");
    }
    if (st->volume) {
        const int rows = (p->flags & SE_TRACK_VOLUME) ? nsub + 1 : 2;
        double add = 0.0;
        if (f32) {
            add = p->eta_ref * m->h.Av_total;
        }
        HIP_TRY(launch_vol_reduce(a.vol_part, P.ntiles, rows, add, st->volume, s), "volume");
    }
    return SE_OK;
}

extern "C" {

se_status se_subcycle_plain(se_mesh *m, const se_params *p, se_state *st, const se_forcing *fo,
                            int32_t nsub, double dt, void *ws, void *stream) {
    SE_TRY(check_params(m, p, nsub, dt));
    SE_TRY(check_state(st, fo, ws));
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    const bool f32 = p->precision == SE_F32_MIXED;
    const bool sesm = p->scheme == SE_SCHEME_SESM;
    const bool visc = visc_on(p);
    if (sesm && visc) {
        set_error("se_subcycle_plain: the viscous term is implemented for SE_SCHEME_SE only");
        return SE_ERR_UNSUPPORTED;
    }
    if (visc) SE_TRY(ensure_visc(m));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nv = m->h.nv, ne = m->h.ne;
    const Layout L = fwd_layout(nv, ne, f32, nsub, vol_width(nv), sesm, visc);
    char *w = static_cast<char *>(ws);
    PlainArgs a{};
    a.nv = nv;
    a.ne = ne;
    a.tri = m->d.tri.as<const int32_t>();
    a.row_ptr = m->d.row_ptr.as<const int32_t>();
    a.pcol = m->d.pcol.as<const int32_t>();
    a.geom = f32 ? m->d.geom32.p : m->d.geom64.p;
    a.H0 = fo->H0;
    a.R = fo->R;
    a.f = fo->f;
    a.W = fo->W;
    a.Av = f32 ? m->d.Av32.p : m->d.Av64.p;
    a.Av64 = m->d.Av64.as<const double>();
    a.eta = st->eta;
    a.U = st->U;
    a.phi = w + L.phi;
    a.sum = w + L.sum;
    a.U0c = w + L.U0c;
    a.Uavg = st->Uavg;
    a.vol_part = reinterpret_cast<double *>(w + L.vol);
    a.faults = m->d.faults.as<uint32_t>();
    a.c = make_step(p, nsub, dt);
    a.nblk_v = static_cast<int32_t>((nv + 255) / 256);
    if (sesm) {
        // histories start from the initial state
        const size_t es = f32 ? 4 : 8;
        a.eta1 = w + L.sv[0];
        a.eta2 = w + L.sv[1];
        a.etaA = w + L.sv[2];
        a.U1 = w + L.se[0];
        a.U2 = w + L.se[1];
        a.Uab = w + L.se[6];
        for (void *dst : {a.eta1, a.eta2})
            HIP_TRY(hipMemcpyAsync(dst, st->eta, nv * es, hipMemcpyDeviceToDevice, s), "history");
        for (void *dst : {a.U1, a.U2})
            HIP_TRY(hipMemcpyAsync(dst, st->U, 2 * ne * es, hipMemcpyDeviceToDevice, s), "history");
        for (int mm = 0; mm < nsub; ++mm) {
            a.m = mm;
            HIP_TRY(launch_sesm_step(f32, a, s), "se_subcycle_plain launch");
        }
    } else if (visc) {
        // R^hV of eq. (eq:viscosity_BT) at every substep, its initial value subtracted
        ViscArgs va = visc_args(m, f32, p, fo->H0, st->eta, st->U, w + L.vub);
        va.base = fo->R;
        va.sign = -1;
        va.out = w + L.vRb;
        HIP_TRY(launch_visc(f32, va, s), "se_subcycle_plain viscous term");
        va.base = w + L.vRb;
        va.sign = 1;
        va.out = w + L.vRe;
        a.R = w + L.vRe;
        for (int mm = 0; mm < nsub; ++mm) {
            a.m = mm;
            HIP_TRY(launch_visc(f32, va, s), "se_subcycle_plain viscous term");
            HIP_TRY(launch_plain_step(f32, a, s), "se_subcycle_plain launch");
        }
    } else {
        for (int mm = 0; mm < nsub; ++mm) {
            a.m = mm;
            HIP_TRY(launch_plain_step(f32, a, s), "se_subcycle_plain launch");
        }
    }
    if (st->volume) {
        const int rows = (p->flags & SE_TRACK_VOLUME) ? nsub + 1 : 2;
        double add = 0.0;
        if (f32) {
            add = p->eta_ref * m->h.Av_total;
        }
        HIP_TRY(launch_vol_reduce(a.vol_part, a.nblk_v, rows, add, st->volume, s), "volume");
    }
    return SE_OK;
}

se_status se_trim_zstar(se_mesh *m, int32_t K, const double *H0, const double *eta_new,
                        const double *Uavg, const double *Ustar, const double *hn,
                        const double *h0, const double *W, double tau, double *U, double *hnew,
                        double *w, void *stream) {
    if (!m || !H0 || !eta_new || !Uavg || !Ustar || !hn || !h0 || !U || !hnew || !w) {
        set_error("se_trim_zstar: null argument");
        return SE_ERR_ARG;
    }
    if (K < 1 || K > 64 || !(tau > 0.0) || !std::isfinite(tau)) {
        set_error("se_trim_zstar: need 1 <= K <= 64 and a finite tau > 0");
        return SE_ERR_ARG;
    }
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    TrimArgs a{};
    a.nv = m->h.nv;
    a.ne = m->h.ne;
    a.K = K;
    a.tau = tau;
    a.tri = m->d.tri.as<const int32_t>();
    a.row_ptr = m->d.row_ptr.as<const int32_t>();
    a.pcol = m->d.pcol.as<const int32_t>();
    a.geom = m->d.geom64.as<const double>();
    a.Av = m->d.Av64.as<const double>();
    a.H0 = H0;
    a.eta_new = eta_new;
    a.Uavg = Uavg;
    a.Ustar = Ustar;
    a.hn = hn;
    a.h0 = h0;
    a.W = W;
    a.U = U;
    a.hnew = hnew;
    a.w = w;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (!m->d.slotS.p) {
        // sub-cell flux vectors S_k = -A_e grad N_k of every triangle, built on the host
        // and uploaded synchronously (visible to calls on any stream)
        const HostMesh &h = m->h;
        std::vector<double> S(6 * static_cast<size_t>(h.ne));
        for (int64_t e = 0; e < h.ne; ++e)
            for (int q = 0; q < 6; ++q) S[6 * e + q] = -h.Ae[e] * h.gN[6 * e + q];
        SE_TRY(m->d.slotS.upload(S.data(), S.size() * 8));
    }
    // the tile form (one launch), unless U is Ustar itself (a tile would overwrite
    // transports that a later tile still reads) or one vertex's row exceeds a tile
    const int cap_e = trim_tile_cap_e(K), cap_v = trim_tile_cap_v(K);
    if (U != Ustar && m->d.tt_cap_e != cap_e && m->d.tt_cap_e != -cap_e) {
        TrimTiles tt;
        m->d.tt_cap_e = 0;
        if (build_trim_tiles(m->h, cap_e, kTrimTileOwn, cap_v, tt)) {
            SE_TRY(m->d.tt_hdr.upload(tt.hdr.data(), tt.hdr.size() * 4));
            SE_TRY(m->d.tt_lv.upload(tt.lv.data(), tt.lv.size() * 4));
            SE_TRY(m->d.tt_le.upload(tt.le.data(), tt.le.size() * 4));
            SE_TRY(m->d.tt_rloc.upload(tt.rloc.data(), tt.rloc.size() * 2));
            m->d.tt_ntiles = tt.ntiles;
            m->d.tt_cap_v = cap_v;
            m->d.tt_cap_e = cap_e;
        } else {
            m->d.tt_cap_e = -cap_e;
        }
    }
    if (U != Ustar && m->d.tt_cap_e == cap_e) {
        a.tt_hdr = m->d.tt_hdr.as<const int32_t>();
        a.tt_lv = m->d.tt_lv.as<const int32_t>();
        a.tt_le = m->d.tt_le.as<const int2>();
        a.tt_rloc = m->d.tt_rloc.as<const uint16_t>();
        a.tt_ntiles = m->d.tt_ntiles;
        a.tt_cap_v = m->d.tt_cap_v;
        HIP_TRY(launch_trim_tile(a, m->d.slotS.as<const double>(), s), "se_trim_zstar launch");
        return SE_OK;
    }
    HIP_TRY(launch_trim(a, m->d.slotS.as<const double>(), s), "se_trim_zstar launch");
    return SE_OK;
}

// Neighbour tables of the viscous term, built on first use.
static se_status ensure_visc(se_mesh *m) {
    if (m->d.vnb.p) return SE_OK;
    std::vector<int32_t> nb4;
    std::vector<double> vg;
    SE_TRY(build_visc_tables(m->h, nb4, vg));
    std::vector<float> vg32(vg.begin(), vg.end());
    SE_TRY(m->d.vgeo64.upload(vg.data(), vg.size() * 8));
    SE_TRY(m->d.vgeo32.upload(vg32.data(), vg32.size() * 4));
    SE_TRY(m->d.vnb.upload(nb4.data(), nb4.size() * 4));
    return SE_OK;
}

// Tile-local neighbour tables of the viscous term for the mesh's current plan: for
// every local triangle, the local index of the triangle across each edge when it
// belongs to the tile (0xffff otherwise: a coast, or a neighbour beyond the loaded
// rings, which no updated triangle uses), and the edge geometry.
static se_status ensure_tile_visc(se_mesh *m) {
    DevTiles &P = *m->plan;
    if (P.vnb.p) return SE_OK;
    std::vector<int32_t> nb4;
    std::vector<double> vg;
    SE_TRY(build_visc_tables(m->h, nb4, vg));
    const int64_t nle = static_cast<int64_t>(P.le_gid_host.size());
    std::vector<uint32_t> tnb(2 * nle);
    std::vector<double> tg64(6 * nle);
    std::vector<float> tg32(6 * nle);
    std::vector<int32_t> eloc(m->h.ne, -1);
    for (int32_t t = 0; t < P.ntiles; ++t) {
        const int64_t off = P.hdr_host[t].le_off;
        const int32_t n = P.nE_host[static_cast<size_t>(t) * (P.K + 1) + P.K];
        for (int32_t q = 0; q < n; ++q) eloc[P.le_gid_host[off + q]] = q;
        for (int32_t q = 0; q < n; ++q) {
            const int64_t e = P.le_gid_host[off + q];
            uint32_t l3[3];
            for (int j = 0; j < 3; ++j) {
                const int32_t g = nb4[4 * e + j];
                l3[j] = (g >= 0 && eloc[g] >= 0) ? static_cast<uint32_t>(eloc[g]) : 0xffffu;
                for (int k = 0; k < 2; ++k) {
                    tg64[6 * (off + q) + 2 * j + k] = vg[6 * e + 2 * j + k];
                    tg32[6 * (off + q) + 2 * j + k] = static_cast<float>(vg[6 * e + 2 * j + k]);
                }
            }
            tnb[2 * (off + q)] = l3[0] | (l3[1] << 16);
            tnb[2 * (off + q) + 1] = l3[2] | (0xffffu << 16);
        }
        for (int32_t q = 0; q < n; ++q) eloc[P.le_gid_host[off + q]] = -1;
    }
    SE_TRY(P.vgeo64.upload(tg64.data(), tg64.size() * 8));
    SE_TRY(P.vgeo32.upload(tg32.data(), tg32.size() * 4));
    SE_TRY(P.vnb.upload(tnb.data(), tnb.size() * 4));
    return SE_OK;
}

static ViscArgs visc_args(const se_mesh *m, bool f32, const se_params *p, const void *H0,
                          const void *eta, const void *U, void *ubar) {
    ViscArgs va{};
    va.ne = m->h.ne;
    va.tri = m->d.tri.as<const int32_t>();
    va.nb = m->d.vnb.as<const int32_t>();
    va.vgeo = f32 ? m->d.vgeo32.p : m->d.vgeo64.p;
    va.geom = f32 ? m->d.geom32.p : m->d.geom64.p;
    va.H0 = H0;
    va.eta = eta;
    va.U = U;
    va.ubar = ubar;
    va.A0 = p->visc_A0;
    va.Cv = p->visc_Cv;
    va.eta_ref = f32 ? p->eta_ref : 0.0;
    va.linear_h = (p->flags & SE_LINEAR_H) ? 1 : 0;
    va.sign = 1;
    return va;
}

se_status se_barotropic_visc(se_mesh *m, int32_t precision, uint32_t flags, double eta_ref,
                             double A0, double Cv, const void *H0, const void *eta,
                             const void *U, void *V, void *ws, void *stream) {
    if (!m || !H0 || !eta || !U || !V || !ws) {
        set_error("se_barotropic_visc: null argument");
        return SE_ERR_ARG;
    }
    if (!(A0 >= 0.0) || !std::isfinite(A0) || !(Cv >= 0.0) || !std::isfinite(Cv) ||
        !std::isfinite(eta_ref)) {
        set_error("se_barotropic_visc: A0, Cv must be finite and >= 0, eta_ref finite");
        return SE_ERR_ARG;
    }
    if (precision != SE_F64 && precision != SE_F32_MIXED) {
        set_error("se_barotropic_visc: precision must be SE_F64 or SE_F32_MIXED");
        return SE_ERR_ARG;
    }
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    SE_TRY(ensure_visc(m));
    se_params p{};
    p.precision = precision;
    p.flags = flags & SE_LINEAR_H;
    p.eta_ref = eta_ref;
    p.visc_A0 = A0;
    p.visc_Cv = Cv;
    const bool f32 = precision == SE_F32_MIXED;
    ViscArgs va = visc_args(m, f32, &p, H0, eta, U, ws);
    va.out = V;
    HIP_TRY(launch_visc(f32, va, static_cast<hipStream_t>(stream)), "se_barotropic_visc launch");
    return SE_OK;
}

se_status se_forcing_assemble(se_mesh *m, int32_t K, const int32_t *nlev, const double *RA,
                     const double *RP, const double *RhV, const double *tau_s, const double *u,
                     double Cd, int32_t precision, void *R, void *stream) {
    if (!m || !R) {
        set_error("se_forcing_assemble: null mesh or output");
        return SE_ERR_ARG;
    }
    if (K < 1 || !(Cd >= 0.0) || !std::isfinite(Cd) || (Cd > 0.0 && !u)) {
        set_error("se_forcing_assemble: need K >= 1, a finite Cd >= 0, and u when Cd > 0");
        return SE_ERR_ARG;
    }
    if (precision != SE_F64 && precision != SE_F32_MIXED) {
        set_error("se_forcing_assemble: precision must be SE_F64 or SE_F32_MIXED");
        return SE_ERR_ARG;
    }
    if (static_cast<int64_t>(m->h.ne) * K > (int64_t(1) << 40)) {
        set_error("se_forcing_assemble: ne * K too large");
        return SE_ERR_ARG;
    }
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    ForcingArgs a{};
    a.ne = m->h.ne;
    a.K = K;
    a.out_f32 = precision == SE_F32_MIXED;
    a.Cd = Cd;
    a.nlev = nlev;
    a.RA = RA;
    a.RP = RP;
    a.RhV = RhV;
    a.u = u;
    a.tau_s = tau_s;
    a.R = R;
    a.faults = m->d.faults.as<uint32_t>();
    HIP_TRY(launch_forcing(a, static_cast<hipStream_t>(stream)), "se_forcing_assemble launch");
    return SE_OK;
}

se_status se_check_faults(void *obj, int32_t kind, void *stream, uint32_t *bits) {
    if (obj && bits && kind == 1) return se_batch_faults_impl(static_cast<se_batch *>(obj), stream, bits);
    if (!obj || !bits || kind != 0) {
        set_error("se_check_faults: bad argument");
        return SE_ERR_ARG;
    }
    se_mesh *m = static_cast<se_mesh *>(obj);
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s), "se_check_faults sync");
    uint32_t v = 0;
    HIP_TRY(hipMemcpy(&v, m->d.faults.p, 4, hipMemcpyDeviceToHost), "se_check_faults copy");
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(m->d.faults.p, &zero, 4, hipMemcpyHostToDevice), "se_check_faults reset");
    *bits = v;
    return SE_OK;
}


se_status se_subcycle_adjoint(se_mesh *m, const se_params *p, const void *eta0, const void *U0,
                              const se_forcing *fo, int32_t nsub, double dt, int32_t ckpt_every,
                              const void *lam_eta, const void *lam_U, const double *lam_Uavg,
                              void *g_eta0, void *g_U0, void *g_R, void *g_H0, void *ws,
                              void *stream) {
    SE_TRY(check_params(m, p, nsub, dt));
    if (p->scheme != SE_SCHEME_SE || visc_on(p)) {
        set_error("se_subcycle_adjoint: only the forward-backward scheme without the viscous "
                  "term has an adjoint");
        return SE_ERR_UNSUPPORTED;
    }
    if (!eta0 || !U0 || !fo || !fo->R || !fo->f || !fo->H0 || !ws) {
        set_error("se_subcycle_adjoint: null input, forcing or workspace");
        return SE_ERR_ARG;
    }
    if (ckpt_every < 1 || ckpt_every > nsub) {
        set_error("se_subcycle_adjoint: need 1 <= ckpt_every <= nsub");
        return SE_ERR_ARG;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return SE_ERR_ARG;
    }
    SE_TRY(check_device(m));
    DeviceGuard dg(m->device);
    const bool f32 = p->precision == SE_F32_MIXED;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nv = m->h.nv, ne = m->h.ne;
    const size_t es = f32 ? 4 : 8;
    const Layout L = fwd_layout(nv, ne, f32, nsub, vol_width(nv));
    const AdjLayout A = adj_layout(nv, ne, f32, nsub, ckpt_every, L.total);
    char *w = static_cast<char *>(ws);
    const size_t st_bytes = al((nv + 2 * ne) * es);
    auto st_eta = [&](size_t off) { return w + off; };
    auto st_U = [&](size_t off) { return w + off + nv * es; };

    // forward substep (state update only) on the plain path
    PlainArgs fa{};
    fa.nv = nv;
    fa.ne = ne;
    fa.tri = m->d.tri.as<const int32_t>();
    fa.row_ptr = m->d.row_ptr.as<const int32_t>();
    fa.pcol = m->d.pcol.as<const int32_t>();
    fa.geom = f32 ? m->d.geom32.p : m->d.geom64.p;
    fa.H0 = fo->H0;
    fa.R = fo->R;
    fa.f = fo->f;
    fa.W = fo->W;
    fa.Av = f32 ? m->d.Av32.p : m->d.Av64.p;
    fa.Av64 = m->d.Av64.as<const double>();
    fa.phi = w + L.phi;
    fa.sum = w + L.sum;
    fa.U0c = w + L.U0c;
    fa.faults = m->d.faults.as<uint32_t>();
    fa.c = make_step(p, nsub, dt);
    fa.nblk_v = static_cast<int32_t>((nv + 255) / 256);
    fa.fwd_only = 1;
    // one forward substep from the state (se, sU) into the workspace state at off
    auto fstep = [&](const void *se, const void *sU, size_t off) -> se_status {
        fa.eta_src = se;
        fa.U_src = sU;
        fa.eta = st_eta(off);
        fa.U = st_U(off);
        HIP_TRY(launch_plain_step(f32, fa, s), "adjoint: forward substep");
        return SE_OK;
    };

    // 1. forward sweep storing a checkpoint every k substeps: state m (m = q k) in
    // checkpoint slot q, the caller's eta0, U0 standing for slot 0; the states between
    // checkpoints go to segment buffer 0 (no copies: each substep writes its result into
    // its slot).  The sweep stops at the last checkpoint: the states after it are
    // recomputed by the reverse sweep anyway.
    const int32_t k = A.k;
    auto ckpt_eta = [&](int32_t q) -> const void * { return q == 0 ? eta0 : st_eta(A.ckpt + st_bytes * q); };
    auto ckpt_U = [&](int32_t q) -> const void * { return q == 0 ? U0 : st_U(A.ckpt + st_bytes * q); };
    // state j of segment sg (j = 0: its checkpoint; else segment buffer sg mod 2)
    auto seg_off = [&](int32_t sg, int32_t j) { return A.traj[sg & 1] + st_bytes * j; };
    auto seg_eta = [&](int32_t sg, int32_t j) -> const void * {
        return j == 0 ? ckpt_eta(sg) : st_eta(seg_off(sg, j));
    };
    auto seg_U = [&](int32_t sg, int32_t j) -> const void * {
        return j == 0 ? ckpt_U(sg) : st_U(seg_off(sg, j));
    };
    const DevTiles *TP = m->plan.get();
    if (TP && TP->ok(f32, false) && TP->prepared[f32 ? 1 : 0]) {
        // The mesh has a tile plan for this precision: each segment runs as temporally
        // blocked launches from checkpoint q to checkpoint q + 1 (the tile path equals
        // the plain path bit for bit).  A segment is a subcycle of k substeps of this
        // dt_s; chunk i reads state B_i and writes B_{i+1} (B_0, B_n the checkpoints, the
        // others alternating between two free slots of the segment buffers).
        StepC c = fa.c;
        c.nsub = k;
        c.flags &= ~KF_TRACK_VOLUME;
        c.ntiles = TP->ntiles;
        c.vol_off = 0;
        TileArgs ta = tile_args(m, *TP, f32, fo, w, L, c);
        const size_t lds = TP->lds(f32, false);
        const int32_t nch = (k + TP->K - 1) / TP->K;
        for (int32_t q = 0; q + 1 < A.nseg; ++q) {
            for (int32_t i = 0; i < nch; ++i) {
                void *se = i == 0 ? const_cast<void *>(ckpt_eta(q)) : st_eta(seg_off((i - 1) & 1, 1));
                void *sU = i == 0 ? const_cast<void *>(ckpt_U(q)) : st_U(seg_off((i - 1) & 1, 1));
                void *de = i + 1 == nch ? st_eta(A.ckpt + st_bytes * (q + 1)) : st_eta(seg_off(i & 1, 1));
                void *dU = i + 1 == nch ? st_U(A.ckpt + st_bytes * (q + 1)) : st_U(seg_off(i & 1, 1));
                // an even chunk reads (eta_u, U_u) and writes (eta_w, U_w); an odd one the reverse
                ta.eta_u = (i & 1) ? de : se;
                ta.U_u = (i & 1) ? dU : sU;
                ta.eta_w = (i & 1) ? se : de;
                ta.U_w = (i & 1) ? sU : dU;
                ta.chunk = i;
                HIP_TRY(launch_tile(f32, 0, TP->ept, TP->block, ta, TP->ntiles, lds, s),
                        "adjoint: forward sweep");
            }
        }
    } else {
        const void *ce = eta0, *cU = U0;
        const int32_t last_ckpt = (A.nseg - 1) * k;
        for (int32_t n1 = 1; n1 <= last_ckpt; ++n1) {   // n1: index of the state produced
            const size_t dst = n1 % k == 0 ? A.ckpt + st_bytes * (n1 / k) : seg_off(0, n1 % k);
            SE_TRY(fstep(ce, cU, dst));
            ce = st_eta(dst);
            cU = st_U(dst);
        }
    }

    auto seg_len = [&](int32_t sg) { return std::min(nsub, sg * k + k) - sg * k; };
    AdjArgs aa{};
    aa.nv = nv;
    aa.ne = ne;
    aa.tri = fa.tri;
    aa.row_ptr = fa.row_ptr;
    aa.pcol = fa.pcol;
    aa.geom = fa.geom;
    aa.H0 = fo->H0;
    aa.Av = fa.Av;
    aa.f = fo->f;
    aa.lam_eta = w + A.lam_eta;
    aa.lam_U = w + A.lam_U;
    aa.lam_Uavg = lam_Uavg;
    aa.gR = g_R ? g_R : static_cast<void *>(w + A.gR);
    aa.gH0 = g_H0 ? g_H0 : static_cast<void *>(w + A.gH0);
    aa.psi = w + A.psi;
    aa.c = fa.c;
    aa.rM = 1.0 / static_cast<double>(nsub);
    aa.thrM = p->theta * aa.rM;

    if (TP && TP->ok(f32, false) && TP->prepared[f32 ? 1 : 0] && TP->adj_ready[f32 ? 1 : 0]) {
        // 2'. reverse sweep on the tile plan, segment by segment from the last.  A
        // segment's forward elevations are recomputed from its checkpoint on the tile
        // kernel (mode 3: each substep's owned elevations to the segment's trajectory
        // buffer, two buffers alternating by segment), its reverse substeps run up to K
        // per launch on the reverse tile kernel (the adjoint state alternating between
        // two buffers).  The recompute of segment sg - 1 shares the launches of the
        // reverse substeps of segment sg (independent work on disjoint arrays); only
        // the last segment's recompute runs alone.  The sweep's first launch starts from
        // the seeds and its last one writes the gradients of the initial state (the
        // seed and final kernels of the per-substep path folded in).
        const DevTiles &P = *TP;
        StepC c = fa.c;
        c.flags &= ~KF_TRACK_VOLUME;
        c.ntiles = P.ntiles;
        c.vol_off = 0;
        const size_t traj_bytes = al(static_cast<size_t>(k) * nv * es);
        auto traj_of = [&](int32_t sg) { return static_cast<void *>(w + A.etraj + (sg & 1) * traj_bytes); };
        AdjTileArgs ra{};
        ra.hdr = P.hdr.as<const TileHdrK>();
        ra.nV = P.nV.as<const int32_t>();
        ra.nE = P.nE.as<const int32_t>();
        ra.lv_gid = P.lv_gid.as<const int32_t>();
        ra.le_rec = P.le_rec.as<const uint32_t>();
        ra.cs_row = P.cs_row.as<const uint16_t>();
        ra.lgeo = f32 ? P.geo32.p : P.geo64.p;
        ra.lae = f32 ? P.ae32.p : P.ae64.p;
        ra.Av = fa.Av;
        ra.H0 = fo->H0;
        ra.f = fo->f;
        ra.traj_stride = nv;
        ra.lam_Uavg = lam_Uavg;
        ra.gR = aa.gR;
        ra.gH0 = aa.gH0;
        ra.c = fa.c;
        ra.rM = aa.rM;
        ra.thrM = aa.thrM;
        ra.K = P.K;
        ra.ntiles = P.ntiles;
        ra.xcd = 1;
        ra.ell = P.ell ? 1 : 0;
        ra.cap_nv = P.max_nv;
        ra.cap_ne = P.max_ne;
        ra.cap_nvu = P.max_nvu;
        ra.cap_cs = P.max_cs;
        void *lam_e[2] = {w + A.lam_eta, w + A.lam_eta2};
        void *lam_u[2] = {w + A.lam_U, w + A.lam_U2};
        int cur = 0;
        const size_t lds_f = P.lds(f32, false), lds_r = P.lds_adj[f32 ? 1 : 0];
        const size_t lds_p = std::max(lds_f, lds_r);
        // recompute launches of segment sg (none when it has a single substep)
        auto recompute = [&](int32_t sg) {
            std::vector<TileArgs> v;
            const int32_t len = seg_len(sg);
            if (len <= 1) return v;
            StepC cs = c;
            cs.nsub = len;
            TileArgs ta = tile_args(m, P, f32, fo, w, L, cs);
            ta.traj = traj_of(sg);
            ta.traj_stride = nv;
            const int32_t nch = (len + P.K - 1) / P.K;
            for (int32_t i = 0; i < nch; ++i) {
                void *se = i == 0 ? const_cast<void *>(ckpt_eta(sg)) : st_eta(seg_off((i - 1) & 1, 1));
                void *sU = i == 0 ? const_cast<void *>(ckpt_U(sg)) : st_U(seg_off((i - 1) & 1, 1));
                void *de = st_eta(seg_off(i & 1, 1));
                void *dU = st_U(seg_off(i & 1, 1));
                ta.eta_u = (i & 1) ? de : se;
                ta.U_u = (i & 1) ? dU : sU;
                ta.eta_w = (i & 1) ? se : de;
                ta.U_w = (i & 1) ? sU : dU;
                ta.chunk = i;
                v.push_back(ta);
            }
            return v;
        };
        for (const TileArgs &ta : recompute(A.nseg - 1))
            HIP_TRY(launch_tile(f32, 3, P.ept, P.block, ta, P.ntiles, lds_f, s),
                    "adjoint: last segment recompute");
        for (int32_t sg = A.nseg - 1; sg >= 0; --sg) {
            const std::vector<TileArgs> rec = sg > 0 ? recompute(sg - 1) : std::vector<TileArgs>();
            ra.eta_s0 = ckpt_eta(sg);
            ra.traj = traj_of(sg);
            size_t i = 0;
            for (int32_t s_hi = seg_len(sg); s_hi > 0; ++i) {
                const int32_t cntr = std::min(P.K, s_hi);
                const bool first = sg == A.nseg - 1 && i == 0, last = sg == 0 && s_hi == cntr;
                ra.cnt = cntr;
                ra.s_hi = s_hi;
                ra.seed = first ? 1 : 0;
                ra.lam_eta_in = first ? lam_eta : lam_e[cur];
                ra.lam_U_in = first ? lam_U : lam_u[cur];
                ra.lam_eta_out = lam_e[cur ^ 1];
                ra.lam_U_out = lam_u[cur ^ 1];
                ra.fin = last ? 1 : 0;
                ra.g_eta0 = last ? g_eta0 : nullptr;
                ra.g_U0 = last ? g_U0 : nullptr;
                if (i < rec.size())
                    HIP_TRY(launch_adj_tile_pair(f32, P.ept, P.block, ra, rec[i], lds_p, s),
                            "adjoint: reverse substeps and recompute");
                else
                    HIP_TRY(launch_adj_tile(f32, P.ept, P.block, ra, lds_r, s),
                            "adjoint: reverse substeps");
                cur ^= 1;
                s_hi -= cntr;
            }
            for (; i < rec.size(); ++i)
                HIP_TRY(launch_tile(f32, 3, P.ept, P.block, rec[i], P.ntiles, lds_f, s),
                        "adjoint: segment recompute");
        }
        return SE_OK;
    }
    HIP_TRY(launch_adj_init(f32, aa, lam_eta, lam_U, s), "adjoint: init");

    // 2. reverse sweep, segment by segment.  Segment sg (substeps m0 .. m1 - 1) needs its
    // states m0 + 1 .. m1 - 1, recomputed from its checkpoint into segment buffer sg mod 2.
    // The last segment is recomputed alone; every other segment's recompute runs in the
    // same launches as the reverse substeps of the segment after it (independent work on
    // disjoint buffers), which halves the chain of dependent launches.
    {
        const int32_t sg = A.nseg - 1;
        for (int32_t j = 1; j < seg_len(sg); ++j)
            SE_TRY(fstep(seg_eta(sg, j - 1), seg_U(sg, j - 1), seg_off(sg, j)));
    }
    for (int32_t sg = A.nseg - 1; sg >= 0; --sg) {
        const int32_t nrev = seg_len(sg);                 // reverse substeps of sg
        const int32_t nrec = sg > 0 ? seg_len(sg - 1) - 1 : 0;   // recompute of sg - 1
        for (int32_t i = 0; i < std::max(nrev, nrec); ++i) {
            const bool rev = i < nrev, rec = i < nrec;
            if (rev) aa.eta_m = seg_eta(sg, nrev - 1 - i);
            if (rec) {
                fa.eta_src = seg_eta(sg - 1, i);
                fa.U_src = seg_U(sg - 1, i);
                fa.eta = st_eta(seg_off(sg - 1, i + 1));
                fa.U = st_U(seg_off(sg - 1, i + 1));
            }
            if (rev && rec)
                HIP_TRY(launch_adj_pair(f32, aa, fa, s), "adjoint: reverse substep and recompute");
            else if (rev)
                HIP_TRY(launch_adj_step(f32, aa, s), "adjoint: reverse substep");
            else
                HIP_TRY(launch_plain_step(f32, fa, s), "adjoint: recompute");
        }
    }
    HIP_TRY(launch_adj_final(f32, aa, g_eta0, g_U0, s), "adjoint: final");
    return SE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched ensemble: a disjoint union of member meshes sharing one tile table
// ---------------------------------------------------------------------------
struct se_batch {
    int device = 0;
    std::vector<sesub::HostMesh> h;
    std::vector<int64_t> voff, eoff;
    int64_t nv = 0, ne = 0;
    std::vector<double> atot;            // per member total area
    sesub::DevBuf Av64, Av32, faults, table, lists;
    std::vector<sesub::StepC> table_host;
    // one-launch epilogue of a call: volume rows of every member, final states that
    // ended in the workspace copied back (per configuration, host copies to compare)
    sesub::DevBuf voltab, cpytab;
    std::vector<sesub::VolMember> voltab_host;
    std::vector<sesub::CopyRange> cpytab_host;
    std::vector<int32_t> list_off;       // per launch offset into lists (size nlaunch + 1)
    std::unique_ptr<sesub::DevTiles> plan;
    int32_t plan_T = 768, plan_K = 4, plan_block = 512;
    std::vector<int32_t> mtiles, mtile_first;
    struct Graph {
        std::vector<uint64_t> key;
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
    };
    std::vector<Graph> graphs;
    void drop_graphs() {
        for (auto &gr : graphs) {
            if (gr.x) (void)hipGraphExecDestroy(gr.x);
            if (gr.g) (void)hipGraphDestroy(gr.g);
        }
        graphs.clear();
    }
    ~se_batch() { drop_graphs(); }
};

namespace sesub {
namespace {

std::vector<const HostMesh *> batch_members(const se_batch *b) {
    std::vector<const HostMesh *> v;
    for (const auto &m : b->h) v.push_back(&m);
    return v;
}

se_status batch_install_plan(se_batch *b, int32_t T, int32_t K, int32_t block) {
    std::unique_ptr<DevTiles> p;
    SE_TRY(make_plan(batch_members(b), b->voff, b->eoff, T, K, block, p));
    const size_t n = b->h.size();
    b->mtiles.assign(n, 0);
    b->mtile_first.assign(n, -1);
    for (size_t t = 0; t < p->hdr_host.size(); ++t) {
        const int mb = p->hdr_host[t].member;
        if (b->mtile_first[mb] < 0) b->mtile_first[mb] = static_cast<int32_t>(t);
        b->mtiles[mb]++;
    }
    b->plan = std::move(p);
    b->plan_T = T;
    b->plan_K = K;
    b->plan_block = block;
    b->table_host.clear();   // forces a new schedule
    b->drop_graphs();
    return SE_OK;
}

se_status batch_ensure_plan(se_batch *b) {
    if (b->plan) return SE_OK;
    static const int32_t cand[][3] = {{768, 4, 512}, {512, 4, 512}, {512, 2, 512}, {256, 4, 512},
                                      {256, 2, 256}, {128, 2, 256}, {64, 1, 256}};
    for (const auto &c : cand) {
        HostTiles ht;
        se_plan_stats_t st;
        if (plan_host(batch_members(b), b->voff, b->eoff, c[0], c[1], c[2], ht, st) != SE_OK)
            continue;
        if (!st.ok_f32 || !st.ok_f64 || !st.ok_sesm_f32 || !st.ok_sesm_f64) continue;
        return batch_install_plan(b, c[0], c[1], c[2]);
    }
    set_error("no default plan fits this batch");
    return SE_ERR_ARG;
}

int64_t batch_vol_rows(const se_params *p, const int32_t *nsub, size_t i) {
    return (p->flags & SE_TRACK_VOLUME) ? nsub[i] + 1 : 2;
}

struct BatchLayout {
    size_t eta_alt, U_alt, sum, U0c, vol, total;
    std::vector<int64_t> vol_off;   // per member offset (elements) into vol partials
};

BatchLayout batch_layout(const se_batch *b, bool f32, const se_params *p, const int32_t *nsub) {
    const size_t s = f32 ? 4 : 8;
    BatchLayout L{};
    size_t o = 0;
    L.eta_alt = o;
    o += al(b->nv * s);
    L.U_alt = o;
    o += al(2 * b->ne * s);
    L.sum = o;
    o += al(16 * b->ne);
    L.U0c = o;
    o += al(2 * b->ne * s);
    L.vol = o;
    int64_t acc = 0;
    for (size_t i = 0; i < b->h.size(); ++i) {
        L.vol_off.push_back(acc);
        acc += batch_vol_rows(p, nsub, i) * ((b->h[i].nv + 63) / 64);
    }
    o += al(acc * 8);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace sesub

extern "C" {

se_status se_batch_create(se_mesh *const *members, int32_t n, se_batch **out) {
    if (!members || n < 1 || !out) {
        set_error("se_batch_create: need n >= 1 members and an output pointer");
        return SE_ERR_ARG;
    }
    *out = nullptr;
    auto b = std::make_unique<se_batch>();
    b->device = members[0] ? members[0]->device : -1;
    b->voff.push_back(0);
    b->eoff.push_back(0);
    for (int32_t i = 0; i < n; ++i) {
        if (!members[i] || members[i]->device != b->device) {
            set_error("se_batch_create: null member or members on different devices");
            return SE_ERR_ARG;
        }
        b->h.push_back(members[i]->h);
        b->voff.push_back(b->voff.back() + members[i]->h.nv);
        b->eoff.push_back(b->eoff.back() + members[i]->h.ne);
    }
    b->nv = b->voff.back();
    b->ne = b->eoff.back();
    if (b->nv >= (int64_t(1) << 31) || b->ne >= (int64_t(1) << 30)) {
        set_error("se_batch_create: batch too large for 32-bit indices");
        return SE_ERR_ARG;
    }
    std::vector<double> av;
    av.reserve(b->nv);
    for (const auto &m : b->h) {
        b->atot.push_back(m.Av_total);
        av.insert(av.end(), m.Av.begin(), m.Av.end());
    }
    if (b->device >= 0) {
        DeviceGuard dg(b->device);
        SE_TRY(b->Av64.upload(av.data(), av.size() * 8));
        std::vector<float> av32(av.begin(), av.end());
        SE_TRY(b->Av32.upload(av32.data(), av32.size() * 4));
        const uint32_t zero = 0;
        SE_TRY(b->faults.upload(&zero, 4));
    }
    *out = b.release();
    return SE_OK;
}

void se_batch_destroy(se_batch *b) {
    if (!b) return;
    if (b->device < 0) {
        delete b;
        return;
    }
    DeviceGuard dg(b->device);
    delete b;
}

se_status se_batch_info(const se_batch *b, int64_t *nv_total, int64_t *ne_total,
                        int64_t *vert_offset, int64_t *elem_offset) {
    if (!b) {
        set_error("se_batch_info: null batch");
        return SE_ERR_ARG;
    }
    if (nv_total) *nv_total = b->nv;
    if (ne_total) *ne_total = b->ne;
    if (vert_offset) std::memcpy(vert_offset, b->voff.data(), b->voff.size() * 8);
    if (elem_offset) std::memcpy(elem_offset, b->eoff.data(), b->eoff.size() * 8);
    return SE_OK;
}

se_status se_batch_workspace_bytes(const se_batch *b, const se_params *p, const int32_t *nsub,
                                   size_t *bytes) {
    if (!b || !p || !nsub || !bytes) {
        set_error("se_batch_workspace_bytes: bad argument");
        return SE_ERR_ARG;
    }
    for (size_t i = 0; i < b->h.size(); ++i)
        if (nsub[i] < 1) {
            set_error("se_batch_workspace_bytes: nsub must be >= 1");
            return SE_ERR_ARG;
        }
    *bytes = batch_layout(b, p->precision == SE_F32_MIXED, p, nsub).total;
    return SE_OK;
}

se_status se_subcycle_batched(se_batch *b, const se_params *p, se_state *st, const se_forcing *fo,
                              const int32_t *nsub, const double *dt, int use_graph, void *ws,
                              void *stream) {
    if (!b || !p || !nsub || !dt) {
        set_error("se_subcycle_batched: null argument");
        return SE_ERR_ARG;
    }
    if (p->scheme != SE_SCHEME_SE || visc_on(p)) {
        set_error("se_subcycle_batched: only the forward-backward scheme without the viscous "
                  "term is batched");
        return SE_ERR_UNSUPPORTED;
    }
    SE_TRY(check_state(st, fo, ws));
    if (b->device < 0) {
        set_error("host-only batch cannot run kernels");
        return SE_ERR_ARG;
    }
    const size_t n = b->h.size();
    // per-member validation (CFL uses each member's own spectral bound)
    for (size_t i = 0; i < n; ++i) {
        se_mesh probe;
        probe.h.mu_max = b->h[i].mu_max;
        SE_TRY(check_params(&probe, p, nsub[i], dt[i]));
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (use_graph && s == nullptr) {
        set_error("se_subcycle_batched: graph capture needs a non-default stream");
        return SE_ERR_ARG;
    }
    DeviceGuard dg(b->device);
    SE_TRY(batch_ensure_plan(b));
    const DevTiles &P = *b->plan;
    const bool f32 = p->precision == SE_F32_MIXED;
    if (!(f32 ? P.ok32 : P.ok64)) {
        set_error("se_subcycle_batched: plan does not fit this precision");
        return SE_ERR_ARG;
    }
    const BatchLayout L = batch_layout(b, f32, p, nsub);
    const int32_t K = P.K;

    // member constants and launch offsets (balance the active tiles per launch)
    std::vector<StepC> tab(n);
    std::vector<int32_t> Lm(n), order(n);
    int32_t Lmax = 0;
    for (size_t i = 0; i < n; ++i) {
        Lm[i] = (nsub[i] + K - 1) / K;
        Lmax = std::max(Lmax, Lm[i]);
        order[i] = static_cast<int32_t>(i);
    }
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return Lm[x] != Lm[y] ? Lm[x] > Lm[y] : b->mtiles[x] > b->mtiles[y];
    });
    std::vector<int64_t> load(Lmax, 0);
    std::vector<int32_t> off(n, 0);
    for (int32_t i : order) {
        int32_t best = 0;
        int64_t best_peak = -1;
        for (int32_t o = 0; o + Lm[i] <= Lmax; ++o) {
            int64_t peak = 0;
            for (int32_t c = o; c < o + Lm[i]; ++c) peak = std::max(peak, load[c]);
            if (best_peak < 0 || peak < best_peak) {
                best_peak = peak;
                best = o;
            }
        }
        off[i] = best;
        for (int32_t c = best; c < best + Lm[i]; ++c) load[c] += b->mtiles[i];
    }
    for (size_t i = 0; i < n; ++i) {
        tab[i] = make_step(p, nsub[i], dt[i]);
        tab[i].ntiles = b->mtiles[i];
        tab[i].vol_off = L.vol_off[i];
        tab[i].chunk0 = off[i];
    }
    const bool same = b->table_host.size() == n &&
                      std::memcmp(b->table_host.data(), tab.data(), n * sizeof(StepC)) == 0;
    if (!same) {
        // new configuration: upload constants and per-launch tile lists
        HIP_TRY(hipStreamSynchronize(s), "batched: sync before table update");
        std::vector<int32_t> lists;
        std::vector<int32_t> loff{0};
        for (int32_t c = 0; c < Lmax; ++c) {
            for (size_t i = 0; i < n; ++i)
                if (c >= off[i] && c < off[i] + Lm[i])
                    for (int32_t t = 0; t < b->mtiles[i]; ++t) lists.push_back(b->mtile_first[i] + t);
            loff.push_back(static_cast<int32_t>(lists.size()));
        }
        SE_TRY(b->table.upload(tab.data(), n * sizeof(StepC)));
        SE_TRY(b->lists.upload(lists.data(), std::max<size_t>(lists.size(), 1) * 4));
        b->list_off = loff;
        b->table_host = tab;
        b->drop_graphs();
    }
    // epilogue tables: volume rows per member, and the word ranges of the members
    // whose last chunk wrote the workspace buffers (an odd number of chunks)
    const size_t es = f32 ? 4 : 8;
    std::vector<VolMember> vt;
    int32_t vrows = 0;
    for (size_t i = 0; i < n; ++i) {
        const int32_t rows = static_cast<int32_t>(batch_vol_rows(p, nsub, i));
        VolMember vm{};
        vm.part_off = L.vol_off[i];
        vm.out_off = vrows;
        vm.width = b->mtiles[i];
        vm.row0 = vrows;
        vm.add = f32 ? p->eta_ref * b->atot[i] : 0.0;
        vt.push_back(vm);
        vrows += rows;
    }
    std::vector<CopyRange> ct;
    int64_t cwords = 0;
    const int64_t wpe = static_cast<int64_t>(es / 4);   // 32-bit words per value
    for (size_t i = 0; i < n; ++i) {
        if (Lm[i] % 2 == 0) continue;
        CopyRange re{b->voff[i] * wpe, cwords, 0, 0};
        ct.push_back(re);
        cwords += b->h[i].nv * wpe;
        CopyRange ru{2 * b->eoff[i] * wpe, cwords, 1, 0};
        ct.push_back(ru);
        cwords += 2 * b->h[i].ne * wpe;
    }
    auto differs = [](const auto &x, const auto &y) {
        return x.size() != y.size() ||
               (!x.empty() && std::memcmp(x.data(), y.data(), x.size() * sizeof(x[0])) != 0);
    };
    if (differs(vt, b->voltab_host) || differs(ct, b->cpytab_host)) {
        HIP_TRY(hipStreamSynchronize(s), "batched: sync before epilogue table update");
        b->drop_graphs();
        SE_TRY(b->voltab.upload(vt.data(), vt.size() * sizeof(VolMember)));
        if (ct.empty())
            SE_TRY(b->cpytab.alloc(sizeof(CopyRange)));   // never read (no ranges)
        else
            SE_TRY(b->cpytab.upload(ct.data(), ct.size() * sizeof(CopyRange)));
        b->voltab_host = vt;
        b->cpytab_host = ct;
    }
    char *w = static_cast<char *>(ws);
    TileArgs a{};
    a.nt = stream_policy(b->nv, f32);
    a.hdr = P.hdr.as<const TileHdrK>();
    a.nV = P.nV.as<const int32_t>();
    a.nE = P.nE.as<const int32_t>();
    a.lv_gid = P.lv_gid.as<const int32_t>();
    a.le_rec = P.le_rec.as<const uint32_t>();
    a.cs_row = P.cs_row.as<const uint16_t>();
    a.lgeo = f32 ? P.geo32.p : P.geo64.p;
    a.lae = f32 ? P.ae32.p : P.ae64.p;
    a.lv_av = f32 ? P.lav32.p : P.lav64.p;
    a.mem = b->table.as<const StepC>();
    a.R = fo->R;
    a.f = fo->f;
    a.H0 = fo->H0;
    a.W = fo->W;
    a.Av = f32 ? b->Av32.p : b->Av64.p;
    a.Av64 = b->Av64.as<const double>();
    a.sum = w + L.sum;
    a.U0c = w + L.U0c;
    a.Uavg = st->Uavg;
    a.vol_part = reinterpret_cast<double *>(w + L.vol);
    a.faults = b->faults.as<uint32_t>();
    a.K = K;
    a.ksub = K;
    a.xcd = 1;
    a.cap_nv = P.max_nv;
    a.cap_ne = P.max_ne;
    a.cap_nvu = P.max_nvu;
    a.cap_cs = P.max_cs;
    a.ell = P.ell ? 1 : 0;
    a.eta_u = st->eta;
    a.eta_w = w + L.eta_alt;
    a.U_u = st->U;
    a.U_w = w + L.U_alt;
    const size_t lds = f32 ? P.lds_bytes32 : P.lds_bytes64;
    HIP_TRY(prepare_tile(f32, 0, P.ept, P.block), "batched prepare");

    auto enqueue = [&]() -> se_status {
        for (int32_t c = 0; c < Lmax; ++c) {
            const int32_t cnt = b->list_off[c + 1] - b->list_off[c];
            if (cnt == 0) continue;
            a.chunk = c;
            a.tile_list = b->lists.as<const int32_t>() + b->list_off[c];
            a.ntiles = cnt;
            HIP_TRY(launch_tile(f32, 0, P.ept, P.block, a, cnt, lds, s), "batched launch");
        }
        HIP_TRY(launch_copy_ranges(reinterpret_cast<const uint32_t *>(w + L.eta_alt),
                                   static_cast<uint32_t *>(st->eta),
                                   reinterpret_cast<const uint32_t *>(w + L.U_alt),
                                   static_cast<uint32_t *>(st->U),
                                   b->cpytab.as<const CopyRange>(),
                                   static_cast<int32_t>(b->cpytab_host.size()), cwords, s),
                "batched copy of final states");
        if (st->volume)
            HIP_TRY(launch_vol_reduce_batch(a.vol_part, b->voltab.as<const VolMember>(),
                                            static_cast<int32_t>(n), vrows, st->volume, s),
                    "batched volume");
        return SE_OK;
    };

    if (!use_graph) return enqueue();
    std::vector<uint64_t> key = {
        reinterpret_cast<uint64_t>(st->eta), reinterpret_cast<uint64_t>(st->U),
        reinterpret_cast<uint64_t>(st->Uavg), reinterpret_cast<uint64_t>(st->volume),
        reinterpret_cast<uint64_t>(fo->R), reinterpret_cast<uint64_t>(fo->f),
        reinterpret_cast<uint64_t>(fo->H0), reinterpret_cast<uint64_t>(fo->W),
        reinterpret_cast<uint64_t>(ws), reinterpret_cast<uint64_t>(s),
        static_cast<uint64_t>(p->precision), static_cast<uint64_t>(p->flags)};
    for (auto &gr : b->graphs) {
        if (gr.key == key) {
            HIP_TRY(hipGraphLaunch(gr.x, s), "batched graph launch");
            return SE_OK;
        }
    }
    se_batch::Graph gr;
    gr.key = key;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    const se_status es_ = enqueue();
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (es_ != SE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return es_;
    }
    if (ee != hipSuccess) return hip_fail(ee, "end capture");
    gr.g = g;
    HIP_TRY(hipGraphInstantiate(&gr.x, g, nullptr, nullptr, 0), "graph instantiate");
    b->graphs.push_back(gr);
    HIP_TRY(hipGraphLaunch(gr.x, s), "batched graph launch");
    return SE_OK;
}


se_status se_batch_set_plan_impl(se_batch *b, int32_t tile, int32_t k_fused, int32_t block) {
    if (b->device < 0) {
        HostTiles ht;
        se_plan_stats_t st;
        SE_TRY(plan_host(batch_members(b), b->voff, b->eoff, tile, k_fused, block, ht, st));
        b->plan_T = tile;
        b->plan_K = k_fused;
        b->plan_block = block;
        return SE_OK;
    }
    DeviceGuard dg(b->device);
    return batch_install_plan(b, tile, k_fused, block);
}

se_status se_batch_get_plan_impl(const se_batch *b, int32_t *tile, int32_t *k_fused,
                                 int32_t *block) {
    if (tile) *tile = b->plan_T;
    if (k_fused) *k_fused = b->plan_K;
    if (block) *block = b->plan_block;
    return SE_OK;
}

se_status se_batch_plan_stats_impl(const se_batch *b, int32_t tile, int32_t k_fused,
                                   int32_t block, se_plan_stats_t *stats) {
    HostTiles ht;
    return plan_host(batch_members(b), b->voff, b->eoff, tile, k_fused, block, ht, *stats);
}

se_status se_batch_faults_impl(se_batch *b, void *stream, uint32_t *bits) {
    if (b->device < 0) {
        set_error("host-only batch has no fault word");
        return SE_ERR_ARG;
    }
    DeviceGuard dg(b->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamSynchronize(s), "se_check_faults sync");
    uint32_t v = 0;
    HIP_TRY(hipMemcpy(&v, b->faults.p, 4, hipMemcpyDeviceToHost), "se_check_faults copy");
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(b->faults.p, &zero, 4, hipMemcpyHostToDevice), "se_check_faults reset");
    *bits = v;
    return SE_OK;
}

}  // extern "C"
