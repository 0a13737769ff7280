// HIP kernels (gfx950, wave64) of the split-explicit barotropic subcycle.
//
// One substep (Banerjee et al., arXiv 2311.08241, Sec. 2.2, eq. (eq4_10),
// pressure sign of eq. (eq4_5)):
//   triangle phase  grad eta (P1, difference form), H = mean(H0 + eta),
//                   U' = (I + aJ)^-1 [(I - aJ) U + dt_s(-g H grad eta + R)],
//                   a = f dt_s / 2, J = e_z x;  F = (1+theta) U' - theta U;
//                   flux of F through each vertex's median-dual sub-cell
//                   boundary inside the triangle: phi_k = F . (-A_e grad N_k)
//   vertex phase    eta' = eta - dt_s (sum_k phi / A_v + W), summed over the
//                   vertex's triangles in ascending triangle order
// plus the running sum of U' for the averaged transport of eq. (eq4_12) and
// the volume sum_v A_v eta_v.
//
// All floating-point code is compiled without FMA contraction so that every
// path (plain, any tile plan) performs the same IEEE operations in the same
// order: FP64 results do not depend on the plan.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sesub {

namespace {


template <typename T> __device__ __forceinline__ T cdts(const StepC &c);
template <> __device__ __forceinline__ double cdts<double>(const StepC &c) { return c.dts; }
template <> __device__ __forceinline__ float cdts<float>(const StepC &c) { return c.dts_f; }
template <typename T> __device__ __forceinline__ T cg(const StepC &c);
template <> __device__ __forceinline__ double cg<double>(const StepC &c) { return c.g; }
template <> __device__ __forceinline__ float cg<float>(const StepC &c) { return c.g_f; }
template <typename T> __device__ __forceinline__ T cth(const StepC &c);
template <> __device__ __forceinline__ double cth<double>(const StepC &c) { return c.theta; }
template <> __device__ __forceinline__ float cth<float>(const StepC &c) { return c.theta_f; }
template <typename T> __device__ __forceinline__ T copt(const StepC &c);
template <> __device__ __forceinline__ double copt<double>(const StepC &c) { return c.opt; }
template <> __device__ __forceinline__ float copt<float>(const StepC &c) { return c.opt_f; }

// Per-triangle update.  ea..ec: eta at the vertices (FP64: absolute; FP32:
// deviation from eta_ref), ha..hc: H0, al = f dt_s / 2 (0.5 f first, then dt_s).
// Returns U' and the three sub-cell fluxes; dry is set when the triangle's total depth
// is not positive.  The CPU definition's divisions by 3 and by 1 + a^2 are
// multiplications by reciprocals here (one FP64 division per triangle and substep
// instead of three; agreement with the definition to rounding), the same in every
// path and plan.
template <typename T, bool F32>
__device__ __forceinline__ void tri_update(T ea, T eb, T ec, T ha, T hb, T hc, T gbx, T gby,
                                           T gcx, T gcy, T Ae, T Ux, T Uy, T Rx, T Ry, T al,
                                           const StepC &c, bool linear_h, T &Unx, T &Uny,
                                           T &pa, T &pb, T &pc, bool &dry) {
    const T dts = cdts<T>(c), g = cg<T>(c), th = cth<T>(c), opt = copt<T>(c);
    const T db = eb - ea, dc = ec - ea;
    const T gx = db * gbx + dc * gcx;
    const T gy = db * gby + dc * gcy;
    const T third = T(1) / T(3);
    T He;
    if (linear_h) {
        He = (ha + hb + hc) * third;
    } else if (!F32) {
        He = ((ha + ea) + (hb + eb) + (hc + ec)) * third;
    } else {
        He = ((ha + hb + hc) + (ea + eb + ec)) * third + c.eta_ref_f;
    }
    dry = !(He > T(0));
    const T rx = Ux + al * Uy + dts * (-g * He * gx + Rx);
    const T ry = Uy - al * Ux + dts * (-g * He * gy + Ry);
    const T rden = T(1) / (T(1) + al * al);
    Unx = (rx + al * ry) * rden;
    Uny = (ry - al * rx) * rden;
    const T Fx = opt * Unx - th * Ux;
    const T Fy = opt * Uny - th * Uy;
    const T gax = -(gbx + gcx), gay = -(gby + gcy);
    pa = Fx * (-Ae * gax) + Fy * (-Ae * gay);
    pb = Fx * (-Ae * gbx) + Fy * (-Ae * gby);
    pc = Fx * (-Ae * gcx) + Fy * (-Ae * gcy);
}

// FP32 triangle update with per-triangle constants of the call: a = f dt/2 (al),
// 1/(1 + a^2) (rk), dt R (dRx, dRy), -A_e (mAe), mean H0 (+ eta_ref unless H is
// linear) (rH); gd = g dt.  The Crank-Nicolson step is evaluated as the increment
//   U' = U + C (q - 2 a J U),  C = (I + aJ)^-1,  q = dt (R - g H grad eta),
// algebraically equal to C [(I - aJ) U + q]; in FP32 the rounded rotation
// coefficients then perturb only the small increment instead of scaling U by
// 1 + O(eps) every substep, which would bias its amplitude over many substeps.
__device__ __forceinline__ void tri_update_f32(float ea, float eb, float ec, float rH, float gbx,
                                               float gby, float gcx, float gcy, float mAe,
                                               float ux, float uy, float dRx, float dRy,
                                               float al, float rk, float gd, float th,
                                               bool linear_h, float &Unx, float &Uny, float &pa,
                                               float &pb, float &pc, bool &dry) {
    // fused multiply-adds (one rounding each) where a product feeds a sum
    const float db = eb - ea, dc = ec - ea;
    const float gx = __builtin_fmaf(db, gbx, dc * gcx);
    const float gy = __builtin_fmaf(db, gby, dc * gcy);
    const float He = linear_h ? rH : __builtin_fmaf(ea + eb + ec, 1.0f / 3.0f, rH);
    dry = !(He > 0.0f);
    const float gHe = gd * He;
    const float al2 = 2.0f * al;
    const float px = __builtin_fmaf(al2, uy, __builtin_fmaf(-gHe, gx, dRx));
    const float py = __builtin_fmaf(-al2, ux, __builtin_fmaf(-gHe, gy, dRy));
    const float dx = __builtin_fmaf(al, py, px) * rk;
    const float dy = __builtin_fmaf(-al, px, py) * rk;
    Unx = ux + dx;
    Uny = uy + dy;
    const float Fx = __builtin_fmaf(th, dx, Unx);   // (1 + theta) U' - theta U
    const float Fy = __builtin_fmaf(th, dy, Uny);
    pb = mAe * __builtin_fmaf(Fx, gbx, Fy * gby);
    pc = mAe * __builtin_fmaf(Fx, gcx, Fy * gcy);
    pa = -(pb + pc);
}

// FP32 vertex update eta - dt (sum / A_v + W) with the reciprocal area 1 / A_v
// (identical in every path).
template <typename T>
__device__ __forceinline__ T vtx_update_f32(T eta, T acc, T rav, T w, T dts) {
    return __builtin_fmaf(-dts, __builtin_fmaf(acc, rav, w), eta);
}

// Per-triangle constants of the FP32 update (identical in every path).
__device__ __forceinline__ void tri_consts_f32(float f, float dts, float &al, float &rk) {
    al = 0.5f * f * dts;
    rk = 1.0f / (1.0f + al * al);
}

// Non-temporal accesses of the tile kernels.  A tile's own triangle records, geometry
// and areas are read by that tile alone, once per launch, and what a launch writes is
// next read by the following launch; streaming both past L2 leaves L2 to the state that
// neighbouring tiles' halo gathers share (lat-lon workload, FP32: 150 -> 137 us per
// launch).  The smaller per-tile tables (local vertex ids, the owned running sums; in
// FP32 also the row offsets and owned FP64 areas) measured faster as ordinary loads.
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <typename T> struct NtVec2;
template <> struct NtVec2<float> { using type = nt_f2; };
template <> struct NtVec2<double> { using type = nt_d2; };

__device__ __forceinline__ uint4 ld_nt(const uint4 *p) {
    const nt_u4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld_nt(const uint2 *p) {
    const nt_u2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u2 *>(p));
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld_nt(const float2 *p) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2 *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p));
    return make_double2(v.x, v.y);
}
template <typename S> __device__ __forceinline__ S ld_nt(const S *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T> __device__ __forceinline__ void st_nt2(void *p, int64_t i, T x, T y) {
    using V = typename NtVec2<T>::type;
    const V v = {x, y};
    __builtin_nontemporal_store(v, static_cast<V *>(p) + i);
}
// The same accesses under a launch-wide policy (a template parameter of the tile
// kernel, so that no access carries a branch): non-temporal when the launch streams
// more than the last-level cache can keep between launches (large meshes), ordinary
// when the whole working set stays cached from one launch to the next (small meshes,
// where bypassing the caches would turn hits into device-memory reads).
template <bool NT, typename V> __device__ __forceinline__ V ldp(const V *p) {
    if constexpr (NT)
        return ld_nt(p);
    else
        return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st2(void *p, int64_t i, T x, T y) {
    if constexpr (NT) {
        st_nt2<T>(p, i, x, y);
    } else {
        using T2 = typename Vec2<T>::type;
        T2 v;
        v.x = x;
        v.y = y;
        static_cast<T2 *>(p)[i] = v;
    }
}
template <bool NT, typename T> __device__ __forceinline__ void st1(T v, T *p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Running sum of the substep transports, always accumulated in FP64 (the FP32 path
// converts each FP32 transport exactly and adds it in FP64: on this hardware an FP64
// add issues at the FP32 rate, and the sum carries no FP32 rounding).
template <bool F32> struct SumT {
    double x, y;
    template <typename V> __device__ __forceinline__ void init(V ux, V uy) {
        x = (double)ux;
        y = (double)uy;
    }
    template <typename V> __device__ __forceinline__ void add(V ux, V uy) {
        x += (double)ux;
        y += (double)uy;
    }
    __device__ __forceinline__ void load(const void *p, int64_t i) {
        const nt_d2 v = static_cast<const nt_d2 *>(p)[i];
        x = v.x;
        y = v.y;
    }
    template <bool NT = false> __device__ __forceinline__ void store(void *p, int64_t i) const {
        const nt_d2 v = {x, y};
        if constexpr (NT)
            __builtin_nontemporal_store(v, static_cast<nt_d2 *>(p) + i);
        else
            static_cast<nt_d2 *>(p)[i] = v;
    }
    __device__ __forceinline__ double vx() const { return x; }
    __device__ __forceinline__ double vy() const { return y; }
};


// ---------------------------------------------------------------------------
// Plain two-kernel path
// ---------------------------------------------------------------------------
// Triangle phase of one plain substep for triangle e (any e; out of range returns).
template <typename T, bool F32>
__device__ __forceinline__ void plain_tri_at(const PlainArgs &a, int64_t e) {
    using T2 = typename Vec2<T>::type;
    if (e >= a.ne) return;
    const StepC &c = a.c;
    const T *eta = static_cast<const T *>(a.eta_src ? a.eta_src : a.eta);
    const T *H0 = static_cast<const T *>(a.H0);
    const T *geom = static_cast<const T *>(a.geom);
    const int32_t va = a.tri[3 * e], vb = a.tri[3 * e + 1], vc = a.tri[3 * e + 2];
    T2 *U = static_cast<T2 *>(a.U);
    const T2 u = (a.U_src ? static_cast<const T2 *>(a.U_src) : U)[e];
    const T2 r = static_cast<const T2 *>(a.R)[e];
    const T fc = static_cast<const T *>(a.f)[e];
    T Unx, Uny, pa, pb, pc;
    bool dry;
    const bool linear_h = (c.flags & KF_LINEAR_H) != 0;
    if constexpr (F32) {
        float al, rk;
        tri_consts_f32(fc, c.dts_f, al, rk);
        const float rH = (H0[va] + H0[vb] + H0[vc]) * (1.0f / 3.0f) + (linear_h ? 0.0f : c.eta_ref_f);
        tri_update_f32(eta[va], eta[vb], eta[vc], rH, geom[e], geom[a.ne + e],
                       geom[2 * a.ne + e], geom[3 * a.ne + e], -geom[4 * a.ne + e], u.x, u.y,
                       c.dts_f * r.x, c.dts_f * r.y, al, rk, c.g_f * c.dts_f, c.theta_f,
                       linear_h, Unx, Uny, pa, pb, pc, dry);
    } else {
        tri_update<T, F32>(eta[va], eta[vb], eta[vc], H0[va], H0[vb], H0[vc], geom[e],
                           geom[a.ne + e], geom[2 * a.ne + e], geom[3 * a.ne + e],
                           geom[4 * a.ne + e], u.x, u.y, r.x, r.y, T(0.5) * fc * cdts<T>(c), c,
                           linear_h, Unx, Uny, pa, pb, pc, dry);
    }
    if (dry) set_fault(a.faults, 1u);
    T *phi = static_cast<T *>(a.phi);
    phi[3 * e] = pa;
    phi[3 * e + 1] = pb;
    phi[3 * e + 2] = pc;
    T2 un;
    un.x = Unx;
    un.y = Uny;
    U[e] = un;
    if (a.fwd_only) return;
    const bool first = a.m == 0, last = a.m == c.nsub - 1;
    SumT<F32> s;
    if (first) {
        s.init(Unx, Uny);
        static_cast<T2 *>(a.U0c)[e] = u;
    } else {
        s.load(a.sum, e);
        s.add(Unx, Uny);
    }
    if (last) {
        if (!a.Uavg) return;
        const T2 u0 = first ? u : static_cast<const T2 *>(a.U0c)[e];
        a.Uavg[2 * e] = s.vx() / c.Mdbl + c.thM * ((double)Unx - (double)u0.x);
        a.Uavg[2 * e + 1] = s.vy() / c.Mdbl + c.thM * ((double)Uny - (double)u0.y);
    } else {
        s.store(a.sum, e);
    }
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_plain_tri(PlainArgs a) {
    plain_tri_at<T, F32>(a, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// Vertex phase of one plain substep for vertex v < nv: the new elevation, and the
// volume terms A_v eta of the new and old elevation.
template <typename T, bool F32>
__device__ __forceinline__ void plain_vtx_at(const PlainArgs &a, int64_t v, double &v_new,
                                             double &v_old) {
    const StepC &c = a.c;
    T *eta = static_cast<T *>(a.eta);
    const T *phi = static_cast<const T *>(a.phi);
    T acc = T(0);
    const int32_t j1 = a.row_ptr[v + 1];
    for (int32_t j = a.row_ptr[v]; j < j1; ++j) acc += phi[a.pcol[j]];
    const T eo = a.eta_src ? static_cast<const T *>(a.eta_src)[v] : eta[v];
    const T wv = a.W ? static_cast<const T *>(a.W)[v] : T(0);
    const T av = static_cast<const T *>(a.Av)[v];
    const T en = F32 ? vtx_update_f32(eo, acc, T(1) / av, wv, cdts<T>(c))
                     : eo - cdts<T>(c) * (acc * (T(1) / av) + wv);
    eta[v] = en;
    if (!finite_val(en)) set_fault(a.faults, 2u);
    const double av64 = a.Av64[v];
    v_new = av64 * (double)en;
    v_old = av64 * (double)eo;
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_plain_vtx(PlainArgs a) {
    __shared__ double red[2][4];
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const StepC &c = a.c;
    const bool first = a.m == 0, last = a.m == c.nsub - 1;
    const bool track = (c.flags & KF_TRACK_VOLUME) != 0;
    double v_new = 0.0, v_old = 0.0;
    if (v < a.nv) plain_vtx_at<T, F32>(a, v, v_new, v_old);
    if (a.fwd_only || !(track || first || last)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v_new = wave_sum(v_new);
    v_old = wave_sum(v_old);
    if (lane == 0) {
        red[0][w] = v_new;
        red[1][w] = v_old;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sn = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
        const int64_t row = track ? (a.m + 1) : 1;
        if (track || last) a.vol_part[row * a.nblk_v + blockIdx.x] = sn;
        if (first) a.vol_part[blockIdx.x] = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
    }
}

// ---------------------------------------------------------------------------
// AB3-AM4 (SESM) substep pieces, shared by the plain kernels and the tile kernel.
// FP64: the operations of the definition in its order (as the oracle);
// FP32: the same steps with fused multiply-adds and per-triangle constants
// (dt f: fd, dt R: dRx/dRy, -A_e: mAe, mean H0 (+ eta_ref unless H is linear): rH).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T sesm_ab(const StepC &c, T u, T u1, T u2);
template <> __device__ __forceinline__ double sesm_ab<double>(const StepC &c, double u, double u1,
                                                             double u2) {
    return c.ab0 * u - c.ab1 * u1 + c.ab2 * u2;
}
template <> __device__ __forceinline__ float sesm_ab<float>(const StepC &c, float u, float u1,
                                                           float u2) {
    return __builtin_fmaf(c.ab2_f, u2, __builtin_fmaf(-c.ab1_f, u1, c.ab0_f * u));
}

template <typename T> __device__ __forceinline__ T sesm_am(const StepC &c, T en, T e, T e1, T e2);
template <> __device__ __forceinline__ double sesm_am<double>(const StepC &c, double en, double e,
                                                             double e1, double e2) {
    return c.am0 * en + c.am1 * e + c.am2 * e1 + c.am3 * e2;
}
template <> __device__ __forceinline__ float sesm_am<float>(const StepC &c, float en, float e,
                                                           float e1, float e2) {
    return __builtin_fmaf(c.am3_f, e2, __builtin_fmaf(c.am2_f, e1, __builtin_fmaf(c.am1_f, e, c.am0_f * en)));
}

// Sub-cell fluxes F . S_k of a transport F (FP64: as in tri_update).
// FP32 form with mAe = -A_e (as in tri_update_f32)
__device__ __forceinline__ void slot_fluxes_f32(float Fx, float Fy, float gbx, float gby, float gcx,
                                                float gcy, float mAe, float &pa, float &pb,
                                                float &pc) {
    pb = mAe * __builtin_fmaf(Fx, gbx, Fy * gby);
    pc = mAe * __builtin_fmaf(Fx, gcx, Fy * gcy);
    pa = -(pb + pc);
}

// Transport update of eq. (eq4_8): U + dt (-f e_z x U_ab - g H_am grad eta_am + R).
// FP64: eAa..eAc eta_am at the vertices, ha..hc H0.
__device__ __forceinline__ void sesm_u_f64(const StepC &c, bool linear_h, double eAa, double eAb,
                                           double eAc, double ha, double hb, double hc, double gbx,
                                           double gby, double gcx, double gcy, double fc,
                                           double Rx, double Ry, double ux, double uy, double ax,
                                           double ay, double &Unx, double &Uny, bool &dry) {
    const double db = eAb - eAa, dc = eAc - eAa;
    const double gx = db * gbx + dc * gcx;
    const double gy = db * gby + dc * gcy;
    const double He = linear_h ? (ha + hb + hc) / 3.0 : ((ha + eAa) + (hb + eAb) + (hc + eAc)) / 3.0;
    dry = !(He > 0.0);
    const double dts = c.dts, g = c.g;
    Unx = ux + dts * (fc * ay - g * He * gx + Rx);
    Uny = uy + dts * (-fc * ax - g * He * gy + Ry);
}
// FP32: rH mean H0 (+ eta_ref unless linear), gd = g dt, fd = f dt, dR = dt R.
__device__ __forceinline__ void sesm_u_f32(bool linear_h, float eAa, float eAb, float eAc, float rH,
                                           float gbx, float gby, float gcx, float gcy, float fd,
                                           float dRx, float dRy, float gd, float ux, float uy,
                                           float ax, float ay, float &Unx, float &Uny, bool &dry) {
    const float db = eAb - eAa, dc = eAc - eAa;
    const float gx = __builtin_fmaf(db, gbx, dc * gcx);
    const float gy = __builtin_fmaf(db, gby, dc * gcy);
    const float He = linear_h ? rH : __builtin_fmaf(eAa + eAb + eAc, 1.0f / 3.0f, rH);
    dry = !(He > 0.0f);
    const float gHe = gd * He;
    Unx = ux + __builtin_fmaf(fd, ay, __builtin_fmaf(-gHe, gx, dRx));
    Uny = uy + __builtin_fmaf(-fd, ax, __builtin_fmaf(-gHe, gy, dRy));
}

// ---- plain three-kernel form: AB3 transport and fluxes; elevation; transport
template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_sesm_ab(PlainArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.ne) return;
    const StepC &c = a.c;
    const T *geom = static_cast<const T *>(a.geom);
    const T2 u = static_cast<const T2 *>(a.U)[e];
    const T2 u1 = static_cast<const T2 *>(a.U1)[e];
    const T2 u2 = static_cast<const T2 *>(a.U2)[e];
    T2 ab;
    ab.x = sesm_ab<T>(c, u.x, u1.x, u2.x);
    ab.y = sesm_ab<T>(c, u.y, u1.y, u2.y);
    static_cast<T2 *>(a.Uab)[e] = ab;
    T pa, pb, pc;
    if constexpr (F32)
        slot_fluxes_f32(ab.x, ab.y, geom[e], geom[a.ne + e], geom[2 * a.ne + e],
                        geom[3 * a.ne + e], -geom[4 * a.ne + e], pa, pb, pc);
    else
        slot_fluxes(ab.x, ab.y, geom[e], geom[a.ne + e], geom[2 * a.ne + e], geom[3 * a.ne + e],
                    geom[4 * a.ne + e], pa, pb, pc);
    T *phi = static_cast<T *>(a.phi);
    phi[3 * e] = pa;
    phi[3 * e + 1] = pb;
    phi[3 * e + 2] = pc;
    SumT<F32> s;
    if (a.m == 0)
        s.init(ab.x, ab.y);
    else {
        s.load(a.sum, e);
        s.add(ab.x, ab.y);
    }
    if (a.m == c.nsub - 1) {
        if (a.Uavg) {
            a.Uavg[2 * e] = s.vx() / c.Mdbl;
            a.Uavg[2 * e + 1] = s.vy() / c.Mdbl;
        }
    } else {
        s.store(a.sum, e);
    }
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_sesm_vtx(PlainArgs a) {
    __shared__ double red[2][4];
    const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const StepC &c = a.c;
    const bool first = a.m == 0, last = a.m == c.nsub - 1;
    const bool track = (c.flags & KF_TRACK_VOLUME) != 0;
    double v_new = 0.0, v_old = 0.0;
    if (v < a.nv) {
        T *eta = static_cast<T *>(a.eta);
        T *eta1 = static_cast<T *>(a.eta1);
        T *eta2 = static_cast<T *>(a.eta2);
        const T *phi = static_cast<const T *>(a.phi);
        T acc = T(0);
        const int32_t j1 = a.row_ptr[v + 1];
        for (int32_t j = a.row_ptr[v]; j < j1; ++j) acc += phi[a.pcol[j]];
        const T eo = eta[v], e1 = eta1[v], e2 = eta2[v];
        const T wv = a.W ? static_cast<const T *>(a.W)[v] : T(0);
        const T av = static_cast<const T *>(a.Av)[v];
        const T en = F32 ? vtx_update_f32(eo, acc, T(1) / av, wv, cdts<T>(c))
                         : eo - cdts<T>(c) * (acc * (T(1) / av) + wv);
        static_cast<T *>(a.etaA)[v] = sesm_am<T>(c, en, eo, e1, e2);
        eta2[v] = e1;
        eta1[v] = eo;
        eta[v] = en;
        if (!finite_val(en)) set_fault(a.faults, 2u);
        const double av64 = a.Av64[v];
        v_new = av64 * (double)en;
        v_old = av64 * (double)eo;
    }
    if (!(track || first || last)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v_new = wave_sum(v_new);
    v_old = wave_sum(v_old);
    if (lane == 0) {
        red[0][w] = v_new;
        red[1][w] = v_old;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double sn = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
        const int64_t row = track ? (a.m + 1) : 1;
        if (track || last) a.vol_part[row * a.nblk_v + blockIdx.x] = sn;
        if (first) a.vol_part[blockIdx.x] = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
    }
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_sesm_u(PlainArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.ne) return;
    const StepC &c = a.c;
    const bool linear_h = (c.flags & KF_LINEAR_H) != 0;
    const T *eA = static_cast<const T *>(a.etaA);
    const T *H0 = static_cast<const T *>(a.H0);
    const T *geom = static_cast<const T *>(a.geom);
    const int32_t va = a.tri[3 * e], vb = a.tri[3 * e + 1], vc = a.tri[3 * e + 2];
    T2 *U = static_cast<T2 *>(a.U);
    T2 *U1 = static_cast<T2 *>(a.U1);
    T2 *U2 = static_cast<T2 *>(a.U2);
    const T2 u = U[e];
    const T2 ab = static_cast<const T2 *>(a.Uab)[e];
    const T2 r = static_cast<const T2 *>(a.R)[e];
    const T fc = static_cast<const T *>(a.f)[e];
    T Unx, Uny;
    bool dry;
    if constexpr (F32) {
        const float rH = (H0[va] + H0[vb] + H0[vc]) * (1.0f / 3.0f) + (linear_h ? 0.0f : c.eta_ref_f);
        sesm_u_f32(linear_h, eA[va], eA[vb], eA[vc], rH, geom[e], geom[a.ne + e],
                   geom[2 * a.ne + e], geom[3 * a.ne + e], fc * c.dts_f, c.dts_f * r.x,
                   c.dts_f * r.y, c.g_f * c.dts_f, u.x, u.y, ab.x, ab.y, Unx, Uny, dry);
    } else {
        sesm_u_f64(c, linear_h, eA[va], eA[vb], eA[vc], H0[va], H0[vb], H0[vc], geom[e],
                   geom[a.ne + e], geom[2 * a.ne + e], geom[3 * a.ne + e], fc, r.x, r.y, u.x,
                   u.y, ab.x, ab.y, Unx, Uny, dry);
    }
    if (dry) set_fault(a.faults, 1u);
    U2[e] = U1[e];
    U1[e] = u;
    T2 un;
    un.x = Unx;
    un.y = Uny;
    U[e] = un;
}

// Final step of the tile form of AB3-AM4: the transport update of the last
// substep (pending at the end of the last launch) into the caller's U, and the
// final elevation into the caller's eta.  U1: U^{M-1}, Uab: U_ab^{M-1}, etaA:
// eta_am^{M-1}, eta1: eta^M (global numbering, written by the last launch).
template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_sesm_fin(PlainArgs a) {
    using T2 = typename Vec2<T>::type;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const StepC &c = a.c;
    if (i < a.nv) static_cast<T *>(a.eta)[i] = static_cast<const T *>(a.eta1)[i];
    if (i >= a.ne) return;
    const int64_t e = i;
    const bool linear_h = (c.flags & KF_LINEAR_H) != 0;
    const T *eA = static_cast<const T *>(a.etaA);
    const T *H0 = static_cast<const T *>(a.H0);
    const T *geom = static_cast<const T *>(a.geom);
    const int32_t va = a.tri[3 * e], vb = a.tri[3 * e + 1], vc = a.tri[3 * e + 2];
    const T2 u = static_cast<const T2 *>(a.U1)[e];
    const T2 ab = static_cast<const T2 *>(a.Uab)[e];
    const T2 r = static_cast<const T2 *>(a.R)[e];
    const T fc = static_cast<const T *>(a.f)[e];
    T Unx, Uny;
    bool dry;
    if constexpr (F32) {
        const float rH = (H0[va] + H0[vb] + H0[vc]) * (1.0f / 3.0f) + (linear_h ? 0.0f : c.eta_ref_f);
        sesm_u_f32(linear_h, eA[va], eA[vb], eA[vc], rH, geom[e], geom[a.ne + e],
                   geom[2 * a.ne + e], geom[3 * a.ne + e], fc * c.dts_f, c.dts_f * r.x,
                   c.dts_f * r.y, c.g_f * c.dts_f, u.x, u.y, ab.x, ab.y, Unx, Uny, dry);
    } else {
        sesm_u_f64(c, linear_h, eA[va], eA[vb], eA[vc], H0[va], H0[vb], H0[vc], geom[e],
                   geom[a.ne + e], geom[2 * a.ne + e], geom[3 * a.ne + e], fc, r.x, r.y, u.x,
                   u.y, ab.x, ab.y, Unx, Uny, dry);
    }
    if (dry) set_fault(a.faults, 1u);
    T2 un;
    un.x = Unx;
    un.y = Uny;
    static_cast<T2 *>(a.U)[e] = un;
}

// ---------------------------------------------------------------------------
// Temporally blocked tile kernel: up to K substeps of one tile per launch
// ---------------------------------------------------------------------------
__device__ __forceinline__ int align16(int b) { return (b + 15) & ~15; }

// SM: the AB3-AM4 (SESM) substep instead of the forward-backward one.  The state a
// launch hands to the next is (eta, eta^{-1}, eta^{-2}, eta_am) at vertices and
// (U, U^{-1}, U_ab) at triangles, with the transport update of the last substep
// still pending (it needs eta_am on a ring the launch does not hold); the next
// launch, or k_sesm_fin after the last one, applies it.
// MODE 2: the forward-backward substep with the barotropic viscous term, whose
// evaluation on a triangle needs its edge neighbours one ring further out: a launch
// loading K rings runs K / 2 substeps, each with a velocity phase (u = U / H_e of the
// triangles one ring beyond those updated) before the triangle phase; R holds
// R - V(eta^0, U^0) and the triangle phase adds V(eta^m, U^m).
// MODE 3: MODE 0 that also writes the owned vertices' elevation after every substep to
// a trajectory (the adjoint's recompute).
// The body of one tile's launch work for block index b of a grid of G blocks.
// NT: the access policy of the launch (non-temporal accesses of the tile's own tables
// and of the write-back; see ldp), chosen by the host per mesh size.
template <typename T, bool F32, int EPT, int BLOCK, int MODE, bool NT = false>
__device__ __forceinline__ void tile_body(const TileArgs &a, int b, int G) {
    constexpr bool SM = MODE == 1, VI = MODE == 2, TR = MODE == 3, FB = MODE == 0 || TR;
    using T2 = typename Vec2<T>::type;
    constexpr int NW = BLOCK / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.xcd) {
        // consecutive tiles on the same XCD (blocks are dealt round-robin to 8 XCDs)
        const int x = b & 7, q = b >> 3;
        const int base = G >> 3, rem = G & 7;
        b = x * base + (x < rem ? x : rem) + q;
    }
    if (b >= a.ntiles) return;
    if (a.tile_list) b = a.tile_list[b];
    const TileHdrK h = a.hdr[b];
    constexpr bool nt = NT;   // access policy of the launch (ldp, st1, st2)
    // step constants: the member's table row (batches) or the launch's own copy,
    // moved word by word so that both sources stay in scalar registers
    StepC c;
    {
        constexpr int NWD = sizeof(StepC) / 4;
        static_assert(sizeof(StepC) % 4 == 0, "StepC size");
        uint32_t wd[NWD];
        const uint32_t *kw = reinterpret_cast<const uint32_t *>(&a.c0);
        if (a.mem) {
            const uint32_t *gw = reinterpret_cast<const uint32_t *>(a.mem + h.member);
#pragma unroll
            for (int q = 0; q < NWD; ++q) wd[q] = gw[q];
        } else {
#pragma unroll
            for (int q = 0; q < NWD; ++q) wd[q] = kw[q];
        }
        __builtin_memcpy(&c, wd, sizeof(StepC));
    }
    const int K = a.K, KS = a.ksub;   // rings per tile, substeps per launch
    const int ch = a.chunk - c.chunk0;   // this member's chunk index
    if (ch < 0) return;
    const int m0 = ch * KS;
    if (m0 >= c.nsub) return;
    const bool even = (ch & 1) == 0;
    const int cnt = min(KS, c.nsub - m0);
    const int rings = VI ? 2 * cnt : cnt;   // rings this launch needs
    const bool first = m0 == 0, last = m0 + cnt == c.nsub;
    const bool track = (c.flags & KF_TRACK_VOLUME) != 0;
    const bool linear_h = (c.flags & KF_LINEAR_H) != 0;
    const bool hasW = a.W != nullptr;
    const int *nV = a.nV + b * (K + 1);   // level counts of the tile (uniform loads)
    const int *nE = a.nE + b * (K + 1);
    const int nv_load = nV[rings], ne_load = nE[rings], nvu = nV[rings - 1 - (VI ? 1 : 0)];
    const int tid = threadIdx.x;

    // LDS carve-up: the vertex arrays filled by direct-to-LDS loads come first
    int off = 0;
    T *sEta = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nv);
    T *sE1 = nullptr, *sE2 = nullptr, *sEA = nullptr;   // SM: eta^{-1}, eta^{-2}, eta_am
    if constexpr (SM) {
        sE1 = reinterpret_cast<T *>(smem + off);
        off = align16(off + (int)sizeof(T) * a.cap_nv);
        sE2 = reinterpret_cast<T *>(smem + off);
        off = align16(off + (int)sizeof(T) * a.cap_nv);
        sEA = reinterpret_cast<T *>(smem + off);
        off = align16(off + (int)sizeof(T) * a.cap_nv);
    }
    T *sH = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nv);
    T *sAv = reinterpret_cast<T *>(smem + off);   // 1 / A_v
    off = align16(off + (int)sizeof(T) * a.cap_nvu);
    T *sW = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nvu);
    double *red = reinterpret_cast<double *>(smem + off);
    off = align16(off + 8 * NW * 9);
    int *sLev = reinterpret_cast<int *>(smem + off);   // level counts: V_0..V_8, E_0..E_8
    off = align16(off + 4 * 18);
    T *sAcc = reinterpret_cast<T *>(smem + off);   // sub-cell fluxes in local CSR order
    off = align16(off + (int)sizeof(T) * a.cap_cs);
    uint16_t *sRow = reinterpret_cast<uint16_t *>(smem + off);
    // VI: u = U / H_e per local triangle (after the row offsets), then the triangles'
    // local edge-neighbour ids (three 16-bit ids in a uint2)
    const int ub_off = align16(off + 2 * (a.cap_nvu + 4));
    T *sUb = reinterpret_cast<T *>(smem + ub_off);
    uint2 *sNb = reinterpret_cast<uint2 *>(smem + align16(ub_off + 2 * (int)sizeof(T) * a.cap_ne));

    // ---- load phase in two rounds of independent loads: (A) index and static data
    // (local vertex ids, triangle records, geometry, row offsets, running sums), one
    // wait, then (B) the gathers through those indices, one wait before the barrier.
    // FP32 vertex gathers go straight to LDS (global_load_lds, the LDS address from
    // M0), FP64 ones through registers.
    constexpr bool dma = F32;
    // inputs: SE ping-pongs (caller's arrays, workspace); SM reads the caller's
    // arrays at the member's first chunk, else the set the previous chunk wrote
    const int rs = (ch - 1) & 1;
    const bool pend = SM && ch > 0;   // SM: transport update of the previous substep pending
    const T *eta_in = static_cast<const T *>(
        SM ? (ch == 0 ? a.eta_u : a.sm_v[rs][0]) : (even ? a.eta_u : a.eta_w));
    const T *e1_in = SM ? static_cast<const T *>(ch == 0 ? a.eta_u : a.sm_v[rs][1]) : nullptr;
    const T *e2_in = SM ? static_cast<const T *>(ch == 0 ? a.eta_u : a.sm_v[rs][2]) : nullptr;
    const T *eA_in = SM ? static_cast<const T *>(a.sm_v[rs][3]) : nullptr;
    const T *H0 = static_cast<const T *>(a.H0);
    const T *Wt = static_cast<const T *>(a.W);
    const T *lav = static_cast<const T *>(a.lv_av) + h.lv_off;   // 1 / A_v
    const int32_t *lv = a.lv_gid + h.lv_off;
    // vertex slots per thread staged in the rounds (the rest, for large tiles on
    // small workgroups, in a loop afterwards)
    constexpr int VS = F32 ? (BLOCK >= 512 ? 3072 / BLOCK : 8) : 2;
    int gv[VS];
#pragma unroll
    for (int u = 0; u < VS; ++u) gv[u] = lv[min(tid + u * BLOCK, nv_load - 1)];

    const uint4 *lrec = reinterpret_cast<const uint4 *>(a.le_rec) + h.le_off;
    const T *lgeo = static_cast<const T *>(a.lgeo) + 4 * (int64_t)h.le_off;
    const T *lae = static_cast<const T *>(a.lae) + h.le_off;
    const T2 *Uin = static_cast<const T2 *>(
        SM ? (ch == 0 ? a.U_u : a.sm_e[rs][0]) : (even ? a.U_u : a.U_w));
    const T2 *U1in = SM ? static_cast<const T2 *>(ch == 0 ? a.U_u : a.sm_e[rs][1]) : nullptr;
    const T2 *UAin = SM ? static_cast<const T2 *>(a.sm_e[rs][2]) : nullptr;
    const T2 *Rg = static_cast<const T2 *>(a.R);
    const T *fg = static_cast<const T *>(a.f);
    const T dts = cdts<T>(c);
    T rUx[EPT], rUy[EPT], rRx[EPT], rRy[EPT], rf[EPT], rk[EPT], g0[EPT], g1[EPT], g2[EPT],
        g3[EPT], g4[EPT];
    // SM: U^{-1} and the AB3 transport of the previous substep
    T pUx[SM ? EPT : 1], pUy[SM ? EPT : 1], aUx[SM ? EPT : 1], aUy[SM ? EPT : 1];
    // local vertices and flux positions, 16 bits each (slots past the tile's triangles
    // hold copies of its last triangle's)
    uint32_t t0[EPT] = {}, t1[EPT] = {}, t2[EPT] = {};
    int gt[EPT];
    // running sums only in the slots that can hold owned triangles (the plan keeps
    // every tile's owned triangles within them); osl(r) names slot r's sum
    constexpr int OS = own_slots(EPT);
    SumT<F32> sm[OS];
    auto osl = [](int r) { return r < OS ? r : 0; };
    // VI: the edge geometry of the first HV slots held in registers for the whole launch
    // (the other slots read it from memory at every substep).  Measured on the lat-lon
    // workload: faster with FP32 and up to three triangles per thread in 256- and
    // 512-thread workgroups (the same register tier), slower elsewhere
    constexpr int HV = (VI && F32 && BLOCK <= 512 && EPT <= 3) ? EPT : 0;
    T vgh[HV > 0 ? 6 * HV : 1];
    if (ne_load > 0) {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int lc = min(tid + r * BLOCK, ne_load - 1);
            const uint4 rec = ldp<nt>(lrec + lc);
            gt[r] = (int)rec.x;
            t0[r] = rec.y;
            t1[r] = rec.z;
            t2[r] = rec.w;
            if constexpr (F32) {
                const float4 gg = ldp<nt>(reinterpret_cast<const float4 *>(lgeo) + lc);
                g0[r] = gg.x;
                g1[r] = gg.y;
                g2[r] = gg.z;
                g3[r] = gg.w;
            } else {
                const double2 ga = ldp<nt>(reinterpret_cast<const double2 *>(lgeo) + 2 * lc);
                const double2 gb = ldp<nt>(reinterpret_cast<const double2 *>(lgeo) + 2 * lc + 1);
                g0[r] = ga.x;
                g1[r] = ga.y;
                g2[r] = gb.x;
                g3[r] = gb.y;
            }
            g4[r] = ldp<nt>(lae + lc);
        }
        if constexpr (HV > 0) {
#pragma unroll
            for (int r = 0; r < HV; ++r) {
                const int lc = min(tid + r * BLOCK, ne_load - 1);
                const T *vg = static_cast<const T *>(a.vgeo) + 6 * (int64_t)(h.le_off + lc);
#pragma unroll
                for (int q = 0; q < 6; ++q) vgh[6 * r + q] = ldp<nt>(vg + q);
            }
        }
        if (!first && h.nown > 0) {
            // running sums of owned triangles (the tile's contiguous global range)
#pragma unroll
            for (int r = 0; r < OS; ++r) sm[r].load(a.sum, h.ebase + min(tid + r * BLOCK, h.nown - 1));
        }
    }
    // FP64 dual-cell areas of owned vertices, for the volume sums of this launch
    constexpr int VO = 2;   // owned-vertex slots held in registers
    const bool need_vol = first || track || last;
    double rAv64[VO];
    if (need_vol) {
#pragma unroll
        for (int k = 0; k < VO; ++k) {
            const double *pa = a.Av64 + h.vbase + min(tid + k * BLOCK, h.nv0 - 1);
            rAv64[k] = F32 ? *pa : ldp<nt>(pa);
        }
    }
    // level counts for the substep loop
    const int lev_cnt = tid <= K ? nV[tid] : 0;
    const int lev_cnt_e = tid <= K ? nE[tid] : 0;
    // local CSR row offsets (chunks padded to multiples of 4 entries)
    const uint2 *crow = reinterpret_cast<const uint2 *>(a.cs_row + h.rw_off);
    const int nrow4 = (nvu + 1 + 3) >> 2;
    const uint2 row0 = F32 ? crow[min(tid, nrow4 - 1)] : ldp<nt>(crow + min(tid, nrow4 - 1));
    __builtin_amdgcn_s_waitcnt(0);   // round A complete

    auto stage_vertex = [&](int i, int g) {   // register path
        const T ve = eta_in[g], vh = H0[g];
        const T va = i < nvu ? ldp<nt>(lav + i) : T(0);
        const T vw = (i < nvu && hasW) ? Wt[g] : T(0);
        if constexpr (SM) {
            const T v1 = e1_in[g], v2 = e2_in[g];
            const T vA = pend ? eA_in[g] : T(0);
            sE1[i] = v1;
            sE2[i] = v2;
            sEA[i] = vA;
        }
        sEta[i] = ve;
        sH[i] = vh;
        if (i < nvu) {
            sAv[i] = va;
            sW[i] = vw;
        }
    };
    auto dma_vertex = [&](int i, int g) {   // lane l of the wave writes LDS element i0 + l
        const int i0 = i - (tid & 63);
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(eta_in + g),
                                         (__attribute__((address_space(3))) void *)(sEta + i0), 4, 0, 0);
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(H0 + g),
                                         (__attribute__((address_space(3))) void *)(sH + i0), 4, 0, 0);
        if constexpr (SM) {
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(e1_in + g),
                                             (__attribute__((address_space(3))) void *)(sE1 + i0), 4, 0, 0);
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(e2_in + g),
                                             (__attribute__((address_space(3))) void *)(sE2 + i0), 4, 0, 0);
            if (pend)
                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(eA_in + g),
                                                 (__attribute__((address_space(3))) void *)(sEA + i0), 4, 0, 0);
        }
        if (i < nvu) {
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(lav + i),
                                             (__attribute__((address_space(3))) void *)(sAv + i0), 4, 0, 0);
            if (hasW)
                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(Wt + g),
                                                 (__attribute__((address_space(3))) void *)(sW + i0), 4, 0, 0);
            else
                sW[i] = T(0);
        }
    };
    // round B
    if constexpr (F32) {
        if (dma) {
#pragma unroll
            for (int u = 0; u < VS; ++u) {
                const int i = tid + u * BLOCK;
                if (i < nv_load) dma_vertex(i, gv[u]);
            }
        }
    }
    if (ne_load > 0) {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int g = gt[r];
            const T2 u = Uin[g];
            rUx[r] = u.x;
            rUy[r] = u.y;
            const T2 rr = Rg[g];
            rRx[r] = rr.x;
            rRy[r] = rr.y;
            rf[r] = fg[g];
            if constexpr (SM) {
                const T2 u1 = U1in[g];
                pUx[r] = u1.x;
                pUy[r] = u1.y;
                if (pend) {
                    const T2 ua = UAin[g];
                    aUx[r] = ua.x;
                    aUy[r] = ua.y;
                } else {
                    aUx[r] = T(0);
                    aUy[r] = T(0);
                }
            }
        }
    }
    {
        uint2 *srow2 = reinterpret_cast<uint2 *>(sRow);
        if (tid < nrow4) srow2[tid] = row0;
        if (tid <= K) {
            sLev[tid] = lev_cnt;
            sLev[9 + tid] = lev_cnt_e;
        }
    }
    if (!dma) {
#pragma unroll
        for (int u = 0; u < VS; ++u) {
            const int i = tid + u * BLOCK;
            if (i < nv_load) stage_vertex(i, gv[u]);
        }
    }
    // remainders: vertices beyond the staged slots, rows beyond the first chunk
    for (int i = tid + VS * BLOCK; i < nv_load; i += BLOCK) {
        if constexpr (F32) {
            if (dma) {
                dma_vertex(i, lv[i]);
                continue;
            }
        }
        stage_vertex(i, lv[i]);
    }
    for (int i = tid + BLOCK; i < nrow4; i += BLOCK) reinterpret_cast<uint2 *>(sRow)[i] = ldp<nt>(crow + i);
    if constexpr (VI) {
        const uint2 *nbt = reinterpret_cast<const uint2 *>(a.vnb) + h.le_off;
        for (int i = tid; i < ne_load; i += BLOCK) sNb[i] = ldp<nt>(nbt + i);
    }
    if (a.ell) {
        // fixed-width rows: the entries past a vertex's triangles are never written
        // and must read as zero (adding +0 leaves every row sum unchanged)
        const int nz = (kEllWidth * nvu * (int)sizeof(T) + 15) / 16;
        for (int i = tid; i < nz; i += BLOCK) reinterpret_cast<uint4 *>(sAcc)[i] = make_uint4(0, 0, 0, 0);
    }
    if (first && !SM) {
#pragma unroll
        for (int r = 0; r < OS; ++r) {
            const int le = tid + r * BLOCK;
            if (le < h.nown) {
                T2 u;
                u.x = rUx[r];
                u.y = rUy[r];
                st2<nt, T>(a.U0c, h.ebase + le, u.x, u.y);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // round B complete (direct-to-LDS loads included)
    __syncthreads();
    if constexpr (F32) {
        // FP32: per-triangle constants of the launch (see tri_update_f32)
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int le = tid + r * BLOCK;
            if (le < ne_load) {
                if constexpr (SM) {
                    rf[r] = rf[r] * dts;   // f dt
                } else {
                    float al, kk;
                    tri_consts_f32(rf[r], dts, al, kk);
                    rk[r] = kk;
                    rf[r] = al;
                }
                if constexpr (!VI) {   // VI: R + V, scaled at every substep
                    rRx[r] = dts * rRx[r];
                    rRy[r] = dts * rRy[r];
                }
                g4[r] = -g4[r];
            }
        }
    } else if constexpr (!SM) {
        // FP64 forward-backward: a = f dt_s / 2 of the launch in place of f
#pragma unroll
        for (int r = 0; r < EPT; ++r) rf[r] = T(0.5) * rf[r] * dts;
    }
    T rH[F32 ? EPT : 1];
    if constexpr (F32) {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int le = tid + r * BLOCK;
            if (le < ne_load) {
                const int ia = t0[r] & 0xffffu, ib = t0[r] >> 16, ic = t1[r] & 0xffffu;
                rH[r] = (sH[ia] + sH[ib] + sH[ic]) * (1.0f / 3.0f) + (linear_h ? 0.0f : c.eta_ref_f);
            }
        }
    }

    double v0 = 0.0;
    if (first) {
#pragma unroll
        for (int k = 0; k < VO; ++k) {
            const int i = tid + k * BLOCK;
            if (i < h.nv0) v0 += rAv64[k] * (double)sEta[i];
        }
        for (int i = tid + VO * BLOCK; i < h.nv0; i += BLOCK) v0 += a.Av64[h.vbase + i] * (double)sEta[i];
    }
    bool dry_any = false, bad_any = false;
    const T gd = cg<T>(c) * dts, th = cth<T>(c);
    const float eref = F32 ? c.eta_ref_f : 0.0f;
    for (int j = 0; j < cnt; ++j) {
        // levels: triangles updated through ring lev, vertices through lev - 1; VI also
        // needs the velocities of ring lev + 1
        const int lev = VI ? 2 * (cnt - j) - 1 : cnt - j;
        const int ne_act = sLev[9 + lev], nv_act = sLev[lev - 1];
        // VI: the thread index, the packed local indices and the geometry pass through an
        // empty asm once per substep, so addresses, indices and values derived from them
        // are recomputed instead of held in registers for every triangle across the loop
        int tidv = tid;
        if constexpr (VI) {
            asm volatile("" : "+v"(tidv));
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                asm volatile("" : "+v"(t0[r]), "+v"(t1[r]), "+v"(t2[r]));
                asm volatile("" : "+v"(g0[r]), "+v"(g1[r]), "+v"(g2[r]), "+v"(g3[r]), "+v"(g4[r]));
            }
        }
        // FP64 forward-backward: likewise the packed indices and the geometry (the FP64
        // values derived from them would otherwise double the registers held per
        // triangle; three triangles per thread then fit two 512-thread tiles per CU)
        if constexpr (!F32 && FB) {
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                asm volatile("" : "+v"(t0[r]), "+v"(t1[r]), "+v"(t2[r]));
                asm volatile("" : "+v"(g0[r]), "+v"(g1[r]), "+v"(g2[r]), "+v"(g3[r]), "+v"(g4[r]));
            }
        }
        // FP32 forward-backward: the three elevations of every slot read before any
        // update, so that all slots wait for one LDS round trip
        float hE[(F32 && FB) ? 3 * EPT : 1];
        if constexpr (F32 && FB) {
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                hE[3 * r] = sEta[t0[r] & 0xffffu];
                hE[3 * r + 1] = sEta[t0[r] >> 16];
                hE[3 * r + 2] = sEta[t1[r] & 0xffffu];
            }
        }
        if constexpr (VI) {
            const int ne_u = sLev[9 + lev + 1];
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                const int le = tid + r * BLOCK;
                if (le < ne_u) {
                    const int ia = t0[r] & 0xffffu, ib = t0[r] >> 16, ic = t1[r] & 0xffffu;
                    const T He = visc_tri_depth<T, F32>(linear_h, eref, sH[ia], sH[ib], sH[ic],
                                                        sEta[ia], sEta[ib], sEta[ic]);
                    sUb[2 * le] = rUx[r] / He;
                    sUb[2 * le + 1] = rUy[r] / He;
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int le = tid + r * BLOCK;
            if (le < ne_act) {
                const int ia = t0[r] & 0xffffu, ib = t0[r] >> 16, ic = t1[r] & 0xffffu;
                if constexpr (SM) {
                    // pending transport update of the previous substep, then U_ab
                    T Px = rUx[r], Py = rUy[r], Qx = pUx[r], Qy = pUy[r], abx, aby;
                    if (pend || j > 0) {
                        T Unx, Uny;
                        bool dry;
                        const T eAa = sEA[ia], eAb = sEA[ib], eAc = sEA[ic];
                        if constexpr (F32)
                            sesm_u_f32(linear_h, eAa, eAb, eAc, rH[r], g0[r], g1[r], g2[r], g3[r],
                                       rf[r], rRx[r], rRy[r], gd, Px, Py, aUx[r], aUy[r], Unx,
                                       Uny, dry);
                        else
                            sesm_u_f64(c, linear_h, eAa, eAb, eAc, sH[ia], sH[ib], sH[ic], g0[r],
                                       g1[r], g2[r], g3[r], rf[r], rRx[r], rRy[r], Px, Py,
                                       aUx[r], aUy[r], Unx, Uny, dry);
                        dry_any |= dry;
                        abx = sesm_ab<T>(c, Unx, Px, Qx);
                        aby = sesm_ab<T>(c, Uny, Py, Qy);
                        Qx = Px;
                        Qy = Py;
                        Px = Unx;
                        Py = Uny;
                    } else {   // first substep: the histories equal U^0
                        abx = sesm_ab<T>(c, Px, Qx, Qx);
                        aby = sesm_ab<T>(c, Py, Qy, Qy);
                    }
                    T pa, pb, pc;
                    if constexpr (F32)
                        slot_fluxes_f32(abx, aby, g0[r], g1[r], g2[r], g3[r], g4[r], pa, pb, pc);
                    else
                        slot_fluxes(abx, aby, g0[r], g1[r], g2[r], g3[r], g4[r], pa, pb, pc);
                    sAcc[t1[r] >> 16] = pa;
                    sAcc[t2[r] & 0xffffu] = pb;
                    sAcc[t2[r] >> 16] = pc;
                    rUx[r] = Px;
                    rUy[r] = Py;
                    pUx[r] = Qx;
                    pUy[r] = Qy;
                    aUx[r] = abx;
                    aUy[r] = aby;
                    if (r < OS && le < h.nown) {
                        if (first && j == 0)
                            sm[osl(r)].init(abx, aby);
                        else
                            sm[osl(r)].add(abx, aby);
                    }
                    continue;
                }
                T Unx, Uny, pa, pb, pc;
                T rx = rRx[r], ry = rRy[r];
                if constexpr (VI) {
                    // V(eta^m, U^m): edges to local neighbours (0xffff: coast)
                    const uint2 nbp = sNb[le];
                    const int lq = h.le_off + tidv + r * BLOCK;   // = h.le_off + le
                    const T *vg = r < HV ? vgh + 6 * (r < HV ? r : 0)
                                         : static_cast<const T *>(a.vgeo) + 6 * (int64_t)lq;
                    const int nbs[3] = {static_cast<int>(nbp.x & 0xffffu),
                                        static_cast<int>(nbp.x >> 16),
                                        static_cast<int>(nbp.y & 0xffffu)};
                    const int iv[3] = {ia, ib, ic};
                    const T uex = sUb[2 * le], uey = sUb[2 * le + 1];
                    const T A0 = static_cast<T>(a.vA0), Cv = static_cast<T>(a.vCv);
                    T Hv[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        Hv[k] = visc_vtx_depth<T, F32>(linear_h, eref, sH[iv[k]], sEta[iv[k]]);
                    T sx = 0, sy = 0;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const int n = nbs[q];
                        if (n == 0xffff) continue;
                        visc_edge<T>(A0, Cv, static_cast<T>(0.5) * (Hv[q] + Hv[(q + 1) % 3]),
                                     vg[2 * q], vg[2 * q + 1], sUb[2 * n] - uex,
                                     sUb[2 * n + 1] - uey, sx, sy);
                    }
                    const T Ae = F32 ? -g4[r] : g4[r];
                    rx = rRx[r] + sx / Ae;
                    ry = rRy[r] + sy / Ae;
                    if constexpr (F32) {
                        rx = dts * rx;
                        ry = dts * ry;
                    }
                }
                if constexpr (F32) {
                    bool dry;
                    const float ea = FB ? hE[FB ? 3 * r : 0] : sEta[ia];
                    const float eb = FB ? hE[FB ? 3 * r + 1 : 0] : sEta[ib];
                    const float ec = FB ? hE[FB ? 3 * r + 2 : 0] : sEta[ic];
                    tri_update_f32(ea, eb, ec, rH[r], g0[r], g1[r], g2[r],
                                   g3[r], g4[r], rUx[r], rUy[r], rx, ry, rf[r], rk[r],
                                   gd, th, linear_h, Unx, Uny, pa, pb, pc, dry);
                    dry_any |= dry;
                } else {
                    bool dry;
                    tri_update<T, F32>(sEta[ia], sEta[ib], sEta[ic], sH[ia], sH[ib], sH[ic],
                                       g0[r], g1[r], g2[r], g3[r], g4[r], rUx[r], rUy[r],
                                       rx, ry, rf[r], c, linear_h, Unx, Uny, pa, pb,
                                       pc, dry);
                    dry_any |= dry;
                }
                sAcc[t1[r] >> 16] = pa;
                sAcc[t2[r] & 0xffffu] = pb;
                sAcc[t2[r] >> 16] = pc;
                rUx[r] = Unx;
                rUy[r] = Uny;
                if (r < OS && le < h.nown) {
                    if (first && j == 0)
                        sm[osl(r)].init(Unx, Uny);
                    else
                        sm[osl(r)].add(Unx, Uny);
                }
            }
        }
        __syncthreads();
        // vertex phase.  The update of vertex i from its row sum acc (and its elevation,
        // area term and W read beforehand)
        auto finish = [&](int i, T acc, T e_i, T av_i, T w_i) -> T {
            T en;
            if constexpr (F32)
                en = vtx_update_f32(e_i, acc, av_i, w_i, dts);
            else
                en = e_i - dts * (acc * av_i + w_i);
            if constexpr (SM) {
                const T e1 = sE1[i], e2 = sE2[i];
                sEA[i] = sesm_am<T>(c, en, e_i, e1, e2);
                sE2[i] = e1;
                sE1[i] = e_i;
            }
            sEta[i] = en;
            bad_any |= !finite_val(en);
            return en;
        };
        // fixed-width rows: the row's entries in ascending triangle order, then zeros
        auto ell_sum = [&](int i) -> T {
            const T *row = sAcc + kEllWidth * i;
            T b[kEllWidth];
#pragma unroll
            for (int q = 0; q < kEllWidth; ++q) b[q] = row[q];
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < kEllWidth; ++q) acc += b[q];
            return acc;
        };
        // local CSR rows: row sums in entry order, loads issued four (or the last up to
        // three) at a time; reads past a row end stay inside the flux array (its 64
        // scratch slots) and are not summed
        auto csr_sum = [&](int i) -> T {
            T acc = T(0);
            int q = sRow[i];
            const int q1 = sRow[i + 1];
            for (; q + 4 <= q1; q += 4) {
                const T b0 = sAcc[q], b1 = sAcc[q + 1], b2 = sAcc[q + 2], b3 = sAcc[q + 3];
                acc += b0;
                acc += b1;
                acc += b2;
                acc += b3;
            }
            const int rem = q1 - q;
            const T b0 = sAcc[q], b1 = sAcc[q + 1], b2 = sAcc[q + 2];
            if (rem > 0) acc += b0;
            if (rem > 1) acc += b1;
            if (rem > 2) acc += b2;
            return acc;
        };
        auto vertex = [&](int i) -> T {
            const T acc = a.ell ? ell_sum(i) : csr_sum(i);
            return finish(i, acc, sEta[i], sAv[i], sW[i]);
        };
        const bool vol_j = track || (last && j == cnt - 1);
        // adjoint recompute: the owned vertices' elevation after member substep
        // m0 + j + 1 to the trajectory (all but the final state)
        T *trj = nullptr;
        if (TR && m0 + j + 1 < c.nsub)
            trj = static_cast<T *>(a.traj) + (int64_t)(m0 + j + 1) * a.traj_stride + h.vbase;
        double vp = 0.0;
        if (F32 && a.ell) {
            // every read of the thread's vertex slots issued before any update (slots
            // past nv_act read a valid row and are not updated)
            T vacc[VO], ve[VO], vav[VO], vw[VO];
#pragma unroll
            for (int k = 0; k < VO; ++k) {
                const int i = min(tid + k * BLOCK, max(nv_act - 1, 0));
                vacc[k] = ell_sum(i);
                ve[k] = sEta[i];
                vav[k] = sAv[i];
                vw[k] = sW[i];
            }
#pragma unroll
            for (int k = 0; k < VO; ++k) {
                const int i = tid + k * BLOCK;
                if (i < nv_act) {
                    const T en = finish(i, vacc[k], ve[k], vav[k], vw[k]);
                    if (vol_j && i < h.nv0) vp += rAv64[k] * (double)en;
                    if (TR && trj && i < h.nv0) trj[i] = en;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < VO; ++k) {
                const int i = tid + k * BLOCK;
                if (i < nv_act) {
                    const T en = vertex(i);
                    if (vol_j && i < h.nv0) vp += rAv64[k] * (double)en;
                    if (TR && trj && i < h.nv0) trj[i] = en;
                }
            }
        }
        for (int i = tid + VO * BLOCK; i < nv_act; i += BLOCK) {
            const T en = vertex(i);
            if (vol_j && i < h.nv0) vp += a.Av64[h.vbase + i] * (double)en;
            if (TR && trj && i < h.nv0) trj[i] = en;
        }
        if (vol_j) {   // by DPP: no LDS round trips before the barrier
            vp = wave_sum_last(vp);
            if ((tid & 63) == 63) red[j * NW + (tid >> 6)] = vp;
        }
        __syncthreads();
    }
    if (dry_any) set_fault(a.faults, 1u);
    if (bad_any) set_fault(a.faults, 2u);

    // write back owned vertices and triangles
    if constexpr (SM) {
        const int wsel = ch & 1;
        T *o0 = static_cast<T *>(a.sm_v[wsel][0]) + h.vbase;
        T *o1 = static_cast<T *>(a.sm_v[wsel][1]) + h.vbase;
        T *o2 = static_cast<T *>(a.sm_v[wsel][2]) + h.vbase;
        T *o3 = static_cast<T *>(a.sm_v[wsel][3]) + h.vbase;
        for (int i = tid; i < h.nv0; i += BLOCK) {
            st1<nt>(sEta[i], o0 + i);
            st1<nt>(sE1[i], o1 + i);
            st1<nt>(sE2[i], o2 + i);
            st1<nt>(sEA[i], o3 + i);
        }
        T2 *u0 = static_cast<T2 *>(a.sm_e[wsel][0]);
        T2 *u1 = static_cast<T2 *>(a.sm_e[wsel][1]);
        T2 *u2 = static_cast<T2 *>(a.sm_e[wsel][2]);
#pragma unroll
        for (int r = 0; r < OS; ++r) {   // owned triangles lie in the first OS slots
            const int le = tid + r * BLOCK;
            if (le < h.nown) {
                const int g = h.ebase + le;
                st2<nt, T>(u0, g, rUx[r], rUy[r]);
                st2<nt, T>(u1, g, pUx[r], pUy[r]);
                st2<nt, T>(u2, g, aUx[r], aUy[r]);
                if (last) {
                    if (a.Uavg) {
                        st2<nt, double>(a.Uavg, g, sm[r].vx() / c.Mdbl, sm[r].vy() / c.Mdbl);
                    }
                } else {
                    sm[r].template store<nt>(a.sum, g);
                }
            }
        }
    } else {
    T *eta_out = static_cast<T *>(even ? a.eta_w : a.eta_u);
    for (int i = tid; i < h.nv0; i += BLOCK) st1<nt>(sEta[i], eta_out + h.vbase + i);
    T2 *Uout = static_cast<T2 *>(even ? a.U_w : a.U_u);
#pragma unroll
    for (int r = 0; r < OS; ++r) {   // owned triangles lie in the first OS slots
        const int le = tid + r * BLOCK;
        if (le < h.nown) {
            const int g = h.ebase + le;
            T2 u;
            u.x = rUx[r];
            u.y = rUy[r];
            st2<nt, T>(Uout, g, u.x, u.y);
            if (last) {
                if (!a.Uavg) continue;
                const T2 u0 = ldp<nt>(static_cast<const T2 *>(a.U0c) + g);
                st2<nt, double>(a.Uavg, g, sm[r].vx() / c.Mdbl + c.thM * ((double)u.x - (double)u0.x),
                               sm[r].vy() / c.Mdbl + c.thM * ((double)u.y - (double)u0.y));
            } else {
                sm[r].template store<nt>(a.sum, g);
            }
        }
    }
    }
    // volume partials of this tile
    if (first) {
        v0 = wave_sum_last(v0);
        if ((tid & 63) == 63) red[8 * NW + (tid >> 6)] = v0;
    }
    __syncthreads();
    if (tid == 0) {
        double *vp = a.vol_part + c.vol_off;
        if (first) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += red[8 * NW + w];
            vp[h.mtile] = s;
        }
        for (int j = 0; j < cnt; ++j) {
            const bool keep = track || (last && j == cnt - 1);
            if (!keep) continue;
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += red[j * NW + w];
            const int64_t row = track ? (m0 + j + 1) : 1;
            vp[row * c.ntiles + h.mtile] = s;
        }
    }
}

template <typename T, bool F32, int EPT, int BLOCK, int MODE, bool NT>
__global__ void __launch_bounds__(BLOCK) k_tile(TileArgs a) {
    tile_body<T, F32, EPT, BLOCK, MODE, NT>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Adjoint of one substep (reverse of the triangle and vertex phases)
// ---------------------------------------------------------------------------
// Reverse triangle phase for triangle e (any e; out of range returns).
template <typename T, bool F32>
__device__ __forceinline__ void adj_tri_at(const AdjArgs &a, int64_t e) {
    using T2 = typename Vec2<T>::type;
    if (e >= a.ne) return;
    const StepC &c = a.c;
    const T dts = cdts<T>(c), g = cg<T>(c), th = cth<T>(c), opt = copt<T>(c);
    const T *geom = static_cast<const T *>(a.geom);
    const T gbx = geom[e], gby = geom[a.ne + e], gcx = geom[2 * a.ne + e],
            gcy = geom[3 * a.ne + e], Ae = geom[4 * a.ne + e];
    const T gax = -(gbx + gcx), gay = -(gby + gcy);
    const int32_t v0 = a.tri[3 * e], v1 = a.tri[3 * e + 1], v2 = a.tri[3 * e + 2];
    const T *le = static_cast<const T *>(a.lam_eta);
    const T *Av = static_cast<const T *>(a.Av);
    // lambda_F = -dt_s sum_k (lambda_eta_k / A_k) S_k,  S_k = -A_e grad N_k; the
    // adjoint multiplies by reciprocals (1 / A_k, 1 / (1 + a^2), 1 / 3) where the
    // forward divides: the gradients agree with the CPU adjoint to rounding, and the
    // per-substep and tile kernels evaluate the same operations
    T lFx = T(0), lFy = T(0);
    {
        const T w0 = -dts * le[v0] * (T(1) / Av[v0]);
        lFx += w0 * (-Ae * gax);
        lFy += w0 * (-Ae * gay);
        const T w1 = -dts * le[v1] * (T(1) / Av[v1]);
        lFx += w1 * (-Ae * gbx);
        lFy += w1 * (-Ae * gby);
        const T w2 = -dts * le[v2] * (T(1) / Av[v2]);
        lFx += w2 * (-Ae * gcx);
        lFy += w2 * (-Ae * gcy);
    }
    T2 *lU = static_cast<T2 *>(a.lam_U);
    T2 lu = lU[e];
    if (a.lam_Uavg) {   // U^{m+1} enters the running sum with weight 1/M
        lu.x = lu.x + (T)(a.rM * a.lam_Uavg[2 * e]);
        lu.y = lu.y + (T)(a.rM * a.lam_Uavg[2 * e + 1]);
    }
    const T lUnx = lu.x + opt * lFx, lUny = lu.y + opt * lFy;
    T lUox = -th * lFx, lUoy = -th * lFy;
    // triangle quantities of the forward substep
    const T *eta = static_cast<const T *>(a.eta_m);
    const T *H0 = static_cast<const T *>(a.H0);
    const T ea = eta[v0], eb = eta[v1], ec = eta[v2];
    const T db = eb - ea, dc = ec - ea;
    const T gx = db * gbx + dc * gcx;
    const T gy = db * gby + dc * gcy;
    const T third = T(1) / T(3);
    T He;
    if (c.flags & KF_LINEAR_H) {
        He = (H0[v0] + H0[v1] + H0[v2]) * third;
    } else if (!F32) {
        He = ((H0[v0] + ea) + (H0[v1] + eb) + (H0[v2] + ec)) * third;
    } else {
        He = ((H0[v0] + H0[v1] + H0[v2]) + (ea + eb + ec)) * third + c.eta_ref_f;
    }
    const T al = T(0.5) * static_cast<const T *>(a.f)[e] * dts;
    const T rden = T(1) / (T(1) + al * al);
    // U' = C r with C = (I + aJ)^-1:  lambda_r = C^T lambda_U'
    const T lrx = (lUnx - al * lUny) * rden;
    const T lry = (lUny + al * lUnx) * rden;
    // r = (I - aJ) U + dt_s(-g H grad eta + R)
    lUox += lrx - al * lry;
    lUoy += lry + al * lrx;
    T2 *gR = static_cast<T2 *>(a.gR);
    T2 gr = gR[e];
    gr.x += dts * lrx;
    gr.y += dts * lry;
    gR[e] = gr;
    const T lgx = -dts * g * He * lrx, lgy = -dts * g * He * lry;
    const T lHe = -dts * g * (gx * lrx + gy * lry);
    T *psi = static_cast<T *>(a.psi) + 4 * e;
    psi[0] = gax * lgx + gay * lgy;
    psi[1] = gbx * lgx + gby * lgy;
    psi[2] = gcx * lgx + gcy * lgy;
    psi[3] = lHe * third;
    T2 lo;
    lo.x = lUox;
    lo.y = lUoy;
    lU[e] = lo;
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_adj_tri(AdjArgs a) {
    adj_tri_at<T, F32>(a, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// Reverse vertex phase for vertex v (any v; out of range returns).
template <typename T>
__device__ __forceinline__ void adj_vtx_at(const AdjArgs &a, int64_t v) {
    if (v >= a.nv) return;
    const bool nonlin = !(a.c.flags & KF_LINEAR_H);
    T *le = static_cast<T *>(a.lam_eta);
    T *gH0 = static_cast<T *>(a.gH0);
    const T *psi = static_cast<const T *>(a.psi);
    T acc = le[v];
    T gh = gH0[v];
    const int32_t j1 = a.row_ptr[v + 1];
    for (int32_t j = a.row_ptr[v]; j < j1; ++j) {
        const int32_t q = a.pcol[j];
        const int32_t e = q / 3, k = q - 3 * e;
        acc += psi[4 * e + k];
        const T chi = psi[4 * e + 3];
        if (nonlin) acc += chi;
        gh += chi;
    }
    le[v] = acc;
    gH0[v] = gh;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_vtx(AdjArgs a) {
    adj_vtx_at<T>(a, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
}

// A reverse substep of one checkpoint segment and an independent forward substep (state
// update only) of the recompute of the previous segment in one launch: blocks
// [0, nb_adj) run the reverse phase, the others the forward phase.  The two parts read
// and write disjoint arrays (the reverse reads the states of its own segment; the
// forward writes the other segment buffer, its fluxes and nothing the reverse touches),
// so their order inside the launch does not matter and each element's arithmetic is
// that of the separate kernels.
template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_pair_tri(AdjArgs aa, PlainArgs fa, int32_t nb_adj) {
    const int64_t b = blockIdx.x;
    if (b < nb_adj)
        adj_tri_at<T, F32>(aa, b * 256 + threadIdx.x);
    else
        plain_tri_at<T, F32>(fa, (b - nb_adj) * 256 + threadIdx.x);
}

template <typename T, bool F32>
__global__ void __launch_bounds__(256) k_pair_vtx(AdjArgs aa, PlainArgs fa, int32_t nb_adj) {
    const int64_t b = blockIdx.x;
    if (b < nb_adj) {
        adj_vtx_at<T>(aa, b * 256 + threadIdx.x);
    } else {
        const int64_t v = (b - nb_adj) * 256 + threadIdx.x;
        double vn, vo;
        if (v < fa.nv) plain_vtx_at<T, F32>(fa, v, vn, vo);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_init(AdjArgs a, const T *seed_eta, const T *seed_U) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < a.nv) {
        static_cast<T *>(a.lam_eta)[i] = seed_eta ? seed_eta[i] : T(0);
        static_cast<T *>(a.gH0)[i] = T(0);
    }
    if (i < 2 * a.ne) {
        T u = seed_U ? seed_U[i] : T(0);
        if (a.lam_Uavg) u = u + (T)(a.thrM * a.lam_Uavg[i]);
        static_cast<T *>(a.lam_U)[i] = u;
        static_cast<T *>(a.gR)[i] = T(0);
    }
}

// Endpoint term of the average for U^0, and the gradients with respect to the initial
// state written out (either output may be null).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_final(AdjArgs a, T *g_eta0, T *g_U0) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < 2 * a.ne) {
        T *lU = static_cast<T *>(a.lam_U);
        T u = lU[i];
        if (a.lam_Uavg) {
            u = u - (T)(a.thrM * a.lam_Uavg[i]);
            lU[i] = u;
        }
        if (g_U0) g_U0[i] = u;
    }
    if (i < a.nv && g_eta0) g_eta0[i] = static_cast<const T *>(a.lam_eta)[i];
}

// ---------------------------------------------------------------------------
// Reverse substeps on a tile plan
// ---------------------------------------------------------------------------
// cnt reverse substeps per launch on a tile and cnt rings of halo (the rings of the
// forward tile kernel: the reverse substep has the forward one's stencil, a triangle
// reading its three vertices and a vertex summing over its triangles), with the
// arithmetic of adj_tri_at / adj_vtx_at operation for operation, so the gradients equal
// those of the per-substep kernels bit for bit.  Inner step j runs the reverse of the
// forward substep of trajectory slot s_hi - 1 - j; triangles E_lev and vertices
// V_lev-1 are updated at level lev = cnt - j.  LDS holds the adjoint elevation, H0, A_v,
// the forward elevations of the launch's slots and the deposits (three slot terms and
// lambda_H / 3 per triangle, at the forward kernel's flux positions); registers hold
// the adjoint transport, the R gradient of owned triangles and the H0 gradient of owned
// vertices (the plan keeps a tile's owned vertices within two slots per thread).
template <typename T, bool F32, int EPT, int BLOCK>
__device__ __forceinline__ void adj_tile_body(const AdjTileArgs &a, int b, int G) {
    using T2 = typename Vec2<T>::type;
    constexpr int NVO = 2;   // owned-vertex slots per thread
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.xcd) {
        const int x = b & 7, q = b >> 3;
        const int base = G >> 3, rem = G & 7;
        b = x * base + (x < rem ? x : rem) + q;
    }
    if (b >= a.ntiles) return;
    const TileHdrK h = a.hdr[b];
    // ordinary accesses: the adjoint's workloads are small enough to stay cached from
    // launch to launch (non-temporal loads cost the 65k-vertex basin about 10%)
    constexpr bool nt = false;
    const StepC c = a.c;
    const int K = a.K, cnt = a.cnt;
    const int *nV = a.nV + b * (K + 1);
    const int *nE = a.nE + b * (K + 1);
    const int nv_load = nV[cnt], ne_load = nE[cnt], nvu = nV[cnt - 1];
    const int tid = threadIdx.x;
    const bool nonlin = !(c.flags & KF_LINEAR_H);
    const bool linear_h = !nonlin;

    int off = 0;
    T *sLe = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nv);
    T *sH = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nv);
    T *sAv = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_nv);
    T *sEm = reinterpret_cast<T *>(smem + off);   // [cnt][cap_nv] forward elevations
    off = align16(off + (int)sizeof(T) * a.cap_nv * cnt);
    int *sLev = reinterpret_cast<int *>(smem + off);   // V_0..V_8, E_0..E_8
    off = align16(off + 4 * 18);
    T *sPsi = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_cs);
    T *sChi = reinterpret_cast<T *>(smem + off);
    off = align16(off + (int)sizeof(T) * a.cap_cs);
    uint16_t *sRow = reinterpret_cast<uint16_t *>(smem + off);

    // ---- load phase: (A) contiguous per-tile data and owned gradients, (B) gathers
    const int32_t *lv = a.lv_gid + h.lv_off;
    const uint4 *lrec = reinterpret_cast<const uint4 *>(a.le_rec) + h.le_off;
    const T *lgeo = static_cast<const T *>(a.lgeo) + 4 * (int64_t)h.le_off;
    const T *lae = static_cast<const T *>(a.lae) + h.le_off;
    constexpr int OS = own_slots(EPT);
    // den: 1 / (1 + a^2)
    T g0[EPT], g1[EPT], g2[EPT], g3[EPT], g4[EPT], lUx[EPT], lUy[EPT], al[EPT], den[EPT];
    T sux[EPT], suy[EPT];
    T grx[OS], gry[OS];
    uint32_t t0[EPT] = {}, t1[EPT] = {}, t2[EPT] = {};
    int gt[EPT] = {};
    if (ne_load > 0) {
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int lc = min(tid + r * BLOCK, ne_load - 1);
            const uint4 rec = ldp<nt>(lrec + lc);
            gt[r] = (int)rec.x;
            t0[r] = rec.y;
            t1[r] = rec.z;
            t2[r] = rec.w;
            if constexpr (F32) {
                const float4 gg = ldp<nt>(reinterpret_cast<const float4 *>(lgeo) + lc);
                g0[r] = gg.x;
                g1[r] = gg.y;
                g2[r] = gg.z;
                g3[r] = gg.w;
            } else {
                const double2 ga = ldp<nt>(reinterpret_cast<const double2 *>(lgeo) + 2 * lc);
                const double2 gb = ldp<nt>(reinterpret_cast<const double2 *>(lgeo) + 2 * lc + 1);
                g0[r] = ga.x;
                g1[r] = ga.y;
                g2[r] = gb.x;
                g3[r] = gb.y;
            }
            g4[r] = ldp<nt>(lae + lc);
        }
    }
    const T2 *gRg = static_cast<const T2 *>(a.gR);
#pragma unroll
    for (int r = 0; r < OS; ++r) {
        grx[r] = T(0);
        gry[r] = T(0);
    }
    if (h.nown > 0 && !a.seed) {   // a tile may own no triangle (then ebase may equal ne)
#pragma unroll
        for (int r = 0; r < OS; ++r) {
            const T2 v = gRg[h.ebase + min(tid + r * BLOCK, h.nown - 1)];
            grx[r] = v.x;
            gry[r] = v.y;
        }
    }
    T gh[NVO];
    const T *gHg = static_cast<const T *>(a.gH0);
#pragma unroll
    for (int k = 0; k < NVO; ++k) gh[k] = a.seed ? T(0) : gHg[h.vbase + min(tid + k * BLOCK, h.nv0 - 1)];
    const uint2 *crow = reinterpret_cast<const uint2 *>(a.cs_row + h.rw_off);
    const int nrow4 = (nvu + 1 + 3) >> 2;
    const int lev_cnt = tid <= K ? nV[tid] : 0;
    const int lev_cnt_e = tid <= K ? nE[tid] : 0;
    __builtin_amdgcn_s_waitcnt(0);   // round A complete

    const T *lein = static_cast<const T *>(a.lam_eta_in);
    const T *H0g = static_cast<const T *>(a.H0);
    const T *Avg = static_cast<const T *>(a.Av);
    for (int i = tid; i < nv_load; i += BLOCK) {
        const int g = ldp<nt>(lv + i);
        sLe[i] = lein ? lein[g] : T(0);   // null only for a zero seed
        sH[i] = H0g[g];
        sAv[i] = T(1) / Avg[g];   // reciprocal area
        for (int j = 0; j < cnt; ++j) {
            const int sl = a.s_hi - 1 - j;
            const T *es = sl == 0 ? static_cast<const T *>(a.eta_s0)
                                  : static_cast<const T *>(a.traj) + (int64_t)sl * a.traj_stride;
            sEm[j * a.cap_nv + i] = es[g];
        }
    }
    const T dts = cdts<T>(c);
    if (ne_load > 0) {
        const T2 *lUin = static_cast<const T2 *>(a.lam_U_in);
        const T *fg = static_cast<const T *>(a.f);
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int g = gt[r];
            T2 u;
            if (lUin) {
                u = lUin[g];
            } else {   // zero seed
                u.x = T(0);
                u.y = T(0);
            }
            if (a.seed && a.lam_Uavg) {   // the endpoint term of <<U>> for U^M
                u.x = u.x + (T)(a.thrM * a.lam_Uavg[2 * (int64_t)g]);
                u.y = u.y + (T)(a.thrM * a.lam_Uavg[2 * (int64_t)g + 1]);
            }
            lUx[r] = u.x;
            lUy[r] = u.y;
            al[r] = T(0.5) * fg[g] * dts;
            den[r] = T(1) / (T(1) + al[r] * al[r]);   // reciprocal
            if (a.lam_Uavg) {   // U^{m+1} enters the running sum with weight 1/M
                sux[r] = (T)(a.rM * a.lam_Uavg[2 * (int64_t)g]);
                suy[r] = (T)(a.rM * a.lam_Uavg[2 * (int64_t)g + 1]);
            } else {
                sux[r] = T(0);
                suy[r] = T(0);
            }
        }
    }
    for (int i = tid; i < nrow4; i += BLOCK) reinterpret_cast<uint2 *>(sRow)[i] = ldp<nt>(crow + i);
    if (tid <= K) {
        sLev[tid] = lev_cnt;
        sLev[9 + tid] = lev_cnt_e;
    }
    if (a.ell) {   // fixed-width rows: unused entries read as zero
        const int nz = (kEllWidth * nvu * (int)sizeof(T) + 15) / 16;
        for (int i = tid; i < nz; i += BLOCK) {
            reinterpret_cast<uint4 *>(sPsi)[i] = make_uint4(0, 0, 0, 0);
            reinterpret_cast<uint4 *>(sChi)[i] = make_uint4(0, 0, 0, 0);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    const T g = cg<T>(c), th = cth<T>(c), opt = copt<T>(c);
    const bool seeded = a.lam_Uavg != nullptr;
    for (int j = 0; j < cnt; ++j) {
        const int lev = cnt - j;
        const int ne_act = sLev[9 + lev], nv_act = sLev[lev - 1];
        const T *em = sEm + j * a.cap_nv;
        // the packed indices and the geometry pass through an empty asm once per substep,
        // so that values derived from them are recomputed instead of held in registers
        // across the loop
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            asm volatile("" : "+v"(t0[r]), "+v"(t1[r]), "+v"(t2[r]));
            asm volatile("" : "+v"(g0[r]), "+v"(g1[r]), "+v"(g2[r]), "+v"(g3[r]), "+v"(g4[r]));
        }
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int le = tid + r * BLOCK;
            if (le >= ne_act) continue;
            const int ia = t0[r] & 0xffffu, ib = t0[r] >> 16, ic = t1[r] & 0xffffu;
            const T gbx = g0[r], gby = g1[r], gcx = g2[r], gcy = g3[r], Ae = g4[r];
            const T gax = -(gbx + gcx), gay = -(gby + gcy);
            // lambda_F = -dt_s sum_k (lambda_eta_k / A_k) S_k,  S_k = -A_e grad N_k
            T lFx = T(0), lFy = T(0);
            {
                const T w0 = -dts * sLe[ia] * sAv[ia];
                lFx += w0 * (-Ae * gax);
                lFy += w0 * (-Ae * gay);
                const T w1 = -dts * sLe[ib] * sAv[ib];
                lFx += w1 * (-Ae * gbx);
                lFy += w1 * (-Ae * gby);
                const T w2 = -dts * sLe[ic] * sAv[ic];
                lFx += w2 * (-Ae * gcx);
                lFy += w2 * (-Ae * gcy);
            }
            T lux = lUx[r], luy = lUy[r];
            if (seeded) {
                lux = lux + sux[r];
                luy = luy + suy[r];
            }
            const T lUnx = lux + opt * lFx, lUny = luy + opt * lFy;
            T lUox = -th * lFx, lUoy = -th * lFy;
            const T ea = em[ia], eb = em[ib], ec = em[ic];
            const T db = eb - ea, dc = ec - ea;
            const T gx = db * gbx + dc * gcx;
            const T gy = db * gby + dc * gcy;
            const T third = T(1) / T(3);
            T He;
            if (linear_h) {
                He = (sH[ia] + sH[ib] + sH[ic]) * third;
            } else if (!F32) {
                He = ((sH[ia] + ea) + (sH[ib] + eb) + (sH[ic] + ec)) * third;
            } else {
                He = ((sH[ia] + sH[ib] + sH[ic]) + (ea + eb + ec)) * third + c.eta_ref_f;
            }
            const T lrx = (lUnx - al[r] * lUny) * den[r];
            const T lry = (lUny + al[r] * lUnx) * den[r];
            lUox += lrx - al[r] * lry;
            lUoy += lry + al[r] * lrx;
            if (r < OS) {
                grx[r < OS ? r : 0] += dts * lrx;
                gry[r < OS ? r : 0] += dts * lry;
            }
            const T lgx = -dts * g * He * lrx, lgy = -dts * g * He * lry;
            const T lHe = -dts * g * (gx * lrx + gy * lry);
            const T chi = lHe * third;
            const int p0 = t1[r] >> 16, p1 = t2[r] & 0xffffu, p2 = t2[r] >> 16;
            sPsi[p0] = gax * lgx + gay * lgy;
            sPsi[p1] = gbx * lgx + gby * lgy;
            sPsi[p2] = gcx * lgx + gcy * lgy;
            sChi[p0] = chi;
            sChi[p1] = chi;
            sChi[p2] = chi;
            lUx[r] = lUox;
            lUy[r] = lUoy;
        }
        __syncthreads();
        // vertex phase: lambda_eta += sum over the vertex's triangles (ascending) of
        // the slot term and lambda_H / 3; the H0 gradient of owned vertices
        auto vsum = [&](int i, T &ghv, bool own) {
            T acc = sLe[i];
            if (a.ell) {
                const int q0 = kEllWidth * i;
#pragma unroll
                for (int q = 0; q < kEllWidth; ++q) {
                    acc += sPsi[q0 + q];
                    const T ch = sChi[q0 + q];
                    if (nonlin) acc += ch;
                    if (own) ghv += ch;
                }
            } else {
                const int q1 = sRow[i + 1];
                for (int q = sRow[i]; q < q1; ++q) {
                    acc += sPsi[q];
                    const T ch = sChi[q];
                    if (nonlin) acc += ch;
                    if (own) ghv += ch;
                }
            }
            sLe[i] = acc;
        };
#pragma unroll
        for (int k = 0; k < NVO; ++k) {
            const int i = tid + k * BLOCK;
            if (i < nv_act) vsum(i, gh[k], i < h.nv0);
        }
        for (int i = tid + NVO * BLOCK; i < nv_act; i += BLOCK) {
            T dummy = T(0);
            vsum(i, dummy, false);
        }
        __syncthreads();
    }

    // write back the owned entries (the last launch: with the final step's work)
    T *leout = static_cast<T *>(a.lam_eta_out) + h.vbase;
    T *gHo = static_cast<T *>(a.gH0) + h.vbase;
    T *ge0 = (a.fin && a.g_eta0) ? static_cast<T *>(a.g_eta0) + h.vbase : nullptr;
#pragma unroll
    for (int k = 0; k < NVO; ++k) {
        const int i = tid + k * BLOCK;
        if (i < h.nv0) {
            leout[i] = sLe[i];
            gHo[i] = gh[k];
            if (ge0) ge0[i] = sLe[i];
        }
    }
    T2 *lUout = static_cast<T2 *>(a.lam_U_out);
    T2 *gRo = static_cast<T2 *>(a.gR);
    T2 *gU0 = (a.fin && a.g_U0) ? static_cast<T2 *>(a.g_U0) : nullptr;
#pragma unroll
    for (int r = 0; r < OS; ++r) {
        const int le = tid + r * BLOCK;
        if (le < h.nown) {
            const int64_t e = h.ebase + le;
            T2 u;
            u.x = lUx[r];
            u.y = lUy[r];
            if (a.fin && a.lam_Uavg) {   // the endpoint term of <<U>> for U^0
                u.x = u.x - (T)(a.thrM * a.lam_Uavg[2 * e]);
                u.y = u.y - (T)(a.thrM * a.lam_Uavg[2 * e + 1]);
            }
            lUout[e] = u;
            if (gU0) gU0[e] = u;
            u.x = grx[r];
            u.y = gry[r];
            gRo[e] = u;
        }
    }
}

template <typename T, bool F32, int EPT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_adj_tile(AdjTileArgs a) {
    adj_tile_body<T, F32, EPT, BLOCK>(a, blockIdx.x, gridDim.x);
}

// The reverse substeps of one checkpoint segment (blocks [0, nrev)) and the recompute,
// with trajectory output, of the segment before it (the other blocks) in one launch:
// the two read and write disjoint arrays (the reverse reads its own segment's
// trajectory buffer, the recompute writes the other one), so their order does not
// matter and each part's arithmetic is that of its own kernel.
template <typename T, bool F32, int EPT, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_adj_tile_pair(AdjTileArgs ra, TileArgs fa, int nrev) {
    if ((int)blockIdx.x < nrev)
        adj_tile_body<T, F32, EPT, BLOCK>(ra, blockIdx.x, nrev);
    else
        tile_body<T, F32, EPT, BLOCK, 3>(fa, blockIdx.x - nrev, gridDim.x - nrev);
}

// Deterministic sum of each row of partials: out[r] = add + sum_i part[r*width + i].
__global__ void __launch_bounds__(256) k_vol_reduce(const double *part, int64_t width,
                                                    double add, double *out) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < width; i += 256) s += part[r * width + i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = add + ((red[0] + red[1]) + (red[2] + red[3]));
}

template <typename T, bool F32, int EPT, int BLOCK, int SM>
hipError_t launch_tile_t(const TileArgs *a, int grid, size_t lds, hipStream_t s) {
    auto *kern = k_tile<T, F32, EPT, BLOCK, SM, false>;
    auto *kern_nt = k_tile<T, F32, EPT, BLOCK, SM, true>;
    if (!a) {   // prepare only: both access policies
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 160 * 1024);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern_nt),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }
    hipLaunchKernelGGL(a->nt ? kern_nt : kern, dim3(grid), dim3(BLOCK), lds, s, *a);
    return hipGetLastError();
}

template <typename T, bool F32, int BLOCK, int SM>
hipError_t launch_tile_ept(int ept, const TileArgs *a, int grid, size_t lds, hipStream_t s) {
    switch (ept) {
        case 1: return launch_tile_t<T, F32, 1, BLOCK, SM>(a, grid, lds, s);
        case 2: return launch_tile_t<T, F32, 2, BLOCK, SM>(a, grid, lds, s);
        case 3: return launch_tile_t<T, F32, 3, BLOCK, SM>(a, grid, lds, s);
        case 4: return launch_tile_t<T, F32, 4, BLOCK, SM>(a, grid, lds, s);
        case 6: return launch_tile_t<T, F32, 6, BLOCK, SM>(a, grid, lds, s);
        case 8: return launch_tile_t<T, F32, 8, BLOCK, SM>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

// 1024-thread workgroups must fit 128 VGPRs: FP32 up to 4 triangles per thread; FP64
// forward-backward (modes 0 and 3) up to 3, the other FP64 modes one.
template <typename T, bool F32, int SM>
hipError_t launch_tile_1024(int ept, const TileArgs *a, int grid, size_t lds, hipStream_t s) {
    if constexpr (F32) {
        switch (ept) {
            case 1: return launch_tile_t<T, F32, 1, 1024, SM>(a, grid, lds, s);
            case 2: return launch_tile_t<T, F32, 2, 1024, SM>(a, grid, lds, s);
            case 3: return launch_tile_t<T, F32, 3, 1024, SM>(a, grid, lds, s);
            case 4: return launch_tile_t<T, F32, 4, 1024, SM>(a, grid, lds, s);
            default: return hipErrorInvalidValue;
        }
    } else if constexpr (SM == 0 || SM == 3) {
        switch (ept) {
            case 1: return launch_tile_t<T, F32, 1, 1024, SM>(a, grid, lds, s);
            case 2: return launch_tile_t<T, F32, 2, 1024, SM>(a, grid, lds, s);
            case 3: return launch_tile_t<T, F32, 3, 1024, SM>(a, grid, lds, s);
            default: return hipErrorInvalidValue;
        }
    } else {
        return ept == 1 ? launch_tile_t<T, F32, 1, 1024, SM>(a, grid, lds, s) : hipErrorInvalidValue;
    }
}

template <int SM>
hipError_t launch_tile_sm(bool f32, int ept, int block, const TileArgs *a, int grid, size_t lds,
                          hipStream_t s) {
    if (block == 1024)
        return f32 ? launch_tile_1024<float, true, SM>(ept, a, grid, lds, s)
                   : launch_tile_1024<double, false, SM>(ept, a, grid, lds, s);
    if (block == 256)
        return f32 ? launch_tile_ept<float, true, 256, SM>(ept, a, grid, lds, s)
                   : launch_tile_ept<double, false, 256, SM>(ept, a, grid, lds, s);
    if (block == 512)
        return f32 ? launch_tile_ept<float, true, 512, SM>(ept, a, grid, lds, s)
                   : launch_tile_ept<double, false, 512, SM>(ept, a, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tile_any(bool f32, int mode, int ept, int block, const TileArgs *a, int grid,
                           size_t lds, hipStream_t s) {
    switch (mode) {
        case 0: return launch_tile_sm<0>(f32, ept, block, a, grid, lds, s);
        case 1: return launch_tile_sm<1>(f32, ept, block, a, grid, lds, s);
        case 2: return launch_tile_sm<2>(f32, ept, block, a, grid, lds, s);
        case 3: return launch_tile_sm<3>(f32, ept, block, a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int tile_lds_bytes(bool f32, bool sm, int block, int K, int cap_nv, int cap_ne, int cap_nvu,
                   int cap_cs) {
    (void)K;
    (void)cap_ne;
    const int ts = f32 ? 4 : 8;
    int off = 0;
    auto al = [](int b) { return (b + 15) & ~15; };
    off = al(off + ts * cap_nv);
    if (sm)
        for (int k = 0; k < 3; ++k) off = al(off + ts * cap_nv);
    off = al(off + ts * cap_nv);
    off = al(off + ts * cap_nvu);
    off = al(off + ts * cap_nvu);
    off = al(off + 8 * (block / 64) * 9);
    off = al(off + 4 * 18);
    off = al(off + ts * cap_cs);
    off = al(off + 2 * (cap_nvu + 4));
    return off;
}

hipError_t prepare_tile(bool f32, int mode, int ept, int block) {
    return launch_tile_any(f32, mode, ept, block, nullptr, 0, 0, nullptr);
}

hipError_t launch_tile(bool f32, int mode, int ept, int block, const TileArgs &a, int grid,
                       size_t lds, hipStream_t s) {
    return launch_tile_any(f32, mode, ept, block, &a, grid, lds, s);
}

namespace {
template <typename T, bool F32, int EPT, int BLOCK>
hipError_t launch_adj_tile_t(const AdjTileArgs *a, size_t lds, hipStream_t s) {
    auto *kern = k_adj_tile<T, F32, EPT, BLOCK>;
    if (!a)   // prepare only
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipLaunchKernelGGL(kern, dim3(a->ntiles), dim3(BLOCK), lds, s, *a);
    return hipGetLastError();
}

template <typename T, bool F32, int EPT, int BLOCK>
hipError_t launch_adj_pair_t(const AdjTileArgs *a, const TileArgs *f, size_t lds, hipStream_t s) {
    auto *kern = k_adj_tile_pair<T, F32, EPT, BLOCK>;
    if (!a)   // prepare only
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipLaunchKernelGGL(kern, dim3(a->ntiles + f->ntiles), dim3(BLOCK), lds, s, *a, *f,
                       a->ntiles);
    return hipGetLastError();
}

// f null: the reverse kernel alone; else the reverse paired with a recompute launch
template <typename T, bool F32, int BLOCK>
hipError_t launch_adj_tile_ept(int ept, const AdjTileArgs *a, const TileArgs *f, size_t lds,
                               hipStream_t s, bool pair) {
    switch (ept) {
        case 1: return pair ? launch_adj_pair_t<T, F32, 1, BLOCK>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 1, BLOCK>(a, lds, s);
        case 2: return pair ? launch_adj_pair_t<T, F32, 2, BLOCK>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 2, BLOCK>(a, lds, s);
        case 3: return pair ? launch_adj_pair_t<T, F32, 3, BLOCK>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 3, BLOCK>(a, lds, s);
        case 4: return pair ? launch_adj_pair_t<T, F32, 4, BLOCK>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 4, BLOCK>(a, lds, s);
        default: return hipErrorInvalidValue;
    }
}

// 1024-thread workgroups (128 VGPRs without spills): FP32 up to three triangles per
// thread, FP64 two
template <typename T, bool F32>
hipError_t launch_adj_tile_1024(int ept, const AdjTileArgs *a, const TileArgs *f, size_t lds,
                                hipStream_t s, bool pair) {
    if (ept > (F32 ? 3 : 2)) return hipErrorInvalidValue;
    switch (ept) {
        case 1: return pair ? launch_adj_pair_t<T, F32, 1, 1024>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 1, 1024>(a, lds, s);
        case 2: return pair ? launch_adj_pair_t<T, F32, 2, 1024>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 2, 1024>(a, lds, s);
        default:
            if constexpr (F32)
                return pair ? launch_adj_pair_t<T, F32, 3, 1024>(a, f, lds, s)
                            : launch_adj_tile_t<T, F32, 3, 1024>(a, lds, s);
            return hipErrorInvalidValue;
    }
}

// reverse tile kernels exist for 256-, 512- and 1024-thread workgroups, up to four
// triangles per thread (three in FP32 and two in FP64 at 1024 threads)
hipError_t launch_adj_tile_any(bool f32, int ept, int block, const AdjTileArgs *a,
                               const TileArgs *f, size_t lds, hipStream_t s, bool pair) {
    if (block == 1024)
        return f32 ? launch_adj_tile_1024<float, true>(ept, a, f, lds, s, pair)
                   : launch_adj_tile_1024<double, false>(ept, a, f, lds, s, pair);
    if (block == 256)
        return f32 ? launch_adj_tile_ept<float, true, 256>(ept, a, f, lds, s, pair)
                   : launch_adj_tile_ept<double, false, 256>(ept, a, f, lds, s, pair);
    if (block == 512)
        return f32 ? launch_adj_tile_ept<float, true, 512>(ept, a, f, lds, s, pair)
                   : launch_adj_tile_ept<double, false, 512>(ept, a, f, lds, s, pair);
    return hipErrorInvalidValue;
}
}  // namespace

int adj_tile_lds_bytes(bool f32, int block, int cnt, int cap_nv, int cap_nvu, int cap_cs) {
    (void)block;
    const int ts = f32 ? 4 : 8;
    int off = 0;
    auto al = [](int b) { return (b + 15) & ~15; };
    off = al(off + ts * cap_nv);
    off = al(off + ts * cap_nv);
    off = al(off + ts * cap_nv);
    off = al(off + ts * cap_nv * cnt);
    off = al(off + 4 * 18);
    off = al(off + ts * cap_cs);
    off = al(off + ts * cap_cs);
    off = al(off + 2 * (cap_nvu + 4));
    return off;
}

hipError_t prepare_adj_tile(bool f32, int ept, int block) {
    const hipError_t e = launch_adj_tile_any(f32, ept, block, nullptr, nullptr, 0, nullptr, false);
    if (e != hipSuccess) return e;
    return launch_adj_tile_any(f32, ept, block, nullptr, nullptr, 0, nullptr, true);
}

hipError_t launch_adj_tile(bool f32, int ept, int block, const AdjTileArgs &a, size_t lds,
                           hipStream_t s) {
    return launch_adj_tile_any(f32, ept, block, &a, nullptr, lds, s, false);
}

hipError_t launch_adj_tile_pair(bool f32, int ept, int block, const AdjTileArgs &a,
                                const TileArgs &f, size_t lds, hipStream_t s) {
    return launch_adj_tile_any(f32, ept, block, &a, &f, lds, s, true);
}

hipError_t launch_plain_step(bool f32, const PlainArgs &a, hipStream_t s) {
    const int ge = static_cast<int>((a.ne + 255) / 256), gv = static_cast<int>((a.nv + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL((k_plain_tri<float, true>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_plain_vtx<float, true>), dim3(gv), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_plain_tri<double, false>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_plain_vtx<double, false>), dim3(gv), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_sesm_fin(bool f32, const PlainArgs &a, hipStream_t s) {
    const int g = static_cast<int>((std::max(a.nv, a.ne) + 255) / 256);
    if (f32)
        hipLaunchKernelGGL((k_sesm_fin<float, true>), dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_sesm_fin<double, false>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sesm_step(bool f32, const PlainArgs &a, hipStream_t s) {
    const int ge = static_cast<int>((a.ne + 255) / 256), gv = static_cast<int>((a.nv + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL((k_sesm_ab<float, true>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_sesm_vtx<float, true>), dim3(gv), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_sesm_u<float, true>), dim3(ge), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_sesm_ab<double, false>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_sesm_vtx<double, false>), dim3(gv), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_sesm_u<double, false>), dim3(ge), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_adj_step(bool f32, const AdjArgs &a, hipStream_t s) {
    const int ge = static_cast<int>((a.ne + 255) / 256), gv = static_cast<int>((a.nv + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL((k_adj_tri<float, true>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_adj_vtx<float>), dim3(gv), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_adj_tri<double, false>), dim3(ge), dim3(256), 0, s, a);
        hipLaunchKernelGGL((k_adj_vtx<double>), dim3(gv), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_adj_pair(bool f32, const AdjArgs &rev, const PlainArgs &fwd, hipStream_t s) {
    if (rev.nv != fwd.nv || rev.ne != fwd.ne || !fwd.fwd_only) return hipErrorInvalidValue;
    const int ge = static_cast<int>((rev.ne + 255) / 256), gv = static_cast<int>((rev.nv + 255) / 256);
    if (f32) {
        hipLaunchKernelGGL((k_pair_tri<float, true>), dim3(2 * ge), dim3(256), 0, s, rev, fwd, ge);
        hipLaunchKernelGGL((k_pair_vtx<float, true>), dim3(2 * gv), dim3(256), 0, s, rev, fwd, gv);
    } else {
        hipLaunchKernelGGL((k_pair_tri<double, false>), dim3(2 * ge), dim3(256), 0, s, rev, fwd, ge);
        hipLaunchKernelGGL((k_pair_vtx<double, false>), dim3(2 * gv), dim3(256), 0, s, rev, fwd, gv);
    }
    return hipGetLastError();
}

hipError_t launch_adj_init(bool f32, const AdjArgs &a, const void *seed_eta, const void *seed_U,
                           hipStream_t s) {
    const int64_t n = std::max<int64_t>(a.nv, 2 * a.ne);
    const int g = static_cast<int>((n + 255) / 256);
    if (f32)
        hipLaunchKernelGGL((k_adj_init<float>), dim3(g), dim3(256), 0, s, a,
                           static_cast<const float *>(seed_eta), static_cast<const float *>(seed_U));
    else
        hipLaunchKernelGGL((k_adj_init<double>), dim3(g), dim3(256), 0, s, a,
                           static_cast<const double *>(seed_eta),
                           static_cast<const double *>(seed_U));
    return hipGetLastError();
}

hipError_t launch_adj_final(bool f32, const AdjArgs &a, void *g_eta0, void *g_U0, hipStream_t s) {
    const int g = static_cast<int>((std::max<int64_t>(a.nv, 2 * a.ne) + 255) / 256);
    if (f32)
        hipLaunchKernelGGL((k_adj_final<float>), dim3(g), dim3(256), 0, s, a,
                           static_cast<float *>(g_eta0), static_cast<float *>(g_U0));
    else
        hipLaunchKernelGGL((k_adj_final<double>), dim3(g), dim3(256), 0, s, a,
                           static_cast<double *>(g_eta0), static_cast<double *>(g_U0));
    return hipGetLastError();
}

hipError_t launch_vol_reduce(const double *part, int64_t width, int32_t rows, double add,
                             double *out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vol_reduce, dim3(rows), dim3(256), 0, s, part, width, add, out);
    return hipGetLastError();
}

}  // namespace sesub
