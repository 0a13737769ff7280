// Internal structures of the barotropic subcycle library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sesub.h"

namespace sesub {

void set_error(const std::string &msg);

// ---------------------------------------------------------------------------
// Host mesh after reordering: integer connectivity plus FP64 geometry.
// ---------------------------------------------------------------------------
struct HostMesh {
    int64_t nv = 0, ne = 0;
    uint32_t flags = 0;
    double period_x = 0, period_y = 0, radius = 0;
    std::vector<int32_t> vperm, eperm;   // new -> input
    std::vector<int32_t> tri;            // [ne*3], smallest vertex first
    std::vector<int32_t> row_ptr, col;   // vertex -> (tri << 2 | slot)
    std::vector<double> x, y;            // reordered coordinates
    std::vector<double> Ae, gN, Av;      // gN [ne][3][2]
    double Av_total = 0;                 // sum of Av in vertex order (FP32 volume offset)
    double mu_max = 0;                   // Gershgorin bound of -div grad
};

// Build the reordered mesh; returns SE_OK or an error with set_error().
se_status build_host_mesh(const se_mesh_desc &d, HostMesh &m);

// Element neighbours across each local edge (nb4 [ne][4], -1 on coasts, slot 3
// unused) and per edge (length, length / centroid distance) (vg [ne][6]).
se_status build_visc_tables(const HostMesh &m, std::vector<int32_t> &nb4,
                            std::vector<double> &vg);

// Tiles of the trim/z* consumer: runs of consecutive vertices, each with every triangle
// of its vertices' CSR rows (at most cap_e), the vertices of those triangles (at most
// cap_v) and at most cap_o vertices of its own.  hdr [ntiles][8]: first vertex v0, own
// vertices nvo, local vertices nvl (own first, then the others ascending: lv), local
// triangles nel, owned triangles neo (smallest vertex in the run; the first neo local
// triangles, ascending), offset into lv, offset into le, CSR entries of the run's rows.
// le [2 per local triangle]: global id, local vertices a | b << 10 | c << 20.  rloc [3 ne]
// (CSR order): local index of the entry's triangle in the tile owning the row.  Returns
// false when one vertex's row alone exceeds a capacity.
struct TrimTiles {
    int32_t ntiles = 0;
    std::vector<int32_t> hdr, lv, le;
    std::vector<uint16_t> rloc;
};
bool build_trim_tiles(const HostMesh &m, int cap_e, int cap_o, int cap_v, TrimTiles &out);

// ---------------------------------------------------------------------------
// Tile plan of the temporally blocked kernel (one mesh or a disjoint union).
// Tile t owns vertices [vbase, vbase + nv0) and the triangles whose smallest
// vertex it owns.  Level sets: V_0 = owned vertices, E_i = triangles touching
// V_{i-1}, V_i = vertices of E_i, i = 1..K.  Local vertex order: V_0, then
// V_1 \ V_0, ...; local triangle order: owned, E_1 \ owned, E_2 \ E_1, ...
// ---------------------------------------------------------------------------
struct TileHdr {
    int32_t vbase, nv0;     // owned vertex range (global, union numbering)
    int32_t ebase, nown;    // owned triangle range
    int32_t lv_off, le_off; // offsets into local vertex / triangle arrays
    int32_t cs_off, rw_off; // (unused) / offset into local CSR rows
    int32_t member;         // batch member (0 for a single mesh)
    int32_t mtile;          // tile index within its member
    int32_t pad0, pad1;
};

struct HostTiles {
    int32_t T = 0, K = 0;
    std::vector<TileHdr> hdr;
    std::vector<int32_t> nV;      // [ntiles][K+1] cumulative |V_i|
    std::vector<int32_t> nE;      // [ntiles][K+1] cumulative |E_i| (entry 0 = owned)
    std::vector<int32_t> lv_gid;  // local vertex -> global vertex
    std::vector<int32_t> le_gid;  // local triangle -> global triangle
    // [3 per local triangle]: a | b << 16, c | p0 << 16, p1 | p2 << 16 with local
    // vertex indices a, b, c and the CSR positions p0..p2 of the three incidences
    std::vector<uint32_t> le_tri;
    std::vector<uint16_t> cs_row; // per tile: nV[K-1] + 1 row offsets (local), padded to 4
    int64_t n_ent = 0;            // local CSR entries over all tiles
    int32_t max_nv = 0, max_ne = 0, max_nvu = 0, max_cs = 0;   // max_cs: rows + 64 scratch
    int32_t max_nown = 0;         // most owned triangles of a tile
    bool ell = false;             // fixed-width rows of kEllWidth deposits per vertex
};

// T vertices per tile (the last tile of a member the rest); split_cap > 0: tiles with
// more local triangles than split_cap are halved (repeatedly, at most four times).
se_status build_tiles(const std::vector<const HostMesh *> &members,
                      const std::vector<int64_t> &voff, const std::vector<int64_t> &eoff,
                      int32_t T, int32_t K, HostTiles &out, int32_t split_cap = 0);

// ---------------------------------------------------------------------------
// Device-side arrays
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    ~DevBuf();
    se_status alloc(size_t bytes);
    se_status upload(const void *src, size_t bytes);
    template <class T> T *as() const { return static_cast<T *>(p); }
};

struct DevTiles {
    int32_t T = 0, K = 0, block = 256, ept = 0, ntiles = 0;
    bool ell = false;   // fixed-width deposit rows (HostTiles::ell)
    int32_t max_nv = 0, max_ne = 0, max_nvu = 0, max_cs = 0;
    size_t lds_bytes64 = 0, lds_bytes32 = 0;
    bool ok32 = false, ok64 = false;
    size_t lds_sm64 = 0, lds_sm32 = 0;   // AB3-AM4 scheme
    bool ok_sm32 = false, ok_sm64 = false;
    // forward-backward tile kernel of this plan's shape ready to launch (its LDS limit
    // raised when the plan was made), indexed by f32
    bool prepared[2] = {false, false};
    // the adjoint's tile path ready (recompute and reverse kernels prepared), its LDS
    bool adj_ready[2] = {false, false};
    size_t lds_adj[2] = {0, 0};
    size_t lds(bool f32, bool sm) const {
        return sm ? (f32 ? lds_sm32 : lds_sm64) : (f32 ? lds_bytes32 : lds_bytes64);
    }
    bool ok(bool f32, bool sm) const { return sm ? (f32 ? ok_sm32 : ok_sm64) : (f32 ? ok32 : ok64); }
    std::vector<TileHdr> hdr_host;
    DevBuf hdr, nV, nE, lv_gid, le_rec, cs_row;
    DevBuf geo64, geo32, ae64, ae32;   // per local triangle: 4 gradient values; A_e
    DevBuf lav64, lav32;          // per local vertex: 1 / A_v (FP64, FP32)
    // host copies for tables built on first use: global id of each local triangle,
    // level counts [ntiles][K+1]
    std::vector<int32_t> le_gid_host, nE_host;
    // viscous term, built on first use: local edge neighbours (uint2 per local
    // triangle) and edge (l, l/d) [3][2] per local triangle
    DevBuf vnb, vgeo64, vgeo32;
};

// Mesh geometry and connectivity on the device (global numbering).
struct DevMesh {
    int64_t nv = 0, ne = 0;
    DevBuf tri, row_ptr, pcol;    // pcol = 3 * tri + slot, CSR order
    DevBuf geom64, geom32;        // 5 SoA arrays [ne]: gbx gby gcx gcy Ae
    DevBuf Av64, Av32;
    DevBuf faults;                // uint32 fault word
    // barotropic viscous term, built on first use: neighbours int32 [ne][4],
    // edge (l, l/d) [ne][3][2] in FP64 and FP32
    DevBuf vnb, vgeo64, vgeo32;
    // trim/z* consumer, built on first use: sub-cell flux vectors [ne][3][2] FP64; the
    // tile tables (TrimTiles) for the triangle capacity tt_cap_e (0: not built, -1: the
    // mesh has a row beyond it) and local vertex capacity tt_cap_v
    DevBuf slotS;
    DevBuf tt_hdr, tt_lv, tt_le, tt_rloc;
    int32_t tt_cap_e = 0, tt_cap_v = 0, tt_ntiles = 0;
};

// The forward subcycle on the tile kernel (se_subcycle); may_alloc false: fail instead
// of building a missing plan or missing viscous tables (se_subcycle_noalloc).
se_status subcycle_tile(se_mesh *m, const se_params *p, se_state *st, const se_forcing *fo,
                        int32_t nsub, double dt, void *ws, void *stream, bool may_alloc);

}  // namespace sesub

struct se_mesh {
    int device = 0;
    sesub::HostMesh h;
    sesub::DevMesh d;
    std::unique_ptr<sesub::DevTiles> plan;
    int32_t plan_T = 1024, plan_K = 4, plan_block = 256;
};
