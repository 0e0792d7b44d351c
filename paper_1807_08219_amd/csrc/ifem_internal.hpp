// Plan layout shared by the host side (ifem_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ifem_device.hpp"

namespace ifem {

// Everything the per-particle force kernel reads (all device pointers).
struct ForceArgs {
  const int32_t* node_start;  // [n_p + 1]
  const int32_t* law;
  const double* mu;
  const double* mu2;
  const double* kb;
  const double* c0;
  const int32_t* pcol_tri;   // [n_p + 1] first colour of each particle
  const int32_t* colb_tri;   // [n_colours + 1] first element slot of each colour
  const int32_t* tri_local;  // [3][n_tris] particle-local node ids, colour-sorted slots
  const double* tri_ref;     // [4][n_tris] G11 G12 G22 A0
  const int32_t* pcol_tet;
  const int32_t* colb_tet;
  const int32_t* tet_local;  // [4][n_tets]
  const double* tet_ref;     // [10][n_tets] inverse reference edge matrix (row-major: the shape gradients
                             // of nodes 1..3), V0
  const int32_t* ring_start; // [n_nodes + 1]: one-rings of bending and (when all close) membrane nodes, or null
  const int32_t* ring;       // one-ring neighbours, particle-local ids
  const int32_t* lds_part;   // [grid of k_forces] the particles it takes, or null for all of them
  unsigned long long* status;
  int32_t n_nodes, n_tris, n_tets;
  int32_t cap;               // largest particle k_forces takes (nodes): the stride of its LDS arrays
  int32_t cap_mem;           // largest membrane (the volume correction's LDS)
  int32_t cap_solid;         // largest solid (the fluid-stress kernel's LDS)
  int32_t has_bending;       // the force kernel's LDS holds a curvature array
};

// Particles too large for one workgroup's LDS (their forces by the global-memory kernels).
struct LargeArgs {
  int32_t n_part, n_tri, n_tet, n_node, any_bending;
  const int32_t* part;          // [n_part] particle ids
  const int32_t* tri_begin;     // [n_part + 1] first large triangle of each large particle
  const int32_t* tet_begin;     // [n_part + 1]
  const int32_t* tri_slot;      // [n_tri] element slot of each large triangle
  const int32_t* tri_part;      // [n_tri] its particle
  const int32_t* tet_slot;      // [n_tet]
  const int32_t* tet_part;      // [n_tet]
  const int32_t* node_part;     // [n_node] particle of each large node (compact numbering)
  const int32_t* node_base;     // [n_node] compact index of that particle's first node
  const int32_t* node_lp;       // [n_node] index of that particle in part
  const int32_t* part_base;     // [n_part + 1] compact index of each large particle's first node
  const int32_t* gather_start;  // [n_node + 1]
  const int32_t* gather;        // element shares of each node: e * 4 + corner, tetrahedra after triangles
  void* ef_tri;                 // [3 corners][n_tri][4] element nodal forces, x y z and a pad (sized for float64)
  void* ef_tet;                 // [4 corners][n_tet][4]
  void* kh;                     // [n_node] kH - kH0
  void* fb;                     // [3][n_node] bending force
  double* red_terms;            // [5][n_tri + n_tet] element terms of the reductions
  double* red_part;             // [n_part][16][5] their sums over 16 shares of each particle's elements
  double* vol_terms;            // [4][n_node] node terms of the volume correction's sums
  double* lam;                  // [n_part] its multipliers
};

// Room a carried spread list gets beyond half as many entries again as it had (see k_scan).
constexpr int kBucketSlack = 32;

// Everything the transfer kernels read.
struct TransferArgs {
  const int32_t* node_particle;   // [n_nodes]
  const int32_t* particle_box;    // [n_p]
  const BoxDev* boxes;            // [n_boxes]
  const int32_t* tile_box;        // [n_tiles]
  int32_t* tile_count;            // [3 n_tiles] list lengths: nodes whose stencil the tile takes, per component
  int32_t* tile_off;              // [3 n_tiles]
  int32_t* place;                 // [2] running totals of the list placement: this call's lists, the next one's
  int32_t* tile_cursor;           // [3 n_tiles]
  int32_t* bin_list;              // [list_cap] node ids, grouped by (component, tile)
  int32_t* tile_flag;             // [3 n_tiles] 1 if the tile wrote a halo shell this call
  uint32_t* tile_fmax;            // [3 n_tiles] bound on |F| of each list, float32 bits (atomic max)
  void* halo;                     // [3 n_tiles][halo_cells] y/z halo shell rows (float or double)
  int32_t* bk_list;               // [bk_cap] node ids in lists laid out from the previous call's counts (NULL: none)
  int2* bk_lay;                   // [2][3 n_tiles] two such layouts, this call's and the next one's: per list
                                  // its first slot in bk_list and its room
  int32_t* bk_state;              // [2] index of this call's layout; 1 if a list outgrew its room this call
  unsigned long long* status;
  int64_t list_cap;
  int64_t bk_cap;
  int64_t total_cells;
  int32_t n_nodes, n_boxes, n_tiles;
  int32_t tile[3];        // cells per tile and axis (powers of two)
  int32_t tile_shift[3];  // log2 of tile
  int32_t region_cells;   // (tile_x + 5)(tile_y + 2)(tile_z + 2): rows of tile_x cells, two pad cells on each
                          // side, one more for an odd pitch
  int32_t halo_cells;     // tile_x (2 (tile_y + tile_z) + 4): the region's y/z shell rows
};

// The box of particle p.  With one box (a kernel argument, uniform over the grid) its fields come from
// scalar loads and the per-node gather of the particle's box index is skipped.
__device__ __forceinline__ BoxDev box_of(const TransferArgs& a, int p) {
  if (a.n_boxes == 1) return a.boxes[0];
  return a.boxes[a.particle_box[p]];
}

// Index of region row (iy, iz) among the y/z shell rows of a region with ry x rz rows: the two z
// faces (every y), then the two y faces without the z-face rows.  (iy, iz) must be a shell row.
__device__ __forceinline__ int halo_row(int iy, int iz, int ry, int rz) {
  if (iz == 0) return iy;
  if (iz == rz - 1) return ry + iy;
  return 2 * ry + (iy == 0 ? 0 : rz - 2) + (iz - 1);
}

// One periodic box's grid of contact cells (node-face anti-sticking).
struct ContactBoxDev {
  int32_t nc[3];      // cells per axis
  int32_t base;       // first cell of this box
  double origin[3];
  double inv_cs[3];   // 1 / cell width per axis
  double len[3];      // box length per axis (periodic minimum image)
  double inv_len[3];
};

// A node as binned for the anti-sticking search: its absolute position, id and particle.
struct alignas(16) ContactNode {
  double x, y, z;
  int32_t k, p;
};

// Everything the anti-sticking kernels read.
struct ContactArgs {
  const int32_t* node_particle;  // [n_nodes]
  const int32_t* particle_box;   // [n_p]
  const ContactBoxDev* boxes;    // [n_boxes]
  const int32_t* tri;            // [3][n_tris] membrane triangles, global node ids (input order)
  const int32_t* bface;          // [3][n_bfaces] boundary faces of the solids, outward
  int32_t* count;                // [n_cells] nodes per cell
  int32_t* off;                  // [n_cells] first record of each cell
  int32_t* cursor;               // [n_cells]
  int32_t* owner;                // [n_cells] particle of all the cell's nodes, -2 mixed, -1 empty
  int32_t *near_lo, *near_hi;  // [n_cells] least / greatest owner over the 3^3 cells around each cell
  ContactNode* rec;              // [n_nodes] the nodes grouped by cell
  unsigned long long* keys;      // [n_nodes] float64 bits of the least distance below d_min (atomic min)
  int32_t* keyf;                 // [n_nodes] least face id at exactly that distance (second pass)
  uint2* work;                   // [work_cap] (face, cell) pairs to search
  int32_t* work_count;           // [256 + 3]: items per work-list segment, slow faces, hits, cell placement
  int32_t* slow_count;           // work_count + 256
  int32_t* hit_count;            // work_count + 257
  int32_t* place;                // work_count + 258: running total of the cell placement
  int32_t* hits;                 // [work_cap] work-list slots of items that found a pair below d_min
  int32_t* slow;                 // [n_tris + n_bfaces] faces searched whole
  unsigned long long* status;    // the plan's status counters
  int32_t work_cap;
  int32_t n_nodes, n_tris, n_bfaces, n_cells, n_boxes;
};

// The contact box of particle p (scalar loads when there is one box).
__device__ __forceinline__ ContactBoxDev cbox_of(const ContactArgs& a, int p) {
  if (a.n_boxes == 1) return a.boxes[0];
  return a.boxes[a.particle_box[p]];
}

// Kernel slots of the per-kernel event timer.
enum KernelSlot {
  K_FORCES = 0,
  K_BIN_COUNT = 1,
  K_SCAN = 2,
  K_BIN_FILL = 3,
  K_SPREAD_HOME = 4,
  K_SPREAD_MERGE = 8,
  K_SPREAD_ATOMIC = 5,
  K_INTERP = 6,
  K_FILL = 7,
  K_VOLUME = 9,
  K_ADVANCE = 10,
  K_INTERP_CELLS = 11,
  K_FLUID = 12,
  K_CONTACT = 13,
  K_NSLOTS = 16
};

// Optional host-side timer: when enabled, every kernel launch of a step call
// is bracketed by two events recorded on the launch stream.  Events come from
// a pool created when timing is switched on; nothing is allocated per call.
struct KernelTimer {
  bool enabled = false;
  std::vector<hipEvent_t> ev;  // 2 per record
  std::vector<int> slot;       // slot of each record
  size_t used = 0, dropped = 0;
  void begin(int s, hipStream_t st) {
    if (!enabled) return;
    if (used >= slot.size()) {
      ++dropped;
      return;
    }
    slot[used] = s;
    (void)hipEventRecord(ev[2 * used], st);
  }
  void end(hipStream_t st) {
    if (!enabled || used >= slot.size()) return;
    (void)hipEventRecord(ev[2 * used + 1], st);
    ++used;
  }
};

struct PlanDev {
  int32_t n_particles, n_nodes, n_tris, n_tets, n_boxes;
  int64_t total_cells;
  int32_t cap;          // largest particle (nodes)
  int32_t has_bending;  // any particle with kb != 0
  // setup-only views
  const int32_t* tri_src;     // slot -> original triangle
  const int32_t* tri_global;  // [3][n_tris] original connectivity
  double* tri_ref;
  const int32_t* tet_src;
  const int32_t* tet_global;
  double* tet_ref;
  unsigned long long* status;  // [5]
  double* vref;                // [n_p] enclosed volume of every membrane in the reference configuration
  ForceArgs fargs;
  int32_t n_lds_part;  // particles k_forces takes
  LargeArgs large;     // the others
  TransferArgs targs;
  ContactArgs cargs;
  KernelTimer* timer;  // host object owned by the plan
};

// ---- launchers (ifem_forces.hip)
hipError_t launch_ref_setup(const PlanDev& P, const double* X, hipStream_t st);
hipError_t prepare_force_kernels(const PlanDev& P);
size_t force_lds_bytes(const PlanDev& P, int dtype);
hipError_t launch_forces(const PlanDev& P, int dtype, const void* x, const double* anchor, void* f, double* red,
                         int block, hipStream_t st);
// LDS of k_forces for a particle of nn nodes (float64 sizing): a particle above the limit is large
size_t force_lds_per_node(bool has_bending);

// ---- launchers (ifem_volume.hip)
hipError_t prepare_volume_kernels(const PlanDev& P);
hipError_t launch_ref_volume(const PlanDev& P, const double* X, double* vref, hipStream_t st);
hipError_t launch_volume(const PlanDev& P, int dtype, const void* x, const double* V0, void* x_out, double* lam,
                         hipStream_t st);

// ---- launchers (ifem_advance.hip)
hipError_t launch_advance(const PlanDev& P, int dtype, const void* x, const void* v, const void* v_prev, double dt,
                          void* x_out, hipStream_t st);

// ---- launchers (ifem_fluid.hip)
hipError_t prepare_fluid_kernels(const PlanDev& P);
hipError_t launch_interp_cells(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* grid,
                               int ncomp, void* out, hipStream_t st);
hipError_t launch_fluid(const PlanDev& P, int dtype, const void* x, const void* v, const void* C, double eta, double G,
                        void* f, hipStream_t st);

// ---- launchers (ifem_transfer.hip)
hipError_t prepare_transfer_kernels(const PlanDev& P);
hipError_t launch_spread_atomic(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* F,
                                void* grid, int block, hipStream_t st);
// `a` is P.targs, or a copy whose workspace pointers lead elsewhere (the allocation-free entry point)
hipError_t launch_spread_tiled(const PlanDev& P, const TransferArgs& a, int dtype, const void* x, const double* anchor,
                               const void* F, void* grid, hipStream_t st);
hipError_t launch_interp(const PlanDev& P, int dtype, const void* x, const double* anchor, const void* grid,
                         void* v, int block, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);

// ---- launchers (ifem_contact.hip)
hipError_t launch_antistick(const PlanDev& P, int dtype, const void* x, const double* anchor, double d_min,
                            void* x_out, int64_t* face_out, hipStream_t st);
int32_t contact_scan_blocks(int32_t n_cells);
size_t spread_tile_lds_bytes(const PlanDev& P, int dtype);

}  // namespace ifem
