// Internal declarations shared by the HIP translation units of libsrf.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/srf.h"

namespace srf {

// ----------------------------------------------------------------- errors
// Internal failures throw srf::Error; the C entry points catch it and turn
// it into a status code (nothing propagates across the ABI).
struct Error {
    int status;
    std::string msg;
};

[[noreturn]] void fail(int status, const std::string& msg);
void check_hip(hipError_t e, const char* what);

#define SRF_HIP(call) ::srf::check_hip((call), #call)

// ------------------------------------------------------------ device memory
// Size-bucketed cache of device blocks.  Blocks freed on one stream and
// reused on another are synchronised first.
void* dev_alloc(size_t bytes, hipStream_t stream);
void dev_free(void* p, hipStream_t stream);
void dev_release_all();

// A second stream of the current device (non-blocking, default priority),
// for work that overlaps the caller's stream; created on first use and kept
// until the process ends.  Work on it is ordered by events only, and every
// buffer it touches is allocated on the caller's stream.
hipStream_t aux_stream();

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(size_t count, hipStream_t stream) { alloc(count, stream); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(size_t count, hipStream_t stream) {
        reset();
        s = stream;
        n = count;
        p = static_cast<T*>(dev_alloc(count * sizeof(T) + 16, stream));
    }
    void reset() {
        if (p) dev_free(p, s);
        p = nullptr;
        n = 0;
    }
    T* get() const { return p; }
};

// ------------------------------------------------------------- structures
constexpr int kMaxLevel = 21;           // deepest octree level (21 key bits per axis)
constexpr int kLevels = kMaxLevel + 1;  // levels 0..21

// Cell record in DFS preorder, 32 bytes: integer cell coordinates at the
// cell's level, level, leaf flag, particle range and the preorder index of
// the first cell after this cell's subtree ("skip").
struct __align__(16) NodeGeo {
    uint32_t ix, iy, iz;
    uint32_t level_leaf;  // level | (leaf << 8)
};
struct __align__(16) NodeRange {
    int32_t first, count, skip, parent;
};
// The same cell packed into one 16-byte record (the refitted tree's walk
// records hold it):
//   x = ix | (skip & 0x7ff) << 21,  y = iy | ((skip >> 11) & 0x7ff) << 21,
//   z = iz | ((skip >> 22) & 0x3ff) << 21,
//   w = level | leaf << 5 | min(count, kPackCountMax) << 6.
constexpr uint32_t kPackCountMax = 0x3ffffffu;
// and into one 8-byte record for the walk over a built tree, which finds the
// cell's coordinates from those of the cell it visited before (the new
// cell's parent is that cell or one of its ancestors):
//   x = level | leaf << 5 | oct << 6 | min(count, kWalkCountMax) << 9,
//   y = skip,
// oct = the low bits of (ix, iy, iz) as x << 2 | y << 1 | z.
constexpr uint32_t kWalkCountMax = 0x7fffffu;
// A cell of a refitted tree for the list traversal, 32 bytes: the packed
// record and its box rounded outward to multiples of q = 2^-(level + 10),
// per axis a the 16-bit offsets (in q) of its lower and upper bound from
// the cell's dyadic centre, b[a] = lo | hi << 16; b[3] bit 0 is set when the
// box fits those offsets (else the cell is unbounded: never pruned or
// accepted).
struct __align__(32) RefitCell {
    uint4 pk;
    int32_t b[4];
};
constexpr int kRefitShift = 10;         // q = side / 2^kRefitShift
constexpr int64_t kRefitMaxOff = 32767; // largest offset stored, in q

struct Tree {
    uint64_t id = 0;           // generation number, unique per process (lists refer to it)
    int64_t n = 0;
    int64_t n_nodes = 0;
    int64_t n_groups = 0;
    int32_t max_level = 0;
    int32_t n_group = 0, n_leaf = 0;
    bool refit = false;        // cells measured by the boxes of their particles (tree_refit)
    int32_t level_off[kLevels + 1] = {};   // first slot of each level, and the total
    hipStream_t stream = nullptr;
    // sorted particles
    DevBuf<uint64_t> keys;     // sorted keys
    DevBuf<int32_t> perm;      // input index of sorted position s
    DevBuf<double> px, py, pz, pm;   // wrapped positions and masses, sorted
    DevBuf<int32_t> leaf_of;   // preorder id of the leaf holding sorted position s
    // cells, preorder
    DevBuf<NodeGeo> geo;
    DevBuf<NodeRange> range;
    DevBuf<uint2> pack;        // walk records (see kWalkCountMax)
    DevBuf<uint64_t> prefix;
    DevBuf<double> nM, nX, nY, nZ;   // monopoles
    // the cells again as level slots (each level's cells ordered by first
    // particle; a cell's children are one run of the next level's slots):
    // first particle, preorder id and first child slot (-1 for a leaf)
    DevBuf<int32_t> sfirst, spre, schild;
    DevBuf<double> clo, chi;   // [nn*3] boxes of the cells of a refitted tree
    DevBuf<RefitCell> rpack;   // their walk records
    // groups, in order of first
    DevBuf<int32_t> gfirst, gcount;
    DevBuf<double> glo, ghi;   // [ng*3]
    // Work of the build on aux_stream(): the gather of the sorted positions
    // and masses (after `sorted`, recorded on the build's stream; it ends at
    // `gathered`, which the build's stream waits for before the cells) and
    // the groups (after `sized`; they end at `grouped`, which the build's
    // stream waits for before the build returns).
    hipEvent_t sorted = nullptr, gathered = nullptr, sized = nullptr, grouped = nullptr;
    void release_events();   // waits for `gathered` and `grouped`, then destroys all four
    Tree() = default;
    Tree(const Tree&) = delete;
    Tree& operator=(const Tree&) = delete;
    ~Tree() { release_events(); }   // before the buffers the gather writes are freed
};

struct Lists {
    uint64_t tree_id = 0;      // Tree::id of the tree the lists were built from
    int64_t n_groups = 0;
    int64_t n_entries = 0;
    int64_t n_particle_entries = 0;
    int64_t n_node_entries = 0;
    int64_t interactions = 0;
    double r_cut = 0, theta = 0;
    int32_t mac = 0;
    int32_t n_group = 0, n_leaf = 0;
    hipStream_t stream = nullptr;
    DevBuf<int64_t> off;       // [ng+1] entry offsets per group
    DevBuf<int32_t> ent;       // entries: s >= 0 particle (sorted index), -(c+1) cell c
};

// Nearest periodic image of a coordinate difference (unit box).  Targets are
// taken as offsets from their group's centre through it too: in a fresh
// tree a group lies inside one level-1 cell and the offset is unchanged; in
// a refitted tree its box may reach past the unit box.
__device__ __forceinline__ double image(double d) { return d - rint(d); }

// Workgroups are handed to the 8 XCDs (each with its own L2) round-robin in
// launch order.  This maps launch index b of nb to a logical block index so
// that each XCD runs one contiguous run of logical blocks: for work ordered
// in space (groups in Morton order) the blocks sharing an L2 are spatial
// neighbours whose data overlap.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t x = b & 7, y = b >> 3;
    const int64_t q = nb >> 3, r = nb & 7;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + y;
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of n int64 values in place on `stream`; returns
// nothing (the total is out[n] if the caller allocated n+1 entries and
// asked for it with `write_total`).
void exclusive_scan_i64(int64_t* data, int64_t n, bool write_total, hipStream_t stream);
// The same for int32 over the first *nd values (a count on the device, at
// most n_max; data holds n_max + 1 values), the total at data[*nd].
void exclusive_scan_i32_counted(int32_t* data, int64_t n_max, const int32_t* nd, hipStream_t stream);

// ------------------------------------------------------------ launches
// a1-a2: keys, sort, gather.  Sets bits of the device error flag *d_flag
// (bit 0: non-finite position, bit 1: bad mass; bit 3: a run of more than
// kRunMax particles shares the high key word, so the order is incomplete and
// the sort must be run again with `full`).  Without `full` the positions
// and masses are gathered on aux_stream() (t.gathered marks their end).
void build_sorted(Tree& t, const double* x, const double* y, const double* z, int64_t ps,
                  const double* m, int64_t ms, int32_t* d_flag, bool full, hipStream_t stream);
// a3-a5; synchronises `stream` once, then makes it wait for t.gathered, and
// fails with SRF_EDOMAIN if bit 0 or 1 of *d_flag (set by build_sorted) is
// set.  Returns false, having built nothing, if bit 3 is set.
bool build_cells_and_groups(Tree& t, int32_t* d_flag, hipStream_t stream);
// Tree reuse: positions and masses (m may be NULL: masses kept) gathered in
// the tree's sorted order into px..pm, wrapped, with the same checks as
// build_sorted (bits of *d_flag)
void gather_refit(const Tree& t, const double* x, const double* y, const double* z, int64_t ps, const double* m,
                  int64_t ms, int32_t* d_flag, double* px, double* py, double* pz, double* pm, hipStream_t stream);
// moments and cell and group boxes of the tree's current particles, the
// structure held (asynchronous)
void refit_cells_and_groups(Tree& t, hipStream_t stream);
// a6
void build_lists(const Tree& t, Lists& l, hipStream_t stream);
// a7-a8
void launch_force(const Tree& t, const Lists& l, const srf_params& p, double* ax, double* ay, double* az,
                  int64_t os, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);
// a9
void launch_pm(const Tree& t, double G, double r_cut, int n_mesh, double* ax, double* ay, double* az, int64_t os,
               hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);
void launch_kick(int64_t n, double* vx, double* vy, double* vz, int64_t vs, const double* ax, const double* ay,
                 const double* az, int64_t as, double dt, hipStream_t stream);
void launch_drift(int64_t n, double* x, double* y, double* z, int64_t xs, const double* vx, const double* vy,
                  const double* vz, int64_t vs, double dt, hipStream_t stream);
void launch_potential(const Tree& t, const Lists& l, const srf_params& p, double* phi, int64_t os, hipStream_t st);
void launch_quadrupole(const Tree& t, const Lists& l, const srf_params& p, double* ax, double* ay, double* az,
                       int64_t os, hipStream_t st);
void launch_adjoint(const Tree& t, const Lists& l, const srf_params& p, const double* wx, const double* wy,
                    const double* wz, int64_t ws, double* gx, double* gy, double* gz, int64_t gs, double* gm,
                    int64_t gms, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);
// The same on the library's static workspace: no allocation (SRF_EINVAL if
// the tree needs more than SRF_NOALLOC_WORKSPACE_BYTES).
void launch_adjoint_noalloc(const Tree& t, const Lists& l, const srf_params& p, const double* wx, const double* wy,
                            const double* wz, int64_t ws, double* gx, double* gy, double* gz, int64_t gs,
                            double* gm, int64_t gms, hipStream_t stream);
size_t adjoint_workspace_bytes(int64_t n, int64_t n_nodes);

// Fill helpers (kernels, safe under stream capture).
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double* p, double v, int64_t n, hipStream_t s);
void fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);

inline int grid_for(int64_t n, int block, int cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

}  // namespace srf
