// lattice.hpp -- compile-time lattice tables, storage conversion and
// neighbour addressing shared by the gfx950 kernels.
//
// Velocity order and weights follow App. B (stencils figure and weight
// equations): 0 rest; 1/2 = +y/-y; 3/4 = -x/+x; 5/6 = +z/-z; 7-10 the xy
// edges NW NE SW SE; 11-14 TN TS TW TE; 15-18 BN BS BW BE; 19-26 the corners
// TNE TNW TSE TSW BNE BNW BSE BSW.  D3Q15 is the rest + faces + the eight
// corners (in the same corner order); D3Q19 is 0-18; D3Q7 is 0-6.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcp {

// ----------------------------------------------------------------------------
// velocities and weights
// ----------------------------------------------------------------------------
__host__ __device__ constexpr int vel27(int i, int a)
{
    constexpr int t[27][3] = {
        {0, 0, 0},   {0, 1, 0},   {0, -1, 0},  {-1, 0, 0}, {1, 0, 0},   {0, 0, 1},   {0, 0, -1},
        {-1, 1, 0},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {0, 1, 1},   {0, -1, 1},  {-1, 0, 1},
        {1, 0, 1},   {0, 1, -1},  {0, -1, -1}, {-1, 0, -1}, {1, 0, -1}, {1, 1, 1},   {-1, 1, 1},
        {1, -1, 1},  {-1, -1, 1}, {1, 1, -1},  {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
    return t[i][a];
}

// D3Q27 slot of direction i of a Q stencil: D3Q15 maps its corner slots 7..14
// onto D3Q27 slots 19..26, the other stencils are prefixes of D3Q27
template <int Q>
__host__ __device__ constexpr int index27(int i)
{
    return (Q == 15 && i >= 7) ? i + 12 : i;
}

template <int Q>
__host__ __device__ constexpr int vel(int i, int a)
{
    return vel27(index27<Q>(i), a);
}

template <int Q>
__host__ __device__ constexpr double weight(int i)
{
    if (Q == 7) return i == 0 ? 0.0 : 1.0 / 6.0;
    if (Q == 15) return i == 0 ? 16.0 / 72.0 : (i < 7 ? 8.0 / 72.0 : 1.0 / 72.0);
    if (Q == 19) return i == 0 ? 12.0 / 36.0 : (i < 7 ? 2.0 / 36.0 : 1.0 / 36.0);
    return i == 0 ? 64.0 / 216.0 : (i < 7 ? 16.0 / 216.0 : (i < 19 ? 4.0 / 216.0 : 1.0 / 216.0));
}

template <int Q>
__host__ __device__ constexpr int opposite(int i)
{
    for (int j = 0; j < Q; ++j)
        if (vel<Q>(j, 0) == -vel<Q>(i, 0) && vel<Q>(j, 1) == -vel<Q>(i, 1) && vel<Q>(j, 2) == -vel<Q>(i, 2))
            return j;
    return -1;
}

// ----------------------------------------------------------------------------
// storage <-> arithmetic precision
// ----------------------------------------------------------------------------
template <typename R, typename S>
__device__ __forceinline__ R ld(const S *p)
{
    return static_cast<R>(*p);
}

template <typename S, typename R>
__device__ __forceinline__ void st(S *p, R v)
{
    *p = static_cast<S>(v);
}

// Post-collision PDFs are read again only in the next time step, after the
// whole grid has streamed through the caches: stored with the non-temporal
// hint (a vector store that does not keep the line in the caches), which
// raised the stream kernels' bandwidth by about a tenth on MI355X.  Fields
// (u, phi, T) are re-read by the next kernel of the same step and use st().
template <typename S, typename R>
__device__ __forceinline__ void st_pdf(S *p, R v)
{
    __builtin_nontemporal_store(static_cast<S>(v), p);
}

// ----------------------------------------------------------------------------
// D3Q27 index of the offset (dx, dy, dz)
__host__ __device__ constexpr int index_of(int dx, int dy, int dz)
{
    for (int i = 0; i < 27; ++i)
        if (vel27(i, 0) == dx && vel27(i, 1) == dy && vel27(i, 2) == dz) return i;
    return -1;
}

// ----------------------------------------------------------------------------
// geometry and neighbour addressing
// ----------------------------------------------------------------------------
struct Geometry {
    int nx, ny, nz;
    int walls;     // 1: no-slip walls at y = -1/2 and y = ny - 1/2
    int nbx;       // blocks of 64 cells per x-row in the PDF layout: ceil(nx / 64)
    int64_t N;     // nx*ny*nz
    int64_t plane; // nx*ny
};

// Element `idx` of an array that starts at `base`.  Every field or PDF component
// array is limited to 4 GiB (checked at creation), so the byte offset fits in 32
// bits and the load or store uses a uniform base register plus a 32-bit lane
// offset instead of per-lane 64-bit address arithmetic.
template <typename S>
__device__ __forceinline__ const S *elem(const S *base, uint32_t idx)
{
    return reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + (uint32_t)(idx * (uint32_t)sizeof(S)));
}
template <typename S>
__device__ __forceinline__ S *elem(S *base, uint32_t idx)
{
    return reinterpret_cast<S *>(reinterpret_cast<char *>(base) + (uint32_t)(idx * (uint32_t)sizeof(S)));
}

// Offsets of the 3x3x3 neighbourhood of one cell.  Periodic wrap in x and z
// (and y when there are no walls).  With walls, rows beyond the walls are
// clamped onto the wall-adjacent row and flagged so callers apply their
// boundary rule.
struct Nbr {
    uint32_t xo[3]; // x-1, x, x+1 (wrapped)
    uint32_t yr[3]; // y-1, y, y+1 (wrapped or clamped)
    uint32_t yo[3]; // row offsets yr * nx
    uint32_t zo[3]; // plane offsets of z-1, z, z+1 (wrapped)
    uint32_t zi[3]; // z-1, z, z+1 (wrapped)
    uint32_t c;     // own linear index
    bool below;     // y == 0 with a wall below
    bool above;     // y == ny-1 with a wall above

    __device__ __forceinline__ Nbr(const Geometry &g, int x, int y, int z)
    {
        xo[0] = x == 0 ? g.nx - 1 : x - 1;
        xo[1] = x;
        xo[2] = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? (g.walls ? 0 : g.ny - 1) : y - 1;
        const int yp = y == g.ny - 1 ? (g.walls ? g.ny - 1 : 0) : y + 1;
        yr[0] = (uint32_t)ym;
        yr[1] = (uint32_t)y;
        yr[2] = (uint32_t)yp;
        for (int k = 0; k < 3; ++k) yo[k] = yr[k] * (uint32_t)g.nx;
        zi[0] = z == 0 ? g.nz - 1 : z - 1;
        zi[1] = z;
        zi[2] = z == g.nz - 1 ? 0 : z + 1;
        for (int k = 0; k < 3; ++k) zo[k] = zi[k] * (uint32_t)g.plane;
        c = xo[1] + yo[1] + zo[1];
        below = g.walls && y == 0;
        above = g.walls && y == g.ny - 1;
    }
    // index of the cell at offset (dx, dy, dz)
    __device__ __forceinline__ uint32_t at(int dx, int dy, int dz) const
    {
        return xo[dx + 1] + yo[dy + 1] + zo[dz + 1];
    }
    // element of a field at offset (dx, dy, dz): a wave-uniform row pointer
    // (y and z are the same across a wavefront) plus one of the three per-lane
    // x offsets, so a 27-point stencil costs no per-lane address arithmetic
    template <typename T>
    __device__ __forceinline__ T *ptr(T *base, int dx, int dy, int dz) const
    {
        return elem(base + (yo[dy + 1] + zo[dz + 1]), xo[dx + 1]);
    }
    // true when the offset dy leaves the fluid through a wall
    __device__ __forceinline__ bool ghost(int dy) const
    {
        return (dy < 0 && below) || (dy > 0 && above);
    }
    // phi beyond a wall (dy crossing it) from the wall-adjacent value v: the
    // contact-angle ghost v + wet v (1 - v), wet = (4/xi) cos(theta) of that wall
    template <typename R>
    __device__ __forceinline__ R phi_ghost(R v, int dy, const double (&wet)[2]) const
    {
        return v + R(dy < 0 ? wet[0] : wet[1]) * v * (R(1) - v);
    }
    // wall-column index x + nx*z of the neighbour at (dx, dz)
    __device__ __forceinline__ uint32_t col(int dx, int dz, const Geometry &g) const
    {
        return xo[dx + 1] + zi[dz + 1] * (uint32_t)g.nx;
    }
    // A field on the 3x3x3 neighbourhood of the cell, in D3Q27 order (rows
    // beyond a wall are the clamped own row, as ptr()).  (Taking the x - 1
    // and x + 1 values from the neighbouring lanes of one row load, with DPP
    // wave shifts, loads 18 instead of 27 values but made the fused FP32 step
    // 6 % slower on MI355X; loads it is.)
    template <typename R, typename S>
    __device__ __forceinline__ void stencil27(const S *f, R (&v)[27]) const
    {
#pragma unroll
        for (int k = 0; k < 27; ++k) v[k] = ld<R>(ptr(f, vel27(k, 0), vel27(k, 1), vel27(k, 2)));
    }
};

// ----------------------------------------------------------------------------
// PDF layout.  Fields are plain arrays (x fastest).  PDF arrays are blocked:
// each x-row (y, z) holds nbx = ceil(nx/64) blocks of 64 cells, and within a
// block the Q components follow each other as runs of 64 values, so component
// i of cell (x, y, z) sits at
//     ((y + ny z) nbx + x/64) 64 Q + 64 i + x%64.
// A kernel touching Q components then streams from one contiguous region per
// block instead of from Q regions a whole grid apart, which a 27-component copy
// runs a quarter faster with.  A wavefront updates the 64 cells of one block
// (one row), so the row part of every address is wave-uniform (scalar
// registers) and the per-lane part is one of three offsets, for x-1, x, x+1.
// ----------------------------------------------------------------------------
inline int64_t pdf_elems(const Geometry &g, int q) { return (int64_t)g.nbx * 64 * q * g.ny * g.nz; }

template <int Q>
__host__ __device__ __forceinline__ int64_t pdf_index(const Geometry &g, int x, int y, int z, int i)
{
    return ((int64_t)(y + (int64_t)g.ny * z) * g.nbx + (x >> 6)) * (64 * Q) + 64 * i + (x & 63);
}

// per-lane offsets, within a row, of the cells x-1, x, x+1
template <int Q>
struct PdfLanes {
    uint32_t xq[3];
    __device__ __forceinline__ explicit PdfLanes(const Nbr &nb)
    {
        for (int k = 0; k < 3; ++k) xq[k] = (nb.xo[k] >> 6) * (64u * Q) + (nb.xo[k] & 63u);
    }
};

// start of component i of row (y, z): wave-uniform
template <int Q, typename P>
__device__ __forceinline__ P *pdf_row(P *base, const Geometry &g, uint32_t y, uint32_t z, int i)
{
    return base + ((int64_t)(y + (uint32_t)g.ny * z) * g.nbx * (64 * Q) + 64 * i);
}

// ----------------------------------------------------------------------------
// Work-group order.
//
// A work-group updates one kTX x kTY tile of one z plane, one cell per thread.
// The hardware deals work-groups to the eight XCDs (each with its own L2)
// round-robin by linear id.  The id is remapped so that every XCD receives one
// contiguous run of tiles, ordered z fastest within a chunk of kTZ planes,
// then x, then y, then the chunk: the work-groups that read the same phi and T
// stencil planes (z neighbours) and the same edge cache lines of the pulled
// PDFs (x neighbours) then run at the same time in the same L2.
// ----------------------------------------------------------------------------
constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kTZ = 16;
constexpr int kXCD = 8;

struct Tiling {
    int tiles_x, tiles_y, chunks_z;
    int total;   // kTZ * tiles_x * tiles_y * chunks_z work-groups with a tile
    int per_xcd; // total rounded up to a multiple of kXCD, divided by kXCD
};

inline Tiling make_tiling(const Geometry &g)
{
    Tiling t;
    t.tiles_x = (g.nx + kTX - 1) / kTX;
    t.tiles_y = (g.ny + kTY - 1) / kTY;
    t.chunks_z = (g.nz + kTZ - 1) / kTZ;
    t.total = kTZ * t.tiles_x * t.tiles_y * t.chunks_z;
    t.per_xcd = (t.total + kXCD - 1) / kXCD;
    return t;
}

inline dim3 tiling_grid(const Tiling &t) { return dim3((unsigned)(t.per_xcd * kXCD), 1, 1); }
inline dim3 tiling_block() { return dim3(kTX, kTY, 1); }

// Tiling of the kernels that march a 64 x 4 tile up a column of kMarchZ
// planes, staging each plane of their stencil field with a one-cell halo in x
// and y in LDS (three planes held at a time): each input is read from memory
// about (66 x 6) / (64 x 4) = 1.55 times and the stencil comes from LDS.
// Tiles are ordered x fastest, then y, then the column, XCD-aware as above.
constexpr int kMarchZ = 16;
constexpr int kHX = kTX + 2, kHY = kTY + 2;
constexpr int kHalo = kHX * kHY; // 396 cells per staged plane

struct March {
    int tiles_x, tiles_y, chunks_z;
    int total, per_xcd;
};

inline March make_march(const Geometry &g)
{
    March m;
    m.tiles_x = (g.nx + kTX - 1) / kTX;
    m.tiles_y = (g.ny + kTY - 1) / kTY;
    m.chunks_z = (g.nz + kMarchZ - 1) / kMarchZ;
    m.total = m.tiles_x * m.tiles_y * m.chunks_z;
    m.per_xcd = (m.total + kXCD - 1) / kXCD;
    return m;
}

inline dim3 march_grid(const March &m) { return dim3((unsigned)(m.per_xcd * kXCD), 1, 1); }

__host__ __device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// origin of this work-group's tile and the end of its column; false for a
// padding work-group (uniform across the work-group: it reaches no barrier)
__device__ __forceinline__ bool march_tile(const March &m, const Geometry &g, int &x0, int &y0, int &z0, int &z1)
{
    const int w = blockIdx.x;
    const int L = (w % kXCD) * m.per_xcd + w / kXCD;
    if (L >= m.total) return false;
    const int r = L / m.tiles_x;
    x0 = (L % m.tiles_x) * kTX;
    y0 = (r % m.tiles_y) * kTY;
    z0 = (r / m.tiles_y) * kMarchZ;
    z1 = z0 + kMarchZ < g.nz ? z0 + kMarchZ : g.nz;
    return true;
}

// cell index of halo entry i of the plane zz staged by the tile at (x0, y0);
// false for halo rows beyond a wall (never read)
__device__ __forceinline__ bool halo_cell(const Geometry &g, int x0, int y0, int zz, int i, uint32_t &c)
{
    const int gx = wrap(x0 - 1 + i % kHX, g.nx);
    int gy = y0 - 1 + i / kHX;
    if (gy < 0 || gy >= g.ny) {
        if (g.walls) return false;
        gy = wrap(gy, g.ny);
    }
    c = (uint32_t)gx + (uint32_t)gy * (uint32_t)g.nx + (uint32_t)zz * (uint32_t)g.plane;
    return true;
}

// The halo entries a thread stages in the marching kernels (tid and
// tid + 256: kHalo = 396 entries over 256 threads), as offsets within a plane,
// worked out once per work-group: `own` marks an entry of the halo, `in` one
// with a cell to load (not in a row beyond a wall).
constexpr int kHaloPer = (kHalo + kTX * kTY - 1) / (kTX * kTY);
struct HaloSlots {
    uint32_t off[kHaloPer];
    bool own[kHaloPer], in[kHaloPer];
    __device__ __forceinline__ HaloSlots(const Geometry &g, int x0, int y0, int tid)
    {
#pragma unroll
        for (int j = 0; j < kHaloPer; ++j) {
            const int i = tid + j * kTX * kTY;
            uint32_t c = 0;
            own[j] = i < kHalo;
            in[j] = own[j] && halo_cell(g, x0, y0, 0, i, c);
            off[j] = c;
        }
    }
};

// Tile of this work-group in the mapping of cell_of_thread: origin (x0, y0)
// and plane z; false for a padding work-group or a plane beyond the grid
// (both uniform across the work-group).
__device__ __forceinline__ bool tile_of_block(const Tiling &t, const Geometry &g, int &x0, int &y0, int &z)
{
    const int w = blockIdx.x;
    const int L = (w % kXCD) * t.per_xcd + w / kXCD;
    if (L >= t.total) return false;
    const int zz = L % kTZ;
    int r = L / kTZ;
    x0 = (r % t.tiles_x) * kTX;
    r /= t.tiles_x;
    y0 = (r % t.tiles_y) * kTY;
    z = (r / t.tiles_y) * kTZ + zz;
    return z < g.nz;
}

// Cell of this thread; false for padding work-groups and cells outside the grid.
// A wavefront is one x-row of a tile (64 threads with the same threadIdx.y), so
// y and z are wave-uniform; y is read through readfirstlane to tell the compiler.
static_assert(kTX == 64, "a wavefront must cover exactly one 64-cell block of a row");
__device__ __forceinline__ bool cell_of_thread(const Tiling &t, const Geometry &g, int &x, int &y, int &z)
{
    const int w = blockIdx.x;
    const int L = (w % kXCD) * t.per_xcd + w / kXCD;
    if (L >= t.total) return false;
    const int zz = L % kTZ;
    int r = L / kTZ;
    const int tx = r % t.tiles_x;
    r /= t.tiles_x;
    const int ty = r % t.tiles_y;
    const int cz = r / t.tiles_y;
    x = tx * kTX + threadIdx.x;
    y = ty * kTY + __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    z = cz * kTZ + zz;
    return x < g.nx && y < g.ny && z < g.nz;
}

// ----------------------------------------------------------------------------
// heat sources (Eq. HeatSource)
// ----------------------------------------------------------------------------
constexpr int kMaxSources = 16;

struct HeatSources {
    int n;
    double Q[kMaxSources], x[kMaxSources], y[kMaxSources], z[kMaxSources];
    double inv_w2[kMaxSources], dcut2[kMaxSources]; // dcut2 <= 0: no cut-off
};

template <typename R>
__device__ __forceinline__ R heat_source(const HeatSources &hs, int x, int y, int z)
{
    R q = R(0);
    for (int k = 0; k < hs.n; ++k) {
        R dx = R(x) - R(hs.x[k]), dy = R(y) - R(hs.y[k]), dz = R(z) - R(hs.z[k]);
        R d2 = dx * dx + dy * dy + dz * dz;
        if (hs.dcut2[k] > 0.0 && d2 > R(hs.dcut2[k])) continue;
        q += R(hs.Q[k]) * exp(R(-2) * d2 * R(hs.inv_w2[k]));
    }
    return q;
}

// ----------------------------------------------------------------------------
// Inverse central-moment transform restricted to the first-order moments.
//
// All moments of order >= 2 of the phase-field and thermal collisions relax
// with rate one, so f* = f_eq + S/2 + d where d is the unique PDF vector whose
// central moments (basis of the stencil, about u) are zero except the three
// first-order ones, which equal v.  The functions below build d from its raw
// moments (found from the central ones by the binomial shift, which is
// triangular in the polynomial degree) followed by the constant inverse of
// the raw-moment matrix of the stencil.
// ----------------------------------------------------------------------------
template <int Q, typename R>
struct FirstOrder;

template <typename R>
struct FirstOrder<7, R> {
    __host__ __device__ __forceinline__ static void apply(const R u[3], const R v[3], R d[7])
    {
        d[0] = R(-2) * (u[0] * v[0] + u[1] * v[1] + u[2] * v[2]);
        d[1] = v[1] * (u[1] + R(0.5));
        d[2] = v[1] * (u[1] - R(0.5));
        d[3] = v[0] * (u[0] - R(0.5));
        d[4] = v[0] * (u[0] + R(0.5));
        d[5] = v[2] * (u[2] + R(0.5));
        d[6] = v[2] * (u[2] - R(0.5));
    }
};

template <typename R>
struct FirstOrder<15, R> {
    __host__ __device__ __forceinline__ static void apply(const R u[3], const R v[3], R d[15])
    {
        const R ux = u[0], uy = u[1], uz = u[2], vx = v[0], vy = v[1], vz = v[2];
        // raw moments of d
        const R rxx = R(2) * ux * vx, ryy = R(2) * uy * vy, rzz = R(2) * uz * vz;
        const R rxy = ux * vy + uy * vx, rxz = ux * vz + uz * vx, ryz = uy * vz + uz * vy;
        const R rxyy = uy * uy * vx + R(2) * ux * uy * vy;
        const R ryzz = uz * uz * vy + R(2) * uy * uz * vz;
        const R rzxx = ux * ux * vz + R(2) * uz * ux * vx;
        const R rxyz = uy * uz * vx + ux * uz * vy + ux * uy * vz;
        // x^2 y^2 row: on this lattice x^2 y coincides with y z^2
        const R rxxyy = R(-2) * ux * uy * uy * vx + R(2) * uy * uz * uz * vy + R(4) * uy * uy * uz * vz;
        // inverse of the raw-moment matrix: corners by a Walsh-Hadamard sum
#pragma unroll
        for (int k = 7; k < 15; ++k) {
            const R sx = R(vel<15>(k, 0)), sy = R(vel<15>(k, 1)), sz = R(vel<15>(k, 2));
            d[k] = R(0.125) * (rxxyy + sx * rxyy + sy * ryzz + sz * rzxx + sx * sy * rxy + sx * sz * rxz +
                               sy * sz * ryz + sx * sy * sz * rxyz);
        }
        const R ex = rxx - rxxyy, ox = vx - rxyy;
        const R ey = ryy - rxxyy, oy = vy - ryzz;
        const R ez = rzz - rxxyy, oz = vz - rzxx;
        d[4] = R(0.5) * (ex + ox);
        d[3] = R(0.5) * (ex - ox);
        d[1] = R(0.5) * (ey + oy);
        d[2] = R(0.5) * (ey - oy);
        d[5] = R(0.5) * (ez + oz);
        d[6] = R(0.5) * (ez - oz);
        d[0] = R(2) * rxxyy - (rxx + ryy + rzz);
    }
};

template <typename R>
struct FirstOrder<19, R> {
    __host__ __device__ __forceinline__ static void apply(const R u[3], const R v[3], R d[19])
    {
        const R ux = u[0], uy = u[1], uz = u[2], vx = v[0], vy = v[1], vz = v[2];
        // the D3Q19 basis is closed under taking factors, so every raw moment
        // of d is v . grad_u of the monomial evaluated at u
        const R rxx = R(2) * ux * vx, ryy = R(2) * uy * vy, rzz = R(2) * uz * vz;
        const R rxy = ux * vy + uy * vx, rxz = ux * vz + uz * vx, ryz = uy * vz + uz * vy;
        const R rxxy = R(2) * ux * uy * vx + ux * ux * vy, rxyy = uy * uy * vx + R(2) * ux * uy * vy;
        const R rxxz = R(2) * ux * uz * vx + ux * ux * vz, rxzz = uz * uz * vx + R(2) * ux * uz * vz;
        const R ryyz = R(2) * uy * uz * vy + uy * uy * vz, ryzz = uz * uz * vy + R(2) * uy * uz * vz;
        const R rxxyy = R(2) * ux * uy * uy * vx + R(2) * ux * ux * uy * vy;
        const R rxxzz = R(2) * ux * uz * uz * vx + R(2) * ux * ux * uz * vz;
        const R ryyzz = R(2) * uy * uz * uz * vy + R(2) * uy * uy * uz * vz;
#pragma unroll
        for (int k = 7; k < 19; ++k) {
            const int sx = vel<19>(k, 0), sy = vel<19>(k, 1), sz = vel<19>(k, 2);
            R val;
            if (sz == 0) // xy edges
                val = rxxyy + R(sx) * rxyy + R(sy) * rxxy + R(sx * sy) * rxy;
            else if (sy == 0) // xz edges
                val = rxxzz + R(sx) * rxzz + R(sz) * rxxz + R(sx * sz) * rxz;
            else // yz edges
                val = ryyzz + R(sy) * ryzz + R(sz) * ryyz + R(sy * sz) * ryz;
            d[k] = R(0.25) * val;
        }
        const R ex = rxx - rxxyy - rxxzz, ox = vx - rxyy - rxzz;
        const R ey = ryy - rxxyy - ryyzz, oy = vy - rxxy - ryzz;
        const R ez = rzz - rxxzz - ryyzz, oz = vz - rxxz - ryyz;
        d[4] = R(0.5) * (ex + ox);
        d[3] = R(0.5) * (ex - ox);
        d[1] = R(0.5) * (ey + oy);
        d[2] = R(0.5) * (ey - oy);
        d[5] = R(0.5) * (ez + oz);
        d[6] = R(0.5) * (ez - oz);
        d[0] = (rxxyy + rxxzz + ryyzz) - (rxx + ryy + rzz);
    }
};

// D3Q27: the moment matrix is the tensor product of three 3x3 matrices
// (c - u)^p, p = 0..2, c = -1, 0, 1, so its inverse factorises; m_p(c) below is
// column p of the 1-D inverse evaluated at lattice coordinate c.
template <typename R>
struct Axis1D {
    R m0[3], m1[3], m2[3]; // index c + 1
    __host__ __device__ __forceinline__ explicit Axis1D(R u)
    {
        const R u2 = u * u;
        m0[1] = R(1) - u2;
        m0[0] = R(0.5) * (u2 - u);
        m0[2] = R(0.5) * (u2 + u);
        m1[1] = R(-2) * u;
        m1[0] = u - R(0.5);
        m1[2] = u + R(0.5);
        m2[1] = R(-1);
        m2[0] = R(0.5);
        m2[2] = R(0.5);
    }
};

template <typename R>
struct FirstOrder<27, R> {
    __host__ __device__ __forceinline__ static void apply(const R u[3], const R v[3], R d[27])
    {
        const Axis1D<R> X(u[0]), Y(u[1]), Z(u[2]);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int a = vel27(i, 0) + 1, b = vel27(i, 1) + 1, c = vel27(i, 2) + 1;
            d[i] = v[0] * X.m1[a] * Y.m0[b] * Z.m0[c] + v[1] * X.m0[a] * Y.m1[b] * Z.m0[c] +
                   v[2] * X.m0[a] * Y.m0[b] * Z.m1[c];
        }
    }
};

} // namespace tcp
