// Host side of the C ABI declared in include/spdhg.h: validation, geometry tables,
// workspace layout, step sizes (Theorem 2), the SPDHG iteration driver (Algorithm 2),
// objective and checkpoints.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/spdhg.h"
#include "kernels.hip"

using namespace spdhg;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(SPDHG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

#define LAUNCH_CHECK()                                                                  \
    do {                                                                                \
        hipError_t _e = hipGetLastError();                                              \
        if (_e != hipSuccess)                                                           \
            return fail(SPDHG_E_HIP, std::string("kernel launch: ") + hipGetErrorString(_e)); \
    } while (0)

inline unsigned nblocks(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// ---------------------------------------------------------------- recordable launches
// The kernels of the SPDHG iteration are launched through klaunch, which either enqueues
// the launch or, while a Recorder is installed on the calling thread, records it (kernel,
// launch shape and a copy of the argument values) for a persistent epoch graph, whose
// nodes then receive exactly the arguments an eager run would launch with.
struct LaunchRec {
    const void* func = nullptr;
    dim3 grid, block;
    unsigned lds = 0;
    std::shared_ptr<void> vals;  // a std::tuple of the kernel's parameter values
    std::vector<void*> ptrs;     // pointers to its elements (kernel node parameters)
};

struct Recorder {
    std::vector<LaunchRec> recs;
    std::vector<size_t> marks;  // recs.size() at the start of each iteration
};

thread_local Recorder* g_rec = nullptr;

template <typename Tup, size_t... I>
void tuple_ptrs(Tup& t, void** out, std::index_sequence<I...>) {
    ((out[I] = (void*)&std::get<I>(t)), ...);
}

template <typename... KP, typename... A>
int klaunch(void (*k)(KP...), dim3 grid, dim3 block, size_t lds, hipStream_t st, A&&... a) {
    static_assert(sizeof...(KP) == sizeof...(A), "kernel argument count");
    using Tup = std::tuple<std::decay_t<KP>...>;
    if (g_rec) {
        auto t = std::make_shared<Tup>(std::forward<A>(a)...);
        LaunchRec r;
        r.func = (const void*)k;
        r.grid = grid;
        r.block = block;
        r.lds = (unsigned)lds;
        r.ptrs.resize(sizeof...(KP));
        tuple_ptrs(*t, r.ptrs.data(), std::index_sequence_for<KP...>{});
        r.vals = t;
        g_rec->recs.push_back(std::move(r));
        return SPDHG_OK;
    }
    Tup t(std::forward<A>(a)...);
    std::array<void*, sizeof...(KP)> p;
    tuple_ptrs(t, p.data(), std::index_sequence_for<KP...>{});
    HIP_TRY(hipLaunchKernel((const void*)k, grid, block, p.data(), lds, st));
    return SPDHG_OK;
}

int64_t n_planes(const spdhg_geom* g) {
    int64_t n = 0;
    for (int i = 0; i < g->n_seg; ++i) n += g->seg_planes[i];
    return n;
}

// Ring difference of segment i in the order 0, +1, -1, +2, -2, ...
int ring_diff(int i) { return i == 0 ? 0 : ((i + 1) / 2) * (i % 2 ? 1 : -1); }

// Data planes of a sinogram row: the segments' planes, or with span compression the
// planes of the data segments 0, +-1, .. (data segment G: ring sums from G span -
// (span-1)/2 to 2 (rings - 1) minus that; it exists while that smallest |d| is present).
int64_t n_data_planes(const spdhg_geom* g) {
    if (g->span == 0) return n_planes(g);
    const int h = (g->span - 1) / 2;
    int dmax = 0;
    for (int i = 0; i < g->n_seg; ++i) dmax = std::max(dmax, std::abs(ring_diff(i)));
    int64_t n = g->nz;
    for (int G = 1; G * g->span - h <= dmax; ++G) n += 2 * (g->nz - 2 * (G * g->span - h));
    return n;
}

// Largest |bin angle| of the non-arc-corrected sampling, (n_rad - 1) / 2 d_rad / R.
double max_bin_angle(const spdhg_geom* g) { return 0.5 * (g->n_rad - 1) * g->d_rad / g->det_radius; }

int check_geom(const spdhg_geom* g) {
    if (!g) return fail(SPDHG_E_ARG, "geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->n_rad <= 0 || g->n_ang <= 0)
        return fail(SPDHG_E_SHAPE, "geometry sizes must be positive");
    if (!(g->vx > 0) || !(g->vy > 0) || !(g->vz > 0) || !(g->d_rad > 0))
        return fail(SPDHG_E_SHAPE, "voxel sizes and radial spacing must be positive");
    if (g->n_seg <= 0 || g->n_seg > SPDHG_MAX_SEG)
        return fail(SPDHG_E_SHAPE, "n_seg out of range");
    for (int i = 0; i < g->n_seg; ++i) {
        const int pitch = g->seg_pitch[i] == 0 ? 1 : g->seg_pitch[i];
        if (pitch != 1 && pitch != 2) return fail(SPDHG_E_SHAPE, "segment pitch must be 1 or 2");
        const int64_t span = 1 + (int64_t)pitch * ((int64_t)g->seg_planes[i] - 1);
        if (g->seg_planes[i] <= 0 || span > g->nz || ((g->nz - span) & 1))
            return fail(SPDHG_E_SHAPE,
                        "segment plane count N must be >= 1 with nz - 1 - pitch (N - 1) even "
                        "and >= 0");
        if (!std::isfinite(g->seg_tan[i])) return fail(SPDHG_E_SHAPE, "segment slope not finite");
    }
    if (g->nonarc || g->oblique_s) {
        if (!(g->det_radius > 0) || !std::isfinite(g->det_radius))
            return fail(SPDHG_E_SHAPE, "the scanner model needs det_radius > 0");
        if (g->nonarc ? !(max_bin_angle(g) < 1.5) : !(0.5 * (g->n_rad - 1) * g->d_rad < g->det_radius * 0.997))
            return fail(SPDHG_E_SHAPE, "radial bins reach the detector ring");
    }
    if (g->span != 0) {
        if (g->span < 3 || !(g->span & 1)) return fail(SPDHG_E_SHAPE, "span must be odd and >= 3");
        const int rings = g->seg_planes[0];
        if (g->nz != 2 * rings - 1) return fail(SPDHG_E_SHAPE, "span compression needs nz = 2 rings - 1");
        for (int i = 0; i < g->n_seg; ++i) {
            const int pitch = g->seg_pitch[i] == 0 ? 1 : g->seg_pitch[i];
            if (pitch != 2 || g->seg_planes[i] != rings - std::abs(ring_diff(i)))
                return fail(SPDHG_E_SHAPE,
                            "span compression needs the ring-pair segments 0, +1, -1, ... at pitch 2");
        }
    }
    const double nv = (double)g->nx * g->ny * g->nz;
    const double nb = (double)g->n_ang * (double)n_data_planes(g) * g->n_rad;
    if (nv > 4.0e9 || nb > 8.0e9) return fail(SPDHG_E_SHAPE, "problem too large");
    if (g->nx > 16384 || g->ny > 16384 || g->nz > 16384 || g->n_rad > 1 << 20)
        return fail(SPDHG_E_SHAPE, "dimension too large for FP32 index arithmetic");
    return SPDHG_OK;
}

// Host-side tables: per-angle sampling coefficients, per-(angle, segment) axial
// coefficients (FP64) and FP32 step lengths, plane -> segment map.
struct HostTables {
    std::vector<AngleDev> ang;
    std::vector<SegAngleDev> sa;
    std::vector<int32_t> plane_seg;
    std::vector<double> kpos, kobl;     // scanner model (empty when off)
    std::vector<float> kL;
    std::vector<int32_t> cstart, clist; // span compression (empty when off)
    GeomDev G;
};

void build_tables(const spdhg_geom* g, HostTables& T) {
    const double pi = 3.14159265358979323846;
    const int na = g->n_ang, ns = g->n_seg;
    T.ang.resize(na);
    T.sa.resize((size_t)na * ns);
    for (int a = 0; a < na; ++a) {
        const double phi = pi * (double)a / (double)na;
        const double c = std::cos(phi), s = std::sin(phi);
        const bool rowdom = (4 * a <= na) || (4 * a >= 3 * na);
        AngleDev A{};
        double dt_dj, dt_dk, L;
        if (rowdom) {
            const double sec = 1.0 / c, tn = s / c;
            A.du_dk = g->d_rad * sec / g->vx;
            A.du_dj = -tn * g->vy / g->vx;
            A.cu = 0.5 * (g->nx - 1);
            A.cj = 0.5 * (g->ny - 1);
            A.n_prim = g->ny;
            A.n_sec = g->nx;
            dt_dj = g->vy * sec;
            dt_dk = -g->d_rad * tn;
            L = g->vy * std::fabs(sec);
        } else {
            const double csc = 1.0 / s, ct = c / s;
            A.du_dk = g->d_rad * csc / g->vy;
            A.du_dj = -ct * g->vx / g->vy;
            A.cu = 0.5 * (g->ny - 1);
            A.cj = 0.5 * (g->nx - 1);
            A.n_prim = g->nx;
            A.n_sec = g->ny;
            dt_dj = -g->vx * csc;
            dt_dk = g->d_rad * ct;
            L = g->vx * std::fabs(csc);
        }
        A.rowdom = rowdom ? 1 : 0;
        T.ang[a] = A;
        for (int sg = 0; sg < ns; ++sg) {
            const double tau = g->seg_tan[sg];
            SegAngleDev S{};
            S.ez_dj = tau / g->vz * dt_dj;
            S.ez_dk = tau / g->vz * dt_dk;
            S.L = (float)(L * std::sqrt(1.0 + tau * tau));
            T.sa[(size_t)a * ns + sg] = S;
        }
    }
    GeomDev& G = T.G;
    memset(&G, 0, sizeof(G));
    G.nx = g->nx;
    G.ny = g->ny;
    G.nz = g->nz;
    G.n_rad = g->n_rad;
    G.n_ang = na;
    G.n_seg = ns;
    G.ck = 0.5 * (g->n_rad - 1);
    int base = 0;
    for (int sg = 0; sg < ns; ++sg) {
        const int pitch = g->seg_pitch[sg] == 0 ? 1 : g->seg_pitch[sg];
        G.seg_planes[sg] = g->seg_planes[sg];
        G.seg_base[sg] = base;
        G.seg_pitch[sg] = pitch;
        G.seg_off[sg] = (g->nz - 1 - pitch * (g->seg_planes[sg] - 1)) / 2;
        for (int p = 0; p < g->seg_planes[sg]; ++p) T.plane_seg.push_back(sg);
        base += g->seg_planes[sg];
    }
    G.n_planes = base;
    G.n_dplanes = base;
    G.dstride = 1;
    for (int sg = 0; sg < ns; ++sg) G.seg_dbase[sg] = G.seg_base[sg];

    // scanner model: centred radial coordinates s_k / d_rad, slope factors R / sqrt(R^2 -
    // s_k^2), step-length factors sqrt(1 + tau^2 f^2) / sqrt(1 + tau^2)
    if (g->nonarc || g->oblique_s) {
        const double R = g->det_radius;
        T.kpos.resize(g->n_rad);
        T.kobl.assign(g->n_rad, 1.0);
        for (int k = 0; k < g->n_rad; ++k) {
            const double t = ((double)k - G.ck) * g->d_rad;
            const double sk = g->nonarc ? R * std::sin(t / R) : t;
            T.kpos[k] = sk / g->d_rad;
            if (g->oblique_s) T.kobl[k] = R / std::sqrt(R * R - sk * sk);
        }
        if (g->oblique_s) {
            T.kL.resize((size_t)ns * g->n_rad);
            for (int sg = 0; sg < ns; ++sg)
                for (int k = 0; k < g->n_rad; ++k) {
                    const double tau = g->seg_tan[sg], f = T.kobl[k];
                    T.kL[(size_t)sg * g->n_rad + k] =
                        (float)(std::sqrt(1.0 + tau * tau * f * f) / std::sqrt(1.0 + tau * tau));
                }
        } else {
            T.kobl.clear();
        }
        if (g->nonarc) G.krho = R / g->d_rad;
    }

    // span compression: ring-pair plane p of segment i (ring difference d, rings
    // (p, p + |d|) in some order, ring sum 2p + |d|) belongs to data segment G = (|d| + h)
    // / span (sign of d; h = (span - 1) / 2) at its ring sum minus the segment's smallest,
    // G span - h (0 for G = 0): data element dbase_i + 2p
    if (g->span != 0) {
        const int h = (g->span - 1) / 2;
        const int64_t nd = n_data_planes(g);
        std::vector<int> dstart;  // first data plane of data segment j (order 0, +1, -1, ..)
        int64_t acc = 0;
        for (int Gs = 0; acc < nd; ++Gs) {
            const int n = g->nz - 2 * (Gs == 0 ? 0 : Gs * g->span - h);
            dstart.push_back((int)acc);
            acc += n;
            if (Gs > 0) {
                dstart.push_back((int)acc);
                acc += n;
            }
        }
        std::vector<int32_t> owner(base);
        for (int sg = 0; sg < ns; ++sg) {
            const int d = ring_diff(sg), ad = std::abs(d);
            const int Gs = (ad + h) / g->span;
            const int j = Gs == 0 ? 0 : (d > 0 ? 2 * Gs - 1 : 2 * Gs);
            const int smin = Gs == 0 ? 0 : Gs * g->span - h;
            G.seg_dbase[sg] = dstart[j] + ad - smin;
            for (int p = 0; p < g->seg_planes[sg]; ++p)
                owner[G.seg_base[sg] + p] = G.seg_dbase[sg] + 2 * p;
        }
        G.n_dplanes = (int32_t)nd;
        G.dstride = 2;
        // CSR: the ring-pair planes of each data plane, in increasing ring-pair plane order
        T.cstart.assign(nd + 1, 0);
        for (int q = 0; q < base; ++q) T.cstart[owner[q] + 1] += 1;
        for (int64_t q = 0; q < nd; ++q) T.cstart[q + 1] += T.cstart[q];
        T.clist.resize(base);
        std::vector<int32_t> fill(T.cstart.begin(), T.cstart.end() - 1);
        for (int q = 0; q < base; ++q) T.clist[fill[owner[q]]++] = q;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t table_bytes(const HostTables& T) {
    return align256(T.ang.size() * sizeof(AngleDev)) + align256(T.sa.size() * sizeof(SegAngleDev)) +
           align256(T.plane_seg.size() * sizeof(int32_t)) + align256(T.kpos.size() * 8) +
           align256(T.kobl.size() * 8) + align256(T.kL.size() * 4) + align256(T.cstart.size() * 4) +
           align256(T.clist.size() * 4);
}

// Copy the tables to `dev` (table_bytes long, device memory) on `st` and point G at them.
// The host vectors are pageable memory: each copy returns once HIP has staged the source,
// so they may be released after the call; the device copies are ordered on `st` before
// every kernel enqueued after them.
int upload_tables(HostTables& T, char* dev, hipStream_t st) {
    char* p = dev;
    HIP_TRY(hipMemcpyAsync(p, T.ang.data(), T.ang.size() * sizeof(AngleDev),
                           hipMemcpyHostToDevice, st));
    T.G.ang = (const AngleDev*)p;
    p += align256(T.ang.size() * sizeof(AngleDev));
    HIP_TRY(hipMemcpyAsync(p, T.sa.data(), T.sa.size() * sizeof(SegAngleDev),
                           hipMemcpyHostToDevice, st));
    T.G.sa = (const SegAngleDev*)p;
    p += align256(T.sa.size() * sizeof(SegAngleDev));
    HIP_TRY(hipMemcpyAsync(p, T.plane_seg.data(), T.plane_seg.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
    T.G.plane_seg = (const int32_t*)p;
    p += align256(T.plane_seg.size() * sizeof(int32_t));
    // optional tables (scanner model, span compression): NULL when empty
    auto put = [&](const void* src, size_t bytes) -> const void* {
        if (bytes == 0) return nullptr;
        void* dst = p;
        p += align256(bytes);
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess
                   ? dst : (const void*)-1;
    };
    T.G.kpos = (const double*)put(T.kpos.data(), T.kpos.size() * 8);
    T.G.kobl = (const double*)put(T.kobl.data(), T.kobl.size() * 8);
    T.G.kL = (const float*)put(T.kL.data(), T.kL.size() * 4);
    T.G.cstart = (const int32_t*)put(T.cstart.data(), T.cstart.size() * 4);
    T.G.clist = (const int32_t*)put(T.clist.data(), T.clist.size() * 4);
    for (const void* q : {(const void*)T.G.kpos, (const void*)T.G.kobl, (const void*)T.G.kL,
                          (const void*)T.G.cstart, (const void*)T.G.clist})
        if (q == (const void*)-1) return fail(SPDHG_E_HIP, "copying the scanner tables failed");
    return SPDHG_OK;
}

int subset_angles(const spdhg_geom* g, int32_t m, int32_t i, int& ang0, int& step, int& count) {
    if (i < 0) {
        ang0 = 0;
        step = 1;
        count = g->n_ang;
        return SPDHG_OK;
    }
    if (m <= 0 || m > g->n_ang || i >= m) return fail(SPDHG_E_ARG, "bad subset index");
    ang0 = i;
    step = m;
    count = (g->n_ang - i + m - 1) / m;
    return SPDHG_OK;
}

// SplitMix64 (Steele, Lea, Flood 2014), counter form: output k of a generator seeded
// with `seed` is mix(seed + (k + 1) * golden).
inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double grad_norm(int nx, int ny, int nz) {
    // largest singular value of forward differences with Neumann ends: the sum over axes
    // of the path-graph Laplacian maxima 4 sin^2(pi (N-1) / (2N))
    const double pi = 3.14159265358979323846;
    double s = 0.0;
    for (int n : {nx, ny, nz}) {
        const double v = std::sin(pi * (n - 1) / (2.0 * n));
        s += v * v;
    }
    return 2.0 * std::sqrt(s);
}

}  // namespace

namespace {

// Zero padding of the axial column in the forward kernel: every axial cell offset
// floor(e) of a sample inside the in-plane range satisfies |floor(e)| <= pad - 2, since
// |e| <= |ez_dj| (n_prim - 1) / 2 + |ez_dk| (n_rad - 1) / 2 (e is affine in the centred
// indices).
int axial_pad(const HostTables& T) {
    double m = 0.0;
    const int ns = T.G.n_seg;
    for (size_t a = 0; a < T.ang.size(); ++a)
        for (int g = 0; g < ns; ++g) {
            const SegAngleDev& S = T.sa[a * ns + g];
            m = std::max(m, std::fabs(S.ez_dj) * T.ang[a].cj + std::fabs(S.ez_dk) * T.G.ck);
        }
    // scanner model: |kpos| <= ck (|sin x| <= |x|), both coefficients scaled by kobl
    double f = 1.0;
    for (double v : T.kobl) f = std::max(f, v);
    return (int)std::ceil(m * f) + 2;
}

// Rays per lane of the forward kernel: smallest supported power of two >= planes / 64.
int rays_per_lane(int n_planes) {
    const int need = (n_planes + 63) / 64;
    for (int r : {1, 2, 4, 8, 16, 32, 64})
        if (r >= need) return r;
    return -1;
}

int check_kernel_limits(const spdhg_geom* g) {
    if (rays_per_lane((int)n_planes(g)) < 0)
        return fail(SPDHG_E_SHAPE, "more than 4096 sinogram planes");
    if (g->nz > 128) return fail(SPDHG_E_SHAPE, "nz above 128");
    // the forward walk addresses the image through 32-bit byte offsets below 1 GiB
    if ((int64_t)g->nx * g->ny * g->nz * 4 >= (int64_t(1) << 30))
        return fail(SPDHG_E_SHAPE, "image of 1 GiB or more");
    // the gather keeps at most 4 candidate radial bins per voxel column and angle: the
    // radial spacing must be at least half the in-plane voxel size
    if (g->d_rad < 0.5 * std::max(g->vx, g->vy))
        return fail(SPDHG_E_SHAPE, "radial spacing below half the voxel size");
    return SPDHG_OK;
}

// ---------------------------------------------------------------- launch helpers
// Whether the forward walk's RUN instances apply: every segment on consecutive image
// planes, at most 64 runs of FWD_RUN planes, and more than 256 planes (below that the
// interleaved instances have at most 4 rays per lane and the runs would leave most lanes
// idle).
bool walk_runs(const GeomDev& G) {
    if (G.n_planes <= 256) return false;
    int runs = 0;
    for (int g = 0; g < G.n_seg; ++g) {
        if (G.seg_pitch[g] != 1) return false;
        runs += (G.seg_planes[g] + FWD_RUN - 1) / FWD_RUN;
    }
    return runs <= 64;
}

template <int MODE, int NW>
int launch_fwd_nw(int rpl, const FwdArgs& A, int nblk, hipStream_t st) {
    // per wavefront: axial columns and segment tables, also the staging of its partial
    // ray sums (kernel: wstride)
    const size_t lds = NW * std::max<size_t>(2 * (size_t)A.gsize + 8 * (size_t)A.G.n_seg, 64) * 4;
    const int nt = 64 * NW;
    if (!A.interleave && walk_runs(A.G)) {
        // the RUN epilogue also stages the ray sums in plane order
        const size_t tbytes = (size_t)A.G.n_planes * 4;
        return klaunch(fwd_wave<FWD_RUN, MODE, NW, true>, nblk, nt, std::max(lds, tbytes), st,
                       A);
    }
    // the iteration and the objective also have a 14-row instance (837 planes of span 11
    // take 14 rows: no rows past the last plane)
    constexpr bool hot = MODE == F_DUAL || MODE == F_OBJ;
    if (hot && rpl == 16 && (A.G.n_planes + 63) / 64 >= 13 && (A.G.n_planes + 63) / 64 <= 14)
        rpl = 14;
    int rc = SPDHG_OK;
    switch (rpl) {
        case 1: rc = klaunch(fwd_wave<1, MODE, NW>, nblk, nt, lds, st, A); break;
        case 2: rc = klaunch(fwd_wave<2, MODE, NW>, nblk, nt, lds, st, A); break;
        case 4: rc = klaunch(fwd_wave<4, MODE, NW>, nblk, nt, lds, st, A); break;
        case 8: rc = klaunch(fwd_wave<8, MODE, NW>, nblk, nt, lds, st, A); break;
        case 14:
            if constexpr (hot) rc = klaunch(fwd_wave<14, MODE, NW>, nblk, nt, lds, st, A);
            break;
        case 16: rc = klaunch(fwd_wave<16, MODE, NW>, nblk, nt, lds, st, A); break;
        case 32:
            if constexpr (NW <= 4) rc = klaunch(fwd_wave<32, MODE, NW>, nblk, nt, lds, st, A);
            break;
        case 64:
            if constexpr (NW <= 4) rc = klaunch(fwd_wave<64, MODE, NW>, nblk, nt, lds, st, A);
            break;
        default: return fail(SPDHG_E_SHAPE, "unsupported plane count");
    }
    return rc;
}

// Plane-split forward: PS wavefronts per ray bundle, each with RPL rays per lane.
template <int MODE, int PS>
int launch_fwd_ps(const FwdArgs& A, int nblk, hipStream_t st) {
    const size_t lds = (2 * (size_t)A.gsize + 8 * (size_t)A.G.n_seg) * 4;
    const int rpl = rays_per_lane((A.G.n_planes + PS - 1) / PS);
    switch (rpl) {
        case 1: return klaunch(fwd_bundle<1, MODE, PS>, nblk, 64 * PS, lds, st, A);
        case 2: return klaunch(fwd_bundle<2, MODE, PS>, nblk, 64 * PS, lds, st, A);
        case 4: return klaunch(fwd_bundle<4, MODE, PS>, nblk, 64 * PS, lds, st, A);
        case 8: return klaunch(fwd_bundle<8, MODE, PS>, nblk, 64 * PS, lds, st, A);
        case 16: return klaunch(fwd_bundle<16, MODE, PS>, nblk, 64 * PS, lds, st, A);
        default: return fail(SPDHG_E_SHAPE, "unsupported plane count for the plane split");
    }
}

// One block per (angle of the list, radial bin); launches with few blocks split every ray
// walk over 2, 4 or 8 wavefronts (a single angle has only n_rad ray bundles), unless
// A.split fixes the split (the autotuner's choice).
template <int MODE>
int launch_walk(FwdArgs A, int ang0, int step, int cnt, hipStream_t st) {
    A.ang0 = ang0;
    A.ang_step = step;
    A.n_ang_sub = cnt;
    const int64_t nblk = (int64_t)cnt * A.G.n_rad;
    if (nblk == 0) return SPDHG_OK;
    if (nblk > INT32_MAX) return fail(SPDHG_E_SHAPE, "too many rays");
    const int rpl = rays_per_lane(A.G.n_planes);
    if (A.split == 20) return launch_fwd_ps<MODE, 2>(A, (int)nblk, st);
    if (A.split == 40) return launch_fwd_ps<MODE, 4>(A, (int)nblk, st);
    int nw = A.split;
    if (nw != 1 && nw != 2 && nw != 4 && nw != 8)
        nw = nblk < 4 * 256 ? 8 : nblk < 16 * 256 ? 4 : nblk < 64 * 256 ? 2 : 1;
    if (nw == 8 && rpl > 16) nw = 4;
    switch (nw) {
        case 8: return launch_fwd_nw<MODE, 8>(rpl, A, (int)nblk, st);
        case 4: return launch_fwd_nw<MODE, 4>(rpl, A, (int)nblk, st);
        case 2: return launch_fwd_nw<MODE, 2>(rpl, A, (int)nblk, st);
        default: return launch_fwd_nw<MODE, 1>(rpl, A, (int)nblk, st);
    }
}

// The forward projection of the angles ang0 + i * step (i < cnt) with the epilogue MODE.
// With span compression the walk writes ray sums to A.raw (A.raw_angles angles at a time)
// and fwd_compress adds each data bin's ring-pair rays before the epilogue.
template <int MODE>
int launch_fwd(FwdArgs A, int ang0, int step, int cnt, hipStream_t st) {
    if (!A.G.cstart) return launch_walk<MODE>(A, ang0, step, cnt, st);
    if (!A.raw || A.raw_angles <= 0)
        return fail(SPDHG_E_WORKSPACE, "no ray-sum rows for the span-compressed projection");
    for (int c0 = 0; c0 < cnt; c0 += A.raw_angles) {
        const int cc = std::min(A.raw_angles, cnt - c0);
        FwdArgs R = A;
        R.raw_kq = 1;
        int rc = launch_walk<MODE>(R, ang0 + c0 * step, step, cc, st);
        if (rc) return rc;
        FwdArgs C = A;
        C.ang0 = ang0 + c0 * step;
        C.ang_step = step;
        C.n_ang_sub = cc;
        C.ia0 = A.ia0 + c0;
        if ((rc = klaunch(fwd_compress<MODE>, cc * A.G.n_rad, 256, 0, st, C))) return rc;
    }
    return SPDHG_OK;
}

int bwd_cols(int nz) { return nz < BWD_THREADS ? BWD_THREADS / nz : 1; }

// Backprojection kernel choice: the strip gather for 32 <= nz <= 127; else the per-column
// gather.  The rays a strip considers per angle span BS_W + 1 in the secondary coordinate
// plus one radial bin of margin on each side, so at most (BS_W + 1) / min|du_dk| + 5.
struct BwdPlan {
    bool strip = false;
    int KR = 0;
    int pitch = 1;  // the plane pitch every segment shares (the strip kernel's instance)
    int wj = 1;     // strips of consecutive primary indices per workgroup (1 or 4)
    size_t lds = 0; // per wavefront
};

// Smallest distance of neighbouring radial bins in secondary voxel units (non-arc-corrected
// bins are closer towards the edge of the field of view).
double min_bin_spacing(const HostTables& T) {
    double min_du = 1e30;
    for (const AngleDev& A : T.ang) min_du = std::min(min_du, std::fabs(A.du_dk));
    double dk = 1.0;
    for (size_t k = 1; k < T.kpos.size(); ++k) dk = std::min(dk, T.kpos[k] - T.kpos[k - 1]);
    return min_du * dk;
}

// The per-column gather keeps BWD_KC candidate bins per column and angle: bins at least
// half a voxel apart.
int check_column_gather(const HostTables& T) {
    if (!(min_bin_spacing(T) >= 0.5))
        return fail(SPDHG_E_SHAPE, "radial bins closer than half a voxel: only the strip gather "
                                   "(32 <= nz <= 127, one plane pitch) handles them");
    return SPDHG_OK;
}

BwdPlan bwd_plan(const HostTables& T) {
    BwdPlan pl;
    const int nz = T.G.nz, ns = T.G.n_seg;
    const double min_du = min_bin_spacing(T);
    if (nz < 32 || nz > 127 || !(min_du >= 0.25)) return pl;
    for (int g = 1; g < ns; ++g)
        if (T.G.seg_pitch[g] != T.G.seg_pitch[0]) return pl;  // mixed pitches: per column
    const int KR = (int)std::ceil((BS_W + 1) / min_du) + 6;
    const size_t floats = 2 * (size_t)KR + 2 * (BS_W + 1) +
                          (sizeof(TapCoef) / 4) * (size_t)KR * std::min(ns, SEG_CHUNK);
    if (floats * 4 > 64 * 1024) return pl;  // one workgroup's LDS
    pl.strip = true;
    pl.KR = KR;
    pl.pitch = T.G.seg_pitch[0];
    pl.lds = floats * 4;
    return pl;
}

// Gather backprojection of the angles ang0 + i * step (i < cnt) with the epilogue MODE;
// A.d holds their dual change in the dual_row layout.  With the strip kernel the
// row-sampled and column-sampled angles run as two launches; when both classes occur and
// the epilogue needs the whole sum, the first writes its partial image to `partial`.
// The strip gather of the angles ang0 + i * step (i < cnt) (see launch_bwd).
template <int MODE, int PITCH, int NS, int DS = 1>
int launch_strip(const BwdArgs& A, int cnt, int ang0, int step, hipStream_t st,
                 const BwdPlan& plan, const AngleDev* host_ang, float* partial) {
    bool has[2] = {false, false};
    for (int i = 0; i < cnt; ++i) has[host_ang[ang0 + i * step].rowdom] = true;
    const int wj = plan.wj;
    // rows: strips along x, wj rows per workgroup; columns: strips along y
    const int nstr_r = ((A.G.nx + BS_W - 1) / BS_W) * ((A.G.ny + wj - 1) / wj);
    const int nstr_c = ((A.G.ny + BS_W - 1) / BS_W) * ((A.G.nx + wj - 1) / wj);
    const unsigned nt = 64 * wj;
    const size_t lds = plan.lds * wj;
    const float* none = nullptr;
    if (has[1] && has[0]) {
        if (MODE == B_ACCUM) {
            int rc = klaunch(bwd_strip<B_ACCUM, PITCH, NS, DS>, nstr_r, nt, lds, st, A, plan.KR, 1, none);
            if (rc) return rc;
            return klaunch(bwd_strip<B_ACCUM, PITCH, NS, DS>, nstr_c, nt, lds, st, A, plan.KR, 0, none);
        }
        BwdArgs Pp = A;
        Pp.out = partial;
        int rc = klaunch(bwd_strip<B_PARTIAL, PITCH, NS, DS>, nstr_r, nt, lds, st, Pp, plan.KR, 1, none);
        if (rc) return rc;
        return klaunch(bwd_strip<MODE, PITCH, NS, DS>, nstr_c, nt, lds, st, A, plan.KR, 0,
                       (const float*)partial);
    }
    if (has[1]) return klaunch(bwd_strip<MODE, PITCH, NS, DS>, nstr_r, nt, lds, st, A, plan.KR, 1, none);
    if (has[0]) return klaunch(bwd_strip<MODE, PITCH, NS, DS>, nstr_c, nt, lds, st, A, plan.KR, 0, none);
    return SPDHG_OK;
}

template <int MODE>
int launch_bwd(BwdArgs A, int ang0, int step, int cnt, hipStream_t st, const BwdPlan& plan,
               const AngleDev* host_ang, float* partial) {
    A.ang0 = ang0;
    A.ang_step = step;
    A.n_ang_sub = cnt;
    if (plan.strip && plan.pitch == 2)
        return A.G.dstride == 2
                   ? launch_strip<MODE, 2, 0, 2>(A, cnt, ang0, step, st, plan, host_ang, partial)
                   : launch_strip<MODE, 2, 0, 1>(A, cnt, ang0, step, st, plan, host_ang, partial);
    if (plan.strip && A.G.n_seg == 11 && !A.G.kpos && !A.G.kobl && !A.G.kL)
        return launch_strip<MODE, 1, 11>(A, cnt, ang0, step, st, plan, host_ang, partial);
    if (plan.strip)
        return launch_strip<MODE, 1, 0>(A, cnt, ang0, step, st, plan, host_ang, partial);
    // columns per workgroup: as many as the threads cover, within one workgroup's LDS
    const size_t per_col = (size_t)BWD_KC * (sizeof(ColCoord) + sizeof(TapCoef) * A.G.n_seg);
    A.cols = std::max(1, std::min<int>(bwd_cols(A.G.nz), (int)((64 * 1024) / per_col)));
    const int64_t ncol = (int64_t)A.G.nx * A.G.ny;
    const int64_t nblk = (ncol + A.cols - 1) / A.cols;
    const size_t lds = (size_t)A.cols * per_col;
    return klaunch(bwd_col<MODE>, (unsigned)nblk, BWD_THREADS, lds, st, A, (const float*)nullptr);
}

dim3 img_grid(int nx, int ny, int nz) { return dim3((nx + TT - 1) / TT, (nz + TT - 1) / TT, ny); }

// Worker streams of batched epochs, one pool per device (default priority, created on
// first use, kept until the process ends): the first `need` streams of the pool.
int worker_streams(int dev, int need, std::vector<hipStream_t>& out) {
    static std::mutex mu;
    static std::map<int, std::vector<hipStream_t>> pools;
    std::lock_guard<std::mutex> lk(mu);
    std::vector<hipStream_t>& pool = pools[dev];
    while ((int)pool.size() < need) {
        hipStream_t w = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
        pool.push_back(w);
    }
    out.assign(pool.begin(), pool.begin() + need);
    return SPDHG_OK;
}

// Column tile of the prior kernels: as many whole columns as fit in 1024 threads,
// arranged about twice as wide in x as in y (nz <= 128 gives at least 8 columns).
PriorTile prior_tile(const spdhg_geom& g) {
    const int cols = 1024 / g.nz;
    int ty = 1;
    while ((2 * ty) * (4 * ty) <= cols) ty *= 2;
    PriorTile TL;
    TL.ty = std::min(ty, g.ny);
    TL.tx = std::min(cols / TL.ty, g.nx);
    return TL;
}

int prior_blocks(const spdhg_geom& g, const PriorTile& TL) {
    return ((g.nx + TL.tx - 1) / TL.tx) * ((g.ny + TL.ty - 1) / TL.ty);
}

constexpr int TV_WAVE_LY = 8;  // rows per chunk of the wavefront TV kernel
// The wavefront-march prior kernels (one wavefront per 64-voxel run of a column) for
// volumes with at least 32 planes whose `comps`-component fields stay below 4 GiB (32-bit
// buffer offsets); thinner volumes use the column tiles.
bool prior_use_wave(const spdhg_geom& g, int comps) {
    const uint64_t bytes = (uint64_t)comps * 4 * g.nx * g.ny * g.nz;
    return g.nz >= 32 && g.nz <= 128 && bytes < (1ull << 32);
}

int tv_wave_blocks(const spdhg_geom& g, int ly) {
    const int runs = g.nz <= 64 ? 1 : (g.nz + 61) / 63;  // runs of 64 overlapping by one
    const int64_t waves = (int64_t)runs * g.nx * ((g.ny + ly - 1) / ly);
    return (int)((waves + 3) / 4);
}

}  // namespace

// ====================================================================== context
struct spdhg_ctx {
    spdhg_geom geom;
    spdhg_params prm;
    HostTables tab;
    int device = 0;
    int pad = 0, gsize = 0;
    BwdPlan bplan;
    const float* side = nullptr;
    float* x_user = nullptr;
    // workspace regions (internal layouts: images z-fastest, sinograms [a][k][q])
    float *bp = nullptr, *rp = nullptr, *mp = nullptr;  // private b, r, mult
    float *y = nullptr, *sigma = nullptr, *dscr = nullptr;
    float* raw = nullptr;  // span compression: ray sums before the data bins are summed
    int raw_angles = 0;
    float *xa = nullptr, *xb = nullptr, *z = nullptr, *T = nullptr, *scr = nullptr;
    // SPDHG_FLAG_COMPENSATED: low parts of z and of the iterate (in place, not ping-pong)
    float *zlo = nullptr, *xlo = nullptr;
    float *yn[2] = {nullptr, nullptr}, *xi = nullptr;
    // TGV: w (ping-pong), z_w, q2 (ping-pong); data iterations owe w the line-3 steps
    // w -= T_w z_w, applied together before the next use of w
    float *w[2] = {nullptr, nullptr}, *zw = nullptr, *q2[2] = {nullptr, nullptr};
    int w_cur = 0, q2_cur = 0;
    int64_t w_pending = 0;
    double tw = 0.0;
    int fwd_split = 0;  // wavefronts per ray bundle of the subset projection (0: automatic)
    int interleave = 0; // 1: the forward walk keeps interleaved rays (no RUN instances)
    int gather = 0;     // backprojection tiling: 0 automatic (strips where they apply), 2 columns
    BwdPlan bplan_auto; // the automatic plan (bplan is it, or the per-column gather)
    spdhg_graph* graph = nullptr;  // persistent epoch graph of spdhg_epoch_graph (owned)
    float* em_inv = nullptr;  // SPDHG_FLAG_EM: 1 / (A_i^T 1) per subset (m images, z-fastest)
    int64_t em_k = 0;         // EM-type sub-iterations done (subset em_k mod m is next)
    double* part = nullptr;
    double* scal = nullptr;  // 8 doubles of device scalars
    int64_t part_n = 0;
    int x_cur = 0;  // iterate in xa (0) or xb (1)
    int yn_cur = 0;
    int m = 1, n = 1, n_prior = 0;
    std::vector<double> p, cum;
    std::vector<double> data_norm, data_sigma;
    double prior_norm = 0.0, prior_sigma = 0.0;
    double prior_norm2 = 0.0, prior_sigma2 = 0.0;  // TGV block n
    double masked_phi0 = 0.0;  // sum of phi_j(0) over the bins with (A 1)_j = 0
    int64_t k = 0;
    int64_t iters_per_epoch = 1;
    int64_t nv = 0, nb = 0, max_sub_bins = 0;
    // optional per-kernel timing: event pairs around each launch of the iteration (of the
    // kinds in prof_mask)
    bool prof = false;
    int prof_mask = (1 << SPDHG_PROF_KINDS) - 1;
    bool ev_open = false;  // prof_begin recorded the start of a pair
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;  // kernel kind of each recorded pair
    size_t ev_used = 0;
    double prof_ms[SPDHG_PROF_KINDS] = {0};
    int64_t prof_n[SPDHG_PROF_KINDS] = {0};
    float* xcur() { return x_cur ? xb : xa; }
    float* xother() { return x_cur ? xa : xb; }
    FwdArgs fwd_args() const {
        FwdArgs A{};
        A.G = tab.G;
        A.pad = pad;
        A.gsize = gsize;
        A.raw = raw;
        A.raw_angles = raw_angles;
        A.interleave = interleave;
        return A;
    }
    BwdArgs bwd_args() const {
        BwdArgs A{};
        A.G = tab.G;
        A.zlo = zlo;
        A.xlo = xlo;
        return A;
    }
    PriorArgs prior_args() const {
        PriorArgs P{};
        P.nx = geom.nx;
        P.ny = geom.ny;
        P.nz = geom.nz;
        P.sigma = (float)prior_sigma;
        P.alpha = (float)prm.alpha;
        P.gamma_d = (float)prm.gamma_d;
        P.dtv = prm.prior == SPDHG_PRIOR_DTV;
        P.atv = prm.prior == SPDHG_PRIOR_ATV;
        P.zlo = zlo;
        P.xlo = xlo;
        return P;
    }
    TgvArgs tgv_args(int block) const {
        TgvArgs P{};
        P.nx = geom.nx;
        P.ny = geom.ny;
        P.nz = geom.nz;
        P.sigma = (float)(block == 0 ? prior_sigma : prior_sigma2);
        P.alpha = (float)(block == 0 ? prm.alpha : prm.alpha1);
        P.tw = (float)tw;
        return P;
    }
};

namespace {

struct Layout {
    size_t tables, bp, rp, mp, y, sigma, dscr, raw, xa, xb, z, T, scr, yn, xi, w, zw, q2, em,
        lo, part, scal, total;
    int64_t part_n, raw_angles;
};

Layout layout(const spdhg_geom* g, const spdhg_params* p, const HostTables& tab) {
    Layout L{};
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    const int64_t np = n_data_planes(g);
    const int64_t nb = (int64_t)g->n_ang * np * g->n_rad;
    const int m = std::max(1, p->n_subsets);
    // dual change of the largest subset (see dual_row)
    const int64_t max_sub = (int64_t)((g->n_ang + m - 1) / m) * g->n_rad * np;
    // span compression: ray sums of the largest subset's angles (longer launches, such as
    // the objective's, go through in chunks of that many angles)
    L.raw_angles = g->span ? (g->n_ang + m - 1) / m : 0;
    const bool prior = p->prior != SPDHG_PRIOR_NONE;
    const bool tgv = p->prior == SPDHG_PRIOR_TGV;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.tables = take(table_bytes(tab));
    L.bp = take(nb * 4);
    L.rp = take(nb * 4);
    L.mp = take(nb * 4);
    L.y = take(nb * 4);
    L.sigma = take(p->precond ? nb * 4 : 0);
    L.dscr = take(max_sub * 4);
    L.raw = take(L.raw_angles * g->n_rad * n_planes(g) * 4);
    L.xa = take(nv * 4);
    L.xb = take(nv * 4);
    L.z = take(nv * 4);
    L.T = take(nv * 4);
    L.scr = take(nv * 4);
    L.yn = take(prior ? 6 * nv * 4 : 0);
    L.xi = take(p->prior == SPDHG_PRIOR_DTV ? 3 * nv * 4 : 0);
    L.w = take(tgv ? 6 * nv * 4 : 0);
    L.zw = take(tgv ? 3 * nv * 4 : 0);
    L.q2 = take(tgv ? 12 * nv * 4 : 0);
    L.em = take((p->flags & SPDHG_FLAG_EM) ? (size_t)m * nv * 4 : 0);
    L.lo = take((p->flags & SPDHG_FLAG_COMPENSATED) ? 2 * (size_t)nv * 4 : 0);
    const int64_t fwd_blocks = (int64_t)g->n_ang * g->n_rad;
    L.part_n = std::max<int64_t>({(nb + BLOCK - 1) / BLOCK, (3 * nv + BLOCK - 1) / BLOCK,
                                  fwd_blocks, 1}) * 2;
    L.part = take(L.part_n * 8);
    L.scal = take(8 * 8);
    L.total = off;
    return L;
}

int check_params(const spdhg_geom* g, const spdhg_params* p) {
    if (!p) return fail(SPDHG_E_ARG, "params is NULL");
    if (p->n_subsets < 1 || p->n_subsets > g->n_ang)
        return fail(SPDHG_E_ARG, "n_subsets must be in [1, n_ang]");
    if (p->prior < SPDHG_PRIOR_NONE || p->prior > SPDHG_PRIOR_TGV)
        return fail(SPDHG_E_NOTIMPL, "prior not implemented");
    if (p->prior == SPDHG_PRIOR_TGV && !(p->alpha1 >= 0))
        return fail(SPDHG_E_ARG, "TGV weight alpha1 must be >= 0");
    if (p->sampling != SPDHG_SAMPLING_UNIFORM && p->sampling != SPDHG_SAMPLING_BALANCED &&
        p->sampling != SPDHG_SAMPLING_CUSTOM)
        return fail(SPDHG_E_ARG, "unknown sampling");
    if (p->sampling == SPDHG_SAMPLING_CUSTOM && p->prior != SPDHG_PRIOR_NONE) {
        if (!(p->p_prior > 0.0) || !(p->p_prior < 1.0))
            return fail(SPDHG_E_ARG, "custom sampling needs 0 < p_prior < 1");
        if (p->prior == SPDHG_PRIOR_TGV && (!(p->p_tgv_n >= 0.0) || !(p->p_tgv_n < p->p_prior)))
            return fail(SPDHG_E_ARG, "custom sampling needs 0 <= p_tgv_n < p_prior");
    }
    if (!(p->gamma > 0) || !(p->rho > 0) || !(p->rho < 1))
        return fail(SPDHG_E_ARG, "need gamma > 0 and 0 < rho < 1");
    if (p->prior != SPDHG_PRIOR_NONE && !(p->alpha >= 0))
        return fail(SPDHG_E_ARG, "prior weight must be >= 0");
    if (p->prior == SPDHG_PRIOR_DTV && (!(p->eta > 0) || !(p->gamma_d >= 0) || !(p->gamma_d <= 1)))
        return fail(SPDHG_E_ARG, "dTV needs eta > 0 and gamma_d in [0, 1]");
    if (!p->precond && p->power_iters < 1) return fail(SPDHG_E_ARG, "power_iters must be >= 1");
    if (p->flags & ~(SPDHG_FLAG_EM | SPDHG_FLAG_TGV_SPLIT_T | SPDHG_FLAG_COMPENSATED))
        return fail(SPDHG_E_ARG, "unknown flags");
    if ((p->flags & SPDHG_FLAG_COMPENSATED) && p->prior == SPDHG_PRIOR_TGV)
        return fail(SPDHG_E_NOTIMPL, "the compensated primal step is not built for TGV");
    return SPDHG_OK;
}

int reduce_to(double* part, int64_t n, double* out, int slot, double scale, hipStream_t st) {
    reduce_final<<<1, BLOCK, 0, st>>>(part, n, out, slot, scale);
    LAUNCH_CHECK();
    return SPDHG_OK;
}

// Power iteration on A_i^T A_i from the ones image (scalar steps of Theorem 2): norm of
// data block i.  Uses xb, z, scr and dscr as scratch.
int power_norm_data(spdhg_ctx* c, int i, double* out, hipStream_t st) {
    int a0, step, cnt;
    int rc = subset_angles(&c->geom, c->m, i, a0, step, cnt);
    if (rc) return rc;
    const int64_t nv = c->nv;
    float* v = c->xb;
    float* w = c->z;
    float* tmp = c->dscr;  // dual_row layout
    fill_f32<<<nblocks(nv), BLOCK, 0, st>>>(v, nv, 1.0f);
    sumsq<<<nblocks(nv), BLOCK, 0, st>>>(v, nv, c->part);
    if ((rc = reduce_to(c->part, nblocks(nv), c->scal, 0, 1.0, st))) return rc;
    scale_by_rnorm<<<nblocks(nv), BLOCK, 0, st>>>(v, v, nv, c->scal);
    for (int it = 0; it < c->prm.power_iters; ++it) {
        // w = A_i^T A_i v = G^T (mult^2 G v)
        FwdArgs F = c->fwd_args();
        F.x = v;
        F.mult = c->mp;
        F.out = tmp;
        if ((rc = launch_fwd<F_POWER>(F, a0, step, cnt, st))) return rc;
        BwdArgs B = c->bwd_args();
        B.d = tmp;
        B.out = w;
        if ((rc = launch_bwd<B_PLAIN>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr)))
            return rc;
        sumsq<<<nblocks(nv), BLOCK, 0, st>>>(w, nv, c->part);
        if ((rc = reduce_to(c->part, nblocks(nv), c->scal, 0, 1.0, st))) return rc;
        scale_by_rnorm<<<nblocks(nv), BLOCK, 0, st>>>(w, v, nv, c->scal);
    }
    LAUNCH_CHECK();
    double h = 0.0;
    HIP_TRY(hipMemcpyAsync(&h, c->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(std::sqrt(h));
    return SPDHG_OK;
}

// Power iteration on (D grad)^T (D grad) from a checkerboard, 200 iterations: ||D grad||
// for dTV.  Uses xb, z and yn[0] as scratch.
int power_norm_dgrad(spdhg_ctx* c, double* out, hipStream_t st) {
    const int64_t nv = c->nv;
    PriorArgs P = c->prior_args();
    float* v = c->xb;
    float* w = c->z;
    float* pp = c->yn[0];
    int rc;
    checkerboard_zf<<<nblocks(nv), BLOCK, 0, st>>>(P, v);
    sumsq<<<nblocks(nv), BLOCK, 0, st>>>(v, nv, c->part);
    if ((rc = reduce_to(c->part, nblocks(nv), c->scal, 0, 1.0, st))) return rc;
    scale_by_rnorm<<<nblocks(nv), BLOCK, 0, st>>>(v, v, nv, c->scal);
    for (int it = 0; it < 200; ++it) {
        dgrad_apply<<<nblocks(nv), BLOCK, 0, st>>>(P, v, c->xi, pp);
        dgrad_adj<<<nblocks(nv), BLOCK, 0, st>>>(P, pp, c->xi, w);
        sumsq<<<nblocks(nv), BLOCK, 0, st>>>(w, nv, c->part);
        if ((rc = reduce_to(c->part, nblocks(nv), c->scal, 0, 1.0, st))) return rc;
        scale_by_rnorm<<<nblocks(nv), BLOCK, 0, st>>>(w, v, nv, c->scal);
    }
    LAUNCH_CHECK();
    double h = 0.0;
    HIP_TRY(hipMemcpyAsync(&h, c->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = std::sqrt(std::sqrt(h));
    return SPDHG_OK;
}

// TGV: apply the line-3 updates of w owed by the data iterations since the last use.
int settle_w(spdhg_ctx* c, hipStream_t st) {
    if (!c->zw || c->w_pending == 0) return SPDHG_OK;
    const int64_t n3 = 3 * c->nv;
    int rc = klaunch(w_catchup, nblocks(n3), BLOCK, 0, st, c->w[c->w_cur], (const float*)c->zw, n3,
                     (float)((double)c->w_pending * c->tw));
    c->w_pending = 0;
    return rc;
}

// Copy the internal iterate out to the caller's image.
int export_x(spdhg_ctx* c, hipStream_t st) {
    const spdhg_geom& g = c->geom;
    return klaunch(img_from_zf, img_grid(g.nx, g.ny, g.nz), TT * 8, 0, st, g.nx, g.ny, g.nz,
                   (const float*)c->xcur(), c->x_user);
}

// Per-kernel timing (events around launches; collected on demand).
int prof_collect(spdhg_ctx* c) {
    for (size_t i = 0; i < c->ev_used; ++i) {
        HIP_TRY(hipEventSynchronize(c->ev[2 * i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        c->prof_ms[c->ev_kind[i]] += ms;
        c->prof_n[c->ev_kind[i]] += 1;
    }
    c->ev_used = 0;
    return SPDHG_OK;
}

int prof_begin(spdhg_ctx* c, int kind, hipStream_t st) {
    c->ev_open = false;
    if (!c->prof || !((c->prof_mask >> kind) & 1)) return SPDHG_OK;
    if (2 * c->ev_used + 2 > c->ev.size()) {
        int rc = prof_collect(c);
        if (rc) return rc;
    }
    c->ev_kind[c->ev_used] = kind;
    HIP_TRY(hipEventRecord(c->ev[2 * c->ev_used], st));
    c->ev_open = true;
    return SPDHG_OK;
}

int prof_end(spdhg_ctx* c, hipStream_t st) {
    if (!c->prof || !c->ev_open) return SPDHG_OK;
    HIP_TRY(hipEventRecord(c->ev[2 * c->ev_used + 1], st));
    c->ev_used += 1;
    c->ev_open = false;
    return SPDHG_OK;
}

}  // namespace

namespace {

// ---------------------------------------------------------------- fixed scratch
// Device scratch of spdhg_project_noalloc, for callers that cannot allocate: a fixed
// array in the code object, one copy per GPU the library runs on, held until the process
// ends.  Host code never uses the array's name as an address (on the host it names a
// stand-in, not device memory): scratch_ptr() fetches the device address of the current
// GPU's copy once per device with hipGetSymbolAddress and keeps it.
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {nullptr};

int scratch_ptr(char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(SPDHG_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SPDHG_E_HIP, "hipGetSymbolAddress returned NULL for the scratch");
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return SPDHG_OK;
}

// ---------------------------------------------------------------- stand-alone operators
// Workspace of spdhg_project / spdhg_backproject / spdhg_nnz /
// spdhg_normalised_backprojection (caller memory, 256-byte aligned): the geometry tables,
// two z-fastest images, the dual_row staging of up to OP_CHUNK angles, and FP64 partials
// for a reduction over every bin.
constexpr int OP_CHUNK = 16;

struct OpLayout {
    size_t tables, img, raw, img2, rows, part, total;
    size_t project_total;  // what spdhg_project uses: the tables, the first image, raw rows
};

OpLayout op_layout(const spdhg_geom* g, const HostTables& T) {
    OpLayout L{};
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    const int64_t np = n_data_planes(g);
    const int64_t nb = (int64_t)g->n_ang * np * g->n_rad;
    const int64_t chunk = std::min(g->n_ang, OP_CHUNK);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.tables = take(table_bytes(T));
    L.img = take(nv * 4);
    // span compression: the ray sums of OP_CHUNK angles before their data bins are summed
    L.raw = take(g->span ? chunk * g->n_rad * n_planes(g) * 4 : 0);
    L.project_total = off;
    L.img2 = take(nv * 4);
    L.rows = take(chunk * g->n_rad * np * 4);
    L.part = take((std::max<int64_t>(nblocks(nb), 2 * nblocks(nv)) + 1) * 8);
    L.total = off;
    return L;
}

struct OpWork {
    HostTables tab;
    float *img = nullptr, *img2 = nullptr, *rows = nullptr, *raw = nullptr;
    double* part = nullptr;
    int pad = 0;
    BwdPlan plan;
};

// Validate the caller's workspace, carve it and upload the geometry tables on `st`
// (project_only: the workspace need only hold what spdhg_project uses).
int op_begin(const spdhg_geom* g, void* ws, size_t ws_bytes, hipStream_t st, OpWork& W,
             bool project_only = false) {
    if (!ws) return fail(SPDHG_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) & 255) return fail(SPDHG_E_WORKSPACE, "workspace must be 256-byte aligned");
    build_tables(g, W.tab);
    const OpLayout L = op_layout(g, W.tab);
    const size_t need = project_only ? L.project_total : L.total;
    if (ws_bytes < need)
        return fail(SPDHG_E_WORKSPACE, "operator workspace too small: need " + std::to_string(need));
    char* w = (char*)ws;
    int rc = upload_tables(W.tab, w + L.tables, st);
    if (rc) return rc;
    W.img = (float*)(w + L.img);
    W.raw = g->span ? (float*)(w + L.raw) : nullptr;
    W.img2 = (float*)(w + L.img2);
    W.rows = (float*)(w + L.rows);
    W.part = (double*)(w + L.part);
    W.pad = axial_pad(W.tab);
    W.plan = bwd_plan(W.tab);
    if (!W.plan.strip && (rc = check_column_gather(W.tab))) return rc;
    return SPDHG_OK;
}

// y_out = A x for the angles a0 + i * step (i < cnt), caller layouts; W.img holds the
// z-fastest copy of x.
int project_zf_scratch(const spdhg_geom* g, const OpWork& W, const float* mult, const float* x,
                       float* y_out, int a0, int step, int cnt, hipStream_t st) {
    img_to_zf<<<img_grid(g->nx, g->ny, g->nz), TT * 8, 0, st>>>(g->nx, g->ny, g->nz, x, W.img);
    LAUNCH_CHECK();
    FwdArgs F{};
    F.G = W.tab.G;
    F.pad = W.pad;
    F.gsize = g->nz + 2 * W.pad;
    F.x = W.img;
    F.mult = mult;
    F.out = y_out;
    F.raw = W.raw;
    F.raw_angles = std::min(g->n_ang, OP_CHUNK);
    return launch_fwd<F_PLAIN_QK>(F, a0, step, cnt, st);
}

// acc = G^T (mult y) for the angles a0 + i * step (i < cnt) with y packed in the caller's
// subset layout [i][plane][radial] (mult: full caller sinogram, or NULL); acc is a
// z-fastest image, cleared first.  Angles go through W.rows OP_CHUNK at a time.
int backproject_acc(const spdhg_geom* g, const OpWork& W, const float* y, const float* mult,
                    int a0, int step, int cnt, float* acc, hipStream_t st) {
    const GeomDev& G = W.tab.G;
    const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
    fill_f32<<<nblocks(nv), BLOCK, 0, st>>>(acc, nv, 0.0f);
    LAUNCH_CHECK();
    const int chunk = std::min(cnt, OP_CHUNK);
    for (int c0 = 0; c0 < cnt; c0 += chunk) {
        const int cc = std::min(chunk, cnt - c0);
        const int cang0 = a0 + c0 * step;
        const int64_t nsub = (int64_t)cc * G.n_dplanes * G.n_rad;
        to_rows<<<nblocks(nsub), BLOCK, 0, st>>>(G, y + (int64_t)c0 * G.n_dplanes * G.n_rad, 1,
                                                   mult, cang0, step, cc, W.rows);
        LAUNCH_CHECK();
        BwdArgs B{};
        B.G = G;
        B.d = W.rows;
        B.out = acc;
        int rc = launch_bwd<B_ACCUM>(B, cang0, step, cc, st, W.plan, W.tab.ang.data(), nullptr);
        if (rc) return rc;
    }
    return SPDHG_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* spdhg_last_error(void) { return g_err.c_str(); }

int64_t spdhg_subset_bins(const spdhg_geom* geom, int32_t n_subsets, int32_t subset) {
    if (check_geom(geom)) return -1;
    int a0, st, cnt;
    if (subset_angles(geom, n_subsets, subset, a0, st, cnt)) return -1;
    return (int64_t)cnt * n_data_planes(geom) * geom->n_rad;
}

int spdhg_op_workspace_bytes(const spdhg_geom* geom, size_t* bytes) {
    int rc = check_geom(geom);
    if (rc) return rc;
    if (!bytes) return fail(SPDHG_E_ARG, "bytes is NULL");
    HostTables T;
    build_tables(geom, T);
    *bytes = op_layout(geom, T).total;
    return SPDHG_OK;
}

int spdhg_project(const spdhg_geom* geom, int32_t n_subsets, int32_t subset, const float* mult,
                  const float* x, float* y_out, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_geom(geom);
    if (rc || (rc = check_kernel_limits(geom))) return rc;
    if (!x || !y_out) return fail(SPDHG_E_ARG, "NULL image or output");
    int a0, step, cnt;
    rc = subset_angles(geom, n_subsets, subset, a0, step, cnt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    OpWork W;
    if ((rc = op_begin(geom, ws, ws_bytes, st, W, true))) return rc;
    return project_zf_scratch(geom, W, mult, x, y_out, a0, step, cnt, st);
}

int spdhg_project_noalloc(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                          const float* mult, const float* x, float* y_out, void* stream) {
    int rc = check_geom(geom);
    if (rc || (rc = check_kernel_limits(geom))) return rc;
    if (!x || !y_out) return fail(SPDHG_E_ARG, "NULL image or output");
    int a0, step, cnt;
    rc = subset_angles(geom, n_subsets, subset, a0, step, cnt);
    if (rc) return rc;
    {
        HostTables T;
        build_tables(geom, T);
        const size_t need = op_layout(geom, T).project_total;
        if (need > SCRATCH_BYTES)
            return fail(SPDHG_E_WORKSPACE,
                        "spdhg_project_noalloc: the geometry needs " + std::to_string(need) +
                            " bytes of scratch, above the library's fixed " +
                            std::to_string((size_t)SCRATCH_BYTES) +
                            " (use spdhg_project with a workspace)");
    }
    char* ptr = nullptr;
    if ((rc = scratch_ptr(&ptr))) return rc;
    hipStream_t st = (hipStream_t)stream;
    OpWork W;
    if ((rc = op_begin(geom, ptr, SCRATCH_BYTES, st, W, true))) return rc;
    return project_zf_scratch(geom, W, mult, x, y_out, a0, step, cnt, st);
}

int spdhg_backproject(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                      const float* mult, const float* y, float* x_out, void* ws, size_t ws_bytes,
                      void* stream) {
    int rc = check_geom(geom);
    if (rc || (rc = check_kernel_limits(geom))) return rc;
    if (!y || !x_out) return fail(SPDHG_E_ARG, "NULL sinogram or output");
    int a0, step, cnt;
    rc = subset_angles(geom, n_subsets, subset, a0, step, cnt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    OpWork W;
    if ((rc = op_begin(geom, ws, ws_bytes, st, W))) return rc;
    if ((rc = backproject_acc(geom, W, y, mult, a0, step, cnt, W.img, st))) return rc;
    img_from_zf<<<img_grid(geom->nx, geom->ny, geom->nz), TT * 8, 0, st>>>(
        geom->nx, geom->ny, geom->nz, W.img, x_out);
    LAUNCH_CHECK();
    return SPDHG_OK;
}

int spdhg_normalised_backprojection(const spdhg_geom* geom, const float* b, const float* mult,
                                    float* out, double* stats_dev, void* ws, size_t ws_bytes,
                                    void* stream) {
    int rc = check_geom(geom);
    if (rc || (rc = check_kernel_limits(geom))) return rc;
    if (!b || !mult || !out || !stats_dev) return fail(SPDHG_E_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    OpWork W;
    if ((rc = op_begin(geom, ws, ws_bytes, st, W))) return rc;
    // A^T b = G^T (mult b) into img, A^T 1 = G^T mult into img2 (all angles)
    if ((rc = backproject_acc(geom, W, b, mult, 0, 1, geom->n_ang, W.img, st))) return rc;
    if ((rc = backproject_acc(geom, W, mult, nullptr, 0, 1, geom->n_ang, W.img2, st))) return rc;
    const int64_t nv = (int64_t)geom->nx * geom->ny * geom->nz;
    const int64_t nbk = nblocks(nv);
    ratio_on_support<<<nbk, BLOCK, 0, st>>>(W.img, W.img2, nv, W.img, W.part, W.part + nbk);
    reduce_final<<<1, BLOCK, 0, st>>>(W.part, nbk, stats_dev, 0, 1.0);
    reduce_final<<<1, BLOCK, 0, st>>>(W.part + nbk, nbk, stats_dev, 1, 1.0);
    support_scale<<<1, 64, 0, st>>>(stats_dev);
    img_from_zf<<<img_grid(geom->nx, geom->ny, geom->nz), TT * 8, 0, st>>>(
        geom->nx, geom->ny, geom->nz, W.img, out);
    LAUNCH_CHECK();
    return SPDHG_OK;
}

int spdhg_nnz(const spdhg_geom* geom, int32_t n_subsets, int32_t subset, double* out, void* ws,
              size_t ws_bytes, void* stream) {
    int rc = check_geom(geom);
    if (rc) return rc;
    if (!out) return fail(SPDHG_E_ARG, "out is NULL");
    int a0, step, cnt;
    rc = subset_angles(geom, n_subsets, subset, a0, step, cnt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    OpWork W;
    if ((rc = op_begin(geom, ws, ws_bytes, st, W))) return rc;
    const GeomDev& G = W.tab.G;
    const int64_t n = (int64_t)cnt * G.n_planes * G.n_rad;
    const int64_t nbk = nblocks(n);
    fwd_count<<<nbk, BLOCK, 0, st>>>(G, a0, step, cnt, W.part);
    reduce_final<<<1, BLOCK, 0, st>>>(W.part, nbk, W.part + nbk, 0, 1.0);
    LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(out, W.part + nbk, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPDHG_OK;
}

int spdhg_workspace_bytes(const spdhg_geom* geom, const spdhg_params* params, size_t* bytes) {
    int rc = check_geom(geom);
    if (rc) return rc;
    rc = check_params(geom, params);
    if (rc) return rc;
    if (!bytes) return fail(SPDHG_E_ARG, "bytes is NULL");
    HostTables T;
    build_tables(geom, T);
    *bytes = layout(geom, params, T).total;
    return SPDHG_OK;
}

int spdhg_init(spdhg_ctx** out, const spdhg_geom* geom, const spdhg_params* params,
               const float* b, const float* r, const float* mult, const float* side, float* x,
               void* ws, size_t ws_bytes, void* stream) {
    if (!out) return fail(SPDHG_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_geom(geom);
    if (rc || (rc = check_kernel_limits(geom))) return rc;
    rc = check_params(geom, params);
    if (rc) return rc;
    if (!b || !r || !mult || !x) return fail(SPDHG_E_ARG, "NULL b, r, mult or x");
    if (params->prior == SPDHG_PRIOR_DTV && !side) return fail(SPDHG_E_ARG, "dTV needs a side image");
    if (!ws) return fail(SPDHG_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) & 255) return fail(SPDHG_E_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;

    spdhg_ctx* c = new spdhg_ctx();
    auto bail = [&](int code) {
        delete c;
        return code;
    };
    c->geom = *geom;
    c->prm = *params;
    build_tables(geom, c->tab);
    Layout L = layout(geom, params, c->tab);
    if (ws_bytes < L.total)
        return bail(fail(SPDHG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total)));
    {
        hipError_t e = hipGetDevice(&c->device);
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
    }
    char* w = (char*)ws;
    if ((rc = upload_tables(c->tab, w + L.tables, st))) return bail(rc);
    c->pad = axial_pad(c->tab);
    c->gsize = geom->nz + 2 * c->pad;
    c->bplan = bwd_plan(c->tab);
    c->bplan_auto = c->bplan;
    if (!c->bplan.strip && (rc = check_column_gather(c->tab))) return bail(rc);
    c->side = side;
    c->x_user = x;
    c->bp = (float*)(w + L.bp);
    c->rp = (float*)(w + L.rp);
    c->mp = (float*)(w + L.mp);
    c->y = (float*)(w + L.y);
    c->sigma = params->precond ? (float*)(w + L.sigma) : nullptr;
    c->dscr = (float*)(w + L.dscr);
    c->raw = L.raw_angles ? (float*)(w + L.raw) : nullptr;
    c->raw_angles = (int)L.raw_angles;
    c->xa = (float*)(w + L.xa);
    c->xb = (float*)(w + L.xb);
    c->z = (float*)(w + L.z);
    c->T = (float*)(w + L.T);
    c->scr = (float*)(w + L.scr);
    const bool prior = params->prior != SPDHG_PRIOR_NONE;
    c->nv = (int64_t)geom->nx * geom->ny * geom->nz;
    c->nb = (int64_t)geom->n_ang * c->tab.G.n_dplanes * geom->n_rad;
    if (prior) {
        c->yn[0] = (float*)(w + L.yn);
        c->yn[1] = c->yn[0] + 3 * c->nv;
    }
    c->xi = params->prior == SPDHG_PRIOR_DTV ? (float*)(w + L.xi) : nullptr;
    const bool tgv = params->prior == SPDHG_PRIOR_TGV;
    if (tgv) {
        c->w[0] = (float*)(w + L.w);
        c->w[1] = c->w[0] + 3 * c->nv;
        c->zw = (float*)(w + L.zw);
        c->q2[0] = (float*)(w + L.q2);
        c->q2[1] = c->q2[0] + 6 * c->nv;
    }
    c->part = (double*)(w + L.part);
    c->part_n = L.part_n;
    c->em_inv = (params->flags & SPDHG_FLAG_EM) ? (float*)(w + L.em) : nullptr;
    if (params->flags & SPDHG_FLAG_COMPENSATED) {
        c->zlo = (float*)(w + L.lo);
        c->xlo = c->zlo + c->nv;
    }
    c->scal = (double*)(w + L.scal);
    c->m = params->n_subsets;
    c->n_prior = tgv ? 2 : (prior ? 1 : 0);
    c->n = c->m + c->n_prior;
    // probabilities (Section 4.2)
    c->p.assign(c->n, 1.0 / c->n);
    if (params->sampling == SPDHG_SAMPLING_BALANCED && c->n_prior > 0) {
        for (int i = 0; i < c->m; ++i) c->p[i] = 1.0 / (2.0 * c->m);
        for (int j = 0; j < c->n_prior; ++j) c->p[c->m + j] = 0.5 / c->n_prior;
    } else if (params->sampling == SPDHG_SAMPLING_CUSTOM && c->n_prior > 0) {
        const double q = params->p_prior;
        for (int i = 0; i < c->m; ++i) c->p[i] = (1.0 - q) / c->m;
        if (c->n_prior == 1) {
            c->p[c->m] = q;
        } else if (params->p_tgv_n == 0.0) {
            c->p[c->m] = c->p[c->m + 1] = q / 2.0;
        } else {
            c->p[c->m] = q - params->p_tgv_n;
            c->p[c->m + 1] = params->p_tgv_n;
        }
    }
    c->cum.resize(c->n);
    double acc = 0.0;
    for (int i = 0; i < c->n; ++i) {
        acc += c->p[i];
        c->cum[i] = acc;
    }
    c->cum[c->n - 1] = 1.0;
    double pdata = 0.0;
    for (int i = 0; i < c->m; ++i) pdata += c->p[i];
    c->iters_per_epoch = (int64_t)std::llround(c->m / pdata);
    const int64_t nv = c->nv, nb = c->nb;
    const double gam = params->gamma, rho = params->rho;
    const int np = c->tab.G.n_dplanes;

    // private copies of b, r, mult in the [a][k][q] layout
    {
        dim3 grid((geom->n_rad + TT - 1) / TT, (np + TT - 1) / TT, geom->n_ang);
        sino_to_kq<<<grid, TT * 8, 0, st>>>(np, geom->n_rad, b, c->bp);
        sino_to_kq<<<grid, TT * 8, 0, st>>>(np, geom->n_rad, r, c->rp);
        sino_to_kq<<<grid, TT * 8, 0, st>>>(np, geom->n_rad, mult, c->mp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
    }
    // domain check: needs A 1 > 0 per bin (computed into y, zeroed afterwards)
    {
        FwdArgs F = c->fwd_args();
        F.mult = c->mp;
        F.out = c->y;
        F.gr = 1.0f;
        if ((rc = launch_fwd<F_SENS>(F, 0, 1, geom->n_ang, st))) return bail(rc);
        const int64_t nbk = nblocks(nb);
        if (2 * nbk > c->part_n) return bail(fail(SPDHG_E_WORKSPACE, "partials buffer too small"));
        domain_check<<<nbk, BLOCK, 0, st>>>(c->bp, c->rp, c->mp, c->y, nb, c->part, nbk);
        reduce_final<<<1, BLOCK, 0, st>>>(c->part, nbk, c->scal, 0, 1.0);
        reduce_final<<<1, BLOCK, 0, st>>>(c->part + nbk, nbk, c->scal, 1, 1.0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
        double h[2];
        e = hipMemcpyAsync(h, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
        if (h[0] > 0)
            return bail(fail(SPDHG_E_DOMAIN, "b < 0, r < 0, mult < 0 or non-finite data in " +
                                                 std::to_string((long long)h[0]) + " bins"));
        if (h[1] > 0)
            return bail(fail(SPDHG_E_DOMAIN, std::to_string((long long)h[1]) +
                                                 " bins have b > 0, r = 0 and no voxel on the ray"));
        masked_phi0<<<nbk, BLOCK, 0, st>>>(c->bp, c->rp, c->y, nb, c->part);
        reduce_final<<<1, BLOCK, 0, st>>>(c->part, nbk, c->scal, 0, 1.0);
        e = hipMemcpyAsync(h, c->scal, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
        c->masked_phi0 = h[0];
    }
    // the image: caller layout -> z-fastest, the primal step with z = 0: x = max(x0, 0)
    img_to_zf<<<img_grid(geom->nx, geom->ny, geom->nz), TT * 8, 0, st>>>(geom->nx, geom->ny,
                                                                         geom->nz, x, c->xa);
    clip_nonneg<<<nblocks(nv), BLOCK, 0, st>>>(c->xa, nv);
    // step sizes (Theorem 2)
    double t_data_scalar = INFINITY;
    if (params->precond) {
        FwdArgs F = c->fwd_args();
        F.mult = c->mp;
        F.out = c->sigma;
        F.gr = (float)(gam * rho);
        if ((rc = launch_fwd<F_SENS>(F, 0, 1, geom->n_ang, st))) return bail(rc);
        fill_f32<<<nblocks(nv), BLOCK, 0, st>>>(c->T, nv, INFINITY);
        for (int i = 0; i < c->m; ++i) {
            int a0, step, cnt;
            subset_angles(geom, c->m, i, a0, step, cnt);
            const int64_t nsub = (int64_t)cnt * np * geom->n_rad;
            to_rows<<<nblocks(nsub), BLOCK, 0, st>>>(c->tab.G, c->mp, 0, nullptr, a0, step, cnt,
                                                       c->dscr);
            BwdArgs B = c->bwd_args();
            B.d = c->dscr;
            B.scale = (float)(rho * c->p[i] / gam);
            B.T = c->T;
            if ((rc = launch_bwd<B_SENS>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr)))
                return bail(rc);
        }
    } else {
        c->data_norm.resize(c->m);
        c->data_sigma.resize(c->m);
        for (int i = 0; i < c->m; ++i) {
            double nrm = 0.0;
            if ((rc = power_norm_data(c, i, &nrm, st))) return bail(rc);
            c->data_norm[i] = nrm;
            c->data_sigma[i] = gam * rho / nrm;
            t_data_scalar = std::min(t_data_scalar, rho * c->p[i] / (gam * nrm));
        }
        fill_f32<<<nblocks(nv), BLOCK, 0, st>>>(c->T, nv, (float)t_data_scalar);
    }
    double t_prior = INFINITY;
    if (tgv) {
        // block n-1: ||(grad, -I)|| = sqrt(||grad||^2 + 1); block n: the bound ||grad||
        const double gn = grad_norm(geom->nx, geom->ny, geom->nz);
        c->prior_norm = std::sqrt(gn * gn + 1.0);
        // ||E|| <= ||grad|| (||E w||_F^2 <= sum_k ||grad w_k||^2): the closed-form bound keeps
        // the step condition exact, where a truncated power iteration approaches ||E||
        // from below
        c->prior_norm2 = gn;
        c->prior_sigma = gam * rho / c->prior_norm;
        c->prior_sigma2 = gam * rho / c->prior_norm2;
        const double t1 = rho * c->p[c->m] / (gam * c->prior_norm);
        const double t2 = rho * c->p[c->m + 1] / (gam * c->prior_norm2);
        c->tw = std::min(t1, t2);
        // the minimum over all blocks caps u as well, unless block n (0, E), which does not
        // act on u, is kept to w
        t_prior = (params->flags & SPDHG_FLAG_TGV_SPLIT_T) ? t1 : c->tw;
    } else if (prior) {
        if (params->prior == SPDHG_PRIOR_DTV) {
            img_to_zf<<<img_grid(geom->nx, geom->ny, geom->nz), TT * 8, 0, st>>>(
                geom->nx, geom->ny, geom->nz, side, c->scr);
            dtv_field<<<nblocks(nv), BLOCK, 0, st>>>(c->prior_args(), c->scr,
                                                     (float)params->eta, c->xi);
            double nrm = 0.0;
            if ((rc = power_norm_dgrad(c, &nrm, st))) return bail(rc);
            c->prior_norm = nrm;
        } else {
            c->prior_norm = grad_norm(geom->nx, geom->ny, geom->nz);
        }
        c->prior_sigma = gam * rho / c->prior_norm;
        t_prior = rho * c->p[c->m] / (gam * c->prior_norm);
    }
    finalize_T<<<nblocks(nv), BLOCK, 0, st>>>(c->T, nv, (float)t_prior);
    // EM-type updates (eq. OSEM): 1 / (A_i^T 1) of every subset
    if (c->em_inv) {
        for (int i = 0; i < c->m; ++i) {
            int a0, step, cnt;
            subset_angles(geom, c->m, i, a0, step, cnt);
            const int64_t nsub = (int64_t)cnt * np * geom->n_rad;
            to_rows<<<nblocks(nsub), BLOCK, 0, st>>>(c->tab.G, c->mp, 0, nullptr, a0, step, cnt,
                                                       c->dscr);
            BwdArgs B = c->bwd_args();
            B.d = c->dscr;
            B.out = c->em_inv + (int64_t)i * nv;
            if ((rc = launch_bwd<B_PLAIN>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr)))
                return bail(rc);
            reciprocal_on_support<<<nblocks(nv), BLOCK, 0, st>>>(B.out, nv, B.out);
        }
    }
    // y = 0, z = 0, prior duals = 0
    fill_f32<<<nblocks(nb), BLOCK, 0, st>>>(c->y, nb, 0.0f);
    fill_f32<<<nblocks(nv), BLOCK, 0, st>>>(c->z, nv, 0.0f);
    if (c->zlo) fill_f32<<<nblocks(2 * nv), BLOCK, 0, st>>>(c->zlo, 2 * nv, 0.0f);
    if (prior) fill_f32<<<nblocks(6 * nv), BLOCK, 0, st>>>(c->yn[0], 6 * nv, 0.0f);
    if (tgv) {  // w = 0, z_w = 0, q2 = 0
        fill_f32<<<nblocks(6 * nv), BLOCK, 0, st>>>(c->w[0], 6 * nv, 0.0f);
        fill_f32<<<nblocks(3 * nv), BLOCK, 0, st>>>(c->zw, 3 * nv, 0.0f);
        fill_f32<<<nblocks(12 * nv), BLOCK, 0, st>>>(c->q2[0], 12 * nv, 0.0f);
    }
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
    }
    if ((rc = export_x(c, st))) return bail(rc);
    int64_t max_sub = 0;
    for (int i = 0; i < c->m; ++i) {
        int a0, step, cnt;
        subset_angles(geom, c->m, i, a0, step, cnt);
        max_sub = std::max<int64_t>(max_sub, (int64_t)cnt * np * geom->n_rad);
    }
    c->max_sub_bins = max_sub;
    {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return bail(fail(SPDHG_E_HIP, hipGetErrorString(e)));
    }
    *out = c;
    return SPDHG_OK;
}

}  // extern "C"

namespace {

// FP64 objective of x (NULL: the current iterate) into out[0..3] = [psi, data, prior, 0].
int objective_into(spdhg_ctx* c, const float* x, double* out_dev, hipStream_t st) {
    const spdhg_geom& g = c->geom;
    const float* xx = c->xcur();
    if (x) {
        img_to_zf<<<img_grid(g.nx, g.ny, g.nz), TT * 8, 0, st>>>(g.nx, g.ny, g.nz, x, c->scr);
        xx = c->scr;
    }
    const int64_t nv = c->nv;
    FwdArgs F = c->fwd_args();
    F.x = xx;
    F.mult = c->mp;
    F.b = c->bp;
    F.r = c->rp;
    F.part = c->part;
    int rc;
    if ((rc = launch_fwd<F_OBJ>(F, 0, 1, g.n_ang, st))) return rc;
    const int64_t nblk = (int64_t)g.n_ang * g.n_rad;
    reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblk, out_dev, 1, 1.0);
    if (c->zw) {
        if ((rc = settle_w(c, st))) return rc;
        tgv_obj<<<nblocks(nv), BLOCK, 0, st>>>(g.nx, g.ny, g.nz, c->prm.alpha, c->prm.alpha1, xx,
                                               c->w[c->w_cur], c->part);
    } else {
        tv_obj<<<nblocks(nv), BLOCK, 0, st>>>(c->prior_args(), xx, c->xi, c->part,
                                              c->prm.prior != SPDHG_PRIOR_NONE);
    }
    reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblocks(nv), out_dev, 2, 1.0);
    // failure flag: non-finite voxels of the image (and of w for TGV)
    count_nonfinite<<<nblocks(nv), BLOCK, 0, st>>>(xx, nv, c->part);
    if (c->zw && !x)
        count_nonfinite<<<nblocks(3 * nv), BLOCK, 0, st>>>(c->w[c->w_cur], 3 * nv,
                                                           c->part + nblocks(nv));
    reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblocks(nv) + ((c->zw && !x) ? nblocks(3 * nv) : 0),
                                      out_dev, 3, 1.0);
    combine_objective<<<1, 64, 0, st>>>(out_dev);
    LAUNCH_CHECK();
    return SPDHG_OK;
}

}  // namespace

namespace {

// Block of the context's next iteration (Algorithm 2, block sampling): SplitMix64 output k
// mapped through the cumulative probabilities.
int draw_block(const spdhg_ctx* c) {
    const uint64_t zr = splitmix64(c->prm.seed, (uint64_t)c->k);
    const double u = (double)(zr >> 11) * (1.0 / 9007199254740992.0);
    int i = 0;
    while (!(u < c->cum[i])) ++i;
    return i;
}

// The TV-type prior block's fused kernel (dual step, adjoint, z update and primal step)
// from the current iterate and prior dual into the other buffers.
int launch_tv(spdhg_ctx* c, const PriorArgs& P, hipStream_t st) {
    const spdhg_geom& g = c->geom;
    const float* xin = c->xcur();
    const float* yin = c->yn[c->yn_cur];
    const bool pair = c->zlo != nullptr;
    if (prior_use_wave(g, 3)) {
        const int ly = std::min(TV_WAVE_LY, g.ny);
        auto k = P.dtv ? (pair ? tv_wave<true, true> : tv_wave<true, false>)
                       : (pair ? tv_wave<false, true> : tv_wave<false, false>);
        return klaunch(k, tv_wave_blocks(g, ly), 256, 0, st, P, ly, xin, c->xother(), yin,
                       c->yn[1 - c->yn_cur], c->z, (const float*)c->T, (const float*)c->xi);
    }
    const PriorTile TL = prior_tile(g);
    return klaunch(pair ? tv_iter<true> : tv_iter<false>, prior_blocks(g, TL),
                   TL.tx * TL.ty * g.nz, 0, st, P, TL, xin, c->xother(), yin,
                   c->yn[1 - c->yn_cur], c->z, (const float*)c->T, (const float*)c->xi);
}

// One iteration of Algorithm 2 on block i: dual step, backprojected dual change, z update,
// extrapolation and the next primal step (fused), then the state's buffer parities.
int one_iteration(spdhg_ctx* c, int i, hipStream_t st) {
    const float inv_p = (float)(1.0 / c->p[i]);
    int rc;
    if (i < c->m) {
        int a0, step, cnt;
        subset_angles(&c->geom, c->m, i, a0, step, cnt);
        FwdArgs F = c->fwd_args();
        F.x = c->xcur();
        F.mult = c->mp;
        F.b = c->bp;
        F.r = c->rp;
        F.sigma = c->sigma;
        F.sig_s = c->prm.precond ? 0.0f : (float)c->data_sigma[i];
        F.y = c->y;
        F.d = c->dscr;
        F.split = c->fwd_split;
        if ((rc = prof_begin(c, SPDHG_PROF_FWD, st))) return rc;
        if ((rc = launch_fwd<F_DUAL>(F, a0, step, cnt, st))) return rc;
        if ((rc = prof_end(c, st))) return rc;
        BwdArgs B = c->bwd_args();
        B.d = c->dscr;
        B.inv_p = inv_p;
        B.z = c->z;
        B.x = c->xcur();
        B.T = c->T;
        if ((rc = prof_begin(c, SPDHG_PROF_BWD, st))) return rc;
        rc = c->zlo ? launch_bwd<B_PAIR>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr)
                    : launch_bwd<B_ITER>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr);
        if (rc) return rc;
        if ((rc = prof_end(c, st))) return rc;
        if (c->zw) c->w_pending += 1;  // primal step for w: w -= T_w z_w (z_w unchanged)
    } else if (c->zw) {
        const int j = i - c->m;
        if ((rc = settle_w(c, st))) return rc;
        TgvArgs A = c->tgv_args(j);
        A.inv_p = inv_p;
        if ((rc = prof_begin(c, SPDHG_PROF_PRIOR, st))) return rc;
        const PriorTile TL = prior_tile(c->geom);
        const int nb_t = prior_blocks(c->geom, TL), nt_t = TL.tx * TL.ty * c->geom.nz;
        const int ly = std::min(TV_WAVE_LY, c->geom.ny);
        const float* xin = c->xcur();
        const float* win = c->w[c->w_cur];
        float* const* dual = j == 0 ? c->yn : c->q2;
        const int dcur = j == 0 ? c->yn_cur : c->q2_cur;
        const float* qin = dual[dcur];
        float* wout = c->w[1 - c->w_cur];
        const float* T = c->T;
        if (prior_use_wave(c->geom, 6)) {
            const unsigned nbw = tv_wave_blocks(c->geom, ly);
            rc = j == 0 ? klaunch(tgv1_wave, nbw, 256, 0, st, A, ly, xin, c->xother(), win, wout,
                                  qin, dual[1 - dcur], c->z, c->zw, T)
                        : klaunch(tgv2_wave, nbw, 256, 0, st, A, ly, xin, c->xother(), win, wout,
                                  qin, dual[1 - dcur], (const float*)c->z, c->zw, T);
        } else {
            rc = j == 0 ? klaunch(tgv1_iter, nb_t, nt_t, 0, st, A, TL, xin, c->xother(), win,
                                  wout, qin, dual[1 - dcur], c->z, c->zw, T)
                        : klaunch(tgv2_iter, nb_t, nt_t, 0, st, A, TL, xin, c->xother(), win,
                                  wout, qin, dual[1 - dcur], (const float*)c->z, c->zw, T);
        }
        if (rc) return rc;
        if (j == 0)
            c->yn_cur ^= 1;
        else
            c->q2_cur ^= 1;
        if ((rc = prof_end(c, st))) return rc;
        c->x_cur ^= 1;
        c->w_cur ^= 1;
    } else {
        PriorArgs P = c->prior_args();
        P.inv_p = inv_p;
        if ((rc = prof_begin(c, SPDHG_PROF_PRIOR, st))) return rc;
        if ((rc = launch_tv(c, P, st))) return rc;
        if ((rc = prof_end(c, st))) return rc;
        c->x_cur ^= 1;
        c->yn_cur ^= 1;
    }
    c->k += 1;
    return SPDHG_OK;
}

}  // namespace

// ====================================================================== persistent epoch graphs
// One HIP graph holds an epoch of every problem of a batch: per problem a chain of kernel
// nodes, one group per iteration slot (then the end of the epoch: the owed w steps and the
// export of the iterate), where each group holds every kernel that an iteration of any
// block could launch in that slot.  The graph is instantiated once (twice: two executable
// copies alternate, so one can be updated while the other runs).  Before each epoch the
// blocks are drawn on the host exactly as in spdhg_iterate, whose launches are recorded;
// the recorded arguments are written into the matching nodes and the other nodes of each
// group are disabled.  The kernels and their arguments are those of an eager run, so the
// result is bitwise the same.
struct GraphSlot {
    std::vector<hipGraphNode_t> nodes;
    std::vector<const void*> funcs;
};

struct GraphProblem {
    spdhg_ctx* c = nullptr;
    std::vector<GraphSlot> slots;  // iters_per_epoch iteration slots, then the end slot
};

struct spdhg_graph {
    std::vector<GraphProblem> probs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int next = 0;
    std::vector<std::shared_ptr<void>> keep[2];  // argument storage of the last update
};

namespace {

struct CtxState {
    int64_t k, w_pending;
    int x_cur, yn_cur, w_cur, q2_cur;
};

CtxState ctx_state(const spdhg_ctx* c) {
    return {c->k, c->w_pending, c->x_cur, c->yn_cur, c->w_cur, c->q2_cur};
}

void set_ctx_state(spdhg_ctx* c, const CtxState& s) {
    c->k = s.k;
    c->w_pending = s.w_pending;
    c->x_cur = s.x_cur;
    c->yn_cur = s.yn_cur;
    c->w_cur = s.w_cur;
    c->q2_cur = s.q2_cur;
}

// Make `into` a supersequence of `seq` (kernels in launch order).
void merge_seq(std::vector<const void*>& into, const std::vector<const void*>& seq) {
    size_t pos = 0;
    for (const void* f : seq) {
        size_t k = pos;
        while (k < into.size() && into[k] != f) ++k;
        if (k < into.size()) {
            pos = k + 1;
        } else {
            into.insert(into.begin() + pos, f);
            ++pos;
        }
    }
}

// Launches of one iteration on block i (end = -1: the end of an epoch), recorded without
// changing the context's state.  pending: TGV owes w steps first.
int record_block(spdhg_ctx* c, int i, bool pending, Recorder& r) {
    const CtxState s0 = ctx_state(c);
    if (pending && c->zw) c->w_pending = 1;
    g_rec = &r;
    int rc = SPDHG_OK;
    if (i >= 0) {
        rc = one_iteration(c, i, nullptr);
    } else if ((rc = settle_w(c, nullptr)) == SPDHG_OK) {
        rc = export_x(c, nullptr);
    }
    g_rec = nullptr;
    set_ctx_state(c, s0);
    return rc;
}

hipKernelNodeParams node_params(const LaunchRec& r) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(r.func);
    kp.gridDim = r.grid;
    kp.blockDim = r.block;
    kp.sharedMemBytes = r.lds;
    kp.kernelParams = const_cast<void**>(r.ptrs.data());
    kp.extra = nullptr;
    return kp;
}

int graph_build(spdhg_graph* G) {
    HIP_TRY(hipGraphCreate(&G->graph, 0));
    for (GraphProblem& P : G->probs) {
        spdhg_ctx* c = P.c;
        // the kernels any block can launch in an iteration slot, and at the end
        std::vector<const void*> it_funcs, end_funcs;
        std::map<const void*, LaunchRec> proto;
        auto absorb = [&](Recorder& r, std::vector<const void*>& into) {
            std::vector<const void*> seq;
            for (LaunchRec& x : r.recs) {
                seq.push_back(x.func);
                proto.emplace(x.func, x);
            }
            merge_seq(into, seq);
        };
        for (int i = 0; i < c->n; ++i)
            for (int pend = 0; pend < (c->zw ? 2 : 1); ++pend) {
                Recorder r;
                int rc = record_block(c, i, pend != 0, r);
                if (rc) return rc;
                absorb(r, it_funcs);
            }
        for (int pend = 0; pend < (c->zw ? 2 : 1); ++pend) {
            Recorder r;
            int rc = record_block(c, -1, pend != 0, r);
            if (rc) return rc;
            absorb(r, end_funcs);
        }
        const int64_t L = c->iters_per_epoch;
        P.slots.resize((size_t)L + 1);
        hipGraphNode_t prev = nullptr;
        for (int64_t sl = 0; sl <= L; ++sl) {
            GraphSlot& S = P.slots[(size_t)sl];
            S.funcs = sl < L ? it_funcs : end_funcs;
            for (const void* f : S.funcs) {
                hipKernelNodeParams kp = node_params(proto.at(f));
                hipGraphNode_t node = nullptr;
                HIP_TRY(hipGraphAddKernelNode(&node, G->graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                              &kp));
                S.nodes.push_back(node);
                prev = node;
            }
        }
    }
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(hipGraphInstantiate(&G->exec[b], G->graph, nullptr, nullptr, 0));
        HIP_TRY(hipEventCreateWithFlags(&G->done[b], hipEventDisableTiming));
    }
    return SPDHG_OK;
}

// Draw the next epoch of every problem (advancing the contexts as spdhg_iterate does) and
// write its launches into executable copy b.
int graph_update(spdhg_graph* G, int b) {
    G->keep[b].clear();
    hipGraphExec_t ex = G->exec[b];
    for (GraphProblem& P : G->probs) {
        spdhg_ctx* c = P.c;
        Recorder r;
        g_rec = &r;
        int rc = spdhg_iterate(c, c->iters_per_epoch, nullptr);
        g_rec = nullptr;
        if (rc) return rc;
        const size_t L = P.slots.size() - 1;
        if (r.marks.size() != L + 1) return fail(SPDHG_E_STATE, "epoch graph: slot count changed");
        for (size_t sl = 0; sl <= L; ++sl) {
            size_t idx = r.marks[sl];
            const size_t end = sl < L ? r.marks[sl + 1] : r.recs.size();
            GraphSlot& S = P.slots[sl];
            for (size_t n = 0; n < S.nodes.size(); ++n) {
                if (idx < end && r.recs[idx].func == S.funcs[n]) {
                    hipKernelNodeParams kp = node_params(r.recs[idx]);
                    HIP_TRY(hipGraphExecKernelNodeSetParams(ex, S.nodes[n], &kp));
                    HIP_TRY(hipGraphNodeSetEnabled(ex, S.nodes[n], 1));
                    ++idx;
                } else {
                    HIP_TRY(hipGraphNodeSetEnabled(ex, S.nodes[n], 0));
                }
            }
            if (idx != end)
                return fail(SPDHG_E_STATE, "epoch graph: a launch has no node in its slot");
        }
        for (LaunchRec& x : r.recs) G->keep[b].push_back(x.vals);
    }
    return SPDHG_OK;
}

}  // namespace

extern "C" {

int spdhg_graph_create(spdhg_ctx* const* ctxs, int32_t n, spdhg_graph** out) {
    if (!out) return fail(SPDHG_E_ARG, "out is NULL");
    *out = nullptr;
    if (!ctxs || n <= 0) return fail(SPDHG_E_ARG, "bad context list");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(SPDHG_E_ARG, "NULL context in the graph");
        if (ctxs[i]->prof) return fail(SPDHG_E_STATE, "per-kernel profiling is not recorded in graphs");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(SPDHG_E_ARG, "a context appears twice");
    }
    spdhg_graph* G = new spdhg_graph();
    for (int i = 0; i < n; ++i) {
        GraphProblem P;
        P.c = ctxs[i];
        G->probs.push_back(P);
    }
    int rc = graph_build(G);
    if (rc) {
        spdhg_graph_destroy(G);
        return rc;
    }
    *out = G;
    return SPDHG_OK;
}

int spdhg_graph_epoch(spdhg_graph* G, int32_t n_epochs, void* stream) {
    if (!G) return fail(SPDHG_E_ARG, "graph is NULL");
    if (n_epochs < 0) return fail(SPDHG_E_ARG, "n_epochs < 0");
    hipStream_t st = (hipStream_t)stream;
    for (GraphProblem& P : G->probs)
        if (P.c->prof) return fail(SPDHG_E_STATE, "per-kernel profiling is not recorded in graphs");
    for (int e = 0; e < n_epochs; ++e) {
        const int b = G->next;
        if (G->used[b]) HIP_TRY(hipEventSynchronize(G->done[b]));  // its previous run is over
        int rc = graph_update(G, b);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(G->exec[b], st));
        HIP_TRY(hipEventRecord(G->done[b], st));
        G->used[b] = true;
        G->next ^= 1;
    }
    return SPDHG_OK;
}

int spdhg_graph_destroy(spdhg_graph* G) {
    if (!G) return SPDHG_OK;
    for (int b = 0; b < 2; ++b) {
        if (G->used[b] && G->done[b]) (void)hipEventSynchronize(G->done[b]);
        if (G->exec[b]) (void)hipGraphExecDestroy(G->exec[b]);
        if (G->done[b]) (void)hipEventDestroy(G->done[b]);
    }
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return SPDHG_OK;
}

}  // extern "C"

extern "C" {

int spdhg_set_profiling(spdhg_ctx* c, int32_t on) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (on && c->ev.empty()) {
        // timing-only events: no system-scope fence (and so no cache writeback and
        // invalidation) at each record, which would slow the kernels being timed
        const size_t pairs = 1024;
        c->ev.resize(2 * pairs);
        c->ev_kind.resize(pairs);
        for (auto& e : c->ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    if (!on && c->prof) {
        int rc = prof_collect(c);
        if (rc) return rc;
    }
    c->prof = on != 0;
    for (int i = 0; i < SPDHG_PROF_KINDS; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_n[i] = 0;
    }
    return SPDHG_OK;
}

int spdhg_set_profiling_kinds(spdhg_ctx* c, int32_t mask) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (mask <= 0 || mask >= (1 << SPDHG_PROF_KINDS))
        return fail(SPDHG_E_ARG, "mask must name at least one kernel kind and no other bits");
    c->prof_mask = mask;
    return SPDHG_OK;
}

int spdhg_profile(spdhg_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(SPDHG_E_ARG, "NULL argument");
    int rc = prof_collect(c);
    if (rc) return rc;
    for (int i = 0; i < SPDHG_PROF_KINDS; ++i) {
        ms[i] = c->prof_ms[i];
        launches[i] = c->prof_n[i];
    }
    return SPDHG_OK;
}

int spdhg_iterate(spdhg_ctx* c, int64_t n_iters, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (n_iters < 0) return fail(SPDHG_E_ARG, "n_iters < 0");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    for (int64_t it = 0; it < n_iters; ++it) {
        if (g_rec) g_rec->marks.push_back(g_rec->recs.size());
        if ((rc = one_iteration(c, draw_block(c), st))) return rc;
    }
    if (g_rec) g_rec->marks.push_back(g_rec->recs.size());
    if ((rc = settle_w(c, st))) return rc;
    return export_x(c, st);
}

int spdhg_epoch(spdhg_ctx* c, int32_t n_epochs, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (n_epochs < 0) return fail(SPDHG_E_ARG, "n_epochs < 0");
    return spdhg_iterate(c, (int64_t)n_epochs * c->iters_per_epoch, stream);
}

int spdhg_epoch_graph(spdhg_ctx* c, int32_t n_epochs, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (n_epochs < 0) return fail(SPDHG_E_ARG, "n_epochs < 0");
    if (c->prof) return fail(SPDHG_E_STATE, "per-kernel profiling is not recorded in graphs");
    if (!c->graph) {
        spdhg_ctx* one[1] = {c};
        int rc = spdhg_graph_create(one, 1, &c->graph);
        if (rc) return rc;
    }
    return spdhg_graph_epoch(c->graph, n_epochs, stream);
}

int spdhg_pdhg_iterate(spdhg_ctx* c, int64_t n_iters, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (n_iters < 0) return fail(SPDHG_E_ARG, "n_iters < 0");
    if (c->m != 1) return fail(SPDHG_E_STATE, "PDHG needs a context with one data block (m = 1)");
    if (c->zw) return fail(SPDHG_E_NOTIMPL, "PDHG is not built for TGV");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    const spdhg_geom& g = c->geom;
    for (int64_t it = 0; it < n_iters; ++it) {
        // Algorithm 1: the dual step of every block from the same x ...
        FwdArgs F = c->fwd_args();
        F.x = c->xcur();
        F.mult = c->mp;
        F.b = c->bp;
        F.r = c->rp;
        F.sigma = c->sigma;
        F.sig_s = c->prm.precond ? 0.0f : (float)c->data_sigma[0];
        F.y = c->y;
        F.d = c->dscr;
        F.split = c->fwd_split;
        if ((rc = launch_fwd<F_DUAL>(F, 0, 1, g.n_ang, st))) return rc;
        BwdArgs B = c->bwd_args();
        B.d = c->dscr;
        if (c->n_prior == 0) {
            // ... one block: z += dz, x = max(x - T (z + dz), 0)
            B.inv_p = 1.0f;
            B.z = c->z;
            B.x = c->xcur();
            B.T = c->T;
            rc = c->zlo
                     ? launch_bwd<B_PAIR>(B, 0, 1, g.n_ang, st, c->bplan, c->tab.ang.data(), c->scr)
                     : launch_bwd<B_ITER>(B, 0, 1, g.n_ang, st, c->bplan, c->tab.ang.data(), c->scr);
            if (rc) return rc;
            continue;
        }
        // ... with a prior block: the data change dz_data into scr (the other iterate buffer
        // holds the two-class partial), then the prior kernel adds it to its own change
        // before z += dz and x = max(x - T (z + dz), 0)
        B.out = c->scr;
        if ((rc = launch_bwd<B_PLAIN>(B, 0, 1, g.n_ang, st, c->bplan, c->tab.ang.data(), c->xother())))
            return rc;
        PriorArgs P = c->prior_args();
        P.inv_p = 1.0f;
        P.dz_add = c->scr;
        if ((rc = launch_tv(c, P, st))) return rc;
        c->x_cur ^= 1;
        c->yn_cur ^= 1;
    }
    return export_x(c, st);
}

int spdhg_em_iterate(spdhg_ctx* c, int64_t n_subiters, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (n_subiters < 0) return fail(SPDHG_E_ARG, "n_subiters < 0");
    if (!c->em_inv) return fail(SPDHG_E_STATE, "the context was set up without SPDHG_FLAG_EM");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    for (int64_t it = 0; it < n_subiters; ++it) {
        const int i = (int)(c->em_k % c->m);
        int a0, step, cnt;
        subset_angles(&c->geom, c->m, i, a0, step, cnt);
        FwdArgs F = c->fwd_args();
        F.x = c->xcur();
        F.mult = c->mp;
        F.b = c->bp;
        F.r = c->rp;
        F.d = c->dscr;
        F.split = c->fwd_split;
        if ((rc = launch_fwd<F_EM>(F, a0, step, cnt, st))) return rc;
        BwdArgs B = c->bwd_args();
        B.d = c->dscr;
        B.x = c->xcur();
        B.T = c->em_inv + (int64_t)i * c->nv;
        if ((rc = launch_bwd<B_EM>(B, a0, step, cnt, st, c->bplan, c->tab.ang.data(), c->scr)))
            return rc;
        c->em_k += 1;
    }
    if (c->xlo && n_subiters > 0) {  // the EM steps replaced the iterate: its low part restarts
        fill_f32<<<nblocks(c->nv), BLOCK, 0, st>>>(c->xlo, c->nv, 0.0f);
        LAUNCH_CHECK();
    }
    return export_x(c, st);
}

int spdhg_info(const spdhg_ctx* c, int64_t* ipe, int64_t* done) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (ipe) *ipe = c->iters_per_epoch;
    if (done) *done = c->k;
    return SPDHG_OK;
}

int spdhg_objective(spdhg_ctx* c, const float* x, double* out_dev, void* stream) {
    if (!c || !out_dev) return fail(SPDHG_E_ARG, "NULL ctx or output");
    return objective_into(c, x, out_dev, (hipStream_t)stream);
}

int spdhg_gap(spdhg_ctx* c, double U, double* out_dev, void* stream) {
    if (!c || !out_dev) return fail(SPDHG_E_ARG, "NULL ctx or output");
    if (c->zw) return fail(SPDHG_E_NOTIMPL, "the duality gap is infinite for TGV (w has no bound)");
    if (!(U > 0)) return fail(SPDHG_E_ARG, "U must be > 0");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    double* obj = c->scal + 4;  // [psi, data, prior, -]
    if ((rc = objective_into(c, nullptr, obj, st))) return rc;
    const int64_t nb = c->nb, nv = c->nv;
    gap_dual<<<nblocks(nb), BLOCK, 0, st>>>(c->y, c->bp, c->rp, nb, c->part);
    reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblocks(nb), c->scal, 0, 1.0);
    gap_box<<<nblocks(nv), BLOCK, 0, st>>>(c->z, nv, U, c->part);
    reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblocks(nv), c->scal, 1, 1.0);
    if (c->yn[0]) {
        gap_prior<<<nblocks(nv), BLOCK, 0, st>>>(c->yn[c->yn_cur], nv, c->prm.alpha,
                                                 c->prm.prior == SPDHG_PRIOR_ATV, c->part);
        reduce_final<<<1, BLOCK, 0, st>>>(c->part, nblocks(nv), c->scal, 2, 1.0);
    } else {
        fill_f64<<<1, 64, 0, st>>>(c->scal + 2, 1, 0.0);
    }
    combine_gap<<<1, 64, 0, st>>>(out_dev, obj, c->masked_phi0, c->scal, c->scal + 2, c->scal + 1);
    LAUNCH_CHECK();
    return SPDHG_OK;
}

int spdhg_buffer(spdhg_ctx* c, int32_t which, float** ptr, int64_t* n) {
    if (!c || !ptr || !n) return fail(SPDHG_E_ARG, "NULL argument");
    switch (which) {
        case 0: *ptr = c->y; *n = c->nb; break;
        case 1: *ptr = c->z; *n = c->nv; break;
        case 2: *ptr = c->T; *n = c->nv; break;
        case 3: *ptr = c->sigma; *n = c->sigma ? c->nb : 0; break;
        case 4: *ptr = c->yn[c->yn_cur]; *n = c->yn[0] ? 3 * c->nv : 0; break;
        case 5: *ptr = c->w[c->w_cur]; *n = c->zw ? 3 * c->nv : 0; break;
        case 6: *ptr = c->q2[c->q2_cur]; *n = c->zw ? 6 * c->nv : 0; break;
        case 7: *ptr = c->zw; *n = c->zw ? 3 * c->nv : 0; break;
        case 8: *ptr = c->zlo; *n = c->zlo ? c->nv : 0; break;
        case 9: *ptr = c->xlo; *n = c->xlo ? c->nv : 0; break;
        default: return fail(SPDHG_E_ARG, "unknown buffer id");
    }
    return SPDHG_OK;
}

int spdhg_block_info(const spdhg_ctx* c, int32_t i, double* sigma, double* p, double* norm) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (i < 0 || i >= c->n) return fail(SPDHG_E_ARG, "block index out of range");
    if (p) *p = c->p[i];
    if (i < c->m) {
        if (sigma) *sigma = c->prm.precond ? NAN : c->data_sigma[i];
        if (norm) *norm = c->prm.precond ? NAN : c->data_norm[i];
    } else if (i == c->m) {
        if (sigma) *sigma = c->prior_sigma;
        if (norm) *norm = c->prior_norm;
    } else {
        if (sigma) *sigma = c->prior_sigma2;
        if (norm) *norm = c->prior_norm2;
    }
    return SPDHG_OK;
}

}  // extern "C"

namespace {

// Arrays of a checkpoint, in order: the iterate (and, for TGV, w), z (and z_w), y, the
// prior duals, then (SPDHG_FLAG_COMPENSATED) the low parts of z and the iterate.  `cur` gives the current buffers (save), else the first ones (load).
struct StatePart {
    float* p;
    int64_t n;
};

std::vector<StatePart> state_parts(spdhg_ctx* c, bool cur) {
    std::vector<StatePart> v;
    const int64_t nv = c->nv;
    v.push_back({cur ? c->xcur() : c->xa, nv});
    v.push_back({c->z, nv});
    v.push_back({c->y, c->nb});
    if (c->yn[0]) v.push_back({cur ? c->yn[c->yn_cur] : c->yn[0], 3 * nv});
    if (c->zw) {
        v.push_back({cur ? c->w[c->w_cur] : c->w[0], 3 * nv});
        v.push_back({c->zw, 3 * nv});
        v.push_back({cur ? c->q2[c->q2_cur] : c->q2[0], 6 * nv});
    }
    if (c->zlo) v.push_back({c->zlo, 2 * nv});  // low parts of z and x
    return v;
}

}  // namespace

extern "C" {

int spdhg_state_bytes(const spdhg_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(SPDHG_E_ARG, "NULL argument");
    size_t n = 256;
    for (const StatePart& sp : state_parts(const_cast<spdhg_ctx*>(c), true)) n += align256(sp.n * 4);
    *bytes = n;
    return SPDHG_OK;
}

int spdhg_save_state(spdhg_ctx* c, void* dst, size_t bytes, void* stream) {
    size_t need = 0;
    int rc = spdhg_state_bytes(c, &need);
    if (rc) return rc;
    if (!dst || bytes < need) return fail(SPDHG_E_ARG, "state buffer too small");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = settle_w(c, st))) return rc;
    char* p = (char*)dst;
    for (const StatePart& sp : state_parts(c, true)) {
        HIP_TRY(hipMemcpyAsync(p, sp.p, sp.n * 4, hipMemcpyDeviceToDevice, st));
        p += align256(sp.n * 4);
    }
    // iteration counter: the random block sequence continues from it
    int64_t hdr[4] = {c->k, c->nv, c->nb, 0x5350444847ll};
    HIP_TRY(hipMemcpyAsync(p, hdr, sizeof(hdr), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPDHG_OK;
}

int spdhg_load_state(spdhg_ctx* c, const void* src, size_t bytes, void* stream) {
    size_t need = 0;
    int rc = spdhg_state_bytes(c, &need);
    if (rc) return rc;
    if (!src || bytes < need) return fail(SPDHG_E_ARG, "state buffer too small");
    hipStream_t st = (hipStream_t)stream;
    const std::vector<StatePart> parts = state_parts(c, false);
    size_t off = 0;
    for (const StatePart& sp : parts) off += align256(sp.n * 4);
    int64_t hdr[4];
    HIP_TRY(hipMemcpyAsync(hdr, (const char*)src + off, sizeof(hdr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hdr[1] != c->nv || hdr[2] != c->nb || hdr[3] != 0x5350444847ll)
        return fail(SPDHG_E_STATE, "state does not belong to this problem");
    c->x_cur = c->yn_cur = c->w_cur = c->q2_cur = 0;
    c->w_pending = 0;
    const char* p = (const char*)src;
    for (const StatePart& sp : parts) {
        HIP_TRY(hipMemcpyAsync(sp.p, p, sp.n * 4, hipMemcpyDeviceToDevice, st));
        p += align256(sp.n * 4);
    }
    c->k = hdr[0];
    return export_x(c, st);
}

int spdhg_set_walk(spdhg_ctx* c, int32_t interleave) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (interleave != 0 && interleave != 1) return fail(SPDHG_E_ARG, "interleave must be 0 or 1");
    c->interleave = interleave;
    if (c->graph) {  // its kernels may change: rebuilt on the next graph epoch
        spdhg_graph_destroy(c->graph);
        c->graph = nullptr;
    }
    return SPDHG_OK;
}

int spdhg_set_tuning(spdhg_ctx* c, int32_t fwd_split) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (fwd_split != 0 && fwd_split != 1 && fwd_split != 2 && fwd_split != 4 && fwd_split != 8 &&
        fwd_split != 20 && fwd_split != 40)
        return fail(SPDHG_E_ARG, "fwd_split must be 0, 1, 2, 4, 8, 20 or 40");
    c->fwd_split = fwd_split;
    if (c->graph) {  // its kernels may change: rebuilt on the next graph epoch
        spdhg_graph_destroy(c->graph);
        c->graph = nullptr;
    }
    return SPDHG_OK;
}

// The backprojection plan of a gather tiling (1: strips, one per workgroup; 3: strips of
// four consecutive primary indices per workgroup; 2: groups of whole columns); false if
// the tiling does not apply.
static bool gather_plan(const spdhg_ctx* c, int gather, BwdPlan& out) {
    if (gather == 2) {
        out = BwdPlan{};
        return min_bin_spacing(c->tab) >= 0.5;
    }
    if (!c->bplan_auto.strip) return false;
    out = c->bplan_auto;
    if (gather == 3) {
        out.wj = 4;
        if (out.lds * out.wj > 64 * 1024) return false;
    }
    return true;
}

int spdhg_set_gather(spdhg_ctx* c, int32_t gather) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (gather < 0 || gather > 3) return fail(SPDHG_E_ARG, "gather must be 0, 1, 2 or 3");
    BwdPlan plan = c->bplan_auto;
    if (gather != 0 && !gather_plan(c, gather, plan))
        return fail(SPDHG_E_ARG, "the strip gather does not apply to this geometry");
    c->gather = gather;
    c->bplan = plan;
    if (c->graph) {  // its kernels change: rebuilt on the next graph epoch
        spdhg_graph_destroy(c->graph);
        c->graph = nullptr;
    }
    return SPDHG_OK;
}

int spdhg_get_tuning(const spdhg_ctx* c, int32_t* fwd_split, int32_t* gather) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    if (fwd_split) *fwd_split = c->fwd_split;
    if (gather) *gather = !c->bplan.strip ? 2 : c->bplan.wj > 1 ? 3 : 1;
    return SPDHG_OK;
}

int spdhg_autotune(spdhg_ctx* c, int32_t* fwd_split, double* ms, void* stream) {
    if (!c) return fail(SPDHG_E_ARG, "ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    int a0, step, cnt;
    int rc = subset_angles(&c->geom, c->m, 0, a0, step, cnt);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int cand[6] = {1, 2, 4, 8, 20, 40};
    int best = 0;
    double best_ms = INFINITY;
    for (int ci = 0; ci < 6 && rc == SPDHG_OK; ++ci) {
        if (cand[ci] >= 20 && rays_per_lane((c->tab.G.n_planes + cand[ci] / 10 - 1) / (cand[ci] / 10)) > 16)
            continue;
        // the subset projection walk, timed on the objective epilogue (writes partials only)
        FwdArgs F = c->fwd_args();
        F.x = c->xcur();
        F.mult = c->mp;
        F.b = c->bp;
        F.r = c->rp;
        F.part = c->part;
        F.split = cand[ci];
        if ((rc = launch_fwd<F_OBJ>(F, a0, step, cnt, st))) break;  // warm-up
        hipError_t err = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && rc == SPDHG_OK; ++r) rc = launch_fwd<F_OBJ>(F, a0, step, cnt, st);
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) rc = fail(SPDHG_E_HIP, hipGetErrorString(err));
        if (rc == SPDHG_OK && t / 3.0 < best_ms) {
            best_ms = t / 3.0;
            best = cand[ci];
        }
    }
    // the gather's tiling: strips of BS_W columns (where they apply) against groups of whole
    // columns, timed on the subset-0 backprojection of the stale dual change into the
    // scratch image (the other iterate buffer takes the two-class partial: the next prior
    // iteration overwrites all of it)
    int best_gather = c->bplan_auto.strip ? 1 : 2;
    double best_bms = INFINITY;
    const int gcand[3] = {1, 3, 2};
    for (int gi = 0; gi < 3 && rc == SPDHG_OK && c->bplan_auto.strip; ++gi) {
        BwdPlan plan;
        if (!gather_plan(c, gcand[gi], plan)) continue;
        BwdArgs B = c->bwd_args();
        B.d = c->dscr;
        B.out = c->scr;
        if ((rc = launch_bwd<B_PLAIN>(B, a0, step, cnt, st, plan, c->tab.ang.data(), c->xother())))
            break;  // warm-up
        hipError_t err = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && rc == SPDHG_OK; ++r)
            rc = launch_bwd<B_PLAIN>(B, a0, step, cnt, st, plan, c->tab.ang.data(), c->xother());
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) rc = fail(SPDHG_E_HIP, hipGetErrorString(err));
        if (rc == SPDHG_OK && t / 3.0 < best_bms) {
            best_bms = t / 3.0;
            best_gather = gcand[gi];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    c->fwd_split = best;
    c->gather = best_gather;
    gather_plan(c, best_gather, c->bplan);
    if (c->graph) {
        spdhg_graph_destroy(c->graph);
        c->graph = nullptr;
    }
    if (fwd_split) *fwd_split = best;
    if (ms) *ms = best_ms;
    return SPDHG_OK;
}

int spdhg_batch_epoch(spdhg_ctx* const* ctxs, int32_t n, int32_t n_epochs, int32_t n_streams,
                      int32_t use_graph, void* stream) {
    if (!ctxs || n < 0 || n_epochs < 0) return fail(SPDHG_E_ARG, "bad batch arguments");
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(SPDHG_E_ARG, "NULL context in batch");
        if (ctxs[i]->prof) return fail(SPDHG_E_STATE, "profiling is not recorded in batches");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(SPDHG_E_ARG, "a context appears twice in the batch");
    }
    if (n == 0 || n_epochs == 0) return SPDHG_OK;
    hipStream_t st = (hipStream_t)stream;
    if (use_graph) {
        // one persistent graph for the n_epochs batch epochs
        spdhg_graph* G = nullptr;
        int rc = spdhg_graph_create(ctxs, n, &G);
        if (rc) return rc;
        rc = spdhg_graph_epoch(G, n_epochs, stream);
        const hipError_t err = hipStreamSynchronize(st);
        spdhg_graph_destroy(G);
        if (rc == SPDHG_OK && err != hipSuccess) rc = fail(SPDHG_E_HIP, hipGetErrorString(err));
        return rc;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int ns = std::max(1, std::min<int>(std::min(n_streams, 8), n));
    std::vector<hipStream_t> pool;
    int rc0 = worker_streams(dev, ns, pool);
    if (rc0) return rc0;
    std::vector<hipEvent_t> ev(ns + 1, nullptr);
    for (auto& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int rc = SPDHG_OK;
    hipError_t err = hipSuccess;
    // fork: every worker stream waits for the caller's stream; problem i runs on worker
    // i mod ns (its iterations in order, exactly as a solo run); join back
    err = hipEventRecord(ev[ns], st);
    for (int w = 0; w < ns && err == hipSuccess; ++w) err = hipStreamWaitEvent(pool[w], ev[ns], 0);
    for (int i = 0; i < n && err == hipSuccess && rc == SPDHG_OK; ++i)
        rc = spdhg_iterate(ctxs[i], (int64_t)n_epochs * ctxs[i]->iters_per_epoch, pool[i % ns]);
    for (int w = 0; w < ns && err == hipSuccess; ++w) {
        err = hipEventRecord(ev[w], pool[w]);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, ev[w], 0);
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc == SPDHG_OK && err != hipSuccess) rc = fail(SPDHG_E_HIP, hipGetErrorString(err));
    return rc;
}

int spdhg_destroy(spdhg_ctx* c) {
    if (!c) return SPDHG_OK;
    if (c->graph) spdhg_graph_destroy(c->graph);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return SPDHG_OK;
}

}  // extern "C"
