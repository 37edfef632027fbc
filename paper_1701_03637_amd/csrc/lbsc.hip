// Host runtime of the lbsc C ABI (see include/lbsc.h): validation, scratch
// layout, work-item schedules, launches, HIP graphs, the tile tuner and
// checkpoints. Device work is in kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "lbsc.h"
#include "kernels.h"
#include "kernels1.h"

// Scratch for contexts bound with lbsc_bind_static: one array per device,
// held until the process ends. In host code this name is only a stand-in for
// the symbol; its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[LBSC_STATIC_SCRATCH_BYTES];

using lbsc::Inst;
using lbsc::Item;

namespace {

constexpr size_t kAlign = 256;

// Compute units of the current device (256 on an MI355X), which the default
// schedule fills; 256 if the query fails.
int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 256;
    return cus;
}
constexpr uint64_t kMagic = 0x4C4253432D434B31ull;  // "LBSC-CK1"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int prec) { return prec == LBSC_FP64 ? 8 : (prec == LBSC_FP32S ? 4 : 2); }

// The per-node-shift FP16 forms (FP16N, FP16NF): FP32 rest pairs, FP16 moving
// pairs.
bool per_node(int prec) { return prec == LBSC_FP16N || prec == LBSC_FP16NF; }

// Components of an instance: 1 (single-component multiphase form) or 2.
int ncomp_of(const lbsc_params& p) { return p.ncomp == 1 ? 1 : 2; }

// Slab elements per in-plane element (see kSlabPlanes in kernels.h and
// kSlabPlanes1 in kernels1.h).
int slab_planes(int prec, int ncomp)
{
    if (ncomp == 1) return lbsc::kSlabPlanes1;
    return per_node(prec) ? 40 : 2 * lbsc::kQ;
}

// Elements between population planes beyond nx*ny rounded up to 64. A
// negative plane_pad asks for the automatic skew: planes whose byte stride
// is a multiple of 64 KiB put the same node of every plane on the same HBM
// channels, and on the 512^3 lattice (1 MiB planes) 320 elements more
// (1280 B in FP32) measured 6 % faster (FP32S, FP64; FP16N unchanged);
// lattices of fewer than 2^14 nodes per plane showed no effect.
int64_t plane_pad_of(const lbsc_params& p)
{
    if (p.plane_pad >= 0) return p.plane_pad;
    const int64_t n = (int64_t)align_up((size_t)p.nx * p.ny, 64);
    // bytes per node of one plane (pair planes hold both components)
    const int64_t e = ncomp_of(p) == 1 ? (p.precision == LBSC_FP64 ? 8 : 4)
                                       : (p.precision == LBSC_FP64 ? 16 : p.precision == LBSC_FP32S ? 8 : 4);
    return (n >= 16384 && (n * e) % 65536 == 0) ? 320 : 0;
}

struct CkptHeader {
    uint64_t magic;
    int32_t n_inst, precision;
    int64_t step;
    int64_t pop_bytes;
    int32_t cur, pad;
};

}  // namespace

struct lbsc_ctx {
    int n_inst = 0;
    int precision = 0;
    size_t elem = 0;
    std::vector<lbsc_params> params;
    std::vector<Inst> inst;       // host copy of the device table
    std::vector<Item> items;
    lbsc_tiles tiles{0, 0, 0, 0, 0};
    std::vector<lbsc_tiles> inst_tiles;   // per-instance tw, th, nzc (0: the context's)
    int nt = 256;
    int variant = 1;              // resolved k_step variant: 1 keep, 2 re-pull, 3 pipelined
    int cus = 256;                // compute units the default schedule fills
    int static_dev = -1;          // device whose static scratch this context uses (-1: caller's buffer)
    int ncomp = 2;                // components of every instance
    size_t pop_elems = 0;         // elements per population buffer
    size_t max_items = 0;
    int max_nz = 0;
    // scratch layout (byte offsets)
    size_t off_inst = 0, off_items = 0, off_eacc = 0, off_ebase = 0, off_part = 0, off_out = 0, scratch_bytes = 0;
    // bound buffers
    void* pop[2] = {nullptr, nullptr};
    char* scratch = nullptr;
    bool bound = false;
    int cur = 0;                  // buffer holding the stored populations
    int64_t step = 0;
    hipStream_t stream = nullptr;
    // graphs
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_steps = 0;
    std::string err;

    Inst* d_inst() { return reinterpret_cast<Inst*>(scratch + off_inst); }
    Item* d_items() { return reinterpret_cast<Item*>(scratch + off_items); }
    double* d_eacc() { return reinterpret_cast<double*>(scratch + off_eacc); }
    double* d_ebase() { return reinterpret_cast<double*>(scratch + off_ebase); }
    double* d_part() { return reinterpret_cast<double*>(scratch + off_part); }
    double* d_out() { return reinterpret_cast<double*>(scratch + off_out); }
};

namespace {

lbsc_status fail(lbsc_ctx* c, lbsc_status s, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIPCHK(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), LBSC_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Sink in the kernels' coordinates: above a solid wall of z_off planes the
// kernels' lattice starts at the caller's plane z_off, and the caller's
// z = 0 face is solid, not a sink.
lbsc::Sink make_sink(int kind, double rho_h, double radius, const double* center, int z_off)
{
    lbsc::Sink s{};
    s.kind = kind;
    s.no_zlo = z_off > 0 && kind == LBSC_SINK_FACES;
    s.rho_h = rho_h;
    s.r2 = radius * radius;
    s.cx = center[0];
    s.cy = center[1];
    s.cz = center[2] - z_off;
    return s;
}

bool same_sink(const lbsc::Sink& a, const lbsc::Sink& b)
{
    return a.kind == b.kind && a.no_zlo == b.no_zlo && a.rho_h == b.rho_h && a.r2 == b.r2 && a.cx == b.cx &&
           a.cy == b.cy && a.cz == b.cz;
}

// psi of Eq. (psifunc) (rho_0 = 1) or psi = rho, in FP64 on the host.
double psi_host(int psi, double rho) { return psi == LBSC_PSI_EXP ? 1.0 - std::exp(-rho) : rho; }

// FP16S with a sink needs the explicit flag: its constant-shift FP16 rounds
// away the slow relaxation of the vapour, and the sink then books a flux
// that never leaves the droplet.
bool fp16s_sink_refused(int precision, int sink, int flags)
{
    return precision == LBSC_FP16S && sink != LBSC_SINK_NONE && !(flags & LBSC_FLAG_FP16S_SINK);
}

lbsc_status validate(const lbsc_params& p, int k, std::string& why)
{
    char buf[256];
    auto bad = [&](const char* m) {
        snprintf(buf, sizeof buf, "instance %d: %s", k, m);
        why = buf;
        return LBSC_E_ARG;
    };
    if (p.nx < 1 || p.ny < 1 || p.nz < 1 || p.nx > 4096 || p.ny > 4096 || p.nz > 4096) return bad("size out of 1..4096");
    if ((int64_t)p.nx * p.ny * p.nz >= (int64_t(1) << 31)) return bad("nx*ny*nz must be < 2^31");
    if (p.ncomp < 0 || p.ncomp > 2) return bad("ncomp must be 0, 1 or 2");
    if (p.plane_pad < -1 || p.plane_pad > (1 << 20)) return bad("plane_pad out of -1..2^20");
    if ((int64_t)slab_planes(p.precision, ncomp_of(p)) * ((int64_t)p.nx * p.ny + 64 + plane_pad_of(p)) *
            (int64_t)elem_size(p.precision) >= (int64_t(1) << 32))
        return bad("one z-slab of population planes must be < 4 GiB");
    if (!(p.tau[0] > 0.5) || !(p.tau[1] > 0.5)) return bad("tau must be > 0.5");
    if (!std::isfinite(p.g)) return bad("g not finite");
    if (p.psi != LBSC_PSI_RHO && p.psi != LBSC_PSI_EXP) return bad("unknown psi");
    if (p.precision < LBSC_FP64 || p.precision > LBSC_FP16NF) return bad("unknown precision");
    if (p.sink < LBSC_SINK_NONE || p.sink > LBSC_SINK_SPHERE) return bad("unknown sink kind");
    if (!std::isfinite(p.rho_h) || !std::isfinite(p.sink_radius)) return bad("sink parameters not finite");
    if (p.phi_delta[0] == p.phi_delta[1]) return bad("phi_delta[0] must differ from phi_delta[1]");
    if (!std::isfinite(p.shift[0]) || !std::isfinite(p.shift[1])) return bad("shift not finite");
    if (p.flags & ~LBSC_FLAG_FP16S_SINK) return bad("unknown flag bits");
    if (p.solid_z < 0 || p.solid_z >= p.nz) return bad("solid_z out of 0..nz-1");
    if (p.solid_z > 0 && p.wall_z) return bad("solid_z and wall_z exclude each other");
    if (!std::isfinite(p.wall_rho[0]) || !std::isfinite(p.wall_rho[1])) return bad("wall_rho not finite");
    if (p.reserved != 0) return bad("reserved field must be 0");
    if (ncomp_of(p) == 1 && p.precision != LBSC_FP64 && p.precision != LBSC_FP32S) {
        why = "the single-component form stores FP64 or FP32S populations";
        return LBSC_E_UNSUPPORTED;
    }
    if (fp16s_sink_refused(p.precision, p.sink, p.flags)) {
        why = "FP16S storage with an evaporation sink (set LBSC_FLAG_FP16S_SINK to accept it)";
        return LBSC_E_UNSUPPORTED;
    }
    return LBSC_OK;
}

// Work items of one instance for the schedule in `t` (see lbsc_tiles).
// Split [0, n) into parts: fixed width w with a ragged last part, or, with
// w <= 0, `parts` near-equal parts (sizes differ by at most one).
std::vector<int> split_range(int n, int w, int parts)
{
    std::vector<int> b;
    if (w > 0) {
        for (int a = 0; a < n; a += w) b.push_back(a);
    } else {
        for (int k = 0; k < parts; ++k) b.push_back((int)((int64_t)k * n / parts));
    }
    b.push_back(n);
    return b;
}

// Boundaries of `parts` parts of [0, n) with every inner boundary rounded
// to a multiple of `line`; empty where rounding merges two boundaries.
std::vector<int> split_aligned(int n, int parts, int line)
{
    std::vector<int> b(1, 0);
    for (int k = 1; k < parts; ++k) {
        const int64_t e = ((int64_t)k * n / parts + line / 2) / line * line;
        if (e <= b.back() || e >= n) return {};
        b.push_back((int)e);
    }
    b.push_back(n);
    return b;
}

// Weight of a halo column node against a halo row node in the choice of the
// x split: a row streams with the tile, a column node reads a cache line of
// its own for every population. On the 512^3 lattice FP32S ran 128 x 4 tiles
// faster than 64 x 8 (8.68 against 9.05 ms), which pull half the halo row
// nodes and twice the column nodes: there a column node costs more than 16
// row nodes. The FP16 forms, bound by instruction issue rather than memory,
// pay mostly for the decode and densities of every halo node: FP16N ran
// 64 x 8 faster (5.55 against 5.75 ms) in the pipelined step, a column node
// costing fewer than 16 row nodes there.
constexpr double kColumnWeight = 24.0, kColumnWeightF16 = 8.0;

void instance_items(const Inst& I, int inst, const lbsc_tiles& t, int nt, int min_rows, int line, double colw,
                    int64_t total_nodes, int target_items, int cus, std::vector<Item>& out)
{
    // Defaults from tile sweeps on MI355X: a tile spans the whole x extent
    // (contiguous reads, no x halo) while the block still holds min_rows rows
    // of it. Otherwise x splits into near-equal parts of at most 128 (and at
    // most nt / min_rows) nodes; where nx is a whole number of `line`-node
    // 128-byte lines the part boundaries fall on lines (tiles whose rows start
    // inside a line ran the step up to 45 % slower), and of p0 (the fewest
    // parts) to 4 p0 + 3 parts the split with the cheapest halo, a column node
    // weighing `colw` row nodes, is taken. Rows: as many as the block holds,
    // split evenly so that no block runs a thin ragged tile. Chunks: about
    // target_items blocks per context with at least 16 planes per z chunk
    // (each chunk re-derives the densities of two extra planes), shorter only
    // where 16-plane chunks would leave the instance fewer blocks than its
    // share of the CUs (a block's march is latency-bound plane by plane).
    // Explicit tw / th / nzc give fixed sizes with a ragged last tile.
    const int full = std::max(1, nt / min_rows);
    const int cap = std::min(128, full);
    std::vector<int> xb, yb, zb;
    if (t.tw > 0) {
        xb = split_range(I.nx, std::min({t.tw, I.nx, nt}), 0);
    } else if (I.nx <= full) {
        xb = split_range(I.nx, 0, 1);
    } else {
        const int p0 = (I.nx + cap - 1) / cap;
        // (rows start on a line only where a row is a whole number of lines)
        const int ln = I.nx % std::max(1, line) == 0 ? std::max(1, std::min(line, cap)) : 1;
        double best = 1e300;
        for (int p = p0; p <= std::min(I.nx, 4 * p0 + 3); ++p) {
            std::vector<int> b = split_aligned(I.nx, p, ln);
            if (b.empty()) continue;
            int wmax = 0;
            for (size_t k = 0; k + 1 < b.size(); ++k) wmax = std::max(wmax, b[k + 1] - b[k]);
            if (wmax > cap) continue;
            // halo nodes per plane: two rows of nx + 2p per row of tiles, two
            // columns of ny per part
            const int th = std::min(I.ny, std::max(1, nt / wmax));
            const double rows = (double)((I.ny + th - 1) / th);
            const double cost = 2.0 * rows * (I.nx + 2.0 * p) + colw * 2.0 * I.ny * p;
            if (cost < best) {
                best = cost;
                xb = b;
            }
        }
        // none rounds to widths <= cap: parts of the widest multiple of the
        // line that fits, the last one narrower
        if (xb.empty()) xb = split_range(I.nx, cap / ln * ln, 0);
    }
    int twmax = 0;
    for (size_t k = 0; k + 1 < xb.size(); ++k) twmax = std::max(twmax, xb[k + 1] - xb[k]);
    const int thcap = std::min(I.ny, std::max(1, nt / twmax));
    if (t.th > 0) {
        yb = split_range(I.ny, std::min(t.th, thcap), 0);
    } else {
        yb = split_range(I.ny, 0, (I.ny + thcap - 1) / thcap);
    }
    const int cols = (int)((xb.size() - 1) * (yb.size() - 1));
    if (t.nzc > 0) {
        zb = split_range(I.nz, std::min(t.nzc, I.nz), 0);
    } else {
        const double share = (double)I.n / (double)total_nodes / cols;
        const int want = std::max(1, (int)std::ceil(target_items * share));
        const int fill = (int)std::ceil(cus * share);
        const int chunks = std::min({want, std::max({1, I.nz / 16, fill}), I.nz});
        zb = split_range(I.nz, 0, chunks);
    }
    // Order: groups of about cols/8 neighbouring tiles, each with all its z
    // chunks, so that one XCD (a contiguous run of items) holds the chunks
    // above and below each other; odd chunks march downwards (the pipelined
    // step reads each shared boundary plane from both sides at the same
    // time).
    const int nxt = (int)xb.size() - 1, nch = (int)zb.size() - 1;
    const int gsz = std::max(1, cols / 8);
    for (int g0 = 0; g0 < cols; g0 += gsz)
        for (int kz = 0; kz < nch; ++kz)
            for (int cix = g0; cix < std::min(g0 + gsz, cols); ++cix) {
                const int ky = cix / nxt, kx = cix % nxt;
                Item it{};
                it.inst = inst;
                it.x0 = (int16_t)xb[kx];
                it.y0 = (int16_t)yb[ky];
                it.tw = (int16_t)(xb[kx + 1] - xb[kx]);
                it.th = (int16_t)(yb[ky + 1] - yb[ky]);
                it.z0 = (int16_t)zb[kz];
                it.nzc = (int16_t)(zb[kz + 1] - zb[kz]);
                it.down = (int16_t)(kz & 1);
                out.push_back(it);
            }
}

// Relative time of a work item: the nodes it pulls per plane (halo nodes,
// mostly served by L2, at half weight) times its planes plus the two halo
// planes of its chunk.
double item_cost(const Item& it, const Inst& I)
{
    const lbsc::PipeTile p = lbsc::pipe_tile(it.tw, it.th, I.nx, I.ny);
    return ((double)it.tw * it.th + 0.5 * p.nring) * (it.nzc + 2);
}

// Final item list: the step kernels hand XCD j the contiguous run
// [j per, (j + 1) per) of an n = 8 per item list, so the instances' items
// are cut into eight consecutive runs of equal cost (not equal count: the
// items of a batch differ in size), each padded with empty items (nzc = 0)
// to the longest run. Instances go in order of decreasing item cost, so each
// XCD ends on its cheapest items. Every instance's items stay one range
// [item_begin, item_end) (padding inside it books nothing).
void place_items(const std::vector<std::vector<Item>>& per_inst, std::vector<Inst>& inst, std::vector<Item>& items,
                 size_t max_items = SIZE_MAX)
{
    std::vector<int> order(per_inst.size());
    std::vector<double> unit(per_inst.size(), 0.0);
    for (size_t k = 0; k < per_inst.size(); ++k) {
        order[k] = (int)k;
        if (!per_inst[k].empty()) unit[k] = item_cost(per_inst[k][0], inst[k]);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return unit[a] > unit[b]; });
    std::vector<Item> seq;
    std::vector<double> cost;
    double total = 0.0;
    for (int k : order)
        for (const Item& it : per_inst[k]) {
            seq.push_back(it);
            cost.push_back(item_cost(it, inst[k]));
            total += cost.back();
        }
    // run j ends where the running cost first reaches (j + 1) / 8 of the
    // total (each run at least as long as the one before it may need)
    size_t cut[9];
    cut[0] = 0;
    double run = 0.0;
    size_t pos = 0;
    for (int j = 0; j < 8; ++j) {
        const double goal = total * (j + 1) / 8.0;
        while (pos < seq.size() && (j == 7 || run + 0.5 * cost[pos] <= goal)) run += cost[pos++];
        cut[j + 1] = pos;
    }
    size_t per = 0;
    for (int j = 0; j < 8; ++j) per = std::max(per, cut[j + 1] - cut[j]);
    if (8 * per > max_items) {
        // padding would overflow the reserved item table (runs of very
        // unequal counts): equal counts instead, the last run short
        per = (seq.size() + 7) / 8;
        for (int j = 0; j <= 8; ++j) cut[j] = std::min(seq.size(), j * per);
    }
    Item pad{};
    pad.nzc = 0;
    items.assign(8 * per, pad);
    std::vector<int32_t> lo(inst.size(), INT32_MAX), hi(inst.size(), -1);
    for (int j = 0; j < 8; ++j)
        for (size_t q = cut[j]; q < cut[j + 1]; ++q) {
            const int32_t at = (int32_t)(j * per + (q - cut[j]));
            items[at] = seq[q];
            lo[seq[q].inst] = std::min(lo[seq[q].inst], at);
            hi[seq[q].inst] = std::max(hi[seq[q].inst], at);
        }
    for (size_t k = 0; k < inst.size(); ++k) {
        inst[k].item_begin = hi[k] < 0 ? 0 : lo[k];
        inst[k].item_end = hi[k] < 0 ? 0 : hi[k] + 1;
    }
}

lbsc_status build_items(lbsc_ctx* c, const lbsc_tiles& t, std::vector<Item>& items, std::vector<Inst>& inst, int& nt,
                        int& variant)
{
    // FP32-arithmetic forms run 512-thread blocks by default, FP64
    // (register-bound at two waves per SIMD) 256-thread blocks; about 1024
    // (FP16 forms and batches), 512 (a single FP32S lattice) or 256 (FP64)
    // blocks per context. On the 512^3 droplet one 512-plane chunk per tile
    // ran FP32S 0.6 % faster than two of 256 (8.63 against 8.68 ms) and FP16N
    // 2 % slower (5.64 against 5.53 ms); a batch's items differ in cost, and
    // more of them let the XCD runs balance.
    const bool f64 = c->precision == LBSC_FP64;
    nt = t.nt > 0 ? t.nt : (f64 ? 256 : 512);
    const int target_items = f64 ? 256 : (c->precision == LBSC_FP32S && c->n_inst == 1 ? 512 : 1024);
    if (nt != 256 && nt != 512) return fail(c, LBSC_E_ARG, "tiles.nt must be 256 or 512");
    if (t.variant > 3) return fail(c, LBSC_E_ARG, "tiles.variant must be 0, 1, 2 or 3");
    if (t.variant == 3 && c->precision == LBSC_FP64 && nt != 256)
        return fail(c, LBSC_E_ARG, "tiles.variant 3 in FP64 runs 256-thread blocks");
    if (t.tw > 512 || t.th > 512) return fail(c, LBSC_E_ARG, "tiles.tw and tiles.th must be <= 512");
    // Minimum rows of a default tile. A halo row streams like the tile; a
    // halo column node touches its own cache line per population, so full
    // width stays cheaper down to 3 rows for the pipelined step (2-row tiles
    // pulled twice their nodes and lost to 64 x 4 in FP64). The
    // register-keeping steps pay more per halo pull and run best on 8 rows.
    if (c->ncomp == 1 && t.variant > 1)
        return fail(c, LBSC_E_ARG, "the single-component step has one variant (1)");
    const bool pipe_ok = c->ncomp == 2 && (!f64 || nt == 256);
    // nodes per 128-byte line of a plane row (FP16N: of its FP32 rest pairs)
    const int node_bytes = c->ncomp == 1 ? (int)elem_size(c->precision)
                                         : (per_node(c->precision) ? 8 : 2 * (int)elem_size(c->precision));
    const int line = 128 / node_bytes;
    const int want = t.variant > 0 ? t.variant : (pipe_ok ? 3 : 1);
    const double colw =
        want == 3 && (c->precision == LBSC_FP16S || per_node(c->precision)) ? kColumnWeightF16 : kColumnWeight;
    const int min_rows = want == 3 ? 3 : 8;
    int64_t total = 0;
    for (auto& I : inst) total += I.n;
    std::vector<std::vector<Item>> per_inst(inst.size());
    for (int k = 0; k < (int)inst.size(); ++k) {
        // an instance's own tile width, rows and chunk length override the
        // context's
        lbsc_tiles tk = t;
        const lbsc_tiles& o = c->inst_tiles[k];
        if (o.tw > 0) tk.tw = o.tw;
        if (o.th > 0) tk.th = o.th;
        if (o.nzc > 0) tk.nzc = o.nzc;
        if (tk.tw > 512 || tk.th > 512) return fail(c, LBSC_E_ARG, "instance %d: tw and th must be <= 512", k);
        instance_items(inst[k], k, tk, nt, min_rows, line, colw, total, target_items, c->cus, per_inst[k]);
    }
    place_items(per_inst, inst, items, c->max_items);
    if (items.size() > c->max_items)
        return fail(c, LBSC_E_ARG, "schedule needs %zu work items, more than the %zu reserved", items.size(),
                    c->max_items);
    const int foot = nt == 256 ? lbsc::Foot<256>::kMax : lbsc::Foot<512>::kMax;
    bool pipe_fits = pipe_ok;
    for (auto& it : items) {
        if (it.nzc == 0) continue;  // XCD padding
        if (it.tw * it.th > nt || (it.tw + 2) * (it.th + 2) > foot)
            return fail(c, LBSC_E_ARG, "internal: tile %dx%d does not fit %d threads", it.tw, it.th, nt);
        const Inst& I = inst[it.inst];
        if (it.x0 < 0 || it.y0 < 0 || it.z0 < 0 || it.x0 + it.tw > I.nx || it.y0 + it.th > I.ny ||
            it.z0 + it.nzc > I.nz || it.tw < 1 || it.th < 1 || it.nzc < 1)
            return fail(c, LBSC_E_ARG, "internal: tile outside its lattice");
        if (lbsc::pipe_tile(it.tw, it.th, I.nx, I.ny).nring > nt) pipe_fits = false;
        if (per_node(c->precision) && !lbsc::rest_fits(it.tw, it.th, nt)) pipe_fits = false;
    }
    if (t.variant == 3 && !pipe_fits)
        return fail(c, LBSC_E_ARG,
                    "tiles.variant 3: a tile has more halo nodes than the %d threads%s", nt,
                    per_node(c->precision) ? ", or (tw + 4)(th + 4) exceeds 3 nt (FP16N rest footprint)" : "");
    variant = t.variant > 0 ? t.variant : (pipe_fits ? 3 : 1);
    if (variant != 3)
        for (auto& it : items) it.down = 0;  // the register-keeping steps march upwards only
    return LBSC_OK;
}

lbsc_status upload_table(lbsc_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->d_inst(), c->inst.data(), c->inst.size() * sizeof(Inst), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBSC_OK;
}

lbsc_status upload_items(lbsc_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->d_items(), c->items.data(), c->items.size() * sizeof(Item), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBSC_OK;
}

void drop_graphs(lbsc_ctx* c)
{
    for (auto& g : c->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

int fill_grid(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 65536); }

template <class St, int NT, bool KEEP>
hipError_t launch_step_t(lbsc_ctx* c, hipStream_t s, int src)
{
    using T = typename St::T;
    const int n = (int)c->items.size();
    const int grid = ((n + 7) / 8) * 8;
    hipLaunchKernelGGL((lbsc::k_step<St, NT, KEEP>), dim3(grid), dim3(NT), 0, s, c->d_inst(), c->d_items(), n,
                       (const T*)c->pop[src], (T*)c->pop[src ^ 1], c->d_eacc());
    return hipGetLastError();
}

template <class St, bool KEEP>
hipError_t launch_step_k(lbsc_ctx* c, hipStream_t s, int src)
{
    return c->nt == 512 ? launch_step_t<St, 512, KEEP>(c, s, src) : launch_step_t<St, 256, KEEP>(c, s, src);
}

template <class St, int NT>
hipError_t launch_pipe_t(lbsc_ctx* c, hipStream_t s, int src)
{
    using T = typename St::T;
    const int n = (int)c->items.size();
    const int grid = ((n + 7) / 8) * 8;
    hipLaunchKernelGGL((lbsc::k_step_pipe<St, NT>), dim3(grid), dim3(NT), 0, s, c->d_inst(), c->d_items(), n,
                       (const T*)c->pop[src], (T*)c->pop[src ^ 1], c->d_eacc());
    return hipGetLastError();
}

template <class St>
hipError_t launch_step_p(lbsc_ctx* c, hipStream_t s, int src)
{
    if constexpr (std::is_same_v<typename St::A, double>) {
        if (c->variant == 3) return launch_pipe_t<St, 256>(c, s, src);  // one wave per SIMD: 256 threads only
    } else {
        if (c->variant == 3)
            return c->nt == 512 ? launch_pipe_t<St, 512>(c, s, src) : launch_pipe_t<St, 256>(c, s, src);
    }
    return c->variant == 2 ? launch_step_k<St, false>(c, s, src) : launch_step_k<St, true>(c, s, src);
}

template <class St, int NT>
hipError_t launch_step1_t(lbsc_ctx* c, hipStream_t s, int src)
{
    using T = typename St::T;
    const int n = (int)c->items.size();
    const int grid = ((n + 7) / 8) * 8;
    hipLaunchKernelGGL((lbsc::k_step1<St, NT>), dim3(grid), dim3(NT), 0, s, c->d_inst(), c->d_items(), n,
                       (const T*)c->pop[src], (T*)c->pop[src ^ 1], c->d_eacc());
    return hipGetLastError();
}

template <class St>
hipError_t launch_step1(lbsc_ctx* c, hipStream_t s, int src)
{
    return c->nt == 512 ? launch_step1_t<St, 512>(c, s, src) : launch_step1_t<St, 256>(c, s, src);
}

hipError_t launch_step(lbsc_ctx* c, hipStream_t s, int src)
{
    if (c->ncomp == 1)
        return c->precision == LBSC_FP64 ? launch_step1<lbsc::St1F64>(c, s, src)
                                         : launch_step1<lbsc::St1F32S>(c, s, src);
    switch (c->precision) {
    case LBSC_FP64: return launch_step_p<lbsc::StF64>(c, s, src);
    case LBSC_FP32S: return launch_step_p<lbsc::StF32S>(c, s, src);
    case LBSC_FP16S: return launch_step_p<lbsc::StF16S>(c, s, src);
    case LBSC_FP16NF: return launch_step_p<lbsc::StF16NF>(c, s, src);
    default: return launch_step_p<lbsc::StF16N>(c, s, src);
    }
}

bool steady(const lbsc_ctx* c)
{
    for (auto& I : c->inst)
        if (!I.count_reset || !same_sink(I.reset, I.cur)) return false;
    return true;
}

// Device address of each device's static scratch array and the context that
// owns it (binding a context to it takes it over).
constexpr int kMaxDevices = 64;
struct StaticScratch {
    void* ptr = nullptr;
    const lbsc_ctx* owner = nullptr;
};
StaticScratch g_static[kMaxDevices];

lbsc_status scratch_owned(lbsc_ctx* c)
{
    if (c->static_dev >= 0 && g_static[c->static_dev].owner != c)
        return fail(c, LBSC_E_STATE, "the static scratch of device %d was taken over by another context "
                                     "(bind this context again)", c->static_dev);
    return LBSC_OK;
}

void release_static(lbsc_ctx* c)
{
    if (c->static_dev >= 0 && g_static[c->static_dev].owner == c) g_static[c->static_dev].owner = nullptr;
    c->static_dev = -1;
}

lbsc_status check_bound(lbsc_ctx* c)
{
    if (!c) return LBSC_E_ARG;
    if (!c->bound) return fail(c, LBSC_E_STATE, "context has no bound buffers (call lbsc_bind)");
    return scratch_owned(c);
}

lbsc_status check_inst(lbsc_ctx* c, int inst)
{
    lbsc_status s = check_bound(c);
    if (s) return s;
    if (inst < 0 || inst >= c->n_inst) return fail(c, LBSC_E_ARG, "instance %d out of range", inst);
    return LBSC_OK;
}

template <typename F>
hipError_t by_precision(int prec, F&& f)
{
    switch (prec) {
    case LBSC_FP64: return f(lbsc::StF64{});
    case LBSC_FP32S: return f(lbsc::StF32S{});
    case LBSC_FP16S: return f(lbsc::StF16S{});
    case LBSC_FP16NF: return f(lbsc::StF16NF{});
    default: return f(lbsc::StF16N{});
    }
}

// Single-component storage policy of a precision (FP64 or FP32S).
template <typename F>
hipError_t by_precision1(int prec, F&& f)
{
    if (prec == LBSC_FP64) return f(lbsc::St1F64{});
    return f(lbsc::St1F32S{});
}

lbsc_status fold_eacc(lbsc_ctx* c)
{
    hipLaunchKernelGGL(lbsc::k_fold_eacc, dim3((c->n_inst + 63) / 64), dim3(64), 0, c->stream, c->d_inst(),
                       c->n_inst, c->d_eacc(), c->d_ebase());
    HIPCHK(c, hipGetLastError());
    return LBSC_OK;
}

lbsc_status apply_schedule(lbsc_ctx* c, const lbsc_tiles& t)
{
    std::vector<Item> items;
    std::vector<Inst> inst = c->inst;
    int nt = 256, variant = 1;
    lbsc_status s = build_items(c, t, items, inst, nt, variant);
    if (s) return s;
    if (c->bound && (s = scratch_owned(c))) return s;
    if (c->bound) {
        s = fold_eacc(c);  // accumulators belong to the old item list
        if (s) return s;
    }
    c->items.swap(items);
    c->inst.swap(inst);
    c->nt = nt;
    c->variant = variant;
    c->tiles = t;
    drop_graphs(c);
    if (c->bound) {
        if ((s = upload_items(c))) return s;
        if ((s = upload_table(c))) return s;
    }
    return LBSC_OK;
}

// Tuning cache: schedules the tuner kept, by (architecture, lattice size,
// precision, components, context nt, context variant), for the compiled
// kernel sources (LBSC_KERNEL_HASH, a hash of their code). A one-instance
// context stores its whole schedule under nt = variant = 0; an instance of a
// batch its tile width, rows and chunk length under the batch's nt and
// variant.
#ifndef LBSC_KERNEL_HASH
#define LBSC_KERNEL_HASH "unknown"
#endif
using TuneKey = std::tuple<std::string, int, int, int, int, int, int, int>;
std::map<TuneKey, lbsc_tiles> g_tune_cache;
std::mutex g_tune_mutex;

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

TuneKey tune_key(const lbsc_ctx* c, int inst, int nt, int variant, const std::string& arch)
{
    // the kernels' lattice: without the solid planes of a walled instance
    const Inst& I = c->inst[inst];
    return TuneKey{arch, I.nx, I.ny, I.nz, c->precision, c->ncomp, nt, variant};
}

bool cache_get(const TuneKey& k, lbsc_tiles& out)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(k);
    if (it == g_tune_cache.end()) return false;
    out = it->second;
    return true;
}

void cache_put(const TuneKey& k, const lbsc_tiles& t)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[k] = t;
}

// Size class of an instance for the tuner's per-instance pass: boxes of
// similar width take the same tile shapes.
int size_class(const lbsc_params& p)
{
    const int w = std::max(p.nx, p.ny);
    return w < 64 ? 0 : (w < 96 ? 1 : (w < 128 ? 2 : (w < 192 ? 3 : 4)));
}

}  // namespace

extern "C" {

const char* lbsc_status_string(lbsc_status s)
{
    switch (s) {
    case LBSC_OK: return "ok";
    case LBSC_E_ARG: return "invalid argument";
    case LBSC_E_STATE: return "invalid state";
    case LBSC_E_HIP: return "HIP runtime error";
    case LBSC_E_NONFINITE: return "non-finite density";
    case LBSC_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* lbsc_last_error(const lbsc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char* lbsc_version(void) { return "lbsc 0.1 gfx950"; }

lbsc_status lbsc_create(int32_t n_inst, const lbsc_params* params, lbsc_ctx** out)
{
    if (!out || !params || n_inst < 1 || n_inst > 65536) return LBSC_E_ARG;
    *out = nullptr;
    for (int k = 0; k < n_inst; ++k) {
        std::string why;
        if (lbsc_status st = validate(params[k], k, why)) return st;
        if (params[k].precision != params[0].precision) return LBSC_E_ARG;
        if (ncomp_of(params[k]) != ncomp_of(params[0])) return LBSC_E_ARG;
    }
    lbsc_ctx* c = new lbsc_ctx();
    c->cus = device_cus();
    c->ncomp = ncomp_of(params[0]);
    c->n_inst = n_inst;
    c->precision = params[0].precision;
    c->elem = elem_size(c->precision);
    c->params.assign(params, params + n_inst);
    size_t off = 0;
    int64_t total_nodes = 0;
    for (int k = 0; k < n_inst; ++k) {
        const lbsc_params& p = params[k];
        Inst I{};
        // a solid wall of h planes: the kernels see the fluid planes above it,
        // bounded by the seam wall on both ends (see Inst)
        const int h = p.solid_z;
        I.nx = p.nx; I.ny = p.ny; I.nz = p.nz - h; I.wall_z = (p.wall_z || h > 0) ? 1 : 0;
        I.z_off = h;
        I.psi_wall = h > 0;
        for (int cc = 0; cc < 2; ++cc) {
            I.psi_w[cc] = h > 0 ? psi_host(p.psi, p.wall_rho[cc]) : 0.0;
            I.psi_wf[cc] = (float)I.psi_w[cc];
        }
        I.psi_exp = p.psi == LBSC_PSI_EXP;
        I.count_reset = 0;
        I.n = (int64_t)p.nx * p.ny * I.nz;
        I.ps = (int64_t)align_up((size_t)p.nx * p.ny, 64) + (int64_t)align_up((size_t)plane_pad_of(p), 64);
        I.slab = slab_planes(p.precision, ncomp_of(p)) * I.ps;
        I.ncomp = ncomp_of(p);
        I.base = (int64_t)off + (int64_t)h * I.slab;
        off = align_up(off + (size_t)p.nz * (size_t)I.slab, 256);
        I.tau[0] = p.tau[0]; I.tau[1] = p.tau[1];
        I.omega[0] = 1.0 / p.tau[0]; I.omega[1] = 1.0 / p.tau[1];
        I.g = p.g;
        I.shift[0] = c->precision == LBSC_FP64 ? 0.0 : p.shift[0];
        I.shift[1] = c->precision == LBSC_FP64 ? 0.0 : p.shift[1];
        I.phi_in = p.phi_delta[0]; I.phi_out = p.phi_delta[1];
        for (int cc = 0; cc < 2; ++cc) {
            I.shift_f[cc] = (float)I.shift[cc];
            I.omega_f[cc] = (float)I.omega[cc];
            const float tf = (float)I.tau[cc], gf = (float)I.g;
            I.ntg_f[cc] = -tf * gf;
        }
        I.reset = make_sink(p.sink, p.rho_h, p.sink_radius, p.center, h);
        I.cur = I.reset;
        c->inst.push_back(I);
        total_nodes += I.n;
        c->max_nz = std::max(c->max_nz, I.nz);
    }
    c->pop_elems = off;
    c->inst_tiles.assign(n_inst, lbsc_tiles{0, 0, 0, 0, 0});
    // Bound on work items: any schedule with tiles of >= 16 nodes per plane.
    c->max_items = std::max<size_t>(65536, (size_t)(total_nodes / 16) + 64 * (size_t)n_inst);
    size_t o = 0;
    c->off_inst = o; o = align_up(o + n_inst * sizeof(Inst), kAlign);
    c->off_items = o; o = align_up(o + c->max_items * sizeof(Item), kAlign);
    c->off_eacc = o; o = align_up(o + c->max_items * sizeof(double), kAlign);
    c->off_ebase = o; o = align_up(o + n_inst * sizeof(double), kAlign);
    c->off_part = o; o = align_up(o + (size_t)c->max_nz * lbsc::kDiagVals * sizeof(double), kAlign);
    c->off_out = o; o = align_up(o + 64 * sizeof(double), kAlign);
    c->scratch_bytes = o;
    lbsc_tiles t{0, 0, 0, 0, 0};
    if (apply_schedule(c, t)) {
        delete c;
        return LBSC_E_ARG;
    }
    *out = c;
    return LBSC_OK;
}

lbsc_status lbsc_destroy(lbsc_ctx* ctx)
{
    if (!ctx) return LBSC_E_ARG;
    drop_graphs(ctx);
    release_static(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return LBSC_OK;
}

lbsc_status lbsc_required_bytes(const lbsc_ctx* ctx, size_t* pop_bytes, size_t* scratch_bytes)
{
    if (!ctx || !pop_bytes || !scratch_bytes) return LBSC_E_ARG;
    *pop_bytes = ctx->pop_elems * ctx->elem;
    *scratch_bytes = ctx->scratch_bytes;
    return LBSC_OK;
}

lbsc_status lbsc_set_stream(lbsc_ctx* ctx, void* hip_stream)
{
    if (!ctx) return LBSC_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return LBSC_OK;
}

static lbsc_status bind_buffers(lbsc_ctx* c, void* pop0, void* pop1, void* work)
{
    if (!pop0 || !pop1 || !work || pop0 == pop1)
        return fail(c, LBSC_E_ARG, "bind: need two distinct population buffers and a scratch buffer");
    if (((uintptr_t)pop0 | (uintptr_t)pop1 | (uintptr_t)work) % kAlign)
        return fail(c, LBSC_E_ARG, "bind: buffers must be %zu-byte aligned", kAlign);
    c->pop[0] = pop0;
    c->pop[1] = pop1;
    c->scratch = (char*)work;
    c->bound = true;
    c->cur = 0;
    drop_graphs(c);
    // the accumulators start at zero (fill kernels: no memset nodes in
    // anything a caller may capture)
    hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(fill_grid(c->max_items)), dim3(256), 0, c->stream, c->d_eacc(),
                       (int64_t)c->max_items, 0.0);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(1), dim3(256), 0, c->stream, c->d_ebase(), (int64_t)c->n_inst, 0.0);
    HIPCHK(c, hipGetLastError());
    lbsc_status s = upload_items(c);
    if (s) return s;
    return upload_table(c);
}

lbsc_status lbsc_bind(lbsc_ctx* c, void* pop0, void* pop1, void* work)
{
    if (!c) return LBSC_E_ARG;
    release_static(c);
    return bind_buffers(c, pop0, pop1, work);
}

lbsc_status lbsc_bind_static(lbsc_ctx* c, void* pop0, void* pop1)
{
    if (!c) return LBSC_E_ARG;
    if (c->scratch_bytes > (size_t)LBSC_STATIC_SCRATCH_BYTES)
        return fail(c, LBSC_E_ARG, "bind_static: the context needs %zu bytes of scratch, more than the %d-byte "
                                   "static scratch", c->scratch_bytes, (int)LBSC_STATIC_SCRATCH_BYTES);
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, LBSC_E_ARG, "bind_static: device %d out of range", dev);
    // Once per device, with that device current: the array's device address
    // (host code must not use the symbol itself as a device pointer).
    if (!g_static[dev].ptr) {
        void* ptr = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(c, LBSC_E_HIP, "bind_static: no address for the static scratch");
        g_static[dev].ptr = ptr;
    }
    release_static(c);
    c->static_dev = dev;
    g_static[dev].owner = c;
    lbsc_status s = bind_buffers(c, pop0, pop1, g_static[dev].ptr);
    if (s) release_static(c);
    return s;
}

// Nodes of the caller's lattice of instance inst (solid planes included),
// and the offset of the kernels' first node in the caller's arrays.
static int64_t user_nodes(const lbsc_ctx* c, int inst)
{
    const lbsc_params& p = c->params[inst];
    return (int64_t)p.nx * p.ny * p.nz;
}
static int64_t solid_nodes(const lbsc_ctx* c, int inst)
{
    const lbsc_params& p = c->params[inst];
    return (int64_t)p.nx * p.ny * p.solid_z;
}

// Zeros over the solid planes of `planes` caller arrays of user_nodes each.
static lbsc_status zero_solid(lbsc_ctx* c, int inst, double* out, int planes)
{
    const int64_t ns = solid_nodes(c, inst), nu = user_nodes(c, inst);
    for (int q = 0; q < planes && ns > 0; ++q) {
        hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(fill_grid(ns)), dim3(256), 0, c->stream, out + q * nu, ns, 0.0);
        HIPCHK(c, hipGetLastError());
    }
    return LBSC_OK;
}

static lbsc_status begin_init(lbsc_ctx* c, int inst)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    // Clear this instance's evaporation accumulators.
    Inst& I = c->inst[inst];
    const int nit = I.item_end - I.item_begin;
    if (nit > 0) {
        hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(fill_grid(nit)), dim3(256), 0, c->stream, c->d_eacc() + I.item_begin,
                           (int64_t)nit, 0.0);
        HIPCHK(c, hipGetLastError());
    }
    hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(1), dim3(64), 0, c->stream, c->d_ebase() + inst, (int64_t)1, 0.0);
    HIPCHK(c, hipGetLastError());
    I.count_reset = 0;
    I.reset = I.cur;
    c->step = 0;
    return LBSC_OK;
}

lbsc_status lbsc_init_from_density(lbsc_ctx* c, int32_t inst, const double* rhoA, const double* rhoB)
{
    lbsc_status s = begin_init(c, inst);
    if (s) return s;
    if (!rhoA || (!rhoB && c->ncomp == 2)) return fail(c, LBSC_E_ARG, "init: null density pointer");
    const Inst I = c->inst[inst];
    const int64_t off = solid_nodes(c, inst);  // solid nodes hold no fluid
    if (c->ncomp == 1) {
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_init_density1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      rhoA + off, (T*)c->pop[c->cur]);
                   return hipGetLastError();
               }));
        return upload_table(c);
    }
    HIPCHK(c, by_precision(c->precision, [&](auto tag) {
               using S = decltype(tag);
               using T = typename S::T;
               hipLaunchKernelGGL(lbsc::k_init_density<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                  rhoA + off, rhoB + off, (T*)c->pop[c->cur]);
               return hipGetLastError();
           }));
    return upload_table(c);
}

lbsc_status lbsc_init_from_populations(lbsc_ctx* c, int32_t inst, const double* f)
{
    lbsc_status s = begin_init(c, inst);
    if (s) return s;
    if (!f) return fail(c, LBSC_E_ARG, "init: null population pointer");
    const Inst I = c->inst[inst];
    const int64_t off = solid_nodes(c, inst), nu = user_nodes(c, inst);
    if (c->ncomp == 1) {
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_init_pops1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      f + off, nu, (T*)c->pop[c->cur]);
                   return hipGetLastError();
               }));
        return upload_table(c);
    }
    HIPCHK(c, by_precision(c->precision, [&](auto tag) {
               using S = decltype(tag);
               using T = typename S::T;
               hipLaunchKernelGGL(lbsc::k_init_pops<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I, f + off,
                                  nu, (T*)c->pop[c->cur]);
               return hipGetLastError();
           }));
    return upload_table(c);
}

lbsc_status lbsc_set_sink(lbsc_ctx* c, int32_t inst, int32_t kind, double rho_h, double radius)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    if (kind < LBSC_SINK_NONE || kind > LBSC_SINK_SPHERE || !std::isfinite(rho_h) || !std::isfinite(radius))
        return fail(c, LBSC_E_ARG, "set_sink: bad kind or value");
    if (fp16s_sink_refused(c->precision, kind, c->params[inst].flags))
        return fail(c, LBSC_E_UNSUPPORTED,
                    "set_sink: FP16S storage with an evaporation sink (create with LBSC_FLAG_FP16S_SINK to accept it)");
    c->params[inst].sink = kind;
    c->params[inst].rho_h = rho_h;
    c->params[inst].sink_radius = radius;
    c->inst[inst].cur = make_sink(kind, rho_h, radius, c->params[inst].center, c->inst[inst].z_off);
    return upload_table(c);
}

lbsc_status lbsc_set_graph(lbsc_ctx* c, int32_t steps)
{
    if (!c) return LBSC_E_ARG;
    if (steps != 0 && (steps < 2 || (steps & 1))) return fail(c, LBSC_E_ARG, "graph steps must be 0 or even >= 2");
    drop_graphs(c);
    c->graph_steps = steps;
    return LBSC_OK;
}

static lbsc_status graph_for(lbsc_ctx* c, int parity, hipGraphExec_t* out)
{
    if (!c->gexec[parity]) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (int k = 0; k < c->graph_steps && le == hipSuccess; ++k) le = launch_step(c, c->cap_stream, parity ^ (k & 1));
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
        if (le != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(c, LBSC_E_HIP, "graph capture failed: %s", hipGetErrorString(le != hipSuccess ? le : ee));
        }
        hipError_t ie = hipGraphInstantiate(&c->gexec[parity], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(c, LBSC_E_HIP, "graph instantiate: %s", hipGetErrorString(ie));
    }
    *out = c->gexec[parity];
    return LBSC_OK;
}

lbsc_status lbsc_step(lbsc_ctx* c, int64_t n)
{
    lbsc_status s = check_bound(c);
    if (s) return s;
    if (n < 0) return fail(c, LBSC_E_ARG, "negative step count");
    while (n > 0) {
        if (!steady(c)) {
            HIPCHK(c, launch_step(c, c->stream, c->cur));
            c->cur ^= 1;
            c->step += 1;
            n -= 1;
            for (auto& I : c->inst) {
                I.count_reset = 1;
                I.reset = I.cur;
            }
            if ((s = upload_table(c))) return s;
            continue;
        }
        if (c->graph_steps > 0 && n >= c->graph_steps) {
            hipGraphExec_t g;
            if ((s = graph_for(c, c->cur, &g))) return s;
            HIPCHK(c, hipGraphLaunch(g, c->stream));
            c->step += c->graph_steps;
            n -= c->graph_steps;
            continue;
        }
        HIPCHK(c, launch_step(c, c->stream, c->cur));
        c->cur ^= 1;
        c->step += 1;
        n -= 1;
    }
    return LBSC_OK;
}

lbsc_status lbsc_set_tiles(lbsc_ctx* c, const lbsc_tiles* t)
{
    if (!c || !t) return LBSC_E_ARG;
    return apply_schedule(c, *t);
}

lbsc_status lbsc_get_tiles(const lbsc_ctx* c, lbsc_tiles* out)
{
    if (!c || !out) return LBSC_E_ARG;
    *out = c->tiles;
    out->nt = c->nt;
    out->variant = c->variant;
    return LBSC_OK;
}

lbsc_status lbsc_num_items(const lbsc_ctx* c, int32_t* n)
{
    if (!c || !n) return LBSC_E_ARG;
    int32_t real = 0;
    for (const Item& it : c->items) real += it.nzc > 0;
    *n = real;
    return LBSC_OK;
}

lbsc_status lbsc_set_inst_tiles(lbsc_ctx* c, int32_t inst, const lbsc_tiles* t)
{
    if (!c || !t) return LBSC_E_ARG;
    if (inst < 0 || inst >= c->n_inst) return fail(c, LBSC_E_ARG, "instance %d out of range", inst);
    if (t->tw < 0 || t->th < 0 || t->nzc < 0 || t->tw > 512 || t->th > 512)
        return fail(c, LBSC_E_ARG, "set_inst_tiles: tw, th in 0..512 and nzc >= 0");
    const lbsc_tiles old = c->inst_tiles[inst];
    c->inst_tiles[inst] = lbsc_tiles{0, t->tw, t->th, t->nzc, 0};
    lbsc_status s = apply_schedule(c, c->tiles);
    if (s) {
        c->inst_tiles[inst] = old;
        (void)apply_schedule(c, c->tiles);
    }
    return s;
}

lbsc_status lbsc_get_inst_tiles(const lbsc_ctx* c, int32_t inst, lbsc_tiles* out)
{
    if (!c || !out || inst < 0 || inst >= c->n_inst) return LBSC_E_ARG;
    *out = c->inst_tiles[inst];
    out->nt = c->nt;
    out->variant = c->variant;
    return LBSC_OK;
}

lbsc_status lbsc_tune(lbsc_ctx* c, int32_t steps, lbsc_tiles* chosen)
{
    lbsc_status s = check_bound(c);
    if (s) return s;
    if (steps < 2) return fail(c, LBSC_E_ARG, "tune: steps must be >= 2");
    const std::string arch = device_arch();
    auto report = [&]() {
        if (chosen) {
            *chosen = c->tiles;
            chosen->nt = c->nt;
            chosen->variant = c->variant;
        }
    };
    // A one-instance context tuned before on this architecture and build
    // takes its schedule from the cache.
    if (c->n_inst == 1) {
        lbsc_tiles t;
        if (cache_get(tune_key(c, 0, 0, 0, arch), t) && apply_schedule(c, t) == LBSC_OK) {
            report();
            return LBSC_OK;
        }
    }
    std::vector<lbsc_tiles> cands;
    // Chunks of 1-4 planes are timed only on lattices below 2^22 nodes, where
    // 16-plane chunks of 512-node tiles give fewer than two blocks per CU and
    // each block's march is bound by its serial per-plane latency.
    int64_t total_nodes = 0;
    for (const auto& I : c->inst) total_nodes += I.n;
    std::vector<int> chunks = {0, 8, 16, 32, 64};
    if (total_nodes < (int64_t(1) << 22)) chunks.insert(chunks.end(), {1, 2, 4});
    for (int variant : {1, 2, 3})
        for (int nt : {256, 512}) {
            if (nt == 512 && c->precision == LBSC_FP64 && variant == 1) continue;  // exceeds the register file
            if (variant == 3 && c->precision == LBSC_FP64 && nt != 256)
                continue;
            for (int tw : {0, 32, 64, 128})
                for (int nzc : chunks) cands.push_back(lbsc_tiles{nt, tw, 0, nzc, variant});
        }
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // The live state is left as it was: every timed step reads the stored
    // populations and writes the other buffer without making it current, and
    // the instance table on the device books no evaporation meanwhile.
    const int cur0 = c->cur;
    const int64_t step0 = c->step;
    std::vector<int32_t> count0;
    for (auto& I : c->inst) {
        count0.push_back(I.count_reset);
        I.count_reset = 0;
    }
    auto restore = [&]() -> lbsc_status {
        for (size_t k = 0; k < c->inst.size(); ++k) c->inst[k].count_reset = count0[k];
        c->cur = cur0;
        c->step = step0;
        return upload_table(c);
    };
    const lbsc_tiles before = c->tiles;
    const int graph_before = c->graph_steps;
    c->graph_steps = 0;
    // Time of `n` steps of the schedule in place after a 2-step warm-up
    // (each step from the stored populations; see above).
    auto time_current = [&](int n, float& ms) -> lbsc_status {
        for (int i = 0; i < 2; ++i) HIPCHK(c, launch_step(c, c->stream, c->cur));
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int i = 0; i < n; ++i) HIPCHK(c, launch_step(c, c->stream, c->cur));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        return LBSC_OK;
    };
    // As above for schedule t; negative if the schedule does not apply.
    auto time_schedule = [&](const lbsc_tiles& t, int n, float& ms) -> lbsc_status {
        ms = -1.f;
        if (apply_schedule(c, t) != LBSC_OK) return LBSC_OK;
        return time_current(n, ms);
    };
    std::vector<std::pair<float, lbsc_tiles>> timed;
    std::vector<std::string> seen;
    for (const auto& t : cands) {
        if (apply_schedule(c, t) != LBSC_OK) continue;
        // Skip schedules identical to one already timed.
        std::string key(reinterpret_cast<const char*>(c->items.data()), c->items.size() * sizeof(Item));
        key += std::to_string(c->nt) + "v" + std::to_string(c->variant);
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
        seen.push_back(key);
        float ms;
        if ((s = time_schedule(t, steps, ms))) break;
        if (ms >= 0.f) timed.push_back({ms, t});
    }
    // The three fastest again over three times the steps: a single short
    // run can misorder schedules a few percent apart.
    float best = 1e30f;
    lbsc_tiles best_t = before;
    if (!s) {
        std::stable_sort(timed.begin(), timed.end(),
                         [](const auto& a, const auto& b) { return a.first < b.first; });
        for (size_t k = 0; k < std::min<size_t>(3, timed.size()); ++k) {
            float ms;
            if ((s = time_schedule(timed[k].second, 3 * steps, ms))) break;
            if (ms >= 0.f && ms < best) {
                best = ms;
                best_t = timed[k].second;
            }
        }
    }
    if (!s) s = apply_schedule(c, best_t);
    // Per-instance pass (batches): for each size class in turn, the class's
    // tile width and chunk length that make the whole batch's step fastest,
    // the other instances kept as they are; cached per instance size.
    if (!s && c->n_inst > 1) {
        std::map<int, std::vector<int>> classes;
        for (int k = 0; k < c->n_inst; ++k) classes[size_class(c->params[k])].push_back(k);
        for (auto& kv : classes) {
            const std::vector<int>& members = kv.second;
            bool cached = true;
            std::vector<lbsc_tiles> from_cache(members.size());
            for (size_t q = 0; q < members.size(); ++q)
                cached = cached && cache_get(tune_key(c, members[q], c->nt, c->variant, arch), from_cache[q]);
            if (cached) {
                for (size_t q = 0; q < members.size(); ++q) c->inst_tiles[members[q]] = from_cache[q];
                if ((s = apply_schedule(c, c->tiles))) break;
                continue;
            }
            std::vector<std::pair<float, lbsc_tiles>> ctimed;
            for (int tw : {0, 32, 64, 128})
                for (int nzc : {0, 8, 16, 32}) {
                    const lbsc_tiles o{0, tw, 0, nzc, 0};
                    for (int k : members) c->inst_tiles[k] = o;
                    if (apply_schedule(c, c->tiles) != LBSC_OK) continue;
                    float ms;
                    if ((s = time_current(steps, ms))) break;
                    ctimed.push_back({ms, o});
                }
            if (s) break;
            std::stable_sort(ctimed.begin(), ctimed.end(),
                             [](const auto& a, const auto& b) { return a.first < b.first; });
            float cbest = 1e30f;
            lbsc_tiles cbest_t{0, 0, 0, 0, 0};
            for (size_t q = 0; q < std::min<size_t>(3, ctimed.size()); ++q) {
                for (int k : members) c->inst_tiles[k] = ctimed[q].second;
                if (apply_schedule(c, c->tiles) != LBSC_OK) continue;
                float ms;
                if ((s = time_current(3 * steps, ms))) break;
                if (ms < cbest) {
                    cbest = ms;
                    cbest_t = ctimed[q].second;
                }
            }
            if (s) break;
            for (int k : members) {
                c->inst_tiles[k] = cbest_t;
                cache_put(tune_key(c, k, c->nt, c->variant, arch), cbest_t);
            }
            if ((s = apply_schedule(c, c->tiles))) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->graph_steps = graph_before;
    const lbsc_status sr = restore();
    if (s) return s;
    if (sr) return sr;
    if ((s = apply_schedule(c, c->tiles))) return s;
    if (c->n_inst == 1) {
        lbsc_tiles t = c->tiles;
        t.nt = c->nt;
        t.variant = c->variant;
        cache_put(tune_key(c, 0, 0, 0, arch), t);
    }
    report();
    return LBSC_OK;
}

lbsc_status lbsc_tune_cache_save(const char* path)
{
    if (!path) return LBSC_E_ARG;
    FILE* f = fopen(path, "w");
    if (!f) return LBSC_E_ARG;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const auto& kv : g_tune_cache) {
        const TuneKey& k = kv.first;
        const lbsc_tiles& t = kv.second;
        fprintf(f, "lbsc-tune 1 %s %s %d %d %d %d %d %d %d %d %d %d %d %d\n", LBSC_KERNEL_HASH,
                std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                std::get<5>(k), std::get<6>(k), std::get<7>(k), t.nt, t.tw, t.th, t.nzc, t.variant);
    }
    return fclose(f) == 0 ? LBSC_OK : LBSC_E_ARG;
}

lbsc_status lbsc_tune_cache_load(const char* path, int32_t* n_loaded)
{
    if (!path) return LBSC_E_ARG;
    FILE* f = fopen(path, "r");
    if (!f) return LBSC_E_ARG;
    char hash[65], arch[65];
    int v[13], ver, n = 0;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    while (fscanf(f, " lbsc-tune %d %64s %64s %d %d %d %d %d %d %d %d %d %d %d %d", &ver, hash, arch, &v[0], &v[1],
                  &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10], &v[11]) == 15) {
        // entries of other kernel sources describe other code: skipped
        if (ver != 1 || strcmp(hash, LBSC_KERNEL_HASH) != 0) continue;
        g_tune_cache[TuneKey{arch, v[0], v[1], v[2], v[3], v[4], v[5], v[6]}] =
            lbsc_tiles{v[7], v[8], v[9], v[10], v[11]};
        ++n;
    }
    fclose(f);
    if (n_loaded) *n_loaded = n;
    return LBSC_OK;
}

void lbsc_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache.clear();
}

const char* lbsc_kernel_hash(void) { return LBSC_KERNEL_HASH; }

lbsc_status lbsc_read_density(lbsc_ctx* c, int32_t inst, int32_t comp, double* out)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    if (!out || comp < 0 || comp >= c->ncomp) return fail(c, LBSC_E_ARG, "read_density: bad component or pointer");
    const Inst I = c->inst[inst];
    const int64_t off = solid_nodes(c, inst);
    if (c->ncomp == 1) {
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_read_density1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], out + off);
                   return hipGetLastError();
               }));
        return zero_solid(c, inst, out, 1);
    }
    HIPCHK(c, by_precision(c->precision, [&](auto tag) {
               using S = decltype(tag);
               using T = typename S::T;
               hipLaunchKernelGGL(lbsc::k_read_density<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                  (const T*)c->pop[c->cur], comp == 0 ? out + off : nullptr,
                                  comp == 1 ? out + off : nullptr);
               return hipGetLastError();
           }));
    return zero_solid(c, inst, out, 1);
}

lbsc_status lbsc_read_observables(lbsc_ctx* c, int32_t inst, double* ra, double* rb, double* u)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    if (u && (!ra || (!rb && c->ncomp == 2)))
        return fail(c, LBSC_E_ARG, "read_observables: velocity needs the density arrays");
    const Inst I = c->inst[inst];
    const int64_t off = solid_nodes(c, inst), nu = user_nodes(c, inst);
    if (c->ncomp == 1) {
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   if (ra)
                       hipLaunchKernelGGL(lbsc::k_read_density1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream,
                                          I, (const T*)c->pop[c->cur], ra + off);
                   hipError_t e = hipGetLastError();
                   if (e != hipSuccess || !u) return e;
                   hipLaunchKernelGGL(lbsc::k_read_velocity1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], (const double*)ra + off, u + off, nu);
                   return hipGetLastError();
               }));
        if (ra && (s = zero_solid(c, inst, ra, 1))) return s;
        if (rb) {  // no second component
            hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(fill_grid(nu)), dim3(256), 0, c->stream, rb, nu, 0.0);
            HIPCHK(c, hipGetLastError());
        }
        if (u && (s = zero_solid(c, inst, u, 3))) return s;
        return LBSC_OK;
    }
    HIPCHK(c, by_precision(c->precision, [&](auto tag) {
               using S = decltype(tag);
               using T = typename S::T;
               if (ra || rb)
                   hipLaunchKernelGGL(lbsc::k_read_density<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], ra ? ra + off : nullptr, rb ? rb + off : nullptr);
               hipError_t e = hipGetLastError();
               if (e != hipSuccess || !u) return e;
               hipLaunchKernelGGL(lbsc::k_read_velocity<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                  (const T*)c->pop[c->cur], (const double*)ra + off, (const double*)rb + off, u + off,
                                  nu);
               return hipGetLastError();
           }));
    if (ra && (s = zero_solid(c, inst, ra, 1))) return s;
    if (rb && (s = zero_solid(c, inst, rb, 1))) return s;
    if (u && (s = zero_solid(c, inst, u, 3))) return s;
    return LBSC_OK;
}

lbsc_status lbsc_read_populations(lbsc_ctx* c, int32_t inst, double* f)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    if (!f) return fail(c, LBSC_E_ARG, "read_populations: null pointer");
    const Inst I = c->inst[inst];
    const int64_t off = solid_nodes(c, inst), nu = user_nodes(c, inst);
    if (c->ncomp == 1) {
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_read_pops1<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], f + off, nu);
                   return hipGetLastError();
               }));
        return zero_solid(c, inst, f, lbsc::kQ);
    }
    HIPCHK(c, by_precision(c->precision, [&](auto tag) {
               using S = decltype(tag);
               using T = typename S::T;
               hipLaunchKernelGGL(lbsc::k_read_pops<S>, dim3(fill_grid(I.n)), dim3(256), 0, c->stream, I,
                                  (const T*)c->pop[c->cur], f + off, nu);
               return hipGetLastError();
           }));
    return zero_solid(c, inst, f, 2 * lbsc::kQ);
}

lbsc_status lbsc_diagnostics(lbsc_ctx* c, int32_t inst, lbsc_diag* out)
{
    lbsc_status s = check_inst(c, inst);
    if (s) return s;
    if (!out) return fail(c, LBSC_E_ARG, "diagnostics: null output");
    const Inst I = c->inst[inst];
    if (c->ncomp == 1)
        HIPCHK(c, by_precision1(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_diag_planes1<S>, dim3(I.nz), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], c->d_part());
                   return hipGetLastError();
               }));
    else
        HIPCHK(c, by_precision(c->precision, [&](auto tag) {
                   using S = decltype(tag);
                   using T = typename S::T;
                   hipLaunchKernelGGL(lbsc::k_diag_planes<S>, dim3(I.nz), dim3(256), 0, c->stream, I,
                                      (const T*)c->pop[c->cur], c->d_part());
                   return hipGetLastError();
               }));
    hipLaunchKernelGGL(lbsc::k_diag_final<256>, dim3(1), dim3(256), 0, c->stream, I, (const double*)c->d_part(),
                       (const double*)c->d_eacc(), (const double*)c->d_ebase(), inst, c->d_out());
    HIPCHK(c, hipGetLastError());
    double h[16];
    HIPCHK(c, hipMemcpyAsync(h, c->d_out(), 11 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out->step = c->step;
    out->mass[0] = h[0];
    // one component: the second plane slot held the phase midpoint (for the
    // interface), not a mass
    out->mass[1] = c->ncomp == 1 ? 0.0 : h[1];
    out->momentum[0] = h[2];
    out->momentum[1] = h[3];
    out->momentum[2] = h[4];
    out->r_droplet = std::cbrt(3.0 * h[5] / (4.0 * M_PI));
    out->evap_rate = h[6];
    out->evaporated = h[9] + (I.count_reset ? h[6] : 0.0);
    out->nonfinite = (int64_t)h[7];
    out->nonpositive = (int64_t)h[8];
    out->z_interface = h[10] + I.z_off;  // the caller's plane index
    if (out->nonfinite > 0) return fail(c, LBSC_E_NONFINITE, "instance %d: %lld nodes with non-finite density", inst,
                                        (long long)out->nonfinite);
    return LBSC_OK;
}

lbsc_status lbsc_checkpoint_bytes(const lbsc_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBSC_E_ARG;
    *bytes = align_up(sizeof(CkptHeader) + c->inst.size() * sizeof(Inst), kAlign) + c->pop_elems * c->elem +
             align_up(c->n_inst * sizeof(double), kAlign);
    return LBSC_OK;
}

lbsc_status lbsc_save(lbsc_ctx* c, void* blob)
{
    lbsc_status s = check_bound(c);
    if (s) return s;
    if (!blob || (uintptr_t)blob % kAlign) return fail(c, LBSC_E_ARG, "save: blob must be non-null and aligned");
    if ((s = fold_eacc(c))) return s;
    std::vector<char> head(align_up(sizeof(CkptHeader) + c->inst.size() * sizeof(Inst), kAlign), 0);
    CkptHeader h{kMagic, c->n_inst, c->precision, c->step, (int64_t)(c->pop_elems * c->elem), c->cur, 0};
    memcpy(head.data(), &h, sizeof h);
    memcpy(head.data() + sizeof h, c->inst.data(), c->inst.size() * sizeof(Inst));
    char* b = (char*)blob;
    HIPCHK(c, hipMemcpyAsync(b, head.data(), head.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + head.size(), c->pop[c->cur], c->pop_elems * c->elem, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(b + head.size() + c->pop_elems * c->elem, c->d_ebase(), c->n_inst * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBSC_OK;
}

lbsc_status lbsc_load(lbsc_ctx* c, const void* blob)
{
    lbsc_status s = check_bound(c);
    if (s) return s;
    if (!blob || (uintptr_t)blob % kAlign) return fail(c, LBSC_E_ARG, "load: blob must be non-null and aligned");
    std::vector<char> head(align_up(sizeof(CkptHeader) + c->inst.size() * sizeof(Inst), kAlign), 0);
    const char* b = (const char*)blob;
    HIPCHK(c, hipMemcpyAsync(head.data(), b, head.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    CkptHeader h;
    memcpy(&h, head.data(), sizeof h);
    if (h.magic != kMagic || h.n_inst != c->n_inst || h.precision != c->precision ||
        h.pop_bytes != (int64_t)(c->pop_elems * c->elem))
        return fail(c, LBSC_E_ARG, "load: checkpoint does not match this context");
    std::vector<Inst> saved(c->inst.size());
    memcpy(saved.data(), head.data() + sizeof h, saved.size() * sizeof(Inst));
    for (size_t k = 0; k < saved.size(); ++k) {
        const Inst &a = saved[k], &b2 = c->inst[k];
        if (a.nx != b2.nx || a.ny != b2.ny || a.nz != b2.nz || a.base != b2.base || a.ps != b2.ps)
            return fail(c, LBSC_E_ARG, "load: instance %zu geometry differs", k);
    }
    HIPCHK(c, hipMemcpyAsync(c->pop[c->cur], b + head.size(), c->pop_elems * c->elem, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_ebase(), b + head.size() + c->pop_elems * c->elem, c->n_inst * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(lbsc::k_fill_f64, dim3(fill_grid(c->max_items)), dim3(256), 0, c->stream, c->d_eacc(),
                       (int64_t)c->max_items, 0.0);
    HIPCHK(c, hipGetLastError());
    for (size_t k = 0; k < saved.size(); ++k) {
        Inst& I = c->inst[k];
        I.count_reset = saved[k].count_reset;
        I.reset = saved[k].reset;
        I.cur = saved[k].cur;
        c->params[k].sink = I.cur.kind;
        c->params[k].rho_h = I.cur.rho_h;
        c->params[k].sink_radius = std::sqrt(I.cur.r2);
    }
    c->step = h.step;
    return upload_table(c);
}

lbsc_status lbsc_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream)
{
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return LBSC_E_ARG;
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return LBSC_OK;
    if ((n16 + 255) / 256 > INT32_MAX) return LBSC_E_ARG;
    const int grid = (int)((n16 + 255) / 256);
    hipLaunchKernelGGL(lbsc::k_copy16, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (const uint4*)src,
                       (uint4*)dst, n16);
    return hipGetLastError() == hipSuccess ? LBSC_OK : LBSC_E_HIP;
}

// Pipelined-step halo check of one tile: every stencil read of every tile
// node lands on a footprint cell that the block writes (a tile node or one of
// its nring <= nt halo nodes) and that cell holds the right lattice node.
int pipe_halo_errors(const Item& it, int nx, int ny, int nt)
{
    const int tw = it.tw, th = it.th, row = tw + 2;
    const bool xper = tw == nx, yper = th == ny;
    const lbsc::PipeTile p = lbsc::pipe_tile(tw, th, nx, ny);
    if (p.nring > nt) return 0;  // the pipelined step rejects this tile
    std::vector<int> cell((size_t)row * (th + 2), -1);  // lattice node in each written cell
    auto node = [&](int fx, int fy) { return lbsc::wrap(it.y0 + fy, ny) * nx + lbsc::wrap(it.x0 + fx, nx); };
    int bad = 0;
    for (int ty = 0; ty < th; ++ty)
        for (int tx = 0; tx < tw; ++tx) cell[(size_t)(ty + 1) * row + tx + 1] = node(tx, ty);
    for (int r = 0; r < p.nring; ++r) {
        int fx, fy;
        lbsc::pipe_ring_node(r, p, tw, th, xper, fx, fy);
        if (fx < -1 || fx > tw || fy < -1 || fy > th) { ++bad; continue; }
        int& c = cell[(size_t)(fy + 1) * row + fx + 1];
        if (c != -1) ++bad;  // each cell written once
        c = node(fx, fy);
    }
    for (int ty = 0; ty < th; ++ty)
        for (int tx = 0; tx < tw; ++tx) {
            int cI[3], rI[3];
            lbsc::pipe_stencil(tx, tw, xper, cI);
            lbsc::pipe_stencil(ty, th, yper, rI);
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    const int ci = cI[1 + ex], ri = rI[1 + ey];
                    if (ci < 0 || ci > tw + 1 || ri < 0 || ri > th + 1) { ++bad; continue; }
                    if (cell[(size_t)ri * row + ci] != node(tx + ex, ty + ey)) ++bad;
                }
        }
    return bad;
}

int32_t lbsc_selftest(void)
{
    using namespace lbsc;
    int bad = 0;
    // Lattice: opposites, weights, isotropy up to second order.
    double sw = 0, s1[3] = {0, 0, 0}, s2[3][3] = {{0}};
    for (int i = 0; i < kQ; ++i) {
        if (ex(opp(i)) != -ex(i) || ey(opp(i)) != -ey(i) || ez(opp(i)) != -ez(i)) ++bad;
        const int e2 = ex(i) * ex(i) + ey(i) * ey(i) + ez(i) * ez(i);
        if (wgt(i) != (e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0))) ++bad;
        for (int j = 0; j < i; ++j)
            if (ex(i) == ex(j) && ey(i) == ey(j) && ez(i) == ez(j)) ++bad;
        const int e[3] = {ex(i), ey(i), ez(i)};
        sw += wgt(i);
        for (int a = 0; a < 3; ++a) {
            s1[a] += wgt(i) * e[a];
            for (int b = 0; b < 3; ++b) s2[a][b] += wgt(i) * e[a] * e[b];
        }
    }
    if (std::fabs(sw - 1.0) > 1e-15) ++bad;
    for (int a = 0; a < 3; ++a) {
        if (std::fabs(s1[a]) > 1e-15) ++bad;
        for (int b = 0; b < 3; ++b)
            if (std::fabs(s2[a][b] - (a == b ? 1.0 / 3.0 : 0.0)) > 1e-15) ++bad;
    }
    // Pulls form a permutation of the stored slots, with and without a wall,
    // and the inverse mapping used by the init kernels agrees with it.
    for (int wall = 0; wall < 2; ++wall) {
        const int nx = 3, ny = 2, nz = 4;
        std::vector<int> hits(kQ * nx * ny * nz, 0);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    for (int i = 0; i < kQ; ++i) {
                        PullSrc s = pull_src(i, x, y, z, nx, ny, nz, wall);
                        const int q = s.reflected ? opp(i) : i;
                        if (s.x < 0 || s.x >= nx || s.y < 0 || s.y >= ny || s.z < 0 || s.z >= nz) ++bad;
                        else hits[q * nx * ny * nz + (int)node_of(s.x, s.y, s.z, nx, ny)] += 1;
                        // inverse: slot (q, src) -> target node/population
                        const int zt = s.z + ez(q);
                        int tx, ty, tz, ti;
                        if (wall && (zt < 0 || zt >= nz)) { tx = s.x; ty = s.y; tz = s.z; ti = opp(q); }
                        else { tx = wrap(s.x + ex(q), nx); ty = wrap(s.y + ey(q), ny); tz = wrap(zt, nz); ti = q; }
                        if (tx != x || ty != y || tz != z || ti != i) ++bad;
                    }
        for (int h : hits)
            if (h != 1) ++bad;
    }
    // Every byte of a slab holds exactly one element (c, i) of one in-plane
    // node, and each access is aligned to its width: a pair for the paired
    // forms (one instruction moves both components), one element otherwise.
    auto check_layout = [&](auto tag) {
        using S = decltype(tag);
        for (uint32_t ps : {64u, 4160u, 65536u}) {
            const uint32_t bytes = (uint32_t)kSlabPlanes<S> * ps * (uint32_t)sizeof(typename S::T);
            std::vector<uint8_t> owner(bytes, 0);
            for (int c = 0; c < 2; ++c)
                for (int i = 0; i < kQ; ++i) {
                    const uint32_t e = elem_bytes<S>(i), st = node_stride<S>(i);
                    const uint32_t align = S::kPair ? pair_bytes<S>(i) : e;
                    for (uint32_t xy = 0; xy < ps; ++xy) {
                        const uint32_t o = plane_off<S>(c, i, ps) + xy * st;
                        if (o + e > bytes) { ++bad; continue; }
                        if ((o - (uint32_t)c * (S::kPair ? e : 0u)) % align) ++bad;
                        for (uint32_t b = 0; b < e; ++b) ++owner[o + b];
                    }
                }
            for (uint8_t k : owner)
                if (k != 1) ++bad;
        }
    };
    check_layout(StF64{});
    check_layout(StF32S{});
    check_layout(StF16S{});
    check_layout(StF16N{});
    check_layout(StF16NF{});
    // psi planes stay in range.
    for (int nz : {1, 2, 5})
        for (int wall = 0; wall < 2; ++wall)
            for (int z = -1; z <= nz; ++z) {
                const int p = psi_plane(z, nz, wall);
                if (p < 0 || p >= nz) ++bad;
            }
    // The packed fluid z interval of every column reproduces in_sink node by
    // node (spheres with random, half-integer and outside centres, radii with
    // exact ties; the other kinds).
    {
        uint64_t st = 0x9E3779B97F4A7C15ull;
        auto rnd = [&]() {
            st = st * 6364136223846793005ull + 1442695040888963407ull;   // Knuth's MMIX LCG
            return (double)(st >> 11) * (1.0 / 9007199254740992.0);
        };
        const int dims2[][3] = {{13, 11, 17}, {7, 9, 40}, {5, 5, 3}, {1, 1, 9}, {3, 3, 1}, {2, 2, 2}, {1, 1, 1}};
        for (auto& d : dims2)
            for (int trial = 0; trial < 60; ++trial) {
                Sink sk{};
                // none, z-max, faces, faces without the z = 0 face, spheres
                sk.kind = trial < 4 ? (trial == 3 ? kSinkFaces : trial) : kSinkSphere;
                sk.no_zlo = trial == 3;
                const int mode = trial % 4;
                auto coord = [&](int n) {
                    const double u = rnd() * (n + 6) - 3;
                    return mode == 0 ? u : (mode == 1 ? std::floor(u) + 0.5 : (mode == 2 ? std::floor(u) : u * 3));
                };
                sk.cx = coord(d[0]); sk.cy = coord(d[1]); sk.cz = coord(d[2]);
                const double r = rnd() * 0.8 * (d[0] + d[1] + d[2]) / 2;
                sk.r2 = mode == 2 ? std::floor(r * r) : r * r;
                for (int y = 0; y < d[1]; ++y)
                    for (int x = 0; x < d[0]; ++x) {
                        const uint32_t zr = sink_zrange(sk, x, y, d[0], d[1], d[2]);
                        for (int z = 0; z < d[2]; ++z)
                            if (in_zrange_sink(zr, z) != in_sink(sk, x, y, z, d[0], d[1], d[2])) ++bad;
                    }
            }
    }
    // Stochastic rounding of the rest population: always one of the two FP32
    // neighbours of x (x itself when representable), and unbiased: over
    // 2^16 keys the mean of the rounded values is x to within the sampling
    // error of a two-point draw across one FP32 gap.
    {
        uint64_t st = 0x0123456789ABCDEFull;
        auto rnd = [&]() {
            st = st * 6364136223846793005ull + 1442695040888963407ull;   // Knuth's MMIX LCG
            return (double)(st >> 11) * (1.0 / 9007199254740992.0);
        };
        for (int trial = 0; trial < 64; ++trial) {
            const double mag = std::ldexp(1.0, -(int)(rnd() * 30));
            const double x = (rnd() - 0.5) * mag;
            const float f = (float)x;
            const float lo = f <= x ? f : std::nextafter(f, -INFINITY);
            const float hi = f >= x ? f : std::nextafter(f, INFINITY);
            double sum = 0.0;
            const int n = 1 << 16;
            for (int k = 0; k < n; ++k) {
                const float r = round_sr(x, (uint32_t)k * 2654435761u + (uint32_t)trial);
                if (r != lo && r != hi) ++bad;
                sum += (double)r;
            }
            const double gap = (double)hi - (double)lo;
            if (std::fabs(sum / n - x) > 5.0 * 0.5 * gap / std::sqrt((double)n) + 1e-300) ++bad;
            if ((double)f == x && round_sr(x, 7u) != f) ++bad;
            // the same for the sum of two FP32 values, rounded through TwoSum
            const float a = (float)(x * (0.5 + rnd())), b = (float)(x - (double)a);
            const double xe = (double)a + (double)b;
            const float fe = (float)xe;
            const float lo2 = fe <= xe ? fe : std::nextafter(fe, -INFINITY);
            const float hi2 = fe >= xe ? fe : std::nextafter(fe, INFINITY);
            double sum2 = 0.0;
            for (int k = 0; k < n; ++k) {
                const float r = round_sr_sum(a, b, (uint32_t)k * 2654435761u + (uint32_t)trial);
                if (r != lo2 && r != hi2) ++bad;
                sum2 += (double)r;
            }
            const double gap2 = (double)hi2 - (double)lo2;
            if (std::fabs(sum2 / n - xe) > 5.0 * 0.5 * gap2 / std::sqrt((double)n) + 1e-300) ++bad;
            // both components of a node at once (one hash, 16-bit draws:
            // unbiased to 2^-16 of the gap beyond the sampling error)
            const float a1 = (float)(0.3 * rnd() - 0.1), b1 = (float)((rnd() - 0.5) * 1e-3 * mag);
            const double x1 = (double)a1 + (double)b1;
            const float f1 = (float)x1;
            const float lo3 = f1 <= x1 ? f1 : std::nextafter(f1, -INFINITY);
            const float hi3 = f1 >= x1 ? f1 : std::nextafter(f1, INFINITY);
            double s0 = 0.0, s1 = 0.0;
            for (int k = 0; k < n; ++k) {
                float out[2];
                round_sr_sum2({a, a1}, {b, b1}, (uint32_t)k * 2654435761u + (uint32_t)trial, out);
                if ((out[0] != lo2 && out[0] != hi2) || (out[1] != lo3 && out[1] != hi3)) ++bad;
                s0 += (double)out[0];
                s1 += (double)out[1];
            }
            const double gap3 = (double)hi3 - (double)lo3;
            if (std::fabs(s0 / n - xe) > gap2 * (2.5 / std::sqrt((double)n) + 1.0 / 65536.0) + 1e-300) ++bad;
            if (std::fabs(s1 / n - x1) > gap3 * (2.5 / std::sqrt((double)n) + 1.0 / 65536.0) + 1e-300) ++bad;
        }
    }
    // Item placement: every item once, each instance's items inside its own
    // range (with padding only), the eight XCD runs of near-equal cost, and
    // a single instance of equal items split into equal runs without padding.
    {
        const int boxes[][3] = {{48, 48, 48}, {156, 156, 156}, {97, 97, 97}, {60, 60, 60}, {130, 130, 130},
                                {49, 50, 51}, {150, 150, 20}};
        const int single[][3] = {{128, 128, 128}, {48, 48, 48}};
        for (int nb : {0, 1, 3, 7}) {
            // nb = 0: one 128^3 instance (equal items)
            const int(*bx)[3] = nb == 0 ? single : boxes;
            nb = std::max(nb, 1);
            std::vector<Inst> insts(nb);
            std::vector<std::vector<Item>> per(nb);
            int64_t total = 0, count = 0;
            for (int k = 0; k < nb; ++k) {
                insts[k].nx = bx[k][0]; insts[k].ny = bx[k][1]; insts[k].nz = bx[k][2];
                insts[k].n = (int64_t)bx[k][0] * bx[k][1] * bx[k][2];
                total += insts[k].n;
            }
            for (int k = 0; k < nb; ++k) {
                instance_items(insts[k], k, lbsc_tiles{512, 0, 0, k == 1 ? 8 : 0, 0}, 512, 3, 16, kColumnWeight,
                               total, 4096, 256, per[k]);
                count += (int64_t)per[k].size();
            }
            std::vector<Item> items;
            place_items(per, insts, items);
            if (items.size() % 8) ++bad;
            const size_t run = items.size() / 8;
            int64_t real = 0;
            double c8[8] = {0}, cmax = 0.0;
            for (size_t q = 0; q < items.size(); ++q) {
                const Item& it = items[q];
                if (it.nzc == 0) continue;
                ++real;
                if ((int32_t)q < insts[it.inst].item_begin || (int32_t)q >= insts[it.inst].item_end) ++bad;
                const double cq = item_cost(it, insts[it.inst]);
                c8[q / run] += cq;
                cmax = std::max(cmax, cq);
            }
            if (real != count) ++bad;
            for (int k = 0; k < nb; ++k)
                for (int k2 = 0; k2 < nb; ++k2)
                    if (k != k2 && insts[k].item_begin < insts[k2].item_end && insts[k2].item_begin < insts[k].item_end)
                        ++bad;
            const double mean = (c8[0] + c8[1] + c8[2] + c8[3] + c8[4] + c8[5] + c8[6] + c8[7]) / 8.0;
            for (double cj : c8)
                if (std::fabs(cj - mean) > cmax) ++bad;
            // a table too small for the padding: equal counts instead
            std::vector<Item> tight;
            place_items(per, insts, tight, (size_t)count + 7);
            if (tight.size() > (size_t)count + 7) ++bad;
            int64_t real2 = 0;
            for (size_t q = 0; q < tight.size(); ++q)
                if (tight[q].nzc > 0) {
                    ++real2;
                    if ((int32_t)q < insts[tight[q].inst].item_begin || (int32_t)q >= insts[tight[q].inst].item_end)
                        ++bad;
                }
            if (real2 != count) ++bad;
            place_items(per, insts, items);   // restore the balanced ranges
            bool equal = true;
            for (const Item& it : per[0]) equal = equal && item_cost(it, insts[0]) == item_cost(per[0][0], insts[0]);
            if (nb == 1 && equal && per[0].size() % 8 == 0 && items.size() != per[0].size()) ++bad;
        }
    }
    // Work items tile every lattice exactly once.
    const int dims[][3] = {{4, 4, 128}, {128, 128, 128}, {48, 48, 48}, {156, 156, 156}, {1, 1, 64}, {200, 7, 9},
                           {4096, 2, 3}, {3, 4096, 2}, {2, 3, 4096}, {1, 1, 4096}, {512, 5, 3}, {300, 4, 2},
                           {257, 3, 2}, {384, 6, 2}};
    for (auto& d : dims)
        for (int nt : {256, 512})
            for (int tw : {0, 8, 16, 32, 64, 128, 200, 256})
                for (int nzc : {0, 4, 16})
                for (int target : {256, 4096})
                for (int min_rows : {3, 8})
                for (int line : {1, 8, 16, 32}) {
                    if (tw > 0 && line != 16) continue;   // an explicit width ignores the line
                    Inst I{};
                    I.nx = d[0]; I.ny = d[1]; I.nz = d[2];
                    I.n = (int64_t)d[0] * d[1] * d[2];
                    std::vector<Item> items;
                    instance_items(I, 0, lbsc_tiles{nt, tw, 0, nzc, 0}, nt, min_rows, line,
                                   line == 32 ? kColumnWeightF16 : kColumnWeight, I.n, target, 256, items);
                    std::vector<unsigned char> cover((size_t)I.n, 0);
                    const bool split = tw == 0 && I.nx > std::max(1, nt / min_rows);
                    for (auto& it : items) {
                        if (split && line <= std::min(128, nt / min_rows) && I.nx % line == 0 && it.x0 % line) ++bad;
                        if (it.tw * it.th > nt) ++bad;
                        const int foot = nt == 256 ? Foot<256>::kMax : Foot<512>::kMax;
                        if ((it.tw + 2) * (it.th + 2) > foot) ++bad;
                        for (int z = it.z0; z < it.z0 + it.nzc; ++z)
                            for (int y = it.y0; y < it.y0 + it.th; ++y)
                                for (int x = it.x0; x < it.x0 + it.tw; ++x) {
                                    if (x >= I.nx || y >= I.ny || z >= I.nz) { ++bad; continue; }
                                    cover[(size_t)node_of(x, y, z, I.nx, I.ny)] += 1;
                                }
                    }
                    for (auto v : cover)
                        if (v != 1) { ++bad; break; }
                    for (auto& it : items) bad += pipe_halo_errors(it, I.nx, I.ny, nt);
                }
    return bad;
}

}  // extern "C"
