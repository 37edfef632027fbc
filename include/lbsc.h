/*
 * lbsc: two-component D3Q19 Shan-Chen lattice Boltzmann step with the
 * mass-conserving evaporation sink, for AMD MI355X (gfx950).
 *
 * Method: Hessling, Xie and Harting, "Diffusion dominated evaporation in
 * multicomponent lattice Boltzmann simulations", arXiv:1701.03637, Sec. II:
 *   - BGK update per component, Eq. (LBM), towards the second-order
 *     equilibrium of Eq. (eqdis) on D3Q19 (w = 1/3, 1/18, 1/36, c_s^2 = 1/3);
 *   - densities and velocities as defined after Eq. (eqdis), with the common
 *     velocity u' = sum_c rho^c u^c / sum_c rho^c;
 *   - Shan-Chen inter-component force, Eq. (sc), with psi of Eq. (psifunc)
 *     (psi = 1 - exp(-rho), rho_0 = 1) or psi = rho, applied as the velocity
 *     shift tau^c F^c / rho^c (Sec. II B);
 *   - periodic boundaries, optionally a bounce-back wall on the z seam
 *     (Sec. II A);
 *   - the evaporation sink of Sec. II C: at sink nodes component A (the
 *     evaporating one) is reset to f^eq(rho_H, 0) and component B to
 *     f^eq(rhoA + rhoB - rho_H, 0), from the densities streamed in during the
 *     step, so every sink node keeps its total density; sink nodes neither
 *     collide nor feel the force.
 *
 * Conventions
 *   - Every call returns an lbsc_status; nothing throws across this ABI. On
 *     failure lbsc_last_error(ctx) returns a message for that context.
 *   - The caller owns all device memory: it allocates the two population
 *     buffers and the scratch buffer (sizes from lbsc_required_bytes, every
 *     pointer 256-byte aligned) and hands them over with lbsc_bind. The
 *     library never allocates or frees device memory; it owns only host
 *     metadata, one private capture stream and HIP graph objects.
 *   - Work is enqueued asynchronously on the stream set by lbsc_set_stream
 *     (default: the null stream). Calls that return host data
 *     (lbsc_diagnostics, lbsc_load) and calls that change the instance table
 *     (lbsc_bind, lbsc_init_*, lbsc_set_sink, lbsc_set_tiles, lbsc_tune,
 *     lbsc_step's first step after an init or sink change) synchronise that
 *     stream.
 *   - A context must not be used from two host threads at once.
 *   - A context holds one or more instances (independent lattices with their
 *     own size and fluid parameters) that are stepped together in one launch
 *     per time step. Instance indices run from 0 to n_inst - 1.
 *   - Node order everywhere is z-major: node = (z*ny + y)*nx + x.
 *   - Component 0 is A (held at rho_H by the sink), component 1 is B.
 *   - Direction order: 0 rest, 1..6 = +x,-x,+y,-y,+z,-z, 7..18 = the face
 *     diagonals (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0),(+1,0,+1),(-1,0,-1),
 *     (+1,0,-1),(-1,0,+1),(0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).
 */
#ifndef LBSC_H
#define LBSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbsc_status {
    LBSC_OK = 0,
    LBSC_E_ARG = -1,         /* invalid argument, size or pointer */
    LBSC_E_STATE = -2,       /* call not valid in the context's state (e.g. unbound) */
    LBSC_E_HIP = -3,         /* a HIP runtime call failed */
    LBSC_E_NONFINITE = -4,   /* diagnostics found a non-finite density */
    LBSC_E_UNSUPPORTED = -5  /* option not supported */
} lbsc_status;

/* Storage precision of the populations. FP32S/FP16S store the deviation
 * f - w_i*shift[c] and compute in FP32; FP64 stores f and computes in FP64.
 * FP16N stores a per-node shift: the rest deviation d_0 = f_0 - w_0 shift[c]
 * in FP32 and the moving deviations as d_i - (w_i/w_0) d_0 of the same node
 * in FP16 (zero at rest equilibrium; 160 bytes per lattice update), FP32
 * arithmetic. FP16NF stores the same with the moving deviations times 2^12:
 * deviations down to 1.5e-8 (rather than FP16's smallest normal 6.1e-5) keep
 * FP16's 11 significant bits, which slow diffusion through near-uniform
 * regions needs (its diffusion coefficient matches FP64's where FP16N's comes
 * out low); |d_i - (w_i/w_0) d_0| must stay below 16, and its step costs a
 * few percent more than FP16N's (one more operation per decoded value).
 * Global sums (mass, evaporated mass, interface) are FP64 in every form. */
enum { LBSC_FP64 = 0, LBSC_FP32S = 1, LBSC_FP16S = 2, LBSC_FP16N = 3, LBSC_FP16NF = 4 };
enum { LBSC_PSI_RHO = 0, LBSC_PSI_EXP = 1 };
/* Sink node sets: the plane z = nz-1; the six faces; all nodes at distance
 * >= sink_radius from center. */
enum { LBSC_SINK_NONE = 0, LBSC_SINK_ZMAX = 1, LBSC_SINK_FACES = 2, LBSC_SINK_SPHERE = 3 };
/* Option bits of lbsc_params.flags.
 * LBSC_FLAG_FP16S_SINK: accept FP16S storage together with an evaporation
 * sink. Without it that combination is refused with LBSC_E_UNSUPPORTED: with
 * a constant shift, FP16 rounds away the small per-step changes of slow
 * diffusion, so the vapour near the sink stops relaxing, the sink keeps
 * booking a flux that never leaves the droplet and M^A + E drifts from
 * M^A(0) (use FP16N, which stores a per-node shift). The flag exists to test
 * the FP16S code paths. */
enum { LBSC_FLAG_FP16S_SINK = 1 };

typedef struct lbsc_params {
    int32_t nx, ny, nz;      /* lattice size, each 1..4096, nx*ny*nz < 2^31 and
                                38*nx*ny*element size < 4 GiB */
    int32_t wall_z;          /* 1: half-way bounce-back wall on the z seam */
    double tau[2];           /* relaxation times tau^A, tau^B (> 0.5) */
    double g;                /* interaction strength g^{AB} = g^{BA} */
    int32_t psi;             /* LBSC_PSI_RHO or LBSC_PSI_EXP */
    int32_t precision;       /* LBSC_FP64/FP32S/FP16S/FP16N/FP16NF; equal for all instances */
    double shift[2];         /* rho0^c of shifted storage (ignored for FP64) */
    int32_t sink;            /* LBSC_SINK_* */
    int32_t plane_pad;       /* extra elements between population planes
                                (0 .. 2^20; spreads the plane streams over
                                HBM channels: 38 per slab for FP32S, 19
                                planes of (A, B) pairs for FP64 and FP16);
                                0 = none; -1 = automatic: 320 where a plane's
                                byte size is a multiple of 64 KiB and it
                                holds at least 2^14 nodes, else none */
    double rho_h;            /* density imposed on A at sink nodes */
    double sink_radius;      /* LBSC_SINK_SPHERE only */
    double center[3];        /* sphere centre (x, y, z) in node units */
    double phi_delta[2];     /* rhoA - rhoB inside / outside a droplet, for the
                                volume-fraction radius diagnostic */
    int32_t solid_z;         /* thickness h >= 0 of a solid wall occupying the
                                planes z = 0 .. h-1 (Sec. III A, III B: walls of
                                thickness 2 at the bottom of the film). Fluid
                                links into solid nodes bounce back half-way
                                ("inverting velocities", Sec. II A): below
                                z = h and, through the periodic z wrap, above
                                z = nz-1. Solid nodes hold no fluid; in the
                                force of Eq. (sc) they count with
                                psi(wall_rho[c]). Excludes wall_z; needs
                                nz > h. */
    int32_t flags;           /* LBSC_FLAG_* bits */
    double wall_rho[2];      /* densities of solid nodes in the force of
                                Eq. (sc) (0, 0: the wall does not interact) */
    int32_t ncomp;           /* components: 2 (also 0), or 1 for the
                                single-component multiphase form the method
                                carries over to (Sec. I): the force of
                                Eq. (sc) takes the component itself as the
                                partner with coupling g (g < 0 attracts), and
                                the sink holds it at rho_H with zero velocity;
                                with no partner the removed mass leaves the
                                system and is booked as E (Sec. II C). Uses
                                tau[0], shift[0], wall_rho[0]; phi_delta holds
                                the liquid and vapour densities (the interface
                                is where rho crosses their midpoint). FP64 or
                                FP32S only (LBSC_E_UNSUPPORTED otherwise); all
                                instances of a context alike. */
    int32_t reserved;        /* 0 */
} lbsc_params;

/* FP64 diagnostics of one instance (Sec. II C for the sink bookkeeping,
 * Sec. III B for the film's interface position, Sec. III C for the droplet
 * radius). Solid wall nodes are left out of every sum. */
typedef struct lbsc_diag {
    int64_t step;            /* time steps taken since the last init */
    double mass[2];          /* sum over nodes of rho^A, rho^B */
    double evaporated;       /* mass of A removed by the sink since init: the
                                sum over resets of rhoA_pre - rho_H (Sec. II C) */
    double evap_rate;        /* sum over sink nodes of (rhoA_pre - rho_H) in the
                                reset that formed the current state */
    double momentum[3];      /* sum over nodes and components of j^c */
    double z_interface;      /* x_I of Sec. III B, where rhoA - rhoB = 0: the
                                first zero of its plane mean, scanning up from
                                the lowest fluid plane, linearly interpolated;
                                NaN if none */
    double r_droplet;        /* the droplet radius R_I of Sec. III C, taken as
                                (3 V / 4 pi)^(1/3) with V the sum of the
                                clamped volume fraction of A,
                                (rhoA - rhoB - phi_delta[1]) /
                                (phi_delta[0] - phi_delta[1]) */
    int64_t nonfinite;       /* nodes with a non-finite density */
    int64_t nonpositive;     /* nodes with a density <= 0 */
} lbsc_diag;

typedef struct lbsc_ctx lbsc_ctx;

/* Tile schedule of the fused step kernel: nt threads per block (256 or 512),
 * xy tile tw x th (tw*th <= nt), z chunk of nzc planes, and the
 * kernel variant: 1 keeps a node's pulled populations in registers from its
 * density pass to its collision, 2 pulls the node again for the collision
 * (fewer registers, more blocks per CU), 3 (FP64 with nt = 256, FP32S,
 * FP16S, FP16N, FP16NF) also keeps them but issues each plane's loads one plane ahead
 * of use, with one barrier per plane; it needs one thread per halo node of a
 * tile (the halo of a tile spanning the whole x or y extent is the tile
 * itself), and for FP16N and FP16NF (tw + 4)(th + 4) <= 3 nt (the rest values of the
 * tile and two halo rings are staged through LDS), so tiles that break this
 * are rejected. Variants give bitwise
 * identical populations. Zero or negative fields mean "choose automatically"
 * (variant: 3 where it applies, else 1). */
typedef struct lbsc_tiles {
    int32_t nt, tw, th, nzc, variant;
} lbsc_tiles;

/* Static description of a status code. */
const char* lbsc_status_string(lbsc_status s);
/* Message of the last failure on ctx ("" if none). */
const char* lbsc_last_error(const lbsc_ctx* ctx);
/* Library version string. */
const char* lbsc_version(void);

/* Creates a context of n_inst instances (params[0..n_inst-1]). Validates
 * sizes and parameters; no device memory is touched. */
lbsc_status lbsc_create(int32_t n_inst, const lbsc_params* params, lbsc_ctx** out);
/* Releases host metadata and graphs; never frees the caller's buffers. */
lbsc_status lbsc_destroy(lbsc_ctx* ctx);

/* Bytes the caller must allocate: each of the two population buffers, and the
 * scratch buffer (instance table, work items, FP64 accumulators). */
lbsc_status lbsc_required_bytes(const lbsc_ctx* ctx, size_t* pop_bytes, size_t* scratch_bytes);
/* Binds caller-owned device buffers (borrowed until lbsc_destroy). Clears the
 * evaporation accumulators and uploads the instance table. */
lbsc_status lbsc_bind(lbsc_ctx* ctx, void* pop0, void* pop1, void* scratch);
/* Bytes of the per-device static scratch array used by lbsc_bind_static. */
#define LBSC_STATIC_SCRATCH_BYTES (32 * 1024 * 1024)
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): binds the
 * two caller-owned population buffers like lbsc_bind, with the library's own
 * static scratch array in place of a caller scratch buffer. Allocates no
 * device memory. The array holds LBSC_STATIC_SCRATCH_BYTES (32 MiB) on each
 * device the library runs on, until the process ends; a context whose
 * lbsc_required_bytes scratch exceeds it (about 1.75 bytes per lattice node:
 * lattices up to about 2^24 nodes fit) is refused with LBSC_E_ARG. It is
 * bound on the current device. One context per device uses the array at a
 * time: binding another context to it takes it over, after which calls on
 * the previous one return LBSC_E_STATE until it is bound again. Work from
 * two contexts on one device that overlaps in time races on the array. The
 * evaporation accumulators are cleared at bind, as with lbsc_bind. */
lbsc_status lbsc_bind_static(lbsc_ctx* ctx, void* pop0, void* pop1);
/* Stream for all following work (a hipStream_t; NULL = null stream). */
lbsc_status lbsc_set_stream(lbsc_ctx* ctx, void* hip_stream);

/* Initial state f = f^eq(rho, 0) of instance inst from two FP64 device arrays
 * of nx*ny*nz densities (rhoB is ignored, and may be NULL, with one
 * component), then the initial sink reset, which is not counted as
 * evaporated mass. Resets the step counter and the evaporated mass. */
lbsc_status lbsc_init_from_density(lbsc_ctx* ctx, int32_t inst, const double* rhoA_dev, const double* rhoB_dev);
/* As above from full FP64 device populations f[(c*19 + i)*n + node]
 * (f[i*n + node] with one component). */
lbsc_status lbsc_init_from_populations(lbsc_ctx* ctx, int32_t inst, const double* f_dev);

/* Changes the evaporation sink of instance inst (kind, rho_H, sphere
 * radius): the boundary of Sec. II C that holds component A at rho_H and
 * gives B the rest of the node's density, both at zero velocity. Its nodes
 * skip the next collision; they are reset at the end of that step (the
 * workflow of Sec. III B, III C: equilibrate, then impose rho_H). FP16S
 * storage refuses a sink (LBSC_E_UNSUPPORTED) unless the instance was created
 * with LBSC_FLAG_FP16S_SINK. */
lbsc_status lbsc_set_sink(lbsc_ctx* ctx, int32_t inst, int32_t kind, double rho_h, double radius);

/* Advances every instance by n time steps. */
lbsc_status lbsc_step(lbsc_ctx* ctx, int64_t n);
/* Replays steady-state steps as HIP graphs of `steps` launches (even, >= 2);
 * 0 switches graphs off. */
lbsc_status lbsc_set_graph(lbsc_ctx* ctx, int32_t steps);
/* Sets the tile schedule (see lbsc_tiles). */
lbsc_status lbsc_set_tiles(lbsc_ctx* ctx, const lbsc_tiles* tiles);
/* The schedule in use: tw, th, nzc as requested (0 = automatic) and the
 * resolved nt and kernel variant. */
lbsc_status lbsc_get_tiles(const lbsc_ctx* ctx, lbsc_tiles* out);
/* Times candidate tile schedules (variants x nt x tile widths x chunk
 * lengths; chunks of 1, 2 and 4 planes only for contexts of fewer than 2^22
 * nodes) for `steps` steps each (steps >= 2), re-times the three fastest
 * over three times as many steps, and keeps the best; writes it to *chosen
 * if non-NULL. A context of several instances then tunes per size class
 * (boxes whose larger side is < 64, < 96, < 128, < 192, or more): each
 * class's tile width and chunk length (lbsc_set_inst_tiles) that make the
 * whole context's step fastest, one class after the other.
 * Results go to a process-wide cache keyed by (GPU architecture, fluid
 * lattice size (nz without solid planes), precision, components, and for a
 * batch the context's nt and variant), valid for the compiled kernel
 * sources (lbsc_kernel_hash): a
 * one-instance context, or a size class whose every instance is cached,
 * takes its schedule from the cache without timing. The state is left as
 * it was: the timed steps read the stored populations and write only the
 * other population buffer, and book no evaporation, so the populations, the
 * step count and E are those before the call. The graph setting is kept. */
lbsc_status lbsc_tune(lbsc_ctx* ctx, int32_t steps, lbsc_tiles* chosen);
/* Tile width, rows and chunk length of instance inst (tiles->tw, th, nzc;
 * 0 = the context's; nt and variant are the context's), replacing the
 * context's for that instance only; lbsc_get_inst_tiles reads them back with
 * the context's resolved nt and variant. */
lbsc_status lbsc_set_inst_tiles(lbsc_ctx* ctx, int32_t inst, const lbsc_tiles* tiles);
lbsc_status lbsc_get_inst_tiles(const lbsc_ctx* ctx, int32_t inst, lbsc_tiles* out);
/* The tuning cache as text (one line per entry, tagged with the kernel
 * source hash): save writes every entry; load adds the entries of this
 * build's kernel sources (others are skipped) and reports their number;
 * clear empties it. */
lbsc_status lbsc_tune_cache_save(const char* path);
lbsc_status lbsc_tune_cache_load(const char* path, int32_t* n_loaded);
void lbsc_tune_cache_clear(void);
/* Hash of the kernel sources' code this library was built from. */
const char* lbsc_kernel_hash(void);
/* Number of work items (blocks per step) of the current schedule. */
lbsc_status lbsc_num_items(const lbsc_ctx* ctx, int32_t* n_items);

/* FP64 read-outs of the state S(t) (post-stream, post-sink) of instance inst
 * into caller device arrays: densities of component comp (n values); the
 * densities of both components and the barycentric velocity U of Eq. (velw)
 * (out_u[d*n + node], d = x, y, z; any of the three pointers may be NULL
 * except that U needs both density arrays); all populations f[(c*19+i)*n +
 * node]. With one component: comp 0 only, rhoB (if given) is zero, U needs
 * rhoA, and the populations are f[i*n + node]. */
lbsc_status lbsc_read_density(lbsc_ctx* ctx, int32_t inst, int32_t comp, double* out_dev);
lbsc_status lbsc_read_observables(lbsc_ctx* ctx, int32_t inst, double* rhoA_dev, double* rhoB_dev, double* u_dev);
lbsc_status lbsc_read_populations(lbsc_ctx* ctx, int32_t inst, double* f_dev);

/* FP64 diagnostics of instance inst into a host struct (synchronises).
 * Returns LBSC_E_NONFINITE (with *out filled) if a density is not finite. */
lbsc_status lbsc_diagnostics(lbsc_ctx* ctx, int32_t inst, lbsc_diag* out);

/* Checkpoint of the whole context into a caller device buffer of
 * lbsc_checkpoint_bytes bytes; lbsc_load restores it into a context created
 * with the same parameters. */
lbsc_status lbsc_checkpoint_bytes(const lbsc_ctx* ctx, size_t* bytes);
lbsc_status lbsc_save(lbsc_ctx* ctx, void* blob_dev);
lbsc_status lbsc_load(lbsc_ctx* ctx, const void* blob_dev);

/* Copies `bytes` (a multiple of 16, 16-byte aligned pointers) from src to dst
 * on the given stream with a plain streaming kernel: the HBM bandwidth ceiling
 * the step kernel is measured against, and the calibration of byte counters. */
lbsc_status lbsc_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Host-only checks of the index geometry (no GPU needed); 0 on success,
 * otherwise the number of failed checks. */
int32_t lbsc_selftest(void);

#ifdef __cplusplus
}
#endif

#endif /* LBSC_H */
