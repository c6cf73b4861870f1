/*
 * sph.h -- C ABI of the MI355X (gfx950) weakly-compressible SPH hot path with
 * the dummy-particle wall treatment of Rezavand, Zhang & Hu, "Generalised
 * and efficient wall boundary condition treatment in GPU-accelerated SPH"
 * (arXiv 2110.02621).
 *
 * The library follows the paper's statement of the problem (Sec. 3): fluid
 * particles and fixed wall dummy particles live in device memory for the
 * whole run and are advanced by the paper's compartments -- neighbour search
 * with sorting, density update, wall ("BC") pressure, mass and momentum
 * conservation, time integration -- each one a HIP kernel.  Nothing is
 * copied to the host by these calls.
 *
 * Conventions
 *   - Every pointer inside sph_buffers and every array argument marked
 *     "device" is a device pointer owned by the caller.  The library never
 *     allocates, frees or keeps a pointer between calls, and holds no
 *     global state, with one exception: the fixed device workspace of
 *     sph_diag_noalloc.  Scratch memory is passed in (sph_scratch_bytes).
 *   - T is float when desc->precision == SPH_F32 and double for SPH_F64;
 *     "T[dim][n]" means dim arrays of n values of T, one after the other
 *     (structure of arrays: component k of particle i at index k*n + i).
 *   - Positions are held as an integer cell (linear key) plus an in-cell
 *     offset in [0, L_c) of type T; the absolute position is
 *     lo + cell * L_c + offset.
 *   - "stream" is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work and return; data-dependent faults are counted in the
 *     device status words, to be read after synchronising.
 *   - Return codes are synchronous argument, configuration or launch errors
 *     (SPH_OK, SPH_ERR_ARG, SPH_ERR_CONFIG, SPH_ERR_LAUNCH, and
 *     SPH_ERR_CAPACITY from sph_diag_noalloc).  No call aborts or prints.
 *
 * Per-step schedule (sph_step runs exactly this):
 *   sph_density -> sph_build_cells -> sph_wall_bc -> sph_forces(CONTINUITY)
 *   -> sph_forces(MOMENTUM).
 *
 * Moving tank (desc->motion_freq != 0): every wall dummy translates rigidly
 * with X(t).  The state is held in the tank's frame, where the walls stay
 * where sph_init binned them: positions r - X(t), velocities v - u, where u
 * is the tank velocity of the step's time level.  The step of the fixed
 * frame maps onto it exactly: step n's drift moves the tank by
 * X(t_{n+1}) - X(t_n) = dt Vh, so the half kick (sph_density) adds the
 * uniform X'(t_n) - Vh, the walls are at rest relative to the fluid during
 * the pair sweeps (in the fixed frame they move with Vh), Eq. (12) takes
 * g - a_w - X''(t_{n+1}), and the second kick (sph_forces MOMENTUM) adds
 * Vh - X'(t_{n+1}).  The stored dv/dt (acc) is the fixed-frame one.  Input
 * (sph_init) and output (sph_export, sph_export_walls, sph_diag) are in the
 * fixed frame at t = nstep dt; buf->nstep counts the steps.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_OK 0
#define SPH_ERR_ARG 1    /* null pointer, negative size, size mismatch, bad flag */
#define SPH_ERR_CONFIG 2 /* dim not 2 or 3, precision unknown, dt above the CFL bound of
                            Eqs. (23)-(24), grid too large, L_c < 2h, bad motion */
#define SPH_ERR_LAUNCH 3 /* a kernel launch failed (hipGetLastError after the launch), or
                            sph_diag_noalloc could not look up its device workspace */
#define SPH_ERR_CAPACITY 4 /* sph_diag_noalloc: more fluid particles than its fixed workspace holds */

#define SPH_F32 0
#define SPH_F64 1

#define SPH_CONTINUITY 1u /* sph_forces: mass conservation, Eq. (9), + density update, Eq. (21) */
#define SPH_MOMENTUM 2u   /* sph_forces: momentum, Eqs. (10)-(11), (13), + second kick, Eq. (22) */
#define SPH_NO_KICK 4u    /* with SPH_MOMENTUM: write dv/dt only (initial acceleration) */

/* Device status words (uint32_t[SPH_STATUS_LEN]), counted atomically. */
#define SPH_STATUS_OUT_OF_GRID 0 /* particle steps whose drift left the cell grid (clamped) */
#define SPH_STATUS_FAST 1        /* drifts longer than one cell per step (CFL violated) */
#define SPH_STATUS_NONFINITE 2   /* non-finite values met by sph_diag */
#define SPH_STATUS_LIST_OVERFLOW 3 /* queries with a stencil row of more than 128 candidates
                                      (those walk the cells instead: slower, same result) */
#define SPH_STATUS_LEN 4

/* Diagnostics written by sph_diag (double[SPH_DIAG_LEN], device). */
#define SPH_DIAG_MASS 0     /* sum m */
#define SPH_DIAG_MOM 1      /* sum m v, 3 entries (unused trailing ones 0) */
#define SPH_DIAG_EKIN 4     /* sum m |v|^2 / 2 */
#define SPH_DIAG_EPOT 5     /* -sum m g . r */
#define SPH_DIAG_VMAX 6     /* max |v| */
#define SPH_DIAG_PROBE 7    /* probe integral J = sum over steps of dt * mean(p_w over probe) */
#define SPH_DIAG_STEPS 8    /* steps taken since sph_init (as a double) */
#define SPH_DIAG_LEN 16

/* Run description.  Passed by pointer, read only, except that
 * sph_configure fills the derived fields (cell .. n_cells). */
typedef struct sph_desc {
    int32_t dim;         /* 2 or 3; the last axis is vertical */
    int32_t precision;   /* SPH_F32 or SPH_F64 */
    int32_t penalty_all; /* 1: the penalty force of Eq. (13) acts on every fluid-wall pair;
                            0: on light-phase particles only (none in a single-phase run) */
    int32_t two_phase;   /* 1: fluid particles whose initial index is >= n_heavy form the
                            light phase (reference density rho0_light, same c0): reinitialised
                            by Eq. (18), density from the number density after the drift
                            instead of Eq. (9), Eq. (12) divided by rho_f term by term, wall
                            dummies take the interacting particle's phase (Secs. 2.1-2.6) */
    double dx;           /* initial particle spacing (enters m = rho0 dx^d and Eq. (15)) */
    double h;            /* smoothing length; kernel support 2h (Sec. 4: h = 1.3 dx) */
    double rho0;         /* reference density, Eq. (3) */
    double c0;           /* artificial sound speed, Eq. (3) */
    double mu;           /* dynamic viscosity (0: inviscid) */
    double gamma_p;      /* penalty strength, Eq. (13) (paper: 1) */
    double dt;           /* time step */
    double g[3];         /* body force */
    double a_wall[3];    /* wall acceleration in Eq. (12) */
    double lo[3];        /* lower corner of the cell grid */
    double hi[3];        /* upper corner of the cell grid */
    int64_t n_heavy;     /* two-phase: number of heavy-phase particles (initial indices first) */
    double rho0_light;   /* two-phase: reference density of the light phase */
    double motion_amp[3]; /* prescribed rigid translation of every wall dummy (the tank),   */
    double motion_freq;   /* X(t) = motion_amp sin(2 pi motion_freq t) at t = nstep dt      */
                          /* (Sec. 4.4); 0 = fixed walls.  See "Moving tank" below.        */
    int32_t cross_phase;  /* two phases, momentum of a light particle with a heavy neighbour:
                             0 = p* of Eq. (8) with each side's own state; 1 = the light
                             phase sees the heavy particle as a moving wall dummy (Secs. 2.1,
                             2.5): p* of Eq. (11) with p_w = p_j, density rho0_light +
                             p_w/c0^2, mass rho0_light dx^d; 2 = the same with p_w the
                             pressure extrapolated to the heavy particle from its light
                             neighbours by Eq. (12) divided by rho_f, with the tank's
                             acceleration (computed at the start of sph_forces(MOMENTUM)). */
    int32_t reserved1;
    /* derived by sph_configure: */
    double cell;         /* cell edge L_c = 2h, rounded to T */
    double sigma0;       /* reference number density of Eq. (17): full lattice sum */
    int32_t grid[3];     /* cells per axis (grid[2] = 1 in 2-D) */
    int32_t reserved2;
    int64_t n_cells;     /* grid[0] * grid[1] * grid[2] */
} sph_desc;

/* Device buffers (all caller-owned).  The double-buffered fluid fields have
 * two copies [0] and [1]; sel_vel / sel_rho name the copy that holds the
 * current v and rho - rho0 and are updated by the calls that swap them. */
typedef struct sph_buffers {
    /* at most 2^28 - 1 each in FP32, 2^27 - 1 in FP64 (every record array
       stays below 4 GiB); larger counts get SPH_ERR_ARG */
    int64_t n_fluid;
    int64_t n_wall;
    /* fluid, length n_fluid unless stated */
    int32_t *key[2];  /* linear cell key; [0] = sorted state, [1] = drifted, unsorted */
    int32_t *pid[2];  /* particle id (index in the initial arrays) */
    void *off[2];     /* T[dim][n_fluid] in-cell offsets */
    void *vel[2];     /* T[dim][n_fluid] velocity */
    void *rho[2];     /* T[n_fluid] density minus rho0 */
    void *acc;        /* T[dim][n_fluid] dv/dt of the last momentum sweep */
    int32_t sel_vel;  /* copy holding the current velocity (0 or 1) */
    int32_t sel_rho;  /* copy holding the current density (0 or 1) */
    /* walls, length n_wall, sorted by cell once by sph_init */
    int32_t *wkey;
    int32_t *wpid;    /* wall id (index in the initial wall array) */
    void *woff;       /* T[dim][n_wall] */
    void *pw;         /* T[n_wall] wall pressure, Eq. (12) */
    void *nrm;        /* T[dim][n_wall] wall normal estimate, Eq. (16) */
    /* cell tables, n_cells + 1 entries: particles of cell k are
       [start[k], start[k+1]) of the sorted arrays */
    int32_t *fstart;
    int32_t *wstart;
    void *scratch;         /* >= sph_scratch_bytes(...) bytes, 256-byte aligned */
    size_t scratch_bytes;
    uint32_t *status;      /* uint32_t[SPH_STATUS_LEN] */
    double *diag;          /* double[SPH_DIAG_LEN] */
    void *sigma_out;       /* optional T[n_fluid]: sph_density writes sigma_i (sorted order) */
    const int32_t *probe;  /* optional: wall ids of the probe patch (device) */
    int32_t n_probe;
    /* 1 when the scratch holds sigma_i of the current sorted positions,
     * summed by the last momentum sweep (set by sph_forces(SPH_MOMENTUM),
     * cleared by sph_init, sph_build_cells and sph_density); sph_density
     * then reads it instead of summing again.  A caller that overwrites
     * positions, cell tables or masks must set it to 0. */
    int32_t sigma_ready;
    /* Optional neighbour masks (all three or none).  When given,
     * sph_build_cells fills them for the sorted state and every sweep reads
     * them instead of testing all stencil candidates (same pairs, same
     * order, same arithmetic).  For query q and stencil row r (the rows of
     * three x-adjacent cells around q's cell, r = (dz+1)*3 + (dy+1) in 3-D,
     * dy+1 in 2-D) the words mask[(2*r + w) * n_query + q], w = 0, 1, have
     * bit b set when candidate base_r + 64*w + b of the row's index range is
     * a neighbour.  count[q] is the number of neighbours, or -1 when a row
     * had more than 128 candidates (that query then walks the cells).  Words
     * of rows without candidates, and word 1 of rows of at most 64, are left
     * unwritten (never read). */
    uint64_t *nbr_ff;  /* fluid -> fluid, uint64[rows][2][n_fluid] */
    uint64_t *nbr_fw;  /* fluid -> wall, uint64[rows][2][n_fluid] */
    uint64_t *nbr_wf;  /* wall -> fluid, uint64[rows][2][n_wall] */
    int32_t *cnt_ff, *cnt_fw, *cnt_wf;
    /* Steps taken since sph_init (host side): set to 0 by sph_init and
     * advanced by sph_density, whose drift starts a step; the time of the
     * state is nstep * dt. */
    int64_t nstep;
} sph_buffers;

/* Validates the run description and fills its derived fields: L_c = 2h
 * (rounded to T), the grid covering [lo, hi], and sigma0, the number
 * density sum_j W of a full square/cubic lattice of spacing dx (the initial
 * reference value of Eq. (17)).  Host only.  SPH_ERR_CONFIG for dim not in
 * {2, 3}, unknown precision, h <= 0, dx <= 0, c0 <= 0, hi <= lo, more than
 * 2^31 - 2 cells, a negative or non-finite motion_freq or non-finite
 * motion_amp, or dt more than 1 % above min(0.25 h/(1.1 c0),
 * 0.25 sqrt(h/a)) (Eqs. (23)-(24) with the anticipated maximum velocity
 * c0/10; a = |g| + max |X''|; the slack lets c0 be varied at a fixed dt). */
int sph_configure(sph_desc *desc);

/* Bytes of scratch the calls need for n_fluid fluid and n_wall wall
 * particles (cell counts, sort keys and permutation, reduction partials,
 * the sigma handed from the momentum sweep to the next density update, and
 * packed copies of the sorted state that the sweeps gather from: offset
 * with density and velocity per fluid particle, offset with p_w and the
 * normal per wall particle, 4 T each).  Every call keeps the packed copies
 * equal to the state it leaves; a caller that overwrites state arrays
 * itself must call sph_build_cells (or sph_init) before the next
 * sph_wall_bc or sph_forces. */
size_t sph_scratch_bytes(const sph_desc *desc, int64_t n_fluid, int64_t n_wall);  /* 0 beyond the counts above */

/* Loads the initial state and prepares the run (Sec. 3: the data is copied
 * to the device once, at the start).
 *   fpos, fvel  device double[dim][n_fluid]  absolute positions, velocities
 *   frho        device double[n_fluid]       densities
 *   wpos        device double[dim][n_wall]   wall dummy positions
 * Positions and velocities are those of t = 0 in the fixed frame (a moving
 * tank subtracts X(0) and X'(0)); sets nstep = 0.
 * Converts positions to cell + offset, sorts walls by cell (once: they are
 * fixed, Sec. 2.3) and estimates their normals by Eq. (16), sorts the fluid
 * (sph_build_cells), computes the initial wall pressure (Eq. (12)) and
 * dv/dt (Eq. (10)), and zeroes status and diag.  Particles outside
 * [lo, hi] are clamped into the grid and counted in SPH_STATUS_OUT_OF_GRID.
 * Sets sel_vel and sel_rho. */
int sph_init(const sph_desc *desc, sph_buffers *buf, const double *fpos, const double *fvel,
             const double *frho, const double *wpos, void *stream);

/* Neighbour search with the sorting of particles by cell (Sec. 3, Table 1).
 * Counting sort of the drifted fluid (key[1], off[1], pid[1] and the
 * current velocity and density) by cell key into key[0], off[0], pid[0] and
 * the other velocity/density copy; particles of one cell are ordered by
 * their x offset, ties by their prior order.  Rebuilds fstart and, if
 * present, the neighbour masks.  Swaps sel_vel and sel_rho. */
int sph_build_cells(const sph_desc *desc, sph_buffers *buf, void *stream);

/* Density update (Sec. 2.5 and 2.6): at the current positions
 * sigma_i = sum_{j in fluid and walls} W_ij (j = i included), the
 * reinitialised density of Eq. (17) with rho* the current density, then
 * the half kick of Eq. (19) with the stored dv/dt and the drift of Eq. (20).
 * Writes the new density and the half-step velocity in place (current
 * copies) and the drifted positions to key[1], off[1], pid[1].  When
 * sigma_ready is set, sigma comes from the momentum sweep at these
 * positions (the same pairs summed in the same order, so the same bits).
 * A moving tank adds X'(t_n) - Vh to the kick; nstep advances by one. */
int sph_density(const sph_desc *desc, sph_buffers *buf, void *stream);

/* Wall dummy pressure by force balance with the fluid, Eq. (12), for every
 * wall particle from the current fluid positions and densities:
 * p_w = [sum_f p_f W_wf + (g - a_w) . sum_f rho_f r_wf W_wf] / sum_f W_wf,
 * 0 when no fluid particle is within 2h; a_w = a_wall + X''(nstep dt).  If a probe is set, adds
 * dt * mean(p_w over the probe) to diag[SPH_DIAG_PROBE]. */
int sph_wall_bc(const sph_desc *desc, sph_buffers *buf, void *stream);

/* Pair sweeps over fluid and wall neighbours.
 * SPH_CONTINUITY: drho_i/dt of Eq. (9) with the Riemann intermediate
 *   velocity of Eqs. (7)-(8) (walls: v = 0, p = p_w, rho from the EOS),
 *   then rho^{n+1} = rho + dt drho/dt (Eq. (21)) into the other density
 *   copy; swaps sel_rho.
 * SPH_MOMENTUM: dv_i/dt of Eq. (10) with p* of Eq. (8) (fluid) and
 *   Eq. (11) (walls), the viscous term, the penalty force of Eqs. (13)-(15)
 *   if penalty_all, and g; stores it in acc and, unless SPH_NO_KICK, the
 *   velocity of Eq. (22) into the other velocity copy (a moving tank adds
 *   Vh - X'(t_{n+1}), n + 1 = nstep); swaps sel_vel.
 *   The same sweep sums sigma_i of Eq. (4) for the next density update
 *   into the scratch and sets sigma_ready.
 * Exactly one of the two may be given per call. */
int sph_forces(const sph_desc *desc, sph_buffers *buf, unsigned which, void *stream);

/* nsteps full time steps (the schedule at the top of this file). */
int sph_step(const sph_desc *desc, sph_buffers *buf, int nsteps, void *stream);

/* FP64 global reductions into diag (mass, momentum, energies, max |v|;
 * deterministic order; fixed-frame positions and velocities at nstep dt).  Non-finite values are counted in
 * SPH_STATUS_NONFINITE.  The probe entry and the step count are kept. */
int sph_diag(const sph_desc *desc, sph_buffers *buf, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): sph_diag
 * without its scratch argument.  Computes exactly what sph_diag computes,
 * with the same kernels and the same summation order (bit-identical
 * results); b->scratch and b->scratch_bytes are not read, every other
 * buffer is as for sph_diag.  The per-block partial sums live in a device
 * array of SPH_DIAG_NOALLOC_BYTES that the library holds on each GPU it
 * runs on until the process ends; the call allocates and frees nothing.
 * Every call on one GPU uses that GPU's single array: calls that overlap
 * on one GPU (different streams or host threads) race and must be
 * serialised by the caller.  The partials are written in full by each call
 * before they are read, so nothing needs clearing between calls.
 * Returns SPH_ERR_CAPACITY when n_fluid > SPH_DIAG_NOALLOC_MAX_FLUID, and
 * SPH_ERR_LAUNCH if the workspace's device address cannot be obtained. */
#define SPH_DIAG_NOALLOC_BYTES (4u << 20)          /* 4 MiB per GPU */
#define SPH_DIAG_NOALLOC_MAX_FLUID ((int64_t)1 << 24) /* 65,536 blocks x 256 particles x 8 doubles */
int sph_diag_noalloc(const sph_desc *desc, sph_buffers *buf, void *stream);

/* Copies the fluid state out in particle-id order as doubles (device
 * arrays, any may be NULL): pos double[dim][n_fluid] absolute positions,
 * vel double[dim][n_fluid], rho double[n_fluid] (full density),
 * acc double[dim][n_fluid]; positions and velocities in the fixed frame at
 * t = nstep dt (between steps). */
int sph_export(const sph_desc *desc, const sph_buffers *buf, double *pos, double *vel,
               double *rho, double *acc, void *stream);

/* Copies wall pressure (double[n_wall]), normals (double[dim][n_wall]) and
 * absolute positions (double[dim][n_wall], fixed frame at t = nstep dt) out
 * in wall-id order (device arrays, any may be NULL). */
int sph_export_walls(const sph_desc *desc, const sph_buffers *buf, double *pw, double *nrm,
                     double *pos, void *stream);

/* Neighbour sets as the sweeps enumerate them (pairs with |r_ij|^2 < 4h^2
 * computed from cell + offset in T).  which = 0: for every fluid particle
 * its fluid and wall neighbours, itself included; which = 1: for every wall
 * particle its fluid neighbours.  count (device int32[n_query], indexed by
 * particle/wall id) is always written; if list is not NULL, neighbour ids
 * are written at list[offset[id] ...] (device, offset int64[n_query], the
 * exclusive prefix sum of count) with walls encoded as n_fluid + wall id;
 * entries that would fall outside [0, list_len) are dropped. */
int sph_neighbours(const sph_desc *desc, const sph_buffers *buf, int which, const int64_t *offset,
                   int32_t *count, int32_t *list, int64_t list_len, void *stream);

/* ------------------------------------------------------------------ */
/* Adjoint: reverse-mode derivatives of a probe functional               */
/*   J = sum over steps of dt * mean(p_w over the probe walls)           */
/* with respect to theta = (mu, gamma_p, c0, H), H the initial column    */
/* height (the fluid is stretched vertically, masses unchanged, with the  */
/* hydrostatic initial density).  The backward follows the forward step  */
/* in reverse: momentum and second kick, continuity and density update,  */
/* wall pressure, drift, half kick, reinitialisation, number density.    */
/* Cell keys, sorted order and neighbour sets are taken from the forward */
/* frames (recomputed bit for bit, not differentiated); branches (the    */
/* limiter, max() of Eq. (17), delta < 1) take the forward's side, with  */
/* derivative 0 at max(x, 0)'s kink.  The adjoint runs in FP64.          */
/* It covers the single-phase step, in a fixed or a moving tank (the     */
/* prescribed motion does not depend on theta: its velocity kicks pass   */
/* through, and Eq. (12) takes g - a_w - X'' at each frame's own time);  */
/* every backward call returns SPH_ERR_CONFIG when desc->two_phase is    */
/* set.                                                                  */
/* ------------------------------------------------------------------ */

#define SPH_THETA_MU 0
#define SPH_THETA_GAMMA 1
#define SPH_THETA_C0 2
#define SPH_THETA_H 3
#define SPH_NTHETA 4

/* What the backward of a step needs from the forward, for the state at
 * r^n (device arrays in that state's sorted order, T as in sph_buffers).
 * Frame n+1 carries the quantities step n computed at r^{n+1}. */
typedef struct sph_frame {
    const int32_t *key, *pid; /* sorted state at r^n */
    const void *off;          /* T[dim][n_fluid] */
    const int32_t *fstart;    /* cell table of this state (n_cells + 1) */
    const void *rho;          /* T[n_fluid] rho^n - rho0 */
    const void *sigma;        /* T[n_fluid] sigma at r^n (from step n's density update) */
    const void *vh;           /* T[dim][n_fluid] velocity of the drift into r^n (frame 0: v^0) */
    const void *rt;           /* T[n_fluid] reinitialised density of step n-1, minus rho0 */
    const void *pw;           /* T[n_wall] wall pressure at r^n (frame 0: the initial one) */
    /* optional neighbour masks and counts of this state (see sph_buffers);
     * when all are given the backward sweeps visit them instead of walking */
    const uint64_t *nbr_ff, *nbr_fw, *nbr_wf;
    const int32_t *cnt_ff, *cnt_fw, *cnt_wf;
    /* step count of this state (time nstep * dt): set by sph_step_frame
     * for the state it records; the caller sets it for frame 0 */
    int64_t nstep;
} sph_frame;

/* Adjoint state (device, FP64, particle-id order) and workspace. */
typedef struct sph_adjoint {
    double *xb;    /* [dim][n_fluid] dJ/dr */
    double *vb;    /* [dim][n_fluid] dJ/dv */
    double *rhob;  /* [n_fluid]      dJ/drho */
    double *ab;    /* [dim][n_fluid] dJ/d(dv/dt) carried by the half kick */
    double *theta; /* [SPH_NTHETA] accumulated dJ/dtheta */
    void *work;    /* >= sph_adjoint_work_bytes(...), 256-byte aligned */
    size_t work_bytes;
} sph_adjoint;

size_t sph_adjoint_work_bytes(const sph_desc *desc, int64_t n_fluid, int64_t n_wall);  /* 0 beyond the limits */

/* One forward step (exactly sph_step with nsteps = 1) that also records
 * the frames the backward needs: sigma at r^n into sigma_cur (T[n_fluid],
 * the current sorted order) and the state at r^{n+1} into the arrays of
 * next (written through its pointers, which must be distinct device
 * buffers of the sizes stated in sph_frame; the mask fields are copied only
 * when buf has masks and next provides them), and next->nstep. */
int sph_step_frame(const sph_desc *desc, sph_buffers *buf, void *sigma_cur, sph_frame *next,
                   void *stream);

/* Zeroes the adjoint state and theta. */
int sph_adjoint_zero(const sph_desc *desc, const sph_buffers *buf, sph_adjoint *adj, void *stream);

/* Backward of the momentum sweep with the second kick (Eqs. (10)-(11),
 * (13)-(15), (22)) and of the continuity sweep with the density update
 * (Eqs. (9), (21)) of step n, at the state of frame next = n+1.  Consumes
 * the adjoint of (v^{n+1}, rho^{n+1}, dv/dt^{n+1}); leaves the adjoints of
 * the half-step velocity and the reinitialised density in the workspace and
 * adds to dJ/dr^{n+1}, dJ/dmu, dJ/dgamma_p, dJ/dc0.  buf supplies the walls
 * (sorted once), the probe and nothing else. */
int sph_forces_bwd(const sph_desc *desc, const sph_buffers *buf, const sph_frame *next,
                   sph_adjoint *adj, void *stream);

/* Backward of the wall pressure, Eq. (12), of step n at frame next,
 * including the probe functional's own dt * mean(p_w) term. */
int sph_wall_bc_bwd(const sph_desc *desc, const sph_buffers *buf, const sph_frame *next,
                    sph_adjoint *adj, void *stream);

/* Backward of the drift, the half kick and the reinitialisation of Eq. (17)
 * with the number density sweep of step n, at frame cur = n (positions
 * r^n).  Leaves the adjoint of the state at step n in adj. */
int sph_density_bwd(const sph_desc *desc, const sph_buffers *buf, const sph_frame *cur,
                    sph_adjoint *adj, void *stream);

/* One full step backward: sph_forces_bwd and sph_wall_bc_bwd at next,
 * then sph_density_bwd at cur. */
int sph_step_bwd(const sph_desc *desc, const sph_buffers *buf, const sph_frame *cur,
                 const sph_frame *next, sph_adjoint *adj, void *stream);

/* Backward of sph_init's initial wall pressure and dv/dt at frame 0, then
 * of the initial state itself: adds dJ/dH (vertical stretch of the fluid
 * column of height H above the floor z = 0, hydrostatic initial density)
 * and the initial density's share of dJ/dc0. */
int sph_init_bwd(const sph_desc *desc, const sph_buffers *buf, const sph_frame *f0, double H,
                 sph_adjoint *adj, void *stream);

/* Static text for a return code. */
const char *sph_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
