/*
 * pflb.h -- C ABI of the phase-field lattice Boltzmann library (AMD gfx950, HIP).
 *
 * The library advances the two distribution sets of the conservative Allen-Cahn
 * phase-field lattice Boltzmann method of Otomo, Zhang and Chen ("Improved
 * phase-field-based lattice Boltzmann models with a filtered collision operator"):
 * the order-parameter set h_i (Eq. 1-4) and the hydrodynamic set g_i with the
 * filtered single-relaxation-time collision (Eqs. 5-12) and the high-order
 * equilibrium correction (Eq. 13), on D2Q9 or D3Q19, with central differences for
 * grad(phi) and lap(phi) (Section 2).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer unless its comment says "host".
 *     The caller owns all device memory; the library only borrows pointers.
 *   - Fields are float32, structure of arrays, site index s = (z*ny + y)*nx + x
 *     (D2Q9: s = y*nx + x).  A vector field is [D][N] (D = 2 or 3, N = nx*ny*nz).
 *     A distribution set in "pre-collision form" is [Q][N]: h_i(x) at step n, after
 *     streaming and before collision, velocity ordering:
 *       D2Q9 : 0 rest, then (+x,-x), (+y,-y), (+x+y,-x-y), (+x-y,-x+y)
 *       D3Q19: 0 rest, then (+x,-x), (+y,-y), (+z,-z), (+x+y,-x-y), (+x-y,-x+y),
 *              (+x+z,-x-z), (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z)
 *     so that the opposite of i >= 1 is i+1 (i odd) or i-1 (i even).  T = 1/3.
 *   - Functions return 0 (PFLB_OK) or a negative PFLB_ERR_* code; no exception
 *     crosses the ABI.  pflb_last_error() describes the last failure of a context.
 *     Asynchronous device faults surface at the next synchronous call as
 *     PFLB_ERR_DEVICE.
 *   - Work is enqueued on the given HIP stream (hipStream_t passed as void*; NULL is
 *     the null stream).  Calls that return host values synchronise that stream.
 *   - Calls on one context must not overlap (a context is not thread-safe).
 */
#ifndef PFLB_H
#define PFLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PFLB_OK             0
#define PFLB_ERR_PARAM     -1  /* invalid parameter or argument                     */
#define PFLB_ERR_ALIGN     -2  /* device pointer not 256-byte aligned               */
#define PFLB_ERR_UNBOUND   -3  /* buffers not bound yet                             */
#define PFLB_ERR_DEVICE    -4  /* a HIP call or kernel launch failed                */
#define PFLB_ERR_NONFINITE -5  /* a non-finite population was found                 */
#define PFLB_ERR_IO        -6  /* checkpoint file could not be read or written      */
#define PFLB_ERR_NOMEM     -7  /* host allocation failed                            */

/* ---- enumerations ---- */
#define PFLB_BC_PERIODIC 0
#define PFLB_BC_WALL     1     /* no-slip wall half a site outside the last layer   */

#define PFLB_STORE_FP32  0     /* populations stored as float32                     */
#define PFLB_STORE_FP16S 1     /* rest populations float32; every moving population */
                               /* an fp16 deviation from the first-order equilibrium */
                               /* of its reading site's previous moments (FP32      */
                               /* arithmetic throughout)                             */
#define PFLB_STORE_FP32_INPLACE 2  /* float32 in one state buffer, streamed in place */
                               /* (half the footprint of PFLB_STORE_FP32; not in the */
                               /* paper): each step reads and writes the same slots  */
                               /* of a site, alternating two layouts, after a pass   */
                               /* that writes the phi field into the scratch buffer */

/* buffer ids for pflb_required_bytes / pflb_bind.  A state buffer holds both
 * distribution sets (FP32: float2 (h_i, g_i) per slot, [Q][S]; FP16S: per site the
 * float2 rest pair (h_0, g_0) and a 16-byte word of its pre-collision moments in fp16
 * (sum h, sum g, sum c h, sum c g), then a half2 deviation pair (h_i, g_i) per moving
 * population, [Q-1][S], decoded as w_i (sum h + 3 c_i . sum c h) + dev_h / 2^scale_h
 * and likewise for g, with the moments of the site that reads the slot); the step
 * reads one state buffer and writes the other.  The FP16S moments and deviations must
 * stay within the fp16 range (|sum g|, |sum c g| < 65504; |dev| 2^scale < 65504).
 * PFLB_STORE_FP32_INPLACE uses PFLB_BUF_STATE0 only (Q float arrays of h, then Q of g,
 * [2Q][S]; after an even number of steps since the state was set f_i(x) is in slot
 * (x, i), after an odd number in slot (x - c_i, opp(i)), or in slot (x, i) where x - c_i
 * lies beyond a wall); its PFLB_BUF_STATE1 needs 0 bytes and may be NULL, and its
 * scratch buffer also holds the phi field (N floats). */
#define PFLB_BUF_STATE0  0
#define PFLB_BUF_STATE1  1
#define PFLB_BUF_SCRATCH 2     /* reduction partial sums and flags                  */
#define PFLB_NBUF        3

/*
 * Model and domain parameters (Section 2; Section 4 gives values per case).
 *   lattice      9 (D2Q9) or 19 (D3Q19)
 *   nx, ny, nz   sites per axis (nz = 1 for D2Q9), each >= 1, at most 2^32 - 64 sites
 *   bc[3]        boundary per axis x, y, z: PFLB_BC_PERIODIC or PFLB_BC_WALL (both
 *                faces of an axis alike; walls: halfway bounce-back for h and g,
 *                phi outside a wall equals phi at the adjacent site)
 *   rho_L,rho_H  densities of the light (phi = 0) and heavy (phi = 1) phase, > 0
 *   nu_L, nu_H   kinematic viscosities; tau = nu/T + 1/2 must exceed 1/2
 *   M            mobility (> 0); tau_phi = M/T + 1/2 (Eq. 1)
 *   W            interface thickness (> 0) (Eqs. 4, 8)
 *   sigma        surface tension (>= 0) (Eq. 8)
 *   g[3]         gravitational acceleration; the external force is rho(phi) g
 *   eps          the small constant of the interface normal (text after Eq. 4)
 *   hoc          1: high-order equilibrium correction and modified velocity (Eq. 13)
 *   dtheta_C     C of the dense-bubble correction (Eq. 14, with F = -1 where |phi - 1/2|
 *                > 0.35 and (phi - 1/2) lap(phi) > 0, else 0); 0 switches it off, 10
 *                diffuses dense bubbles away
 *   storage      PFLB_STORE_FP32, PFLB_STORE_FP16S or PFLB_STORE_FP32_INPLACE (the
 *                last without open faces; its contexts are stepped one
 *                by one by pflb_step_many and not taken by the batched read-out and
 *                hand-over of the surrogate's guard)
 *   scale_log2   power-of-two scale exponents of the fp16 deviations of h and g
 *                (FP16S only; each in [-14, 24])
 *   wall_u       velocity of each wall face, rows x-, x+, y-, y+, z-, z+ and columns
 *                (u_x, u_y, u_z) in the axes above (D2Q9: rows 0-3, columns 0-1; the rest
 *                must be 0).  Tangential only (the normal component must be 0) and 0 on
 *                faces of periodic axes; all zeros (e.g. a zero-initialised struct) is a
 *                resting box.  Not in the paper: the momentum correction of halfway
 *                bounce-back for a moving wall (Ladd's method) -- a population sent into
 *                a wall face returns reduced by 2 w_i (c_i . u_w)/T times the sending
 *                site's phi (h) or rho (g); one crossing two or three faces at an edge or
 *                corner takes the mean of their velocities.
 *   wet_cos      cos of the contact angle of each wall face (measured through the
 *                heavy phase), rows as wall_u; each in [-1, 1], 0 on faces of periodic
 *                axes (D2Q9: entries 4, 5 must be 0).  All zeros (90 degrees) is the
 *                mirror ghost above.  Not in the paper, which has no contact angles: the
 *                geometric wetting condition n_w . grad(phi) = -(4/W) cos(theta) phi (1 -
 *                phi) across the half-way wall, i.e. the ghost beyond the face takes
 *                phi_m + (4/W) cos(theta) phi_m (1 - phi_m), phi_m the adjacent site's
 *                phi; a ghost beyond two or three faces adds their terms.
 *   open, open_P a pressure condition on a wall face (Section 4's dam-break top; the
 *                paper does not say how it is imposed): open[f] = 1 makes face f open,
 *                with pressure open_P[f], rows as wall_u (D2Q9: rows 0-3).  An open face
 *                lies on a wall axis of at least 2 sites and has no contact angle, and no
 *                face of the box may move while one is open.  The sites beyond an open
 *                face are copies of the boundary-layer sites they face (zero normal
 *                gradient of phi and u): a population entering a boundary-layer site x
 *                through the face comes from s' = x - c_i with its out-of-range
 *                coordinates put back into the layer, as s' sent it in direction i, plus
 *                2 w_i (P_f - P(s'))/T for g (the filtered collision depends on P only
 *                through w_i P / T); one that crosses several open faces takes the mean
 *                of their P_f, one that also crosses a closed face bounces back.
 *                Populations leaving through the face are lost (outflow), so sum(phi)
 *                changes by the net flux.  A context with an open face is stepped alone
 *                (pflb_step_many does not batch it) and its state buffers also hold the
 *                boundary layers' pressures (pflb_required_bytes includes them).  All
 *                zeros: no open face.
 */
typedef struct pflb_params {
    int lattice;
    int nx, ny, nz;
    int bc[3];
    double rho_L, rho_H;
    double nu_L, nu_H;
    double M, W, sigma;
    double g[3];
    double eps;
    int hoc;
    double dtheta_C;
    int storage;
    int scale_log2[2];
    double wall_u[6][3];
    double wet_cos[6];
    int open[6];
    double open_P[6];
} pflb_params;

typedef struct pflb_ctx pflb_ctx;

/* Validate p and create a context on the current HIP device.  On failure returns
 * PFLB_ERR_PARAM and sets *out = NULL.  The library owns the context. */
int pflb_create(const pflb_params* p, pflb_ctx** out);

/* Destroy a context (NULL is ignored).  Device memory stays the caller's. */
void pflb_destroy(pflb_ctx* ctx);

/* Text of the last error on ctx (static string for ctx == NULL). */
const char* pflb_last_error(const pflb_ctx* ctx);

/* Bytes the caller must allocate for buffer `buffer` (PFLB_BUF_*) with parameters
 * p, or 0 if p is invalid. */
size_t pflb_required_bytes(const pflb_params* p, int buffer);

/* Bind the PFLB_NBUF caller-allocated device buffers, in PFLB_BUF_* order, each at
 * least pflb_required_bytes() long and 256-byte aligned (a buffer that needs 0 bytes
 * may be NULL).  The pointers are borrowed until pflb_destroy or the next pflb_bind. */
int pflb_bind(pflb_ctx* ctx, void* const* dev_ptrs, int n);

/* Pre-collision equilibrium distributions from macroscopic fields (the paper does
 * not state its start; this evaluates Eqs. 2-4 and 6-7 plus Eq. 13 at every site with
 * u := u0 and P := P0, so that the state reads back u0 and P0).
 *   phi [N], u [D][N], P [N] (NULL: zero) -> h_out [Q][N], g_out [Q][N]. */
int pflb_equilibrium(pflb_ctx* ctx, const float* phi, const float* u, const float* P,
                     float* h_out, float* g_out, void* stream);

/* Load a pre-collision state h [Q][N], g [Q][N] as the state at step 0. */
int pflb_set_state(pflb_ctx* ctx, const float* h, const float* g, void* stream);

/* Write the current pre-collision state to h [Q][N], g [Q][N]. */
int pflb_get_state(pflb_ctx* ctx, float* h, float* g, void* stream);

/* Start from macroscopic fields: pflb_equilibrium into `work` (2*Q*N floats of
 * caller device memory) followed by pflb_set_state.  With PFLB_STORE_FP32_INPLACE the
 * equilibria are written straight into the state and `work` is not used (may be NULL). */
int pflb_init_fields(pflb_ctx* ctx, const float* phi, const float* u, const float* P,
                     float* work, void* stream);

/* Allocation-free start, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as pflb_init_fields, bit for bit, with the 2*Q*N floats it stages between its
 * two kernels held in a fixed device array of the library instead of a work buffer.
 *   Limit: 2*Q*N*4 <= PFLB_NOALLOC_SCRATCH_BYTES (64 MiB: N <= 441,505 D3Q19 sites,
 *   932,067 D2Q9 sites); larger domains return PFLB_ERR_PARAM and change nothing.
 *   Contexts with PFLB_STORE_FP32_INPLACE stage nothing and have no such limit.
 *   The call allocates nothing (no hipMalloc, no library allocation).  The array is
 *   one per GPU, held from its first use on that GPU until the process ends, and
 *   shared by every call on that GPU: calls on one GPU that overlap in time (other
 *   threads, other streams not ordered with this one) race on it and must not be
 *   issued.  Asynchronous on stream, like pflb_init_fields. */
#define PFLB_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int pflb_init_fields_noalloc(pflb_ctx* ctx, const float* phi, const float* u, const float* P,
                             void* stream);

/* PFLB_NOALLOC_SCRATCH_BYTES, as compiled into the library. */
size_t pflb_noalloc_scratch_bytes(void);

/* Replace the state by the equilibria of given macroscopic fields (a hand-over from
 * another model of the same flow, e.g. a learned surrogate): u = J / rho' with rho' the
 * density read-out divides by, then the equilibria of pflb_equilibrium and the state
 * load of pflb_init_fields.  Reading back returns phi, P and J up to FP32 rounding.
 *   phi [N], P [N] (NULL: zero), J [D][N]; work: 2*Q*N floats of device memory (the
 *   (2*Q + D)*N floats earlier versions asked for remain enough).
 * The step counter is kept and increased by `advance` (>= 0), the number of steps the
 * given fields lie ahead of the current state. */
int pflb_reconstruct(pflb_ctx* ctx, const float* phi, const float* P, const float* J,
                     float* work, int advance, void* stream);

/* Enqueue nsteps fused stream-and-collide steps of both sets (Eqs. 1 and 10 with
 * the central differences of Section 2).  Returns launch errors only.
 * The launch shape is chosen when the context is created (by pflb_step_many for each
 * call); two environment variables read then override it for tuning (the results do
 * not depend on them):
 * PFLB_BZ (planes per workgroup along z) and PFLB_TILE (D3Q19 tile: 0 64x4, the
 * default; 1 64x8; 2 32x8; 3 32x4). */
int pflb_step(pflb_ctx* ctx, int nsteps, void* stream);

/* The same nsteps steps as pflb_step, enqueued as one HIP graph: the first call for a
 * given nsteps and current state buffer captures the launches pflb_step would issue
 * and instantiates them; later calls with the same nsteps replay that graph (one launch
 * instead of nsteps).  Results are bitwise those of pflb_step.  `stream` must not be
 * the null stream (stream capture needs a created stream).  The graphs are kept until
 * a call with another nsteps, pflb_bind or pflb_destroy.  A device-side way to cut the
 * launch overhead of small, launch-bound domains (Section 4's two-dimensional cases). */
int pflb_step_graph(pflb_ctx* ctx, int nsteps, void* stream);

/* The same steps for n contexts at once (an ensemble of small domains fills the GPU
 * where one alone is launch-bound): each step is one launch per 16 contexts; a context
 * with a moving wall is stepped on its own, as by pflb_step.  The contexts must be
 * distinct, bound and share lattice, storage, sizes and walls; their physical parameters
 * and wall velocities may differ.  Each context ends exactly as
 * pflb_step(ctx[k], nsteps) would leave it, bit for bit.  Asynchronous on stream;
 * errors (PFLB_ERR_PARAM, PFLB_ERR_UNBOUND, PFLB_ERR_DEVICE) are reported on ctx[0]. */
int pflb_step_many(pflb_ctx* const* ctx, int n, int nsteps, void* stream);

/* Macroscopic fields of the current state (end of Section 2):
 *   phi [N]   = sum_i h_i                           (required; also used as input
 *                                                    of the second pass)
 *   P   [N]   = T sum_i g_i + (T rho_dif/2) u.grad(phi)          (NULL: skip)
 *   J   [D][N]= sum_i c_i g_i + (mu grad(phi) + F_ex)/2 (= rho u)  (NULL: skip)
 *   u   [D][N]= J / (rho + lap(rho)/4) (J/rho with hoc = 0)        (NULL: skip) */
int pflb_read(pflb_ctx* ctx, float* phi, float* P, float* J, float* u, void* stream);

/* sum_x phi(x) accumulated in float64 in a fixed order (bitwise reproducible), and
 * *nonfinite = 1 if any population of either set is NaN or Inf.  Synchronous.
 * Returns PFLB_ERR_NONFINITE when *nonfinite is set. */
int pflb_mass(pflb_ctx* ctx, double* sum_phi, int* nonfinite, void* stream);

/* Steps completed since the last pflb_set_state / pflb_init_fields / pflb_load. */
long long pflb_step_count(const pflb_ctx* ctx);

/* Checkpoint the raw state (both sets, storage format, step count, parameters) to a
 * host file / restore it into a context created with identical parameters.
 * Synchronous.  Resuming is bitwise identical to not stopping. */
int pflb_save(pflb_ctx* ctx, const char* path, void* stream);
int pflb_load(pflb_ctx* ctx, const char* path, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PFLB_H */
