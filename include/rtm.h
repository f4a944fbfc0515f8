/*
 * rtm.h -- C ABI of librtm.so: the per-time-step phases of an acoustic reverse-time-migration
 * propagator on one MI355X (gfx950).
 *
 * The paper (section II, "Structure of the Application") describes a PDE solver that applies a
 * high-order stencil to a 3-D block of pressure data every time step, and splits each step into
 * phases: stencil on the halo region, pack of the halo points into messages, non-blocking
 * exchange, stencil on the rest of the block while the messages are in flight, wait, unpack.  The
 * calls below are those phases for one subdomain, plus the source injection, receiver recording
 * and zero-lag imaging that reverse time migration wraps around them.  The halo-first step comes in
 * two forms: the halo region and the rest (rtm_step_halo or rtm_step_halo_pack[_slots], then
 * rtm_step_interior), and the shell form (rtm_step_shell_pack, which computes the cells within R of
 * a face into the face buffer only, then rtm_step_whole_slots over every owned cell); both give the
 * same bits as the one-launch rtm_step_whole.
 *
 * Scheme (3-D isotropic acoustic wave equation, radius-R star stencil, second-order leapfrog,
 * Cerjan sponge on both time levels):
 *
 *     L u     = sum over x, y, z of [ c0 u + sum_{m=1..R} c_m (u(+m) + u(-m)) ]        (dimensionless)
 *     u^{n+1} = g (2 u^n - g u^{n-1} + kappa L u^n),    kappa = (v dt / h)^2,  g = gx[i] gy[j] gz[k].
 *
 * Geometry.  Every field (wavefield time levels, kappa, snapshots, image) is FP32 in the same padded
 * layout: owned cell (i, j, k), 0 <= i < nx etc., lives at element
 *     (k + R) * pitch_z + (j + R) * pitch_y + (i + R)
 * of the base pointer, where R = radius is also the ghost width.  Ghost cells hold what the last
 * rtm_unpack_halo wrote (zero for a physical boundary).  pitch_y >= nx + 2R and
 * pitch_z >= pitch_y * (ny + 2R).  A base pointer that is 16-byte aligned with pitch_y and pitch_z
 * multiples of 4 selects the vectorised kernels; other layouts are accepted and take a scalar path.
 *
 * Ownership and ordering.  All field, index and weight arguments are DEVICE pointers owned by the
 * caller; the library never allocates, frees, copies to the host or synchronises, except
 * rtm_tune_step, which times its settings and waits for them.  Each compute call only enqueues work
 * on `stream` (NULL = the null stream) and returns at once; ordering across streams is the caller's.  The library keeps no pointer after a call returns.  Calls are
 * thread-safe and re-entrant.
 *
 * Errors.  Every call returns RTM_OK or a negative status and enqueues nothing on error.  No C++
 * exception crosses this boundary.
 */
#ifndef RTM_H
#define RTM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTM_ABI_VERSION 1

enum {
    RTM_OK = 0,
    RTM_EINVAL = -1,   /* null pointer, dimension < 2R, radius not 2 or 4, pitch too small, n < 0 */
    RTM_EALIAS = -2,   /* an output overlaps an input it must not overlap (e.g. u_nxt == u_cur) */
    RTM_ELAUNCH = -3,  /* the HIP runtime reported an error when the kernel was launched */
    RTM_EDEVICE = -4,  /* no HIP device, or the current device is not gfx950 */
};

typedef struct rtm_grid {
    int32_t nx, ny, nz;        /* owned cells per axis, each >= 2 * radius */
    int32_t radius;            /* stencil radius R: 4 (8th order) or 2 (4th order); ghost width = R */
    int64_t pitch_y;           /* elements between consecutive y rows, >= nx + 2R */
    int64_t pitch_z;           /* elements between consecutive z planes, >= pitch_y * (ny + 2R) */
    float c[5];                /* c0..cR, second-derivative weights on unit spacing (1/h^2 lives in kappa) */
    const float *gx, *gy, *gz; /* device sponge profiles of length nx, ny, nz (all ones = no sponge) */
} rtm_grid;

/* ---- host-only helpers (no device work) ---------------------------------------------------- */

/* Fill grid->c with the centred Taylor weights of the second derivative for `radius` (Fornberg
 * 1988; R = 4: -205/72, 8/5, -1/5, 8/315, -1/560; R = 2: -5/2, 4/3, -1/12), zero the rest, and set
 * the other fields.  Returns RTM_EINVAL for a bad radius, dims or pitches. */
int rtm_grid_init(rtm_grid *grid, int32_t nx, int32_t ny, int32_t nz, int32_t radius,
                  int64_t pitch_y, int64_t pitch_z, const float *gx, const float *gy, const float *gz);

/* Largest Courant number v dt / h for which this leapfrog scheme is stable in 3-D:
 * 2 / sqrt(3 S) with S = |c0| + 2 sum |c_m| (the checkerboard mode).  0 for a bad radius. */
double rtm_stability_limit(int32_t radius);

/* Time step at `fraction` of the stability limit: *dt = fraction * rtm_stability_limit(radius) * h / vmax
 * (the workloads run at half the limit, fraction = 0.5; a Courant number of 0.5 taken literally would
 * exceed the limit of the radius-4 scheme), computed in FP64 into the host double *dt.  RTM_EINVAL for a bad radius, h <= 0, vmax <= 0, fraction <= 0 or a NULL dt. */
int rtm_stable_dt(int32_t radius, double h, double vmax, double fraction, double *dt);

/* Point-source weights into host memory `out[n]`: out[s] = (v[s] dt)^2 / h^3 in FP64, rounded to
 * FP32.  A source term f(t) delta(x - x_s) of (1/v^2) p_tt - lap p = f delta discretises, after the
 * leapfrog update multiplies the right-hand side by (v dt)^2, to adding (v_s dt)^2 f(t_n) / h^3 at
 * the source cell (the grid delta is 1/h^3).  v: host velocities at the source cells (m/s).
 * RTM_EINVAL for n < 0, h <= 0, dt <= 0 or a NULL pointer with n > 0. */
int rtm_injection_weights(int32_t n, const double *v, double dt, double h, float *out);

/* Cerjan taper along one axis into host memory `out[n]`: exp(-(alpha d)^2), with d = the number
 * of cells into a `width`-cell sponge at either end (d = max(0, width - i, i - (n - 1 - width))). */
int rtm_sponge_profile(int32_t n, int32_t width, double alpha, float *out);

/* Ricker wavelet samples into host memory `out[nsteps]`: f(t_n), t_n = n dt,
 * f(t) = (1 - 2 (pi fp tau)^2) exp(-(pi fp tau)^2), tau = t - t0. */
int rtm_ricker(int32_t nsteps, double dt, double fpeak, double t0, float *out);

/* Offsets (in elements) of the six face slots -X, +X, -Y, +Y, -Z, +Z inside one contiguous face
 * buffer; offsets[6] is the total size.  Slot sizes are R*ny*nz, R*ny*nz, nx*R*nz, nx*R*nz,
 * nx*ny*R, nx*ny*R.  Inside a slot the face's R-thick sub-block is stored x fastest, then y, then z. */
int rtm_face_layout(const rtm_grid *grid, int64_t offsets[7]);

/* Padded-layout element index of owned cell (i, j, k) (no bounds check beyond the grid's own). */
int64_t rtm_index(const rtm_grid *grid, int32_t i, int32_t j, int32_t k);

int rtm_abi_version(void);
const char *rtm_strerror(int status);

/* Process-wide performance options.  They never change results (every variant evaluates the same
 * per-point expression), but the halo and interior calls of one step must see the same options, so
 * change them only between steps.
 *   RTM_OPT_INTERIOR_VARIANT  workgroup shape of the interior call's tiled kernel: 0 = 16x16 threads
 *                             (64x16 cells), 1 = 32x8 (128x8 cells), 2 = 16x8 (64x8 cells; default),
 *                             3 = scalar per-cell kernels for every call, 4 = 32x16 (128x16 cells,
 *                             two workgroups per CU), 5 = 16x32 (64x32 cells).
 *   RTM_OPT_HALO_VARIANT      the halo call's workgroup shape, numbered as above (not 3); default 0.
 *   RTM_OPT_WHOLE_VARIANT     rtm_step_whole's workgroup shape, numbered as above (not 3), or 6 (the
 *                             default): 1 (32x8) at radius 4, 4 (32x16) at radius 2.  The one-launch
 *                             adjoint and gradient calls take it too, except that the adjoint runs 4
 *                             and 5 (tiles held to 128 registers) as 0.
 *   RTM_OPT_ZCHUNK            z planes per workgroup of the tiled kernels; 0 = automatic: at radius 4,
 *                             for one-box launches (interior, whole step, adjoint, gradient) the
 *                             chunking that balances the work of the busiest CU (counted as at least
 *                             the workgroups that hold 6 wavefronts) with the fewest workgroups, for
 *                             the halo call chunks of 12 planes; at radius 2 chunks of 16 planes.
 *   RTM_OPT_XCD_REMAP         1 = give each XCD a contiguous range of tiles (default), 0 = hardware order.
 *   RTM_OPT_HALO_X_WIDTH      width of the halo region's x strips (default 64 = one tile);
 *   RTM_OPT_HALO_Y_WIDTH      height of its y strips (default 8);
 *   RTM_OPT_HALO_Z_WIDTH      depth of its z slabs (default 0 = R); see rtm_halo_region.
 *   RTM_OPT_UNPACK_LINES      1 = (default) where the layout puts a row's +X ghost, its padding and the
 *                             next row's -X ghost in one 128-byte line (radius 4, nx % 32 == 0,
 *                             pitch_y = nx + 32, owned (0,0,0) line-aligned), rtm_unpack_halo writes the
 *                             x faces as whole lines (zeros in the padding, which holds no cell);
 *                             0 = 16-byte pieces.  Ghost and owned cells get the same values either way.
 *   RTM_OPT_TILE_FLAGS        kernel variants.  Bit 0 (default on): non-temporal (streaming) loads of the
 *                             operands every stencil kernel uses once per cell (u_prv and kappa; mu and
 *                             grad; the adjoint's mu_b) and stores of its output, and the same for the
 *                             imaging kernels' operands; the stencil field itself stays cached, since
 *                             neighbouring tiles read it again.  Bit 1: in the radius-4 forward launches,
 *                             each thread's x neighbours from the adjacent lanes' registers (DPP lane
 *                             shifts) instead of LDS (measured: no change).  Default 1.
 *   RTM_OPT_MARKERS           1 = a roctx range named after the call around each per-step call (the
 *                             phase calls, injection, recording, imaging, coding, the adjoint and
 *                             gradient calls), so that a marker trace (rocprofv3 --marker-trace) shows
 *                             each step's phase sequence; RTM_EINVAL when the roctx library cannot
 *                             be opened.  Default 0.
 * Returns RTM_EINVAL for an unknown option or value. */
enum {
    RTM_OPT_INTERIOR_VARIANT = 1,
    RTM_OPT_ZCHUNK = 2,
    RTM_OPT_XCD_REMAP = 3,
    RTM_OPT_HALO_X_WIDTH = 4,
    RTM_OPT_HALO_Y_WIDTH = 5,
    RTM_OPT_HALO_VARIANT = 6,
    RTM_OPT_WHOLE_VARIANT = 7,
    RTM_OPT_UNPACK_LINES = 8,
    RTM_OPT_TILE_FLAGS = 9,
    RTM_OPT_HALO_Z_WIDTH = 10,
    RTM_OPT_MARKERS = 11,
};
int rtm_set_option(int32_t option, int32_t value);
/* The current value of an option (>= 0), or RTM_EINVAL for an unknown option. */
int rtm_get_option(int32_t option);

/* The halo region of a grid under the current options: widths = {wx, hy, hz} with
 * wx = max(R, min(RTM_OPT_HALO_X_WIDTH, nx / 2)), hy = max(R, min(RTM_OPT_HALO_Y_WIDTH, ny / 2)) and
 * hz = max(R, min(RTM_OPT_HALO_Z_WIDTH, nz / 2)) (hz = R when that option is 0).
 * rtm_step_halo updates exactly the owned cells with k < hz or k >= nz - hz or j < hy or j >= ny - hy
 * or i < wx or i >= nx - wx (a superset of the R-shell that neighbours need, widened so that the
 * tiled kernel reads whole cache lines); rtm_step_interior updates the rest.  The region depends
 * only on the grid and the options, never on pointers, so a caller can route each source to the
 * call that owns its cell.  RTM_EINVAL for a bad grid or NULL widths. */
int rtm_halo_region(const rtm_grid *grid, int32_t widths[3]);

/* ---- the per-time-step phases (device work, enqueued on `stream`) -------------------------- */

/* Phase 1 (section II): the update of u_nxt on the halo region (rtm_halo_region): every owned cell
 * within R of a face, which is what the neighbours need, widened in x and y to whole tiles.  Reads
 * u_cur on owned and ghost cells (ghosts from the previous unpack), u_prv and kappa at the cell.
 * u_nxt may equal u_prv (two-buffer in-place update); u_nxt == u_cur is RTM_EALIAS. */
int rtm_step_halo(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                  const float *kappa, hipStream_t stream);

/* Phase 4 (section II): the same update on every owned cell not in the halo region; it reads no
 * ghost cell, so it may run while the halo exchange is in flight.  Halo and interior evaluate the same
 * per-point expression, so any split of one step gives bitwise identical results. */
int rtm_step_interior(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                      const float *kappa, hipStream_t stream);

/* Phases 1 and 4 in one launch, for a subdomain with no exchange to overlap (a single-GPU run with
 * physical or periodic boundaries): the update of every owned cell, reading u_cur on owned and ghost
 * cells.  Bitwise identical to rtm_step_halo followed by rtm_step_interior (the same per-point
 * expression); the face pack and unpack still follow it when ghosts must be refreshed.  Same
 * arguments and status codes as rtm_step_halo. */
int rtm_step_whole(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                   const float *kappa, hipStream_t stream);

/* Measure which tile shape and workgroup order run rtm_step_whole fastest for grids of this shape on
 * the current device, and use them from then on for the one-launch calls on such grids
 * (rtm_step_whole, rtm_adjoint_step, the gradient calls) while RTM_OPT_WHOLE_VARIANT is 6 (its
 * default).  Results never change (every variant evaluates the same per-point expression); only the
 * time does.  Times `reps` launches (1..1000) of each of ten settings on `stream` and WAITS for
 * them: call it once per grid shape, before timing anything.  u_nxt is overwritten and must not be
 * u_prv (RTM_EALIAS); u_cur, u_prv and kappa are read.  choice (host, may be NULL) receives the
 * chosen {tile variant as numbered for RTM_OPT_WHOLE_VARIANT, 1 = contiguous tiles per XCD or 0 =
 * hardware order}, or {-1, -1} when the grid takes the per-cell path (nothing to tune).  Keeps up to
 * 32 shapes (then the oldest is replaced).  Chosen for grids larger than 512^3, where the defaults
 * leave up to 20% (workgroup counts that do not divide evenly over the 256 CUs). */
int rtm_tune_step(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv, const float *kappa,
                  int32_t reps, int32_t choice[2], hipStream_t stream);

/* Phase 2 (section II): copy the R outermost owned layers of u on each face into `faces` (one
 * buffer of rtm_face_layout()[6] elements, slots as described there).  Bitwise copy.  Any slot size
 * (counters are 64-bit where a slot holds 2^31 elements or more). */
int rtm_pack_halo(const rtm_grid *grid, const float *u, float *faces, hipStream_t stream);

/* Phases 1 and 2 in one launch (section II): rtm_step_halo and then rtm_pack_halo of u_nxt into
 * `faces`, bitwise the same fields and face buffer; the halo call's workgroups write each face cell
 * they compute straight into its slot, so the faces are not read back from u_nxt.  Radius 4 with the
 * vectorised layout, nx % 4 == 0 and a 16-byte aligned `faces`; otherwise the two calls run one
 * after the other.  Sources injected afterwards into face cells must be re-copied with
 * rtm_pack_cells.  For schedules that need the faces before the interior call (an exchange that
 * overlaps it); with nothing to overlap, packing after the interior call is cheaper on the whole.
 * Same status codes as the two calls; `faces` must not overlap any field. */
int rtm_step_halo_pack(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                       const float *kappa, float *faces, hipStream_t stream);

/* Phases 1 and 2 of a step with the previous step's phase 5 (section II) folded in: the result of
 * rtm_unpack_halo(u_cur, recv) followed by rtm_step_halo_pack, bitwise (u_nxt's halo-region cells
 * and `faces`), except that u_cur's ghost ring is neither written nor read: the halo call loads
 * each ghost cell it needs from its receive slot.  recv[f] (device) is the receive slot of ghost
 * face f in the layout rtm_unpack_halo reads (what arrived for u_cur's faces); a zero-filled slot
 * stands for a physical boundary.  rtm_step_interior reads no ghost cell, so a step built on this
 * call needs no unpack pass; code that reads u_cur's ghost ring afterwards (rtm_step_whole, the
 * adjoint and gradient calls) must unpack first.  Requires radius 4 with the vectorised layout,
 * nx % 4 == 0, six non-NULL 16-byte aligned slots and a 16-byte aligned `faces`: RTM_EINVAL
 * otherwise.  `faces` must not overlap any field, and no slot may overlap `faces` or u_nxt
 * (RTM_EALIAS): an exchange that hands one step's face buffer to the next step as its receive slots
 * alternates between two face buffers. */
int rtm_step_halo_pack_slots(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                             const float *kappa, const float *const recv[6], float *faces, hipStream_t stream);

/* Phases 1 and 2 (section II) as a shell call: the new values of the owned cells within R of a face
 * (u^{n+1} from u_cur = u^n, u_prv = u^{n-1}, kappa), written to `faces` only (the slots of
 * rtm_face_layout, bitwise what rtm_pack_halo would copy out of a u^{n+1} computed by any other
 * step call).  No field is written: the cells are computed again by rtm_step_whole_slots, which
 * writes u^{n+1}.  The shell call reads u_prv, so a schedule that runs the two calls concurrently
 * must not let rtm_step_whole_slots overwrite u_prv in place.  The ghosts of u_cur come from the
 * receive slots recv[f] (device; the layout rtm_unpack_halo reads; a zero-filled slot is a
 * physical boundary); u_cur's ghost ring is not read.  faces_cur, faces_prv, faces_kappa (device,
 * all three or none): face buffers holding what rtm_pack_halo copies out of u_cur, u_prv and kappa
 * (a schedule has the first two as the face buffers of its last two steps); with them the cells of
 * the x faces read u^n, u^{n-1} and kappa densely from there instead of one 16-byte piece per row of
 * each field (the result is the same bits; wrong copies give wrong faces).  Radius 4 with the
 * vectorised layout, nx % 4 == 0, six non-NULL 16-byte aligned slots and 16-byte aligned face
 * buffers: RTM_EINVAL otherwise.  `faces` must not overlap u_cur, u_prv, kappa or a face copy, and
 * no slot may overlap `faces` (RTM_EALIAS).  Injected sources in face cells must be re-copied
 * afterwards (rtm_pack_cells). */
int rtm_step_shell_pack(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *kappa,
                        const float *faces_cur, const float *faces_prv, const float *faces_kappa,
                        const float *const recv[6], float *faces, hipStream_t stream);

/* Phase 4 (section II) over every owned cell, with the previous step's phase 5 folded in: the result
 * of rtm_unpack_halo(u_cur, recv) followed by rtm_step_whole, bitwise (u_nxt's owned cells), except
 * that u_cur's ghost ring is neither written nor read: the ghosts come from the receive slots, as in
 * rtm_step_halo_pack_slots.  With rtm_step_shell_pack it forms a halo-first step whose halo call only
 * produces the faces for the exchange (cells within R of a face computed twice, about 5% of the
 * cells at 512^3) and whose second call covers the whole block in full-width tiles.  u_nxt may be
 * u_prv (in place) unless a shell call of the same step may still read u_prv.  Requires radius 4
 * with the vectorised layout, nx % 4 == 0 and six non-NULL 16-byte aligned slots: RTM_EINVAL
 * otherwise; no slot may overlap u_nxt (RTM_EALIAS); the field rules of rtm_step_whole apply. */
int rtm_step_whole_slots(const rtm_grid *grid, float *u_nxt, const float *u_cur, const float *u_prv,
                         const float *kappa, const float *const recv[6], hipStream_t stream);

/* For each of the n padded indices idx (int64, device) of owned cells, copy u[idx] into every face
 * slot that holds that cell (as rtm_pack_halo would); indices of cells outside every face, or not
 * owned, are skipped.  Used after injecting sources into face cells of a level packed by
 * rtm_step_halo_pack.  n >= 0; `faces` must not overlap u. */
int rtm_pack_cells(const rtm_grid *grid, const float *u, const int64_t *idx, int32_t n, float *faces,
                   hipStream_t stream);

/* Phase 6 (section II): write slot f of the received faces into the R-wide ghost layer of u on face
 * f (face f of u receives what the neighbour across face f packed from its opposite face).
 * faces[f] is a device pointer to that slot's data (slot size as in rtm_face_layout), or NULL for a
 * physical boundary (zero ghosts).  Passing per-slot pointers lets a periodic self-exchange be a
 * pointer swap.  Edge and corner ghosts are not touched (a star stencil never reads them). */
int rtm_unpack_halo(const rtm_grid *grid, float *u, const float *const faces[6], hipStream_t stream);

/* Source injection: u[idx[s]] += w[s] * amp[s] for s < n (duplicate indices add up).  idx are
 * padded-layout element indices (rtm_index); an index outside the padded block is skipped.  For a
 * point source w = (v_s dt)^2 / h^3 and amp = the wavelet at t_n; in back-propagation amp is the
 * time-reversed trace sample of each receiver. */
int rtm_inject(const rtm_grid *grid, float *u, const int64_t *idx, const float *w, const float *amp,
               int32_t n, hipStream_t stream);

/* rtm_inject(u, src_idx, w, amp, nsrc) followed by rtm_record(u, rec_idx, out, nrec), with the same
 * results (a receiver on a source cell records the injected value): the injection and recording that
 * end a step.  When nsrc + nrec <= 4096 both run in one workgroup of one launch (adds, fence,
 * barrier, gathers), which for short lists costs about one launch instead of two; longer lists take
 * the two launches.  Argument meaning, layout and errors as for the two calls; either count may be
 * zero (its pointers may then be NULL). */
int rtm_inject_record(const rtm_grid *grid, float *u, const int64_t *src_idx, const float *w, const float *amp,
                      int32_t nsrc, const int64_t *rec_idx, float *out, int32_t nrec, hipStream_t stream);

/* Receiver recording: out[r] = u[idx[r]] for r < n (an index outside the padded block gives 0). */
int rtm_record(const rtm_grid *grid, const float *u, const int64_t *idx, float *out, int32_t n,
               hipStream_t stream);

/* Material coefficient on the device: kappa = (v * dt_over_h)^2 in FP32 on the owned cells of the
 * padded `kappa`; `v` is a compact x-fastest nz*ny*nx FP32 velocity array.  Ghost cells of kappa are
 * not written (the stencil never reads them). */
int rtm_kappa_from_velocity(const rtm_grid *grid, float *kappa, const float *v, float dt_over_h,
                            hipStream_t stream);

/* Health check of a time level: *count (a device uint32 the caller zeroes) += the number of owned
 * cells of u that are not finite (NaN or infinite).  A run past the stability limit grows until its
 * values overflow; checking the newest level every K steps catches it within K steps of the first
 * non-finite level.  Reads 4 bytes per owned cell. */
int rtm_count_nonfinite(const rtm_grid *grid, const float *u, uint32_t *count, hipStream_t stream);

/* Zero-lag cross-correlation imaging condition (Claerbout 1971): image += weight * src * rcv on
 * owned cells; src is the source wavefield at a time level and rcv the receiver wavefield at the
 * same level.  image may not overlap src or rcv. */
int rtm_image_accumulate(const rtm_grid *grid, float *image, const float *src, const float *rcv,
                         float weight, hipStream_t stream);

/* ---- exact adjoint and adjoint-state gradient (Tarantola 1984) ------------------------------ */

/* One step of the transposed recursion of the forward update u^{n+1} = G (2 + K L) u^n - G^2 u^{n-1}
 * (G = diag(g), K = diag(kappa), L symmetric with the zero ghosts of a physical boundary):
 *     mu_out = 2 g mu_a + L(kappa g mu_a) - g^2 mu_b,
 * with mu_a the adjoint state one level later and mu_b two levels later.  Cells outside the owned
 * block count as zero in kappa g mu_a, so the ghost values of mu_a, mu_b and kappa do not matter.
 * One launch of the tiled kernel, which forms kappa g mu_a itself as it loads each plane.  `work` is a
 * caller-owned padded field whose ghost cells are zero, used only by the per-cell path (pointers not
 * 16-byte aligned, pitches not multiples of 4, or RTM_OPT_INTERIOR_VARIANT = 3): that path writes
 * kappa g mu_a into its owned cells and then differentiates it; the results are bitwise the same.
 * mu_out may equal mu_b (in-place two-buffer recursion); no ghost cell of mu_out is written.  Adjoint
 * sources (the residual traces, R^T y) are added with rtm_inject afterwards.  Every owned cell is
 * updated. */
int rtm_adjoint_step(const rtm_grid *grid, float *mu_out, const float *mu_a, const float *mu_b, const float *kappa,
                     float *work, hipStream_t stream);

/* Gradient of the least-squares misfit with respect to kappa, one term per step:
 * grad += g * mu^{n+1} * L u^n on owned cells (u's ghosts are read, zero for a physical boundary). */
int rtm_gradient_accumulate(const rtm_grid *grid, float *grad, const float *u, const float *mu, hipStream_t stream);

/* The same recursion in scaled form, which the forward kernel runs.  With w = kappa g mu (kappa, g > 0
 * and time-independent), multiplying the transposed step by kappa g gives
 *     w^m = g (2 w^{m+1} - g w^{m+2} + kappa L w^{m+1}) + kappa g R^T y^{m-1},
 * which is exactly the forward update of rtm_step_whole with u_cur = w^{m+1}, u_prv = w^{m+2} (zero
 * ghosts: cells outside the owned block are zero in w as in kappa g mu), followed by rtm_inject at
 * the receivers with the weights kappa_r g_r.  The adjoint step then costs one forward step.  In this
 * form the gradient is
 *     dJ/dkappa = sum_n g mu^{n+1} L u^n = (1/kappa) sum_n w^{n+1} L u^n,
 *     dJ/dv = 2 v (dt/h)^2 dJ/dkappa = (2 / v) sum_n w^{n+1} L u^n,
 * and the source-side output is w_s mu^{n+1}[s] = w_s w^{n+1}[s] / (kappa_s g_s).  The four calls below
 * provide the pieces the forward calls do not. */

/* grad += w L u on owned cells (u's ghosts are read): one term of G = sum_n w^{n+1} L u^n. */
int rtm_gradient_accumulate_scaled(const rtm_grid *grid, float *grad, const float *u, const float *w,
                                   hipStream_t stream);

/* For the n padded indices idx (int64, device) of owned cells: kg[r] = kappa g at the cell (the receiver
 * weights of the scaled recursion) and inv_kg[r] = 1 / (kappa g) (its source-side output scale), FP32,
 * device arrays of n; either may be NULL, not both.  An index that is not an owned cell gives 0 in both. */
int rtm_scaled_adjoint_factors(const rtm_grid *grid, const float *kappa, const int64_t *idx, int32_t n, float *kg,
                               float *inv_kg, hipStream_t stream);

/* Weighted recording: out[r] = w[r] * u[idx[r]] for r < n (an index outside the padded block gives 0). */
int rtm_record_weighted(const rtm_grid *grid, const float *u, const int64_t *idx, const float *w, float *out,
                        int32_t n, hipStream_t stream);

/* grad_v = 2 G / v (compact x-fastest nz*ny*nx arrays grad_v and v; G a padded field): dJ/dv from the
 * scaled gradient sum G = sum_n w^{n+1} L u^n. */
int rtm_velocity_gradient_scaled(const rtm_grid *grid, float *grad_v, const float *G, const float *v,
                                 hipStream_t stream);

/* resid[i] = d[i] - obs[i] for i < n, and *misfit += 1/2 sum resid^2 accumulated in FP64 in a fixed
 * order (bitwise reproducible; misfit is a device double the caller zeroes).  resid may equal d or
 * obs. */
int rtm_misfit_residual(const float *d, const float *obs, float *resid, int64_t n, double *misfit, hipStream_t stream);

/* The same residual and misfit spread over the whole device: the samples are split into `nchunks`
 * contiguous chunks of ceil(n / nchunks) (one workgroup each), whose FP64 sums of squares go to
 * `partials` (caller-owned device buffer of at least nchunks doubles, overwritten) and are then added
 * in chunk order into *misfit.  The summation order depends only on n and nchunks, so repeated calls
 * give the same bits (not the same bits as rtm_misfit_residual, whose single workgroup sums in
 * another order).  RTM_EINVAL for n < 0, nchunks <= 0 or a NULL pointer; RTM_EALIAS if resid
 * partly overlaps d or obs, or `partials` overlaps d, obs, resid or misfit; n == 0 does nothing. */
int rtm_misfit_residual_chunks(const float *d, const float *obs, float *resid, int64_t n, double *partials,
                               int32_t nchunks, double *misfit, hipStream_t stream);

/* rtm_misfit_residual_chunks without the caller's `partials` buffer, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * per-chunk FP64 sums go to a scratch array inside the library, at most 4096 chunks (32 KiB), which
 * each device that runs this call holds until the process ends.  The call itself allocates nothing
 * and frees nothing.  Same residual, same fixed summation order and so the same bits as
 * rtm_misfit_residual_chunks with the same n and nchunks.  Every call on one device shares that
 * device's scratch: calls that overlap in time on one device (other streams, other host threads)
 * race and must be ordered by the caller.  Each call writes every slot it reads, so nothing carries
 * over from the previous call.  RTM_EINVAL for n < 0, nchunks <= 0 or nchunks > 4096, or a NULL
 * pointer; RTM_EALIAS if resid partly overlaps d or obs; RTM_EDEVICE if the scratch address of the
 * current device cannot be obtained. */
int rtm_misfit_residual_chunks_noalloc(const float *d, const float *obs, float *resid, int64_t n, int32_t nchunks,
                                       double *misfit, hipStream_t stream);

/* Chain rule through kappa = (v dt / h)^2: grad_v = 2 v (dt/h)^2 grad_kappa, with grad_v and v compact
 * x-fastest nz*ny*nx arrays and grad_kappa a padded field. */
int rtm_velocity_gradient(const rtm_grid *grid, float *grad_v, const float *grad_kappa, const float *v,
                          float dt_over_h, hipStream_t stream);

/* ---- reduced-precision source-wavefield snapshots ------------------------------------------- */

enum { RTM_SNAP_BF16 = 1, RTM_SNAP_F16 = 2 };

/* Encode the owned cells of u into a compact snapshot: scales[k] = max |u| over plane k (one FP32
 * scale per z slab, nz values) and codes[(k ny + j) nx + i] = RNE(u / scales[k]) as BF16 or FP16 bits
 * (nx*ny*nz 16-bit values, x fastest); a zero scale gives zero codes.  The division is an IEEE FP32
 * division.  Two kernels on `stream` (a per-plane max, then the quantisation). */
int rtm_snapshot_encode(const rtm_grid *grid, const float *u, uint16_t *codes, float *scales, int32_t format,
                        hipStream_t stream);

/* Imaging with a coded source snapshot: image += weight * (decode(code) * scale) * rcv on owned cells;
 * the decoded value and the accumulation are FP32. */
int rtm_image_accumulate_coded(const rtm_grid *grid, float *image, const uint16_t *codes, const float *scales,
                               int32_t format, const float *rcv, float weight, hipStream_t stream);

/* ---- learned dispersion corrector: a 3-D CNN on BF16 MFMA (FP32 accumulation) --------------- */
/* Not part of the paper, whose §II propagates on one fine grid: these calls correct a coarse-grid
 * propagation (twice the spacing, the radius-2 stencil, twice the step) towards the fine one.  They
 * implement standard operations: 3-D convolution and its weight and data gradients (implicit GEMM),
 * ReLU, Adam (Kingma & Ba 2014), full-weighting restriction (the multigrid restriction operator).
 * Like the propagator calls they only enqueue work on `stream` and return RTM_OK, RTM_EINVAL (null or
 * misaligned pointers, nx not a multiple of 16, sizes or counts out of range), RTM_EALIAS (an output
 * aliasing the input it is computed from), RTM_ELAUNCH or RTM_EDEVICE (not a gfx950 device).
 * Activations are channel-last BF16 volumes of 16 channels with a one-voxel zero halo: channel c of
 * voxel (i, j, k) of an nx*ny*nz volume is element (((k+1)(ny+2) + (j+1))(nx+2) + (i+1)) * 16 + c.
 * "Compact" FP32 channel-last volumes have no halo: element ((k ny + j) nx + i) * 16 + c.  nx must
 * be a multiple of 16.  Weights of a 3x3x3 layer are BF16 [27 taps][16 out][16 in], tap
 * t = 9 (dz+1) + 3 (dy+1) + (dx+1).  The caller zeroes halos once; the kernels write owned voxels only. */

/* y = conv3x3x3(x, w) + bias (bias may be NULL; relu != 0: max(y, 0)), written as compact FP32
 * (y32, [voxel][y32_channels]: only the first y32_channels of the 16 output channels, 1..16) and/or
 * as a BF16 volume with halo (y16, all 16 channels); either may be NULL but not both.  Alignment:
 * x, w and y32 16 bytes, y16 8 bytes; y16 must not alias x. */
int rtm_cnn_conv3d(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const uint16_t *w, const float *bias,
                   int32_t relu, float *y32, int32_t y32_channels, uint16_t *y16, hipStream_t stream);

/* dw[t][co][ci] += sum over voxels of dz[voxel][co] x[voxel + t][ci] and db[co] += sum dz[voxel][co]
 * (x: BF16 with halo, dz: compact FP32, rounded to BF16 for the MFMA; FP32 accumulation, the
 * per-workgroup partial sums added with FP32 atomics, so the summation order is not fixed). */
int rtm_cnn_conv3d_wgrad(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const float *dz, float *dw, float *db,
                         hipStream_t stream);

/* The same weight gradient with a fixed summation order, so that repeated calls (and trainings) give
 * the same bits: each workgroup's partial sums go to its own slot of `partials` (caller-owned device
 * FP32 buffer of at least rtm_cnn_wgrad_partials(nx, ny, nz) elements, contents overwritten), and a
 * second kernel adds the slots in order into dw and db.  RTM_EINVAL for bad dimensions, a NULL pointer
 * or a short buffer; RTM_EALIAS if `partials` overlaps x, dz, dw or db.  The result differs from
 * rtm_cnn_conv3d_wgrad's only by summation order. */
int rtm_cnn_conv3d_wgrad_ordered(int32_t nx, int32_t ny, int32_t nz, const uint16_t *x, const float *dz, float *dw,
                                 float *db, float *partials, int64_t partials_len, hipStream_t stream);

/* Elements of `partials` that rtm_cnn_conv3d_wgrad_ordered needs for this volume (one slot of
 * 27*16*16 + 16 floats per workgroup of 64 x 4 voxels and one plane), or RTM_EINVAL. */
int64_t rtm_cnn_wgrad_partials(int32_t nx, int32_t ny, int32_t nz);

/* dz = dy for channels < channels (0 elsewhere), times the ReLU derivative (y > 0) when relu != 0;
 * written compact FP32 (dz32) and BF16 with halo (dz16). */
int rtm_cnn_relu_backward(int32_t nx, int32_t ny, int32_t nz, const float *y, const float *dy, int32_t relu,
                          int32_t channels, float *dz32, uint16_t *dz16, hipStream_t stream);

/* Gradient of the training loss L = 1/2 sum over voxels and channels < channels of w (out - target)^2,
 * w = weight * mask[voxel] (mask: NULL, or compact FP32 over the voxels, >= 0), with respect to the
 * network output: dz = w (out - target) there, 0 on the other channels, compact FP32 (dz32) and BF16
 * with halo (dz16).  weight >= 0.  When loss is not NULL, L is added into loss[0] (FP64, atomically). */
int rtm_cnn_loss_grad(int32_t nx, int32_t ny, int32_t nz, const float *out, const float *target, int32_t channels,
                      float weight, const float *mask, float *dz32, uint16_t *dz16, double *loss, hipStream_t stream);

/* wt[t][ci][co] = w[26 - t][co][ci]: the weights of the data-gradient convolution
 * dx = rtm_cnn_conv3d(dz, wt). */
int rtm_cnn_weight_flip(const uint16_t *w, uint16_t *wt, hipStream_t stream);

/* One Adam step (Kingma & Ba 2014) on n FP32 parameters with bias correction for step number `step`
 * (>= 1); also writes the BF16 copy param_bf16 when it is not NULL. */
int rtm_cnn_adam(float *param, const float *grad, float *m1, float *m2, int32_t n, float lr, float beta1, float beta2,
                 float eps, int32_t step, uint16_t *param_bf16, hipStream_t stream);

/* b = BF16(a) (round to nearest even) for n values. */
int rtm_cnn_to_bf16(const float *a, uint16_t *b, int32_t n, hipStream_t stream);

/* Network input from a coarse-grid state: channel 0 = a = u^n / s, 1 = d = (u^n - u^{n-1}) / s (the
 * difference formed in FP32), 2 = m a, 3 = m d with m = (velocity[voxel] - v_ref) / v_scale (velocity
 * compact FP32 over the owned cells), channels 4..15 zero, with s = scale[0] read on the device
 * (s = 0 gives zero channels).  v_scale > 0.  noise: NULL, or compact FP32 [voxel][2] added to a and d before the
 * products and the rounding (training-time augmentation; the random numbers are the caller's). */
int rtm_cnn_pack_input(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *velocity,
                       float v_ref, float v_scale, const float *scale, const float *noise, uint16_t *x,
                       hipStream_t stream);

/* Apply the network's correction, given in the input's level-and-difference form (out compact FP32,
 * [voxel][out_channels], out_channels 2..16): u^n += c out[.][0] and u^n - u^{n-1} += c out[.][1], i.e.
 * u^{n-1} += c (out[.][0] - out[.][1]), with c = scale[0] * mask[voxel] (mask: NULL for 1, or compact
 * FP32 over the owned cells, e.g. 0 near injection points). */
int rtm_cnn_apply_correction(const rtm_grid *grid, float *u_cur, float *u_prv, const float *out, int32_t out_channels,
                             const float *mask, const float *scale, hipStream_t stream);

/* The first layer straight from the coarse-grid state, in one launch: y16 = the BF16 output of
 * rtm_cnn_conv3d(x, w, bias, relu) where x is what rtm_cnn_pack_input(grid, u_cur, u_prv, velocity,
 * v_ref, v_scale, scale, NULL) would write, bitwise the same, without x being written or read
 * (the input formed in LDS as each plane is staged).  nx, ny, nz are the grid's; y16 is a BF16
 * volume with halo of that size (8-byte aligned), w 16-byte aligned. */
int rtm_cnn_conv3d_first(const rtm_grid *grid, const float *u_cur, const float *u_prv, const float *velocity,
                         float v_ref, float v_scale, const float *scale, const uint16_t *w, const float *bias,
                         int32_t relu, uint16_t *y16, hipStream_t stream);

/* The last layer applied as the correction, in one launch: the same u_cur and u_prv, bitwise, as
 * rtm_cnn_conv3d(x, w, bias, relu) into a compact FP32 [voxel][2] output followed by
 * rtm_cnn_apply_correction(grid, u_cur, u_prv, that output, 2, mask, scale), without the output
 * being written.  x is a BF16 volume with halo of the grid's size (16-byte aligned, like w); it
 * must not overlap u_cur or u_prv, which must differ. */
int rtm_cnn_conv3d_apply(const rtm_grid *grid, const uint16_t *x, const uint16_t *w, const float *bias, int32_t relu,
                         float *u_cur, float *u_prv, const float *mask, const float *scale, hipStream_t stream);

/* Training target in the same form: channel 0 = (ref^n - u^n) / s, channel 1 =
 * ((ref^n - ref^{n-1}) - (u^n - u^{n-1})) / s, others 0 (compact FP32).  With noise (NULL, or the
 * [voxel][2] array given to rtm_cnn_pack_input) the noise is subtracted too. */
int rtm_cnn_target(const rtm_grid *grid, const float *ref_cur, const float *ref_prv, const float *u_cur,
                   const float *u_prv, const float *scale, const float *noise, float *target, hipStream_t stream);

/* Restriction from a fine grid to one of half the resolution (owned cells of padded fields of the
 * two grids).  RTM_RESTRICT_INJECT: coarse (i, j, k) takes fine (2i, 2j, 2k).  RTM_RESTRICT_FULL: the
 * separable (1/4, 1/2, 1/4) full-weighting average of the 27 fine cells around (2i, 2j, 2k), fine
 * ghost cells included at the boundary; it preserves integrals, so a fine point source maps to the
 * coarse point source.  Both modes need n_fine >= 2 n_coarse - 1 along every axis (full weighting
 * then reads at most one ghost layer of the fine field, which must hold its boundary values). */
#define RTM_RESTRICT_INJECT 0
#define RTM_RESTRICT_FULL 1
int rtm_restrict(const rtm_grid *fine, const rtm_grid *coarse, const float *u_fine, float *u_coarse, int32_t mode,
                 hipStream_t stream);

/* Prolongation from a coarse grid to one of twice the resolution (owned cells of padded fields of the two
 * grids), the transpose of RTM_RESTRICT_FULL up to a factor 8: fine (I, J, K) takes, along each axis,
 * coarse I/2 for even I and the mean of coarse (I-1)/2 and (I+1)/2 for odd I (trilinear interpolation).
 * Needs n_fine <= 2 n_coarse along every axis; the last odd fine cell reads the coarse ghost layer,
 * which must hold its boundary values. */
int rtm_prolong(const rtm_grid *coarse, const rtm_grid *fine, const float *u_coarse, float *u_fine,
                hipStream_t stream);

/* out[0] = max |u| over the owned cells (device; order-independent). */
int rtm_field_absmax(const rtm_grid *grid, const float *u, float *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RTM_H */
