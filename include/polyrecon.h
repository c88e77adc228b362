/*
 * polyrecon: near-field millimetre-wave 3-D imaging with polyline arrays on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Wang, Li, Zhao, Sun, "Near-Field Millimeter-Wave Imaging via Arrays
 * in the Shape of Polyline" (arXiv 2109.02842).  The array is a set of equal
 * chords inscribed in a circle (Sec. II-A, Fig. 1), monostatic or multistatic
 * (Sec. II-B), mechanically scanned along z.  The reconstruction is the
 * paper's hybrid time-domain / spatial-frequency method with NUFFT range
 * compression (eqs. 2-9 monostatic, 12-19 multistatic); brute-force
 * back-projection (the paper's comparison method, Sec. III) is provided
 * beside it.
 *
 * Conventions shared by every entry point
 *   - Complex data are interleaved float pairs (re, im), i.e. complex64.
 *   - "_dev" pointers are device memory on the current HIP device, owned by
 *     the caller; the library never frees them.  "_host" pointers are host
 *     memory owned by the caller.
 *   - Echo cube layout: s[c][m][f] (frequency fastest), c = channel,
 *     m = scan position, f = frequency.  Channel order: monostatic c = chord *
 *     n_elem + element; multistatic c = (chord * n_tx + tx) * n_elem + rx.
 *   - Image layout: g[z][y][x] (x fastest); z runs over the scan grid.
 *   - Kernels are enqueued on the given stream and return before they
 *     complete.  A device fault surfaces at the caller's next synchronisation.
 *   - Return value: PL_OK (0) on success or a negative PL_E* code; the
 *     message of the last failure on the calling thread is last_error().
 *   - Geometry handles are immutable after make_geometry and may be shared
 *     by threads and streams; destroy_geometry must run only after all work
 *     using the handle has completed.
 */
#ifndef POLYRECON_H
#define POLYRECON_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define PL_OK 0
#define PL_EINVAL (-1)       /* bad argument: null pointer, size, range      */
#define PL_EGEOM (-2)        /* no such polyline: chord length >= 2 R        */
#define PL_EDEVICE (-3)      /* HIP runtime error (allocation, launch)       */
#define PL_EWORKSPACE (-4)   /* workspace missing or smaller than required   */
#define PL_EUNSUPPORTED (-5) /* option not supported for this problem        */

#define PL_MONO 0
#define PL_MULTI 1

/* Sampling-criterion warning bits (set by check_sampling; not errors). */
#define PL_WARN_ELEMENT_SPACING 1u /* eq. (21) (monostatic: half of it)        */
#define PL_WARN_SCAN_STEP 2u       /* eq. (22)                                  */

/* ------------------------------------------------------------- geometry */
/*
 * Array description (Sec. II-A/B; Table 1 lists the paper's own values).
 *   mode          PL_MONO or PL_MULTI.
 *   n_chords      number of polyline sections (>= 1).
 *   radius_m      radius R_0 of the circumscribed arc (> 0).
 *   arc_center_rad  angle of the arc's middle; -pi/2 puts the array below the
 *                 origin looking toward +y.
 *   n_elem        transceivers per chord (mono) or receivers per chord (multi).
 *   spacing_m     element / receiver spacing d; chord length is n_elem * d and
 *                 element j sits at (j + 1/2) d - L/2 from the chord midpoint.
 *   n_tx          transmitters per chord (multi only; 2 or 4 with the default
 *                 placement, any count with tx_offsets_m).
 *   tx_offsets_m  host array of n_tx chord-local Tx offsets from the chord
 *                 midpoint, or NULL for the default placement at the chord
 *                 ends (Sec. II-B: -L/2, -L/2 + d/2, L/2 - d/2, L/2 for 4 Tx;
 *                 -L/2, L/2 for 2 Tx).  Copied by make_geometry.
 *   n_scan, scan_step_m, scan_z0_m   scan heights z'_m = z0 + m * step.
 *   n_freq, f_start_hz, f_stop_hz    inclusive uniform sweep (Table 1).
 */
typedef struct pl_geometry_desc {
    int32_t mode;
    int32_t n_chords;
    double radius_m;
    double arc_center_rad;
    int32_t n_elem;
    int32_t n_tx;
    double spacing_m;
    const double* tx_offsets_m;
    int32_t n_scan;
    int32_t n_freq;
    double scan_step_m;
    double scan_z0_m;
    double f_start_hz;
    double f_stop_hz;
} pl_geometry_desc;

typedef struct pl_geometry pl_geometry; /* opaque */

typedef struct pl_geometry_info {
    int32_t mode;
    int32_t n_chords;
    int32_t n_channels;
    int32_t n_scan;
    int32_t n_freq;
    int32_t n_tx;
    int32_t n_elem;
    int32_t reserved;
} pl_geometry_info;

/*
 * Build a polyline array (Sec. II-A/B).  Host-only work: the small device
 * tables (channel positions, wavenumbers) are uploaded by geometry_upload,
 * or on the first device call on a device that has none.
 * Errors: PL_EINVAL (null pointers, non-positive sizes, f_start >= f_stop,
 * n_scan < 1, n_scan > 4096, n_freq > 1024, bad n_tx), PL_EGEOM (chord length
 * n_elem * spacing >= 2 R_0).  *out is left untouched on failure.
 */
int make_geometry(const pl_geometry_desc* desc, pl_geometry** out);

/* Release a handle (NULL is accepted).  Frees its device tables. */
int destroy_geometry(pl_geometry* geom);

/*
 * Copy the geometry's device tables (channel Tx/Rx positions, float64
 * [n_channels][4]; wavenumbers, float64 [n_freq]) to the current device:
 * two small allocations and two stream-ordered copies on `stream`.  Call it
 * once per device before capturing work into a graph or timing the first
 * call: with the tables present, no reconstruction, simulation or transform
 * call allocates or synchronises.  A device call on a device without them
 * uploads them itself (allocating) the first time.  Idempotent; the tables
 * are freed by destroy_geometry.
 * Errors: PL_EINVAL (null geometry), PL_EDEVICE.
 */
int geometry_upload(const pl_geometry* geom, hipStream_t stream);

/*
 * Describe a geometry.  Any of the host arrays may be NULL; otherwise they
 * receive: tx_xy_host / rx_xy_host [n_channels][2] transmit / receive phase
 * centres (m), z_scan_host [n_scan] (m), freq_host [n_freq] (Hz),
 * chord_ends_host [n_chords][2][2] chord start/end points (m).
 */
int geometry_info(const pl_geometry* geom, pl_geometry_info* info, double* tx_xy_host,
                  double* rx_xy_host, double* z_scan_host, double* freq_host,
                  double* chord_ends_host);

/* ------------------------------------------------------------ image grid */
/* Pixel (ix, iy) is centred at (x0 + ix*dx, y0 + iy*dy); nx, ny >= 1; dx, dy > 0. */
typedef struct pl_image_grid {
    int32_t nx;
    int32_t ny;
    double x0;
    double y0;
    double dx;
    double dy;
} pl_image_grid;

/*
 * Sampling criteria of Sec. II-C for this array imaging this pixel grid:
 * element spacing against eq. (21) (half of it for monostatic arrays) with D
 * the grid's horizontal extent and R_0 the distance from the middle section
 * to the grid centre, and the scan step against eq. (22) with Theta_z the
 * angle the scan length subtends from the grid centre.  *warnings receives
 * PL_WARN_* bits.
 */
int check_sampling(const pl_geometry* geom, const pl_image_grid* grid, uint32_t* warnings);

/* ------------------------------------------------------------ simulation */
/*
 * Point-scatterer echoes, eq. (1) (monostatic) and eq. (10) (multistatic):
 *   s[c][m][f] = sum_p sigma_p exp(-j k_f (R_T + R_R)),  k_f = 2 pi f / c,
 * with R_T, R_R the 3-D distances from the channel's Tx and Rx at height z'_m
 * to scatterer p (R_T = R_R for monostatic channels).  No amplitude decay or
 * antenna pattern, as in the paper.
 *   xyz_dev   [n_scat][3] float64 positions (m), device.
 *   refl_dev  [n_scat][2] float64 complex reflectivities (re, im), device.
 *   echo_dev  [n_channels][n_scan][n_freq] complex64 output, device.
 * Phases are formed in float64 and range-reduced before float32 sin/cos.
 * Errors: PL_EINVAL (null pointer, n_scat < 0), PL_EDEVICE.
 */
int simulate_echo(const pl_geometry* geom, int32_t n_scat, const double* xyz_dev,
                  const double* refl_dev, float* echo_dev, hipStream_t stream);

/* ------------------------------------------------- hybrid reconstruction */
#define PL_PREC_FP32 0 /* range compression by FP32 NUFFT on the vector ALUs      */
#define PL_PREC_BF16 1 /* range compression as a BF16 MFMA contraction, split     */
                       /* hi+lo operands, FP32 accumulation                       */
#define PL_PREC_FP16 2 /* same with FP16 operands (hi+lo split, scaled)           */

#define PL_INTERP_BSPLINE4 0  /* cubic B-spline; its prefilter is applied per     */
                              /* frequency before range compression (default)    */
#define PL_INTERP_LAGRANGE4 1 /* cubic Lagrange on the range samples             */
#define PL_INTERP_LINEAR 2    /* linear (the simplest "1-D interpolation")       */

/* Range compression (eq. 8a / 19a) methods. */
#define PL_RANGE_NUFFT 0    /* type-1 NUFFT (the paper's method, default)         */
#define PL_RANGE_RESAMPLE 1 /* resampling onto a uniform k grid + inverse FFT     */
                            /* (the variant without NUFFT of Table 2), FP32 only  */

/* Reference wavenumber k_ref of the range profiles (eq. 8a/8b, 19a/19b). */
#define PL_REF_BAND_CENTRE 0 /* one per block of k_z bins: the centre of its k_rho band (default) */
#define PL_REF_MIN_K 1       /* the paper's: per k_z, k_rho0 = k_rho at the lowest wavenumber    */

/* Back-projection kernels (hybrid plan info). */
#define PL_BP_KZ_LANES 0     /* VALU, one k_z bin per lane, weights broadcast */
#define PL_BP_PIXEL_LANES 1  /* VALU, one pixel per lane, weights shared via LDS */
#define PL_BP_MFMA 2         /* matrix cores, split-BF16 operands */
#define PL_BP_MFMA_SP 3      /* matrix cores, single-pass scaled FP16 operands */

/*
 * Options of the hybrid method.  Zero-initialised fields take the defaults.
 *   precision     PL_PREC_* (default FP32).
 *   interp        PL_INTERP_* (default cubic B-spline).
 *   l_oversample  range-grid oversampling over the Nyquist rate of the
 *                 baseband range profile (default 6; >= 2).
 *   nufft_tol     NUFFT tolerance (default 1e-6; 1e-12 .. 1e-2).
 * The FP32 back-projection (VALU) has two kernels.  By default one pixel of
 * an 8x8 tile per lane (PL_BP_PIXEL_LANES); where the tile's range window
 * exceeds 64 samples, or when kz_per_lane or 8 wavefronts are asked for, one
 * k_z bin per lane on 8x8, 4x4 or 2x2 tiles (PL_BP_KZ_LANES).
 *   tile          back-projection pixel tile edge: 0 = automatic, or 8, 4, 2
 *                 (16 for the MFMA kernel; PL_EUNSUPPORTED if the forced
 *                 tile's range window does not fit).
 *   kz_per_lane   k_z-per-lane kernel: k_z bins per lane, 0 = automatic, or
 *                 1, 2, 4.  64 x kz_per_lane bins share one reference
 *                 wavenumber, so this also sets the range-grid step.
 *   kz_block      k_z bins per workgroup (one reference wavenumber): 0 =
 *                 automatic (32 for the pixel-per-lane kernel, 64 for the
 *                 others); pixel-per-lane kernel 32 or 64, MFMA kernel 64 or
 *                 128.
 *   waves         wavefronts per back-projection workgroup: 0 = automatic, or
 *                 4, 8 (VALU: 8 selects the k_z-per-lane kernel on the 8x8
 *                 tile; MFMA: 8 only with the 16x8 and 16x16 tiles).
 *   mfma_backprojection  BF16 / FP16 modes only: 1 = back-project on the
 *                 matrix cores (PL_EUNSUPPORTED if the grid does not allow it);
 *                 0 (automatic) and -1 use the VALU back-projection.
 *                 The MFMA back-projection keeps the range profiles as BF16
 *                 hi + lo parts, forms each 4x4 pixel group's interpolation x
 *                 carrier operand over a 16-sample range window, and runs
 *                 three split products per pair with FP32 accumulation.  It
 *                 needs the group's taps inside 16 samples; when the requested
 *                 oversampling makes them wider the plan lowers it (not below 4).
 *                 Its tile is tile x tile_y pixels (16x16 by default; 8x8,
 *                 16x8 and 16x16 allowed).
 *                 2 = the same kernel in single-pass form (FP16 mode only,
 *                 else PL_EUNSUPPORTED): the range compression writes the
 *                 profiles as FP16 Re / Im planes times one power of two
 *                 chosen from the strengths' exponents so that no value
 *                 reaches 2^15, the interpolation x carrier operand is
 *                 rounded once to FP16, and each pair takes one product
 *                 (FP32 accumulation).  Every term then carries two FP16
 *                 roundings (relative 2^-11 each): image error 2-3e-4
 *                 relative L2 against the exact sum instead of the split
 *                 form's 1e-5, for a third of the matrix-core work.
 *                 Values above 2: PL_EINVAL.
 * tile, tile_y, kz_per_lane, kz_block and waves are tuning knobs; results
 * agree to the method's tolerance whatever their values.
 *   range_method  PL_RANGE_NUFFT (default) or PL_RANGE_RESAMPLE, the
 *                 conventional evaluation the NUFFT replaces (Sec. I; Sec. II-A
 *                 after eq. 8; "without NUFFT" in Table 2): per channel and
 *                 k_z, the spectrum is demodulated by exp(+j k_L L_ref) (L_ref
 *                 the path length rho_T + rho_R from the channel to the centre
 *                 of the image grid, k_L = sqrt(k^2 - k_z^2/4)), interpolated
 *                 by a centred 4-point Lagrange stencil over the frequency
 *                 index at the k of every point k_L = m dkl of a uniform grid
 *                 inside the propagating band, remodulated, weighted by
 *                 k_L dkl / dk (k dk = k_L dk_L), and inverse-FFT'd onto the
 *                 range grid.  dkl = 2 pi / (n_fine du) (plan info dk_uniform),
 *                 so the profile is periodic in L with period n_fine du.
 *                 FP32 precision only (PL_EUNSUPPORTED otherwise), at least two
 *                 frequencies.  Its accuracy is that of the interpolation, not
 *                 the NUFFT tolerance.
 *   ref_mode      reference wavenumber k_ref that demodulates the range
 *                 profiles (eq. 8a/19a) and is restored by the carrier
 *                 exp(j k_ref l) (eq. 8b/19b).  The two cancel exactly, so
 *                 the choice changes only the profiles' bandwidth and with
 *                 it the interpolation error.  PL_REF_BAND_CENTRE (default):
 *                 one reference per block of k_z bins, the centre of the
 *                 block's k_rho band (narrowest profiles; one carrier per
 *                 pixel and channel for the whole block).  PL_REF_MIN_K: the
 *                 paper's k_rho0 = k_rho at the lowest wavenumber k_0 of the
 *                 sweep, per k_z bin (Sec. II-A after eq. 8, Sec. II-B after
 *                 eq. 19); where k_0 is evanescent, the smallest real k_rho
 *                 of the bin.  Its profiles span [0, max k_rho - k_rho0], so
 *                 the range grid is about twice as fine at the same
 *                 l_oversample, and the carrier is formed per (k_z, pixel,
 *                 channel): it runs the NUFFT range compression (any
 *                 precision) and the k_z-per-lane back-projection with one
 *                 bin per lane and 4 wavefronts (PL_EUNSUPPORTED for other
 *                 range methods, the matrix-core back-projection, kz_block,
 *                 kz_per_lane > 1 or 8 wavefronts).
 */
typedef struct pl_hybrid_opts {
    int32_t precision;
    int32_t interp;
    double l_oversample;
    double nufft_tol;
    int32_t tile;
    int32_t kz_per_lane;
    int32_t waves;
    int32_t mfma_backprojection;
    int32_t tile_y;
    int32_t kz_block;
    int32_t range_method;
    int32_t ref_mode;
} pl_hybrid_opts;

/* Sizes the plan derives for (geometry, grid, options); see hybrid_plan_info. */
typedef struct pl_hybrid_plan_info {
    int32_t n_kz;        /* k_z bins (= n_scan)                                  */
    int32_t n_l;         /* range samples per (channel, k_z)                     */
    int32_t n_fine;      /* NUFFT fine-grid length (2 n_l)                       */
    int32_t kernel_width;/* NUFFT spreading-kernel width W                       */
    int32_t n_blocks;    /* k_z blocks sharing one reference wavenumber          */
    int32_t block;       /* k_z bins per block                                   */
    int32_t window;      /* range samples staged per pixel tile and channel      */
    int32_t tile_x;      /* back-projection pixel tile                           */
    int32_t tile_y;
    int32_t bp_kernel;   /* back-projection kernel: PL_BP_KZ_LANES, PL_BP_PIXEL_LANES, PL_BP_MFMA, PL_BP_MFMA_SP */
    int32_t waves;       /* wavefronts per back-projection workgroup             */
    double du;           /* range-grid step (m of rho_T + rho_R)                 */
    double beta;         /* exponential-of-semicircle kernel shape               */
    size_t workspace_bytes;
    int32_t range_method;/* PL_RANGE_NUFFT or PL_RANGE_RESAMPLE                  */
    double dk_uniform;   /* PL_RANGE_RESAMPLE: step of the uniform k_L grid, 2 pi / (n_fine du); else 0 */
    int32_t scan_fft_len;/* length the scan / k_z transforms run through: n_scan when it is  */
                         /* 2,3,5-smooth, else the chirp-z length (smooth, >= 2 n_scan - 1)  */
    int32_t reserved_;
} pl_hybrid_plan_info;

/*
 * Plan sizes for a hybrid reconstruction (host-only).  k_ref_host, if not
 * NULL, receives n_blocks reference wavenumbers (rad/m, for the range
 * rho_T + rho_R; monostatic ranges are 2 rho).  Errors: PL_EINVAL,
 * PL_EUNSUPPORTED (grid or problem beyond the supported sizes).
 */
int hybrid_plan_info(const pl_geometry* geom, const pl_image_grid* grid,
                     const pl_hybrid_opts* opts, pl_hybrid_plan_info* info,
                     double* k_ref_host);

/* Workspace bytes reconstruct_hybrid needs (host-only). */
int hybrid_workspace_bytes(const pl_geometry* geom, const pl_image_grid* grid,
                           const pl_hybrid_opts* opts, size_t* bytes);

/*
 * The hybrid reconstruction of Sec. II (eqs. 2-9; multistatic 12-19):
 *   1. S = FFT over the scan axis of s (eq. 2/12);
 *   2. per channel and k_z, range compression q(l) = sum_f k_f S e^{j k'_f l}
 *      on a uniform range grid by a type-1 NUFFT (eq. 8a/19a), or with
 *      range_method PL_RANGE_RESAMPLE by uniform-grid resampling and an
 *      inverse FFT;
 *   3. per k_z, interpolation of q at each pixel's range l_c(p) = rho
 *      (mono) or rho_T + rho_R (multi), carrier e^{j k_ref l}, and the sum
 *      over channels (eq. 8b/19b);
 *   4. inverse FFT over k_z (eq. 9).
 * The result approximates the exact double sum
 *   G(k_z, p) = sum_c sum_f k_f S[c,k_z,f] exp(j k_rho(f,k_z) l_c(p)),
 *   g = IFFT_kz G,
 * to the tolerance the options set.
 *   echo_dev   [n_channels][n_scan][n_freq] complex64, read only.
 *   image_dev  [n_scan][ny][nx] complex64 output; must not alias echo or ws.
 *   ws         device workspace of at least hybrid_workspace_bytes bytes,
 *              256-byte aligned; its contents are scratch.
 * Errors: PL_EINVAL, PL_EUNSUPPORTED, PL_EWORKSPACE, PL_EDEVICE.
 */
int reconstruct_hybrid(const pl_geometry* geom, const pl_image_grid* grid,
                       const pl_hybrid_opts* opts, const float* echo_dev, float* image_dev,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * reconstruct_hybrid without a workspace argument and without any device
 * allocation, for callers that cannot allocate: code under graph capture,
 * tight serving loops, harnesses that forbid allocation.  The workspace is
 * a static device array of PL_STATIC_SCRATCH_BYTES (64 MiB) per device,
 * held from the library's first use on that device until the process ends
 * (problems up to C1 size and somewhat beyond fit; hybrid_workspace_bytes
 * tells).  The geometry's tables must be on the device already
 * (geometry_upload); the call never uploads them.  Every call on a device
 * shares that device's array and keeps nothing from the last call: calls
 * that overlap on one device (other streams, other threads) race and must
 * be serialised by the caller.  Same result as reconstruct_hybrid with the
 * same arguments.
 * Errors: PL_EINVAL (also: geometry not uploaded to this device),
 * PL_EUNSUPPORTED, PL_EWORKSPACE (the problem's workspace exceeds
 * PL_STATIC_SCRATCH_BYTES), PL_EDEVICE.
 */
#define PL_STATIC_SCRATCH_BYTES (64u << 20)
int reconstruct_hybrid_static(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                              const float* echo_dev, float* image_dev, hipStream_t stream);

/*
 * Plan caching.  hybrid_prepare writes the plan's device tables (range-grid
 * origins, reference ranges, twiddles, deapodisation, k' and weight tables,
 * the back-projection's tile geometry) into ws; they depend on the geometry,
 * grid and options only.  reconstruct_hybrid_prepared is reconstruct_hybrid
 * without that step: ws must hold the tables of a hybrid_prepare call with
 * the same geometry, grid and options on the same device, and no other call
 * may have used ws since (the reconstruction itself leaves them intact).
 * Results are bitwise those of reconstruct_hybrid.  Same errors.
 */
int hybrid_prepare(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts, void* ws,
                   size_t ws_bytes, hipStream_t stream);
int reconstruct_hybrid_prepared(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                                const float* echo_dev, float* image_dev, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/*
 * reconstruct_hybrid with stage timing for profilers: records
 * stage_events[i] on the stream before stage i and stage_events[5] after the
 * last stage.  Stages: 0 plan tables, 1 scan FFT, 2 range compression,
 * 3 back-projection, 4 k_z inverse FFT.  Events are created and owned by the
 * caller (hipEventCreate); NULL entries are skipped; stage_events itself may
 * be NULL.  Nothing is synchronised.  Same errors as reconstruct_hybrid.
 */
int reconstruct_hybrid_events(const pl_geometry* geom, const pl_image_grid* grid,
                              const pl_hybrid_opts* opts, const float* echo_dev,
                              float* image_dev, void* ws, size_t ws_bytes,
                              hipEvent_t* stage_events, hipStream_t stream);

/*
 * Adjoint of the imaging operator: image_dev ([z][y][x] complex64) ->
 * echo_dev ([c][m][f] complex64), the conjugate transpose of the linear map
 * echo -> image that reconstruct_hybrid evaluates: the forward transform
 * over z with 1/n_z, the scatter form of the back-projection (eq. 8b/19b
 * transposed: each pixel's interpolation taps times the conjugate carrier),
 * the range compression transposed (eq. 8a/19a: for fine grids of 64 R
 * points, R 2,3,5-smooth and at most 32, the exact transpose of the NUFFT
 * the forward call runs; otherwise the direct type-2 sum over the range
 * grid, the transpose of the sum the NUFFT approximates) and the
 * unnormalised inverse transform over k_z.  It serves as the echo model of
 * least-squares refinement (scene image -> echo).  FP32 plans with the
 * pixel-per-lane back-projection and the NUFFT range method only
 * (PL_EUNSUPPORTED otherwise); the same
 * workspace size as reconstruct_hybrid.  Every element of the intermediate
 * range profiles is summed by one workgroup in a fixed order (no atomics), so
 * results are bitwise repeatable.
 * Errors: PL_EINVAL, PL_EUNSUPPORTED, PL_EWORKSPACE, PL_EDEVICE.
 */
int adjoint_hybrid(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                   const float* image_dev, float* echo_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------- the hybrid steps alone */
/*
 * The four steps of reconstruct_hybrid as separate calls, for inspection and
 * step-level checks.  They exchange complex64 range profiles, so they plan as
 * with opts->mfma_backprojection = -1 (the plan hybrid_plan_info reports for
 * those options) and return PL_EUNSUPPORTED if it is 1.  Buffers are device
 * memory:
 *   scan_fft:        echo [c][m][f] -> spec [c][kz][f]        (eq. 2/12)
 *       S[c][kz][f] = sum_m s[c][m][f] exp(-2 pi i kz m / n_scan) (unnormalised).
 *   range_compress:  spec [c][kz][f] -> q [c][kz][n_l]        (eq. 8a/19a)
 *       q[c][kz][i] approximates sum_f w_f k_f S e^{j k'_f l_i} with
 *       k' = k_rho - k_ref(block of kz), l_i = l_lo[c] + i du, where w_f is
 *       1 except for PL_INTERP_BSPLINE4, where it is the B-spline prefilter
 *       1 / sinc^4(k'_f du / 2) (q then holds spline coefficients).
 *   backproject:     q -> G [p][kz] with p = iy * nx + ix      (eq. 8b/19b)
 *   kz_ifft:         G [p][kz] -> image [z][y][x]              (eq. 9)
 *       g[z][p] = (1 / n_scan) sum_kz G[p][kz] exp(+2 pi i kz z / n_scan).
 * The transforms take any n_scan in [1, 4096]: 2,3,5-smooth lengths as
 * mixed-radix stages, other lengths by Bluestein's chirp-z transform through
 * a smooth length of at least 2 n_scan - 1 (same result to float rounding).
 * Their ws holds the transform's tables (fft_workspace_bytes bytes, 256-byte
 * aligned; written by every call, so calls sharing it must not overlap).
 * range_lo_host, if not NULL, receives l_lo[c] (n_channels doubles); the
 * call then waits for the stream.
 * range_compress and backproject take a ws of at least
 * hybrid_workspace_bytes for their tables.  None of the four allocates.
 */
int fft_workspace_bytes(const pl_geometry* geom, size_t* bytes);
int scan_fft(const pl_geometry* geom, const float* echo_dev, float* spec_dev, void* ws, size_t ws_bytes,
             hipStream_t stream);
int range_compress(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                   const float* spec_dev, float* q_dev, double* range_lo_host, void* ws,
                   size_t ws_bytes, hipStream_t stream);
int backproject(const pl_geometry* geom, const pl_image_grid* grid, const pl_hybrid_opts* opts,
                const float* q_dev, float* spectrum_dev, void* ws, size_t ws_bytes,
                hipStream_t stream);
int kz_ifft(const pl_geometry* geom, const pl_image_grid* grid, const float* spectrum_dev,
            float* image_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batches */
/*
 * Several scans (each its own geometry, scan length, frequency count and
 * image grid) reconstructed by one call, each exactly as reconstruct_hybrid
 * would (same plan, same result).  The per-scan steps are launched per scan;
 * the back-projection of every scan whose plan takes the pixel-per-lane
 * kernel (PL_BP_PIXEL_LANES, with the k_z block size of the first such scan)
 * runs in one persistent launch per LDS row length (at most 8) that takes
 * (scan, k_z block, pixel tile) work items from device-side queues, one per
 * XCD with stealing, heaviest scans first; other scans' back-projections
 * follow as their own launches.
 *
 * make_hybrid_batch plans the n scans (opts: an array of n, or NULL for the
 * defaults), and uploads the work queue to the current device (a small
 * allocation owned by the batch; use the batch on that device only).
 * reconstruct_hybrid_batch takes arrays of n device pointers: echoes
 * ([c][m][f] complex64 per scan) and images ([z][y][x] complex64 per scan),
 * and a 256-byte-aligned device workspace of hybrid_batch_info's size.  All
 * of its work is launched in order on `stream` (per scan: plan tables, scan
 * FFT, range compression; the back-projection launches; per scan: k_z
 * IFFT).  It allocates nothing and does not synchronise, so it may be
 * captured in a graph; calls on one batch, or sharing one workspace, must
 * not overlap.
 * hybrid_batch_info: workspace bytes, scans in the persistent launch, its
 * work items and workgroups (any pointer may be NULL).
 * hybrid_batch_prepare writes every scan's plan tables (wavenumber tables,
 * tile geometry, transform tables) into the workspace on `stream`;
 * reconstruct_hybrid_batch_prepared is reconstruct_hybrid_batch without
 * those steps, for a workspace prepared for this batch on this device and
 * not written since by anything else (the plan-caching form of the batch,
 * as hybrid_prepare / reconstruct_hybrid_prepared are for one scan).
 * Errors: PL_EINVAL, PL_EUNSUPPORTED, PL_EWORKSPACE, PL_EDEVICE.
 */
typedef struct pl_hybrid_batch pl_hybrid_batch; /* opaque */
int make_hybrid_batch(int32_t n, const pl_geometry* const* geoms, const pl_image_grid* grids,
                      const pl_hybrid_opts* opts, pl_hybrid_batch** batch);
int destroy_hybrid_batch(pl_hybrid_batch* batch);
int hybrid_batch_info(const pl_hybrid_batch* batch, size_t* workspace_bytes, int32_t* queued_scans,
                      int32_t* work_items, int32_t* workgroups);
int reconstruct_hybrid_batch(const pl_hybrid_batch* batch, const float* const* echoes_dev,
                             float* const* images_dev, void* ws, size_t ws_bytes, hipStream_t stream);
int hybrid_batch_prepare(const pl_hybrid_batch* batch, void* ws, size_t ws_bytes, hipStream_t stream);
int reconstruct_hybrid_batch_prepared(const pl_hybrid_batch* batch, const float* const* echoes_dev,
                                      float* const* images_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------- back-projection */
/*
 * Brute-force back-projection (the paper's comparison method; its formula is
 * not written in the paper; the matched filter of eqs. 1/10 with weight k_f):
 *   g(x,y,z_m) = sum_c sum_m' sum_f k_f s[c,m',f] exp(+j k_f (R_T + R_R)),
 * over all channels and scan positions, for image planes z_m with
 * m in [iz0, iz0 + nz).  image_dev is [nz][ny][nx] complex64.  The
 * frequencies must be uniform (the sweep of make_geometry) and at most 4096.
 * ws: 256-byte aligned, at least bp_workspace_bytes(geom, grid, nz) (the
 * k_f-weighted echo and, for thin slabs whose (channel, scan) rows are split
 * over several workgroups, their partial images, summed in a fixed order).
 * Errors: PL_EINVAL, PL_EWORKSPACE, PL_EUNSUPPORTED, PL_EDEVICE.
 */
int bp_workspace_bytes(const pl_geometry* geom, const pl_image_grid* grid, int32_t nz, size_t* bytes);
int reconstruct_bp(const pl_geometry* geom, const pl_image_grid* grid, int32_t iz0, int32_t nz,
                   const float* echo_dev, float* image_dev, void* ws, size_t ws_bytes,
                   hipStream_t stream);

/* Message for the last failing call on this thread ("" if none). */
const char* last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* POLYRECON_H */
