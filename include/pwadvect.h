/*
 * pwadvect.h -- C ABI of libpwadvect, the MI355X (gfx950) implementation of
 * the Piacsek-Williams (PW) momentum-advection source terms of the MONC
 * model, as ported in N. Brown, "Exploring the acceleration of the Met Office
 * NERC Cloud model using FPGAs" (section 2.1, Listing 1; section 3, Listing 2
 * gives the kernel's external interface: six field arrays plus the grid
 * sizes as scalars).
 *
 * ---------------------------------------------------------------- layout
 * Every field array (u, v, w, the multipliers lu, lv, lw, and the outputs
 * su, sv, sw, gu, gv, gw) is a C-contiguous "storage" array of
 *     (nx + 2*halo) x (ny + 2*halo) x (nz + 2*halo)
 * elements, z fastest, then y, then x: the Fortran F(k, j, i) layout of the
 * paper (section 2.1), in which one column and then consecutive y-columns are
 * contiguous (section 3, Listings 3 and 4).  Interior cell (i, j, k) with
 * 0 <= i < nx, 0 <= j < ny, 0 <= k < nz is element
 *     ((i + halo) * (ny + 2*halo) + (j + halo)) * (nz + 2*halo) + (k + halo).
 * Element type: double for PW_F64, float for PW_F32 and PW_F32_F64, 16-bit
 * for PW_F16 and PW_BF16.
 * tzc1, tzc2 are double arrays of length nz indexed by interior level k, for
 * every dtype (dtypes with float arithmetic round them to float where they
 * use them).  tcx, tcy are passed by value as double (rounded to float by the
 * dtypes with float arithmetic).
 *
 * Placement: the arrays may come from any allocations.  Carving the arrays of
 * one grid out of ONE device allocation (any spacing between them) keeps the
 * large-grid speed steady; over separately allocated arrays the x-marching
 * kernels' time depends on where each allocation lands in HBM (up to about
 * 8% slower on MI355X at 4096 x 4096 x 64).
 *
 * Every pointer is a device pointer (hipMalloc / torch device memory) owned by
 * the caller, except the host field arrays of pw_advect_fwd_host.  The library
 * allocates no memory and reads no environment variables.  The state it keeps
 * is per thread (the tuning knobs of pw_set_tuning and the last error text)
 * or created once per device (two copy streams, a few events and the recent
 * times of pw_advect_fwd_host calls per copy-out mode, from the first such
 * call on that device until the process ends), so every call is thread-safe.
 *
 * ---------------------------------------------------------------- semantics
 * Levels follow Listing 1: Fortran k = 2..z_size is interior k = 1..nz-1.
 *   su, sv: computed on levels 1..nz-1; the top level nz-1 keeps only the
 *           tzc1 term; level 0 is 0.
 *   sw:     computed on levels 1..nz-2; levels 0 and nz-1 are 0.
 * su follows Listing 1.  The paper omits sv and sw ("very similar"); this
 * library computes sv as the x<->y transpose of su and sw as the same
 * upwind-value-times-face-sum scheme staggered in z with tzc1/tzc2.
 * Outputs are ASSIGNED (Listing 1 assigns su), never accumulated.
 * Only interior columns of outputs are written: their interior levels get the
 * result and their 2*halo z-halo levels get 0.  x/y halo columns of outputs are
 * never written.
 * Inputs must have their x/y halos filled (periodic: pw_halo_periodic or
 * pw_pad_periodic).  z-halo levels of inputs are never used; they may hold any
 * value, including NaN.
 *
 * All calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 * stream) and return as soon as the work is queued.
 *
 * ---------------------------------------------------------------- errors
 * Each call returns PW_OK or a negative code and, for a negative code, sets a
 * thread-local message readable with pw_last_error().  Argument checks happen
 * before any GPU work is queued; nothing is written on error.
 *   PW_ERR_ARG          null pointer, nx < 1, ny < 1, nz < 2, halo < 1,
 *                       unknown dtype, not a device pointer, or an array that
 *                       does not fit inside its device allocation
 *   PW_ERR_ALIAS        an output overlaps an input or another output
 *   PW_ERR_ALIGN        a pointer is not aligned to its element type
 *   PW_ERR_SIZE         n + 2*halo overflows int, or a storage byte count
 *                       overflows int64
 *   PW_ERR_UNSUPPORTED  the selected kernel cannot run this shape (the
 *                       x-marching kernels need halo <= 32, 16-byte aligned
 *                       arrays and columns of fewer than 2^30 bytes)
 *   PW_ERR_HIP          the HIP runtime reported an error at launch
 */
#ifndef PWADVECT_H
#define PWADVECT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element type of the field arrays and arithmetic type of the scheme
 * (storage / arithmetic):
 *   PW_F64      double / double
 *   PW_F32      float / float
 *   PW_F32_F64  float / double: operands are widened exactly, each result is
 *               rounded to float once; the bytes of PW_F32 with the
 *               arithmetic of PW_F64
 *   PW_F16      IEEE binary16 / float
 *   PW_BF16     bfloat16 (upper half of a binary32) / float
 * The 16-bit types halve the bytes of PW_F32 again; each result is rounded to
 * the storage type once (round to nearest even).  The utility calls use the
 * storage type only. */
typedef enum { PW_F64 = 0, PW_F32 = 1, PW_F32_F64 = 2, PW_F16 = 3, PW_BF16 = 4 } pw_dtype;

enum {
    PW_OK = 0,
    PW_ERR_ARG = -1,
    PW_ERR_ALIAS = -2,
    PW_ERR_ALIGN = -3,
    PW_ERR_SIZE = -4,
    PW_ERR_UNSUPPORTED = -5,
    PW_ERR_HIP = -6
};

/* Kernel families (tuning knob PW_TUNE_KERNEL). */
enum {
    PW_KERNEL_AUTO = 0,   /* x-marching kernel where it applies, else direct */
    PW_KERNEL_DIRECT = 1, /* one thread per storage level, any nz >= 2 */
    PW_KERNEL_MARCH = 2   /* x-marching, LDS-staged kernel (see PW_ERR_UNSUPPORTED) */
};

/* Tuning knobs (pw_set_tuning).  None changes a result: every kernel family
 * and variant gives the same bits.  Defaults in brackets. */
enum {
    PW_TUNE_KERNEL = 0,        /* kernel family, PW_KERNEL_* [PW_KERNEL_AUTO] */
    PW_TUNE_MARCH_VARIANT = 1, /* x-marching variant 0..PW_MARCH_VARIANTS-1 (strip
                                  width, prefetch depth, halo carriers), or -1 for
                                  the measured default of each storage/arithmetic
                                  type and output set [-1].  Variants 0..6 hold
                                  one wavefront per column and cut columns of
                                  more than 64 levels into z-chunks; variant
                                  PW_MARCH_VARIANTS-1 holds a column of more
                                  than 64 levels in 2 to 4 wavefronts of one
                                  workgroup, a column of more than 256 levels
                                  in z-chunks of 64 * waves - 2 levels (the
                                  default for such columns; for other columns
                                  it selects the default variant) */
    PW_TUNE_MARCH_LX = 2,      /* x-planes per marching workgroup, or 0 to choose
                                  from the grid [0] */
    PW_TUNE_COPY_OUT = 3,      /* how pw_advect_fwd_host returns the source terms,
                                  PW_COPY_OUT_* [PW_COPY_OUT_AUTO] */
    PW_TUNE_BLOCK_ORDER = 4,   /* order of the x-marching workgroups over the
                                  strips: PW_ORDER_XCD, or G in
                                  1..PW_ORDER_MAX_GROUP for groups of G
                                  neighbouring strips per XCD, the 8 XCDs
                                  interleaved group by group (1: natural
                                  order), or -1 for the measured default of
                                  each kernel [-1] */
    PW_TUNE_TALL_WAVES = 5     /* wavefronts per column of variant
                                  PW_MARCH_VARIANTS-1, 2..4, or 0 for the
                                  fewest that hold a column of up to 256
                                  levels and, above that, the most whose
                                  z-chunks idle at most 10% more lanes than
                                  the chunking that idles fewest [0] */
};
enum {
    PW_ORDER_XCD = 0,       /* each of the 8 XCDs takes one contiguous range of strips */
    PW_ORDER_NATURAL = 1,   /* neighbouring strips on all XCDs at once */
    PW_ORDER_MAX_GROUP = 65536
};
enum { PW_MARCH_VARIANTS = 8 };
enum {
    PW_COPY_OUT_RUNTIME = 0, /* the HIP runtime's device-to-host copies */
    PW_COPY_OUT_KERNEL = 1,  /* a copy kernel writing pinned host outputs that are
                                mapped into the device's address space (other
                                outputs still use the runtime's copies) */
    PW_COPY_OUT_DIRECT = 2,  /* the advection kernel itself writes pinned host
                                outputs mapped into the device's address space
                                (no copy out: the kernel's stores cross PCIe
                                while the next slab comes in; other outputs, and
                                outputs whose planes are not 16-byte aligned for
                                the x-marching kernels, use the runtime's
                                copies) */
    PW_COPY_OUT_AUTO = 3     /* per device, the mode of the three that the
                                outputs allow and that has been fastest: every
                                call is timed with two events on `stream`, and
                                a later call reads the times of the calls that
                                have finished (without waiting), trying each
                                allowed mode first and the others again every
                                eighth call.  Only the speed depends on it: the
                                results are identical in every mode. */
};

/*
 * Forward source terms (section 2.1, Listing 1; section 3, Listing 2).
 * Reads u, v, w (storage arrays with filled x/y halos) and writes su, sv, sw.
 */
int pw_advect_fwd(const void *u, const void *v, const void *w,
                  const double *tzc1, const double *tzc2, double tcx, double tcy,
                  int nx, int ny, int nz, int halo,
                  void *su, void *sv, void *sw, int dtype, void *stream);

/*
 * Adjoint (vector-Jacobian product) of pw_advect_fwd, gather form.
 * For L = sum over interior cells of lu*su + lv*sv + lw*sw, writes into the
 * interior of gu, gv, gw the gradient of L with respect to the interior values
 * of u, v, w of the x/y-periodic problem (halos being copies of interior
 * cells).  u, v, w, lu, lv, lw must all have periodic x/y halos filled.  The
 * fields are read again, not stored from the forward; no atomics are used, so
 * the result is bitwise reproducible.  Multipliers on levels whose source
 * term is identically 0 (level 0; level nz-1 of sw) have no effect.
 */
int pw_advect_adj(const void *u, const void *v, const void *w,
                  const void *lu, const void *lv, const void *lw,
                  const double *tzc1, const double *tzc2, double tcx, double tcy,
                  int nx, int ny, int nz, int halo,
                  void *gu, void *gv, void *gw, int dtype, void *stream);

/*
 * pw_advect_fwd and pw_advect_adj in one pass over the inputs: writes
 * su, sv, sw and gu, gv, gw with the values the two separate calls give.
 */
int pw_advect_fwd_adj(const void *u, const void *v, const void *w,
                      const void *lu, const void *lv, const void *lw,
                      const double *tzc1, const double *tzc2, double tcx, double tcy,
                      int nx, int ny, int nz, int halo,
                      void *su, void *sv, void *sw, void *gu, void *gv, void *gw,
                      int dtype, void *stream);

/*
 * Forward source terms combined with their use later in the timestep (section
 * 2.1: after the dynamical core the source terms are integrated into the flow
 * fields).  Writes, on interior cells,
 *     ou = bu + beta*su,   ov = bv + beta*sv,   ow = bw + beta*sw
 * with su, sv, sw the values pw_advect_fwd gives (they are not stored), the
 * product and the sum each rounded once in the arithmetic type (no fused
 * multiply-add), then rounded to the element type.  z-halo levels of interior
 * columns of o get 0; x/y halo columns of o are not written.  Uses:
 *   accumulate   b = o (the same pointers), beta = 1: adds the advective
 *                tendency to source terms that other schemes already hold;
 *                each element is read before the same thread writes it.
 *   Euler step   b = (u, v, w) (the same pointers), o = new arrays, beta = dt:
 *                u + dt*su in one pass; the kernels reuse the field values they
 *                read, so the call moves the bytes of pw_advect_fwd.
 * Any other b must not overlap an output; o must not overlap u, v, w (their
 * neighbours are still being read).  Errors as for pw_advect_fwd; PW_ERR_ALIAS
 * also for a b array that overlaps an output other than its own.
 */
int pw_advect_fwd_update(const void *u, const void *v, const void *w,
                         const double *tzc1, const double *tzc2, double tcx, double tcy,
                         int nx, int ny, int nz, int halo,
                         const void *bu, const void *bv, const void *bw, double beta,
                         void *ou, void *ov, void *ow, int dtype, void *stream);

/*
 * Forward source terms for fields held in HOST memory: the offload measured in
 * the paper's sections 4 and 5 (winds copied to the accelerator, kernel, source
 * terms copied back), with the transfer cut into x-slabs of `chunk` planes and
 * pipelined as its section 6 proposes: the copy in of one slab, the kernel on
 * the previous slab and the copy out of the one before run concurrently.
 *   u, v, w     host storage arrays (layout above, x/y halos filled);
 *   su, sv, sw  host storage arrays; interior columns are written (interior
 *               levels and zero z halo), x/y halo columns are not;
 *   tzc1, tzc2  DEVICE arrays of nz doubles;
 *   workspace   DEVICE memory of at least pw_offload_workspace_bytes(...)
 *               bytes (three slab buffer sets), owned by the caller.
 * Host arrays should be pinned (hipHostMalloc) for the copies to run
 * asynchronously; pageable memory works but the copies then block the host.
 * The call is asynchronous on `stream`: it starts after the work already queued
 * there, and work queued there afterwards sees every result.  Kernels run on
 * `stream`; the copies use two streams the library creates once per device and
 * keeps until the process ends (default priority).  Inputs go in through the
 * runtime's host-to-device copies, outputs come back through the runtime's
 * device-to-host copies, a copy kernel of the library or the advection kernel
 * itself writing pinned outputs mapped into the device's address space, as
 * PW_TUNE_COPY_OUT selects (by default the fastest of these measured on the
 * device, PW_COPY_OUT_AUTO).  Concurrent calls are
 * serialized while they are queued.  Results are identical to pw_advect_fwd on
 * the same data.  Errors as for pw_advect_fwd; PW_ERR_ARG if a field array is
 * device memory, PW_ERR_SIZE if the workspace is too small.
 */
size_t pw_offload_workspace_bytes(int nx, int ny, int nz, int halo, int dtype, int chunk);
int pw_advect_fwd_host(const void *u, const void *v, const void *w,
                       const double *tzc1, const double *tzc2, double tcx, double tcy,
                       int nx, int ny, int nz, int halo,
                       void *su, void *sv, void *sw,
                       int chunk, void *workspace, size_t workspace_bytes, int dtype, void *stream);

/*
 * pw_advect_fwd_host without a workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the three slab buffer sets live in a static scratch
 * array of the library, pw_static_scratch_bytes() bytes (128 MiB) on each
 * device the library runs on, held from module load until the process ends.
 * Arguments, results and errors as for pw_advect_fwd_host, except that
 * PW_ERR_SIZE means pw_offload_workspace_bytes(nx, ny, nz, halo, dtype,
 * chunk) exceeds the static scratch (choose a smaller chunk).  The first call
 * on a device looks up that device's address of the scratch and creates the
 * copy streams and events (set-up); no call allocates device memory.  Calls
 * on one device share its scratch, which keeps the last call's slabs: the
 * library starts each call after the last copy out of the offload call
 * queued before it on that device, so such calls never overlap.
 */
size_t pw_static_scratch_bytes(void);
int pw_advect_fwd_host_static(const void *u, const void *v, const void *w,
                              const double *tzc1, const double *tzc2, double tcx, double tcy,
                              int nx, int ny, int nz, int halo,
                              void *su, void *sv, void *sw,
                              int chunk, int dtype, void *stream);

/*
 * Periodic halo fill in place (the halo swap that precedes advection in each
 * timestep, section 2.1, for a domain that is periodic in x and y): copies
 * whole storage columns so that storage column (i, j) for i or j outside the
 * interior equals interior column (i mod nx, j mod ny), z-halo levels
 * included.  Interior columns are not written.
 */
int pw_halo_periodic(void *storage, int nx, int ny, int nz, int halo, int dtype, void *stream);

/*
 * Builds a storage array from a compact interior array (nx, ny, nz) (C order,
 * same element type): interior columns get the interior values and 0 in their
 * z-halo levels, halo columns get their periodic images.  `interior` and
 * `storage` must not overlap.
 */
int pw_pad_periodic(const void *interior, void *storage, int nx, int ny, int nz, int halo,
                    int dtype, void *stream);

/*
 * Input generator (not part of the scheme): writes interior columns of a
 * storage array with amp * t, where t in [-1, 1) is the SplitMix64
 * counter-based uniform of Steele, Lea and Flood (OOPSLA 2014) for seed
 * `seed`, stream `field_id` and counter = interior linear index
 * (i*ny + j)*nz + k:  z = mix(seed*256 + field_id + (counter+1)*0x9E3779B97F4A7C15),
 * t = ((z >> 11) - 2^52) * 2^-52, value = amp * t rounded to double, then to
 * float for the float-storage dtypes, then to the 16-bit type for PW_F16 and
 * PW_BF16 (each step rounds to nearest even).  With zero_lids != 0 levels 0
 * and nz-1 are 0.
 * z-halo levels are set to 0; x/y halo columns are not written.
 */
int pw_fill_uniform(void *storage, int nx, int ny, int nz, int halo,
                    unsigned long long seed, int field_id, double amp, int zero_lids,
                    int dtype, void *stream);

/*
 * Measurement utility (not part of the scheme): one launch of a plain
 * streaming copy kernel that copies src[q] to dst[q] for q < narrays, each
 * `bytes` long, in units of `unit` bytes (4, 8 or 16), every thread reading
 * its unit of all sources before writing it to all destinations.  It moves
 * the streams of the advection calls over arrays of the same size (3 arrays:
 * the forward's 3 reads and 3 writes; 6 arrays: those of pw_advect_fwd_adj)
 * and so is the achievable-bandwidth reference their rate is read against.
 * src and dst are HOST arrays of narrays device pointers, each aligned to the
 * unit; bytes must be a multiple of the unit; 1 <= narrays <= 8; no
 * destination may overlap any array.  blocks = 0 launches one 256-thread
 * workgroup per 256 units of each array (each thread copies one unit per
 * array; the unit count must stay below 2^32), blocks > 0 launches that many
 * workgroups striding over the arrays.  `hints` is 0 or an OR of
 * PW_COPY_NT_LOADS and PW_COPY_NT_STORES: the non-temporal (streaming) cache
 * policy on the loads and/or the stores.  A copy reads and writes every byte
 * once, and on MI355X the hints make it faster (the FP64 storage arrays of a
 * 4096 x 4096 x 64 grid with halo 2: three arrays 8.09 ms with streaming
 * loads against 8.49 ms, six 16.38 ms with both against 17.49 ms); the
 * advection kernels, whose strips re-read their neighbours' edge columns
 * through the caches, are fastest without them.  Asynchronous on `stream`.
 * Errors: PW_ERR_ARG, PW_ERR_ALIGN, PW_ERR_ALIAS, PW_ERR_SIZE, PW_ERR_HIP.
 */
enum { PW_COPY_NT_LOADS = 1, PW_COPY_NT_STORES = 2 };
int pw_stream_copy(const void *const *src, void *const *dst, int narrays, size_t bytes, int unit, int blocks,
                   int hints, void *stream);

/*
 * Sets tuning knob `knob` (PW_TUNE_*) of the calling thread to `value`: the
 * setting applies to the calls this thread makes afterwards and to no other
 * thread.  Returns PW_OK, or PW_ERR_ARG (nothing changed) for an unknown knob
 * or value.  pw_get_tuning stores the thread's current value in *value.
 * pw_set_kernel sets PW_TUNE_KERNEL and returns the previous selection (a
 * PW_KERNEL_* value) or PW_ERR_ARG; pw_get_kernel returns the selection.
 */
int pw_set_tuning(int knob, int value);
int pw_get_tuning(int knob, int *value);
int pw_set_kernel(int kernel);
int pw_get_kernel(void);

/* Message for the last non-zero return on the calling thread ("" if none). */
const char *pw_last_error(void);

/* Library version: major*10000 + minor*100 + patch. */
int pw_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PWADVECT_H */
