/*
 * mhd.h — C ABI of the MI355X (gfx950) ideal-MHD step library (libmhd.so).
 *
 * The library advances the conserved variables of ideal MHD,
 *     dU/dt + div T(U) = 0,  U = (rho, rho v, B, E)              (paper Sec. 2.1,
 *     E = p/(Gamma-1) + rho v^2/2 + B^2/2                        Eqs. cons_law, mhd, Energy)
 * on a uniform, periodic Cartesian mesh with the semi-discrete finite-volume
 * form of Sec. 2.2, Eq. (FV): primitive recovery (Sec. 2.2, inversion after
 * Eq. reconstruct), piecewise-linear limited reconstruction (Eq. reconstruct),
 * an HLLD or HLL Riemann flux at every interface (Sec. 2.2 flux equation;
 * HLLD as cited for Secs. 4.1-4.2), an upwind constrained-transport EMF on
 * cell edges that keeps div B at round-off (Sec. 2.2, CT), and a two-stage
 * SSP Runge-Kutta step (Sec. 2.2, the SSP family of Eq. RK3).
 *
 * State layout (every call): one contiguous device buffer of 8*nz*ny*nx
 * doubles, field-major, x fastest: element (f,k,j,i) at ((f*nz+k)*ny+j)*nx+i.
 * Fields: 0 rho, 1 m_x, 2 m_y, 3 m_z, 4 E, 5 b_x, 6 b_y, 7 b_z. b_d is the
 * normal field on the LOWER d-face of the cell (b_x(i) at x_{i-1/2}); the face
 * at x_{-1/2} is the periodic image of x_{nx-1/2}. In 2D (nz == 1) field 7 is
 * the cell-centred B_z.
 *
 * Ownership: the caller owns every device buffer (state, adjoint arrays and the
 * workspace `ws` of `ws_bytes` >= mhd_workspace_bytes() bytes, 256-byte
 * aligned; its contents need no initialisation except that the first 256
 * bytes must be zero before the first call). The library allocates no
 * device memory and keeps no device pointer between calls; a context holds
 * host-side metadata only. Work is enqueued on the HIP stream given as
 * `stream` (a hipStream_t; NULL = the default stream). Only calls that return
 * a host value computed on the device (mhd_dt, mhd_check) synchronise.
 * A context is used by one host thread at a time; calls on one workspace must
 * not overlap.
 *
 * Errors: every call returns an mhd_status. MHD_ERR_DEVICE carries the HIP
 * error text in mhd_last_error(). Kernels never abort: a cell with rho <= 0,
 * p <= 0 or a non-finite value raises a sticky flag in the workspace that
 * mhd_dt / mhd_check report as MHD_ERR_UNPHYSICAL (and clear). No floors are
 * applied.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MHD_OK = 0,
  MHD_ERR_INVALID = -1,      /* bad configuration, size, pointer or dt */
  MHD_ERR_UNSUPPORTED = -2,  /* combination not built into this library */
  MHD_ERR_DEVICE = -3,       /* HIP runtime / launch failure (see mhd_last_error) */
  MHD_ERR_UNPHYSICAL = -4,   /* rho <= 0, p <= 0 or non-finite value met */
  MHD_ERR_WORKSPACE = -5     /* workspace missing or too small */
} mhd_status;

/* Reconstruction: PLM with the minmod or van Leer limiter, or fifth-order
 * WENO-Z (Borges et al. 2008, cited with Eq. (reconstruct); FP64 only, with van
 * Leer PLM for the CT edge values; the adjoint does not support it). */
typedef enum { MHD_LIM_MINMOD = 0, MHD_LIM_VANLEER = 1, MHD_LIM_WENOZ = 2 } mhd_limiter;
typedef enum { MHD_RS_HLLD = 0, MHD_RS_HLL = 1 } mhd_riemann;
/* MHD_PREC_MIXED: reconstruction, Riemann solve and EMF in FP32; primitive
 * recovery (incl. pressure), flux/curl differencing, the RK combination and
 * the time step in FP64. The state is FP64 in both modes. */
typedef enum { MHD_PREC_FP64 = 0, MHD_PREC_MIXED = 1 } mhd_precision;
/* Time integrator: the two-stage SSP Runge-Kutta scheme, or the three-stage
 * one of Sec. 2.2 Eq. (RK3) (Shu & Osher). */
typedef enum { MHD_SSP_RK2 = 0, MHD_SSP_RK3 = 1 } mhd_integrator;
/* Edge EMF of constrained transport (Sec. 2.2, CT; the runs of Secs. 4.1-4.2
 * use the UCT-HLLD average, whose formulas the paper does not print):
 * MHD_EMF_UCT_HLL, an upwind average whose weights are the HLL wave-speed
 * bounds of the faces touching the edge (maximised over the two faces);
 * MHD_EMF_UCT_HLLD, an upwind average whose weights and diffusion
 * coefficients are those of the face's Riemann flux of the transverse field
 * (averaged over the two faces), so that with HLLD fluxes and plane-parallel
 * data the EMF is minus the HLLD flux of the transverse field. The adjoint
 * supports MHD_EMF_UCT_HLL only. */
typedef enum { MHD_EMF_UCT_HLL = 0, MHD_EMF_UCT_HLLD = 1 } mhd_emf;
/* Control of div B (Sec. 2.1 lists divergence cleaning beside CT; the
 * strong-scaling runs of Secs. 4.1-4.2 use it): MHD_DIVB_CT, the staggered
 * field with constrained transport; MHD_DIVB_GLM, the mixed GLM cleaning of
 * Dedner et al. (2002) on a cell-centred field with a ninth field psi:
 *   dB/dt + div(vB - Bv) + grad psi = 0,  dpsi/dt + c_h^2 div B = damping,
 * with the (B_n, psi) face problem solved exactly, c_h = C Delta_min / dt (the
 * largest speed the step's dt allows) and psi multiplied by
 * exp(-alpha c_h dt / Delta_min), alpha = 0.1, after each step. With GLM the
 * state holds NINE fields, 9*nz*ny*nx doubles in the order rho, m_x, m_y,
 * m_z, E, B_x, B_y, B_z, psi, all cell-centred; emf must be MHD_EMF_UCT_HLL
 * (it is not used). mhd_rhs, the adjoint and mhd_dt_device_noalloc return
 * MHD_ERR_UNSUPPORTED with GLM. */
typedef enum { MHD_DIVB_CT = 0, MHD_DIVB_GLM = 1 } mhd_divb;

typedef struct {
  int32_t dim;                  /* 2 or 3 */
  int32_t nx, ny, nz;           /* cells per direction; nz == 1 when dim == 2; each >= 4 otherwise;
                                   at most 4e9 cells, and in 3D fewer than 2^29 per x-y plane */
  double xmin, xmax, ymin, ymax, zmin, zmax;  /* periodic box (max > min) */
  double gamma;                 /* adiabatic index, > 1 */
  double cfl;                   /* Courant number C > 0: dt = C min_d,cells dx_d/(|v_d|+c_f,d) */
  int32_t limiter;              /* mhd_limiter */
  int32_t riemann;              /* mhd_riemann */
  int32_t precision;            /* mhd_precision */
  int32_t integrator;           /* mhd_integrator (0, the former reserved field, is SSP-RK2) */
  int32_t emf;                  /* mhd_emf (0: MHD_EMF_UCT_HLL) */
  int32_t divb;                 /* mhd_divb (0: MHD_DIVB_CT) */
} mhd_config;

typedef struct mhd_ctx mhd_ctx;

/* Validate cfg and create a host-side context. No device work.
 * Returns MHD_ERR_INVALID for a bad cfg or null out; *out is set on success. */
mhd_status mhd_init(const mhd_config* cfg, mhd_ctx** out);

/* Release a context (NULL is ignored). */
void mhd_destroy(mhd_ctx* ctx);

/* Bytes of device workspace the calls below need (with_adjoint != 0: enough
 * for mhd_adjoint_step as well). 256-byte alignment is required. */
size_t mhd_workspace_bytes(const mhd_ctx* ctx, int32_t with_adjoint);

/* Time step of the state U (CFL condition; the paper gives no formula, so
 * this is the usual one for ideal MHD): dt = C min over cells and directions d of
 * dx_d / (|v_d| + c_f,d), with c_f,d the fast magnetosonic speed along d.
 * Writes the host double *dt_out; synchronises the stream. Reports (and
 * clears) the unphysical flag as MHD_ERR_UNPHYSICAL, still writing dt. */
mhd_status mhd_dt(mhd_ctx* ctx, const double* U, void* ws, size_t ws_bytes, double* dt_out,
                  void* stream);

/* Same time step, written to the device double *dt_dev; no synchronisation. */
mhd_status mhd_dt_device(mhd_ctx* ctx, const double* U, void* ws, size_t ws_bytes, double* dt_dev,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the time step of
 * mhd_dt_device (the same value, bit for bit) without a workspace. Its
 * scratch, the per-block partials of the reduction (at most 2048 doubles)
 * and the unphysical flag, is a file-scope device array of 16.6 KB that each
 * GPU the library runs on holds until the process ends; the library finds
 * its address on the first call made with a device current. The reduction
 * strides over the grid, so every grid mhd_init accepts fits. The caller
 * passes U and the device double *dt_dev; *flag_dev (a device int32, NULL
 * to skip) receives 1 if a cell of U had rho <= 0, p <= 0 or a non-finite
 * value in this call, else 0 (unlike the workspace flag, it is not sticky).
 * No allocation, no host synchronisation; the current device must be the one
 * that holds U and the stream. Calls that overlap on one GPU share the array
 * and race: serialise them (one stream, or events). MHD_ERR_INVALID for a
 * null ctx, U or dt_dev; MHD_ERR_DEVICE if the array's address cannot be
 * found or a launch fails. */
mhd_status mhd_dt_device_noalloc(mhd_ctx* ctx, const double* U, double* dt_dev,
                                 int32_t* flag_dev, void* stream);

/* One step of size dt, in place. SSP-RK2:
 *   U1 = U + dt L(U);  U <- (U + (U1 + dt L(U1))) / 2;
 * SSP-RK3 (Sec. 2.2 Eq. (RK3), read as the Shu-Osher scheme):
 *   U1 = U + dt L(U);  U2 = (3 U + (U1 + dt L(U1))) / 4;
 *   U <- (U + 2 (U2 + dt L(U2))) / 3,
 * with L the finite-volume right-hand side (Eq. FV) for the cell fields and
 * -curl E on the faces for the staggered field. dt must be > 0 and finite. */
mhd_status mhd_step(mhd_ctx* ctx, double* U, double dt, void* ws, size_t ws_bytes, void* stream);

/* As mhd_step with dt read on the device from *dt_dev (a device double, e.g.
 * written by mhd_dt_device); no host synchronisation. */
mhd_status mhd_step_device_dt(mhd_ctx* ctx, double* U, const double* dt_dev, void* ws,
                              size_t ws_bytes, void* stream);

/* One step of the configured integrator whose dt is the CFL time step of U
 * (as mhd_dt computes it, bit for bit), written to the device double *dt_dev
 * and used by the step; no host synchronisation. The CFL reduction runs
 * inside the first stage's face kernel (in 3D with WENO-Z, its primitive
 * kernel; with GLM, the GLM primitive kernel) instead of as a separate pass
 * over U, except in 2D with WENO-Z, which keeps the separate pass. */
mhd_status mhd_step_cfl(mhd_ctx* ctx, double* U, double* dt_dev, void* ws, size_t ws_bytes,
                        void* stream);

/* Right-hand side L(U) of the semi-discrete equations for all eight stored
 * fields (same layout as U), without time integration. U and L must not
 * alias. */
mhd_status mhd_rhs(mhd_ctx* ctx, const double* U, double* L, void* ws, size_t ws_bytes,
                   void* stream);

/* Adjoint (vector-Jacobian product) of one mhd_step of size dt at the state
 * U_n (left unchanged): Ubar_n = (dPhi/dU_n)^T Ubar_np1 and, if dtbar is
 * non-NULL, the host double *dtbar = (dPhi/d dt)^T Ubar_np1 (this one
 * synchronises). Not part of the paper: the derivative of every
 * non-smooth point (limiter at extrema, min/max, Riemann region switches) is
 * that of the branch the forward step takes. FP64, PLM and MHD_EMF_UCT_HLL,
 * with either integrator (MHD_ERR_UNSUPPORTED otherwise). Ubar_n must not
 * alias Ubar_np1 or U_n. Needs mhd_workspace_bytes(ctx, 1). */
mhd_status mhd_adjoint_step(mhd_ctx* ctx, const double* U_n, double dt, const double* Ubar_np1,
                            double* Ubar_n, double* dtbar, void* ws, size_t ws_bytes,
                            void* stream);

/* As mhd_adjoint_step, with dt-bar written to the device double *dtbar_dev
 * (NULL: not computed) and no host synchronisation, for loops over many
 * steps (the checkpointed N-step gradient). */
mhd_status mhd_adjoint_step_device(mhd_ctx* ctx, const double* U_n, double dt,
                                   const double* Ubar_np1, double* Ubar_n, double* dtbar_dev,
                                   void* ws, size_t ws_bytes, void* stream);

/* Synchronise the stream and report (and clear) the unphysical flag. */
mhd_status mhd_check(mhd_ctx* ctx, void* ws, size_t ws_bytes, void* stream);

/* Measurement support (not part of the method): enable != 0 turns on
 * per-kernel timing for this context — every kernel launch of later calls is
 * bracketed by a pair of HIP events on the call's stream — and resets the
 * totals; enable == 0 turns it off. */
mhd_status mhd_timing(mhd_ctx* ctx, int32_t enable);

/* Read the timing totals of kernel index `kernel` (0, 1, ... until
 * MHD_ERR_INVALID): its name, the summed event time in ms and the number of
 * launches. Waits for the recorded events (synchronises). */
mhd_status mhd_timing_read(mhd_ctx* ctx, int32_t kernel, const char** name, double* total_ms,
                           int64_t* launches);

/* Static text of a status code. */
const char* mhd_strerror(mhd_status s);

/* Text of the last failure on this context ("" if none). */
const char* mhd_last_error(const mhd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MHD_H */
