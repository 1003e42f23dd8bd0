/*
 * qpinn.h - C ABI of the MI355X (gfx950) QPINN circuit engine.
 *
 * The library evaluates, for every collocation point p = (t, x, y), a parametrised quantum
 * circuit as a statevector and returns
 *   - the readouts  f_i(p) = <Z_i>            (section "QPINN architecture and ansatz designs":
 *                                              one Pauli-Z expectation per output qubit),
 *   - the input tangents g_ic(p) = d f_i / d c for c in (t, x, y), by forward-mode tangent
 *     statevectors (the derivatives the Maxwell residuals need),
 *   - the gradient of a loss with respect to the circuit parameters, by an adjoint sweep that
 *     walks the circuit backwards and uncomputes each gate with its inverse instead of storing
 *     intermediate states.
 * The fused entry point evaluates the TE_z Maxwell residual loss (section "PINN architecture
 * and convergence enhancements": eqs. residual_1_vac, residual_1_diel, residuals_2_and_3,
 * phys_loss_vac, phys_loss_diel, mse; section "Stabilizing the dielectric test case":
 * eq. residual_1_intuitive) and its parameter gradient in one call.
 *
 * Conventions (fixed by this library; the paper leaves them open):
 *   - R_P(theta) = exp(-i theta P / 2) for P in {X, Y, Z};
 *   - qubit 0 is the most significant bit of a basis index (leftmost Kronecker factor);
 *   - points are row-major float32 [P][3] with columns (t, x, y);
 *   - outputs are float32 [P][m], tangents float32 [P][m][3] (m = number of output qubits);
 *     the first three outputs are the fields (E_z, H_x, H_y) for the Maxwell loss.
 *
 * Memory and ownership:
 *   - every device pointer argument is caller-owned device memory on the context's device;
 *   - descriptors are copied during the call; the caller may free them afterwards;
 *   - per-call scratch lives in a caller-provided workspace (size from the *_workspace_bytes
 *     query, 256-byte aligned).  Compiling a circuit or a batch uploads its execution plan
 *     once into a small device buffer owned by the returned object; evaluation calls allocate
 *     no device memory.
 *
 * Execution: calls are asynchronous and ordered on the context's HIP stream.  Errors found on
 * the host are returned as status codes (no exceptions or aborts cross this boundary) with a
 * message from qp_last_error(); asynchronous device errors surface at a later call or at
 * qp_sync().  Reductions run in a fixed order, so repeated calls give bitwise equal results.
 * Arithmetic: complex64 state, FP32 accumulation per point and per workgroup; the final
 * cross-workgroup loss and gradient reductions run in FP64.
 */
#ifndef QPINN_H
#define QPINN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum qp_status {
  QP_OK = 0,
  QP_EINVAL = 1,        /* null pointer, bad enum, bad gate operand, P < 0 */
  QP_ESHAPE = 2,        /* sizes inconsistent with the circuit (e.g. fewer than 3 outputs for Maxwell) */
  QP_EUNSUPPORTED = 3,  /* valid request outside this build's range (qubit count, gate kind, P) */
  QP_EWORKSPACE = 4,    /* workspace missing, too small or misaligned */
  QP_EDEVICE = 5        /* HIP runtime error */
} qp_status;

/* Gate kinds.  Rotations take one parameter (param = index into the parameter vector). */
enum { QP_RX = 0, QP_RY = 1, QP_RZ = 2, QP_CNOT = 3, QP_CZ = 4, QP_CRZ = 5 };
/* Encodings (section "QPINN architecture": angle embedding; section "PINN architecture":
 * random Fourier features). */
enum { QP_ENC_CYCLE = 0, QP_ENC_ANGLES = 1, QP_ENC_RFF = 2 };
enum { QP_ENC_RY = 0, QP_ENC_RX = 1 };
/* Input scalings of eq. scale: a, pi a, (a+1) pi/2, asin(a) + pi/2, acos(a). */
enum { QP_SCALE_NONE = 0, QP_SCALE_PI = 1, QP_SCALE_BIAS = 2, QP_SCALE_ASIN = 3, QP_SCALE_ACOS = 4 };
/* Maxwell residual losses: vacuum (eq. phys_loss_vac), split dielectric (eq. phys_loss_diel),
 * intuitive dielectric (eq. phys_loss_intuitive). */
enum { QP_LOSS_VACUUM = 0, QP_LOSS_DIEL_SPLIT = 1, QP_LOSS_DIEL_INTUITIVE = 2 };

/* Flags (bitwise or). */
#define QP_FLAG_NO_TANGENTS 0x1u  /* qp_simulate: tangents not needed (tan may be NULL)      */
#define QP_FLAG_LOSS_SUM    0x2u  /* Maxwell: sum of squared residuals instead of MSE means  */
#define QP_FLAG_TUNE        0x4u  /* Maxwell and batch calls: time the candidate launch shapes
                                     on first use and cache the fastest; for the fused Maxwell
                                     call the candidates also include the dense-block path when
                                     the circuit has one and the workspace covers it
                                     (qp_workspace_bytes with this flag); the first tuned call
                                     per point-count bucket waits for the stream (HIP events), so
                                     it must not run under graph capture                        */
#define QP_FLAG_DENSE_MFMA  0x8u  /* force the dense-block MFMA path (where the plan has one) */
#define QP_FLAG_GATES_FP32  0x10u /* build the 2x2 gate table in FP32 instead of FP64-rounded  */

typedef struct qp_ctx qp_ctx;
typedef struct qp_circuit qp_circuit;
typedef struct qp_batch qp_batch;

typedef struct qp_gate {
  int32_t kind;   /* QP_RX..QP_CRZ                                          */
  int32_t q0;     /* rotation target, or control of CNOT/CRZ, first qubit of CZ */
  int32_t q1;     /* target of CNOT/CRZ, second qubit of CZ; ignored otherwise */
  int32_t param;  /* parameter index for rotations (and CRZ); ignored otherwise */
} qp_gate;

typedef struct qp_encoding {
  int32_t kind;                   /* QP_ENC_*                                             */
  int32_t gate;                   /* QP_ENC_RY or QP_ENC_RX: rotation applied to |0>       */
  int32_t scale;                  /* QP_SCALE_* (QP_ENC_CYCLE only)                       */
  int32_t n_features;             /* QP_ENC_RFF: number of frequencies F                  */
  const int32_t* coord_of_qubit;  /* QP_ENC_CYCLE: host [n] in {0,1,2}, or NULL for q mod 3 */
  const float* rff_B;             /* QP_ENC_RFF: host [F][3] frequencies                  */
  const float* rff_W;             /* QP_ENC_RFF: host [n][2F] map [cos(Bp); sin(Bp)] -> angles */
} qp_encoding;

typedef struct qp_circuit_desc {
  int32_t n_qubits;               /* 3..12 for the fused paths, 1..14 for the plain path  */
  int32_t n_params;               /* K                                                    */
  int32_t n_gates;
  const qp_gate* gates;           /* host [n_gates], time order                          */
  qp_encoding enc;
  int32_t n_out;                  /* m, 1..8                                              */
  const int32_t* out_qubits;      /* host [m]                                             */
} qp_circuit_desc;

typedef struct qp_maxwell_desc {
  int32_t kind;                   /* QP_LOSS_*                                            */
  float eps_r;                    /* relative permittivity of the dielectric half (4)     */
  float x_interface;              /* eps = eps_r where x >= x_interface                   */
} qp_maxwell_desc;

/* ---- context ---------------------------------------------------------------------------
 * qp_ctx_create: binds the calling thread's work to `device` and the HIP stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  One context per stream; not thread-safe.        */
qp_status qp_ctx_create(int device, void* hip_stream, qp_ctx** out);
qp_status qp_ctx_set_stream(qp_ctx* ctx, void* hip_stream);
void qp_ctx_destroy(qp_ctx* ctx);
const char* qp_last_error(const qp_ctx* ctx);
qp_status qp_sync(qp_ctx* ctx);   /* waits for the stream; reports asynchronous device errors */
int32_t qp_device_cu_count(const qp_ctx* ctx);
/* Kernel timing: when enabled, the next fused or batch calls record HIP events on the context
 * stream immediately around their main (per-point) kernel; qp_ctx_last_kernel_ms waits for the
 * second event and returns the elapsed time of the most recent such kernel in milliseconds.  */
qp_status qp_ctx_enable_kernel_timing(qp_ctx* ctx, int32_t on);
qp_status qp_ctx_last_kernel_ms(qp_ctx* ctx, float* ms);

/* ---- circuits --------------------------------------------------------------------------
 * qp_circuit_compile validates the descriptor, fuses consecutive rotations on a qubit into
 * one 2x2 gate, turns runs of CNOT/CZ gates into index permutations with sign functions,
 * schedules the register/LDS rounds and uploads the plan.  Errors: QP_EINVAL (bad operand),
 * QP_EUNSUPPORTED (n outside 3..12 for fused evaluation is reported at evaluation time).     */
qp_status qp_circuit_compile(qp_ctx* ctx, const qp_circuit_desc* desc, qp_circuit** out);
void qp_circuit_destroy(qp_circuit* c);
/* what: 0 n_qubits, 1 n_params, 2 n_out, 3 fused gates, 4 rounds, 5 register-exchange count,
 *       6 threads per workgroup of the fused kernel, 7 points per workgroup tile,
 *       8 LDS exchange planes, 9 persistent workgroups per CU, 10 dense 2^5 blocks,
 *       11 leading rounds folded into the encoding (an opening rotation stage acts on the
 *       product state), 12 fused gates in those rounds, 13 fusion width chosen by the tuner
 *       for Maxwell calls (1: dense 32x32 blocks, 0: 2x2 gates in the fused kernel).  -1 for
 *       an unknown code.                                                                     */
int64_t qp_circuit_info(const qp_circuit* c, int32_t what);

/* Launch shape of the fused kernel for this circuit (what the autotuner sets): exchange_planes
 * 4 = software-pipelined exchanges over two plane pairs, 2 = one plane pair, unpipelined;
 * wg_per_cu = persistent workgroups per CU, 1 at 12 qubits, 1..4 below (above 2 the grid runs
 * in two generations).  The choice changes speed, not results beyond rounding order.
 * QP_EINVAL for other values or a shape whose LDS does not fit a CU.  Circuit compilation
 * applies a choice cached by an earlier tuned run (QP_TUNE_CACHE) for the same circuit shape,
 * the fusion width included; setting a launch shape here puts Maxwell calls back on the fused
 * kernel.                                                                                   */
qp_status qp_circuit_set_launch(qp_circuit* c, int32_t exchange_planes, int32_t wg_per_cu);

/* Points per chunk of the dense-block MFMA path (QP_FLAG_DENSE_MFMA), which streams the
 * statevectors of one chunk of points through HBM at a time: 0 (default) sizes a chunk to about
 * 2 GiB of statevectors; a smaller positive multiple of 64 caps it (more chunks, less workspace).
 * Results do not depend on it beyond rounding order.  QP_EINVAL for other values.            */
qp_status qp_circuit_set_dense_chunk(qp_circuit* c, int32_t points);

/* Host-only introspection: builds the execution plan of `desc` without a device and copies its
 * device image (header, rounds, exchange descriptors, fused gates, gradient map) into host_buf
 * (capacity cap bytes); *bytes receives the image size.  QP_EWORKSPACE if cap is too small.  */
qp_status qp_plan_image(const qp_circuit_desc* desc, void* host_buf, size_t cap, size_t* bytes);

/* Workspace bytes for qp_simulate / qp_vjp / qp_maxwell_fused with P points and `flags`.  With
 * QP_FLAG_TUNE, or once the tuner chose the dense-block path for this circuit, the size also
 * covers that path; a call accepts any workspace that covers the path it must take (the fused
 * kernel's, or the dense path's with QP_FLAG_DENSE_MFMA) and then keeps Maxwell calls on the
 * fused kernel when the dense path does not fit.                                            */
size_t qp_workspace_bytes(const qp_circuit* c, int64_t P, uint32_t flags);

/* ---- evaluation ------------------------------------------------------------------------
 * points [P][3] (read for QP_ENC_CYCLE and QP_ENC_RFF; may be NULL for QP_ENC_ANGLES unless a
 * dielectric loss needs x), angles [P][n] and jac [P][n][3] (QP_ENC_ANGLES only, else NULL).
 * P = 0 is valid and does nothing except zeroing reduced outputs; P above 2^31 - 1 returns
 * QP_EUNSUPPORTED (point indices are 32-bit on the device; split such a call).             */

/* Forward: out [P][m]; tan [P][m][3] unless QP_FLAG_NO_TANGENTS.  Without tangents the fused
 * kernel runs packed (four points in the four statevector slots of a thread group: about a
 * quarter of the cost per point; the outputs equal those of the tangent-carrying kernel).  */
qp_status qp_simulate(qp_ctx* ctx, const qp_circuit* c, const float* params,
                      const float* points, const float* angles, const float* jac, int64_t P,
                      float* out, float* tan, void* ws, size_t ws_bytes, uint32_t flags);

/* Vector-Jacobian product of the scalar s = sum_p [sum_i d_out[p,i] f_i + sum_ic d_tan[p,i,c] g_ic]:
 *   d_params[k] = ds/dtheta_k  ([K]);
 * and, for the angle-given encoding (QP_ENC_ANGLES: the inputs a classical layer in front of the
 * circuit produces, section "QPINN architecture and ansatz designs", angle embedding),
 *   d_angles[p][q] = ds/d angles[p][q]  ([P][n], or NULL),
 *   d_jac[p][q][c] = ds/d jac[p][q][c]  ([P][n][3], or NULL),
 * so that the gradient flows on into that layer.  d_out or d_tan may be NULL (treated as zero).
 * Recomputes the forward internally.  d_angles/d_jac with another encoding: QP_EINVAL; with
 * QP_FLAG_DENSE_MFMA: QP_EUNSUPPORTED.                                                       */
qp_status qp_vjp(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                 const float* angles, const float* jac, int64_t P, const float* d_out,
                 const float* d_tan, float* d_params, float* d_angles, float* d_jac, void* ws,
                 size_t ws_bytes, uint32_t flags);

/* Fused Maxwell evaluation: forward + tangents + residual loss + adjoint gradient in one
 * stream-ordered call.  out/tan may be NULL.  loss: one double (device); d_params: [K];
 * d_angles [P][n] / d_jac [P][n][3]: the loss gradient with respect to the per-point angles and
 * their Jacobian (QP_ENC_ANGLES only, as for qp_vjp), or NULL.                               */
qp_status qp_maxwell_fused(qp_ctx* ctx, const qp_circuit* c, const float* params,
                           const float* points, const float* angles, const float* jac,
                           int64_t P, const qp_maxwell_desc* loss_desc, float* out, float* tan,
                           double* loss, float* d_params, float* d_angles, float* d_jac, void* ws,
                           size_t ws_bytes, uint32_t flags);

/* ---- the paper's total loss -------------------------------------------------------------
 * L_tot = L_phys + w_ic L_IC + w_sym L_sym + w_energy L_energy (eq. 2D_lossTot; the paper's
 * weights are 10, 10, 10) with
 *   L_phys   the residual loss of the collocation points X (as qp_maxwell_fused, means),
 *   L_IC     mean over the initial-condition plane X_0 = {(0, x, y)} of (E_z - E_0)^2 + H_x^2 +
 *            H_y^2, E_0 = exp(-ic_a (x^2 + y^2)) (eqs. pulse_IC_Ez, pulse_IC_Hx, pulse_IC_Hy,
 *            IC_loss; ic_a = 25),
 *   L_sym    mean over X of the parity defects of eq. 2D_symLoss, evaluated at the mirror images
 *            (t, -x, y) and (t, x, -y); the x-mirror terms are left out for the dielectric losses,
 *   L_energy mean over X of the squared local Poynting residual
 *            eps E dE/dt + Hx dHx/dt + Hy dHy/dt - (dE/dx Hy + E dHy/dx) + (dE/dy Hx + E dHx/dy)
 *            (eqs. Poynting_thm, Poynting_value_u, Poynting_value_S, energy_loss).
 * The mirror images couple points, so the call runs stream-ordered phases over the set
 * [X; X_my; X_mx (vacuum); X_0]: the outputs of the mirrored and initial-condition points (whose
 * terms use the fields alone; packed four to a thread group); one fused pass over X (forward
 * with tangents, the residual, energy and symmetry seeds formed in the kernel from the point's
 * fields and its images' outputs, adjoint); the four terms and the seeds of the mirrored and
 * initial-condition points; their adjoint (packed).  points [P][3] (t, x, y) and ic_xy [P0][2]
 * (x, y) are device buffers; out [P][m] and tan
 * [P][m][3] (of X, may be NULL); loss_terms: device double [5] = total, phys, IC, sym, energy;
 * d_params [K].  Point encodings only (cycled or random Fourier features): QP_EINVAL for the
 * angle-given encoding.  Flags: only QP_FLAG_GATES_FP32 (others: QP_EUNSUPPORTED).          */
typedef struct qp_total_loss_desc {
  qp_maxwell_desc phys;
  float w_ic, w_sym, w_energy;    /* weights of eq. 2D_lossTot (10, 10, 10)                 */
  float ic_a;                     /* initial pulse exp(-ic_a (x^2 + y^2)) (25)              */
} qp_total_loss_desc;
size_t qp_total_workspace_bytes(const qp_circuit* c, int64_t P, int64_t P0, int32_t phys_kind);
qp_status qp_total_loss(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* points,
                        int64_t P, const float* ic_xy, int64_t P0, const qp_total_loss_desc* desc,
                        float* out, float* tan, double* loss_terms, float* d_params, void* ws,
                        size_t ws_bytes, uint32_t flags);

/* ---- diagnostics of the "black hole" study --------------------------------------------
 * (section "'Black hole' loss landscape")
 * qp_bloch: for every point, the Bloch vector r_k = (<X_k>, <Y_k>, <Z_k>) of every qubit of the
 * circuit's output state, bloch [P][n][3], and the global Meyer-Wallach entanglement
 *   Q = 2 (1 - (1/n) sum_k Tr rho_k^2) = 1 - (1/n) sum_k |r_k|^2   (rho_k = (I + r_k . sigma) / 2),
 * mw [P] (or NULL): 0 for product states, 1 for GHZ states.  Evaluated on the plain path (the
 * state held in the workspace, any circuit the plain path runs): precision 32 or 64 selects the
 * real type of params, points/angles and the outputs; points [P][3] for point encodings, angles
 * [P][n] for the angle-given encoding; workspace qp_plain_workspace_bytes(c, P, precision).
 * qp_energy_profile: the total field energy U(t_i) = sum over the grid xg x yg of
 *   (eps E_z^2 + H_x^2 + H_y^2) / 2 at every time t_i (device double [Nt]), eps = eps_r where
 *   x >= x_interface for the dielectric losses, else 1, from the fused forward on the Nt Nx Ny grid
 *   points (t-major); the collapse indicator I_BH = 1 - min_{t >= delta} U(t) / U(0) follows on the
 *   host.  Point encodings only; device inputs t [Nt], xg [Nx], yg [Ny]; workspace
 *   qp_energy_workspace_bytes.                                                                */
qp_status qp_bloch(qp_ctx* ctx, const qp_circuit* c, int32_t precision, const void* params,
                   const void* points, const void* angles, int64_t P, void* bloch, void* mw, void* ws,
                   size_t ws_bytes);
size_t qp_energy_workspace_bytes(const qp_circuit* c, int64_t Nt, int64_t Nx, int64_t Ny);
qp_status qp_energy_profile(qp_ctx* ctx, const qp_circuit* c, const float* params, const float* t,
                            int64_t Nt, const float* xg, int64_t Nx, const float* yg, int64_t Ny,
                            const qp_maxwell_desc* desc, double* U, void* ws, size_t ws_bytes,
                            uint32_t flags);

/* ---- fused Maxwell evaluation without allocation ---------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, checks and
 * results as qp_maxwell_fused minus the workspace: the per-call scratch (gate table, dielectric
 * counts, random-Fourier-feature angles, per-workgroup partials, FP64 reductions) lives in a
 * fixed device array of QP_NOALLOC_SCRATCH_BYTES inside the library, one copy per device, held
 * until the process ends.  Nothing in it needs to start at zero: every call writes what it reads.
 * Errors: QP_EWORKSPACE when the call needs more scratch than the array holds
 * (qp_workspace_bytes(c, P, 0) > QP_NOALLOC_SCRATCH_BYTES; only random-Fourier-feature circuits
 * grow with P, by 16 n bytes per point), QP_EUNSUPPORTED with QP_FLAG_TUNE or QP_FLAG_DENSE_MFMA
 * (they need a caller workspace), otherwise as qp_maxwell_fused.  All calls on one device share
 * the array: calls that overlap on one device (several streams or threads) race and must be
 * serialised by the caller.  qp_noalloc_scratch_bytes() returns the array size.            */
#define QP_NOALLOC_SCRATCH_BYTES (16u << 20)
size_t qp_noalloc_scratch_bytes(void);
qp_status qp_maxwell_fused_noalloc(qp_ctx* ctx, const qp_circuit* c, const float* params,
                                   const float* points, const float* angles, const float* jac,
                                   int64_t P, const qp_maxwell_desc* loss_desc, float* out,
                                   float* tan, double* loss, float* d_params, float* d_angles,
                                   float* d_jac, uint32_t flags);

/* ---- uneven batch: many circuits in one persistent launch ------------------------------
 * qp_batch_compile plans `count` circuits with their point counts P[count] (host), orders the
 * (circuit, point-tile) work items longest first and uploads the work list.  qp_batch_run
 * evaluates the fused Maxwell step for every circuit with persistent kernels, one per qubit-count
 * class (3..8, 9..11, 12 qubits; circuits with CRZ phase stages in their own class kernels),
 * followed by one reduction kernel; with QP_FLAG_TUNE the grid size is chosen by timing.  Every
 * circuit the fused path accepts may be batched, with cycled or RFF encodings, except
 * angle-given encodings (qp_batch_io carries no per-point angles: QP_EUNSUPPORTED) and circuits
 * with fewer than 3 outputs (QP_ESHAPE).  io is a host array [count] of per-circuit device
 * pointers.  qp_batch_graph_launch captures the whole step into a hipGraph on first use (per
 * batch, io and workspace) and replays it afterwards; parameters and points may change between
 * replays, the pointers may not.                                                          */
typedef struct qp_batch_io {
  const float* params;    /* [K_c]          */
  const float* points;    /* [P_c][3]       */
  float* out;             /* [P_c][m] or NULL */
  float* tan;             /* [P_c][m][3] or NULL */
  double* loss;           /* [1]            */
  float* d_params;        /* [K_c]          */
} qp_batch_io;

qp_status qp_batch_compile(qp_ctx* ctx, int32_t count, const qp_circuit_desc* descs,
                           const int64_t* P, qp_batch** out);
void qp_batch_destroy(qp_batch* b);
size_t qp_batch_workspace_bytes(const qp_batch* b);
qp_status qp_batch_run(qp_ctx* ctx, qp_batch* b, const qp_batch_io* io,
                       const qp_maxwell_desc* loss_desc, void* ws, size_t ws_bytes,
                       uint32_t flags);
qp_status qp_batch_graph_launch(qp_ctx* ctx, qp_batch* b, const qp_batch_io* io,
                                const qp_maxwell_desc* loss_desc, void* ws, size_t ws_bytes,
                                uint32_t flags);
/* what: 0 circuits, 1 work items, 2 persistent grid when only one stream has work, 3 graph
 * captured (0/1), 4 work items of the low class (3..8 qubits), 5 and 6 the grids of the low and
 * high class (9..11 qubits) when the low class and another have work: the low class then runs
 * on one stream while the high and the 12-qubit classes (one 512-thread workgroup per CU) run one
 * after the other on a second.  By default the high class runs on 2 workgroups per CU and the
 * low class's workgroups come on top (1.25 x its share of estimated work); QP_FLAG_TUNE also
 * times grids of 1..3 workgroups per CU, other shares and an even split of one grid.  7 work
 * items of the 12-qubit class, 8 work items of circuits with CRZ phase stages.              */
int64_t qp_batch_info(const qp_batch* b, int32_t what);

/* ---- plain baseline (the speedup denominator) -----------------------------------------
 * One kernel launch per gate on a statevector batch held in HBM, a readout kernel, input
 * tangents by central finite differences (6 extra forwards with step fd_h): the evaluation
 * pattern a simulator without backpropagation, or quantum hardware, pays for derivatives
 * (the paper's measurement passage in section "QPINN architecture and ansatz designs" names
 * parameter-shift as the hardware route; section "Quantum simulator and performance
 * optimization" uses backpropagation instead).
 * precision 32: complex64 state; 64: complex128 state.  params [K], points [P][3] and the
 * outputs use the matching real type (float or double).  tan may be NULL (forward only).   */
size_t qp_plain_workspace_bytes(const qp_circuit* c, int64_t P, int32_t precision);
qp_status qp_plain_eval(qp_ctx* ctx, const qp_circuit* c, int32_t precision,
                        const void* params, const void* points, int64_t P, double fd_h,
                        void* out, void* tan, void* ws, size_t ws_bytes);
/* Plain Maxwell step: FD tangents, then the loss (FP64 reduction), then central finite
 * differences of the loss for parameters k_begin..k_end-1 (step fd_h_param).  loss: device
 * double [1]; d_params: device [K] (entries outside the range are left untouched).         */
qp_status qp_plain_maxwell_fd(qp_ctx* ctx, const qp_circuit* c, int32_t precision,
                              const void* params, const void* points, int64_t P,
                              const qp_maxwell_desc* loss_desc, double fd_h,
                              double fd_h_param, int32_t k_begin, int32_t k_end,
                              double* loss, void* d_params, void* ws, size_t ws_bytes);

#ifdef __cplusplus
}
#endif
#endif /* QPINN_H */
