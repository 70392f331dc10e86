// Internal declarations shared by the host API and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "setup1d.hpp"

namespace hdg {

constexpr int kMaxNP = 17;     // p <= 16

// Per-degree 1D data the element kernels need, passed by value.
template <typename T>
struct ElemTab {
  T bs0[kMaxNP];   // B_S[k][0]
  T bs1[kMaxNP];   // B_S[k][1]
  T lam[kMaxNP];   // Lambda_k
  T H;             // G + C^T M^-1 C = [[H, H01], [H01, H11]] (low, high face of an axis);
  T H11;           // H01 = 0 and H11 = H for the lumped mass
  T H01;
};

// Per-element data precomputed at set-up: the six face ids (axis a, side s
// at index 2a+s; ids >= n_free_faces are Dirichlet faces), the faces that
// are unknowns with this element alone (bit 2a+s: a face on a Neumann side
// of the box) and the metric factors d0..d3 (paper, section "LDG operator
// structure in three dimensions").  64 bytes, read with scalar loads.
struct ElemInfo {
  int fid[6];
  int nmask;
  int pad;
  double d[4];
};

// Mesh description on the device.  Face ids follow the canonical layout:
// interior faces of axis 0, 1, 2, the faces of the Neumann sides (free), then
// the faces of the Dirichlet sides (see include/hdg.h).
struct MeshDev {
  int n1, n2, n3;
  int neumann;         // bit 2a+s: side s of axis a is a Neumann side
  int64_t n_elem;
  int64_t foff[3];     // first interior face id of each axis
  int64_t boff[6];     // first face id of (axis, side), free or Dirichlet
  int64_t n_int_faces;   // interior faces
  int64_t n_free_faces;  // interior + Neumann faces
  int64_t n_dir_faces;   // faces of the Dirichlet sides
  const double* h1;
  const double* h2;
  const double* h3;
  const double* g1;    // (2/h1)^2 per element index along x1 (likewise g2, g3)
  const double* g2;
  const double* g3;
  const double* lam;   // per element
  const ElemInfo* info; // per element
};

// Device-resident state of one CG run.  The fused apply reads slot A and
// its block 0 writes slot B; the update reads B and its block 0 writes A.
// Because the two kernels strictly alternate, no slot is read and written by
// the same launch.  Reductions are block partials that every block of the
// consuming kernel sums in the same fixed order (no fences, deterministic).
struct CgState {
  double rho;        // A: rho_{k-1} (previous r.z);  B: rho_k
  double alpha;      // A: alpha_{k-1};  B: unused
  double rr_stop;    // absolute threshold on ||r||^2 (set at iteration 0)
  double rtol2;      // rtol^2 from the host
  double rr;         // last ||r||^2 seen (diagnostic)
  double pq;         // last p.q (diagnostic)
  int iter;          // A: k (iterations completed);  B: k
  int maxit;
  int done;          // 0 running, 1 converged, 2 iteration cap, 3 breakdown
  int pad;
};

struct CgScalars {
  CgState A;
  CgState B;
};

// Workspace of one CG solve in precision T (free-trace vectors).
template <typename T>
struct CgWork {
  T* x = nullptr;
  T* z = nullptr;        // preconditioned residual D^-1 r (r itself is not stored)
  T* p[2] = {nullptr, nullptr};
  T* qa = nullptr;       // contribution of the element below each face
  T* qb = nullptr;       // contribution of the element above each face
  // one-kernel CG: second z, s = D^-1 A p (ping-pong), second qa/qb set
  T* zz[2] = {nullptr, nullptr};   // zz[0] aliases z
  T* s[2] = {nullptr, nullptr};
  T* qq[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // qq[i] = {qa_i, qb_i}; qq[0] aliases qa, qb
  T* dinv = nullptr;
  double* partials = nullptr;  // pq[2][pmax] | rz[2][pmax] | rr[2][pmax]
  int pmax = 0;                // partial slots per buffer
  CgScalars* sc = nullptr;
  int64_t n = 0;
  int apply_blocks = 0;
  int update_blocks = 0;
  int pencil_blocks = 0;       // element launches of the pencil CG form
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  int graph_variant = -1;
  // a short graph of the same iterations for the last chunks of a solve
  hipGraphExec_t graph_tail = nullptr;
  int tail_iters = 0;
  int tail_variant = -1;
};

struct KernelConfig {
  int epb = 1;      // elements per block of the element kernels
};

}  // namespace hdg

struct hdg_ctx {
  int n[3] = {0, 0, 0};
  int p = 0, np = 0;
  int tile_variant = 0;           // elements per work unit: epb_max >> variant
  int cg_variant = 1;             // CG form when the options leave it open
  int pencil_ks = 0;              // pencil CG form: elements per x3 segment (0: automatic)
  double tau = 0.0;
  int neumann = 0;                // bit 2a+s: side s of axis a is a Neumann side
  int64_t n_elem = 0, n_free = 0, n_all = 0, n_vol = 0;
  int64_t n_free_faces = 0, n_faces = 0;
  int64_t n_int_faces = 0, n_neu_faces = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;   // private stream for graph capture
  int device = 0;
  hdg::Tables1D tab;
  hdg::MeshDev mesh{};
  std::vector<double> h_host[3];
  double origin[3] = {0.0, 0.0, 0.0};   // coordinates of the mesh corner (hdg_coords only)
  std::vector<double> lam_host;
  // device buffers
  double* d_h[3] = {nullptr, nullptr, nullptr};
  double* d_g[3] = {nullptr, nullptr, nullptr};   // (2/h)^2 per axis
  hdg::ElemInfo* d_info = nullptr;
  double* d_lam = nullptr;
  double* d_mats64 = nullptr;   // St, StM, S, MS (4 n_p^2 doubles)
  float* d_mats32 = nullptr;
  hdg::ElemTab<double> et64{};
  hdg::ElemTab<float> et32{};
  double* d_diag = nullptr;     // diag of K^_ff (FP64)
  float* d_dinv32 = nullptr;
  hdg::CgWork<double> w64;
  hdg::CgWork<float> w32;
  // FP64 free-length scratch: [0] eigen-basis rhs / trace, [1] FP64 solution or FP32
  // inner rhs (mixed), [2] FP64 residual, [3] inverse diagonal (FP64)
  double* d_tmp[4] = {nullptr, nullptr, nullptr, nullptr};
  double* d_vol_tmp = nullptr;
  double* d_guess = nullptr;    // free-length scratch of solves from an initial guess (lazy)
  double* d_red = nullptr;      // small reduction scratch
  unsigned* d_cnt = nullptr;
  hdg::CgScalars* h_scal = nullptr;   // pinned host slots: [0..1] polling, [2] upload
  double* h_red = nullptr;            // pinned host scalar for reductions
};

namespace hdg {

// ---- kernel launchers (defined in the .hip translation units) -------------
// element apply in the eigen basis, output split into qa/qb; with a CG
// state, nothing is done once its slot B reports a finished solve.
template <typename T>
hipError_t launch_elem_apply(const hdg_ctx* c, const T* x_free, const T* x_bdry,
                             T* qa, T* qb, hipStream_t s, CgScalars* skip_if_done = nullptr);
// fused CG apply (see kernels_cg.hip)
template <typename T>
hipError_t launch_cg_apply(const hdg_ctx* c, CgWork<T>& w, hipStream_t s);
template <typename T>
hipError_t launch_cg_update(const hdg_ctx* c, CgWork<T>& w, hipStream_t s);
// two-kernel CG continued on a replaced residual b at iteration `iter`
template <typename T>
hipError_t launch_cg_continue(const hdg_ctx* c, CgWork<T>& w, const T* b, int iter, double pscale,
                              hipStream_t s);
// pencil form of the two-kernel CG (pencil_cg.hip): element launch and
// update launch of one iteration; started by launch_cg_init
template <typename T>
hipError_t launch_pencil_apply(const hdg_ctx* c, CgWork<T>& w, hipStream_t s);
template <typename T>
hipError_t launch_pencil_update(const hdg_ctx* c, CgWork<T>& w, hipStream_t s);
int pencil_blocks(const hdg_ctx* c, int variant);
// one-kernel CG iteration (reads state slot rd, writes rd ^ 1) and its init
template <typename T>
hipError_t launch_cgcg_iter(const hdg_ctx* c, CgWork<T>& w, int rd, hipStream_t s);
template <typename T>
hipError_t launch_cgcg_init(const hdg_ctx* c, CgWork<T>& w, const T* b, hipStream_t s);
template <typename T>
hipError_t launch_cg_init(const hdg_ctx* c, CgWork<T>& w, const T* b, hipStream_t s);
// nodal-basis CG (precond 0 none, 2 diagonal, 3 block; see nodal_cg.hip):
// its start from the right-hand side b and one iteration
hipError_t launch_ncg_init(const hdg_ctx* c, CgWork<double>& w, int precond, const double* b,
                           hipStream_t s);
hipError_t launch_ncg_iter(const hdg_ctx* c, CgWork<double>& w, int precond, hipStream_t s);
int ncg_face_blocks(int np, int64_t n_faces);

// y = qa + qb (optionally scaled); or y = b - (qa + qb) with the squared norm
// reduced into red[0] (FP64)
template <typename T>
hipError_t launch_combine(const T* qa, const T* qb, T* y, int64_t n, hipStream_t s);
hipError_t launch_residual64(const double* b, const double* qa, const double* qb, double* r,
                             int64_t n, double* partials, double* out, int nblocks,
                             hipStream_t s);

// per-face transform A x A of n_faces faces; optional second input added first
template <typename T>
hipError_t launch_face_transform(int np, const T* A, const T* in, const T* in2, T* out,
                                 int64_t n_faces, hipStream_t s);

// diagonal of K^_ff
hipError_t launch_diag(const hdg_ctx* c, double* diag, hipStream_t s);

// volume-source element kernel (RHS / recovery / adjoint)
// (VOL_HYB: the initial-guess flux of a volume field, f = the field,
// x_bdry = the nodal boundary tail for g_N, output into qa / qb)
enum VolMode { VOL_RHS = 0, VOL_RECON = 1, VOL_ADJ = 2, VOL_HYB = 3 };
hipError_t launch_volume(const hdg_ctx* c, int mode, int src_is_forcing,
                         const double* f, const double* x_free, const double* x_bdry,
                         const double* r2, const double* mu_free,
                         double* qa, double* qb, double* out_vol, double* out_elem,
                         hipStream_t s);

// the context's per-face 1D transform matrices by hdg_transform kind
const double* mat64(const hdg_ctx* c, int kind);
const float* mat32(const hdg_ctx* c, int kind);

// misc vector kernels
hipError_t launch_cast_scale_64_32(const double* in, float* out, double scale, int64_t n,
                                   hipStream_t s);
hipError_t launch_axpy_32_64(const float* in, double* out, double scale, int64_t n,
                             hipStream_t s);
hipError_t launch_fill64(double* out, double v, int64_t n, hipStream_t s);
hipError_t launch_copy64(const double* in, double* out, int64_t n, hipStream_t s);
hipError_t launch_add64(const double* in, double* out, int64_t n, hipStream_t s);   // out += in
// both CG state slots zeroed, slot A with rtol^2, maxit and rho = 1
hipError_t launch_state_reset(CgScalars* sc, double rtol2, int maxit, hipStream_t s);
hipError_t launch_fill32(float* out, float v, int64_t n, hipStream_t s);
hipError_t launch_recip_64_32(const double* diag, float* dinv32, double* dinv64, int64_t n,
                              hipStream_t s);
hipError_t launch_dot64(const double* a, const double* b, int64_t n, double* partials,
                        double* out, int nblocks, hipStream_t s);

// grid size of the element apply kernels (number of partials they write) and
// elements per work unit of a tile variant
int elem_apply_blocks(int np, int64_t n_elem, int variant);
int tile_epb(int np, int variant);
int tile_threads(int np, int variant);
constexpr int kNumTileVariants = 3;

}  // namespace hdg
