// Shared device/host definitions of the HIP implementation (gfx950).
//
// Layout conventions (all arrays):
//   nodal arrays      (N_z+1)(N_y+1)(N_x+1) doubles, x fastest (2-D: (N_y+1)(N_x+1))
//   interior arrays   (N_z-1)(N_y-1)(N_x-1) in the working precision, x fastest
//   augmented vector  Q: faces x-, x+, y-, y+[, z-, z+]; inside a face the two
//                     tangential axes row-major, lower axis fastest.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ahoc {

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <typename T> using cx = typename Cx<T>::type;

// Grid geometry of one instance.
struct Geom {
  int dim;
  int n[3];          // intervals N_a (unused axes: 2)
  int ni[3];         // interior counts N_a - 1 (unused axes: 1)
  int nn[3];         // nodal counts N_a + 1 (unused axes: 1)
  double h[3];       // spacings
  long long nint;    // prod ni (interior nodes)
  long long nnodal;  // prod nn
  int px;            // row pitch of interior arrays (ni[0] rounded up to 32 elements)
  long long nalloc;  // px * ni[1] * ni[2]: elements of an interior array incl. row padding
  int nq;            // augmented unknowns
  int face_off[7];   // start of each face in Q, face f = 2*axis + side
  int nb;            // instances in a batch of equal 2-D grids (1 otherwise); every array
                     // holds nb consecutive instances of the per-instance sizes above
};

// Weights of the compact operators, by offset class.
//   3-D L_h: centre, face neighbours (+-x, +-y, +-z), edge neighbours (xy, xz, yz)
//   2-D L_h: centre, (+-x), (+-y), corners (xy)
//   M:       centre m0 and the 2*dim face neighbours m1
struct Weights {
  double c0;
  double cf[3];
  double ce[3];  // ce[0] = xy, ce[1] = xz, ce[2] = yz
  double m0, m1;
  double os[4];  // one-sided normal weights a_0..a_3
  double os_gn;  // Neumann weight 11/3
};

// Status codes of the C ABI (mirrors include/ahoc.h).
enum : int { ST_OK = 0, ST_INVALID = -1, ST_NOMEM = -2, ST_NOCONV = -3, ST_HIP = -4,
             ST_UNSUPPORTED = -5 };

#define AHOC_HIP_TRY(...)                                      \
  do {                                                         \
    hipError_t e__ = (__VA_ARGS__);                            \
    if (e__ != hipSuccess) {                                   \
      ahoc::set_last_error(hipGetErrorString(e__), #__VA_ARGS__); \
      return ahoc::ST_HIP;                                     \
    }                                                          \
  } while (0)

void set_last_error(const char* what, const char* where);

// Return a nonzero status code from the enclosing function.
#define TRY_ST(...)              \
  do {                           \
    const int rc__ = (__VA_ARGS__); \
    if (rc__) return rc__;       \
  } while (0)

// Device memory provider: the caller's callbacks (ahoc_allocator) or, when alloc is null,
// hipMalloc / hipFree.  dev_alloc returns ST_NOMEM (with the last error set) on failure.
struct DevAlloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
int dev_alloc(const DevAlloc& a, void** p, size_t bytes);
void dev_free(const DevAlloc& a, void* p);

// ------------------------------------------------------------------------------------
// DST-I passes (dst.hip)
// ------------------------------------------------------------------------------------

// Precomputed tables for one transform length N (pencil length N-1).
template <typename T> struct DstTables {
  DevAlloc al;        // provider of tw, sn, S (released through it)
  int N = 0;
  int ppt = 0;        // points per thread (compile-time variant selector)
  int nrad = 0;
  int rad[12] = {0};  // radix sequence, product N
  cx<T>* tw = nullptr;   // exp(-2 pi i k / N), k = 0..N-1 (null without an FFT plan)
  T* sn = nullptr;       // sin(pi m / N), m = 0..N/2; without an FFT plan (ppt = 0) the
                         // full period sin(pi j / N), j = 0..2N-1, of the direct pass
  // half sine matrices of the matrix-core pass (even N <= DST_GEMM_MAX_N), [2][HP][HP]
  T* S = nullptr;
  // setup-time choice per plain pass kind (0 rows, 1 strided), dst_tune.hip: method
  // DST_M_DEFAULT (the default FFT kernel), DST_M_GEMM (matrix-core products) or
  // DST_M_TILE (the one-tile FFT kernel with `tile` pencil pairs per work-group), -1 = not
  // timed; the microseconds per pass behind it (-1 = not timed / not applicable)
  int method[2] = {-1, -1};
  int tile[2] = {0, 0};
  double t_default_us[2] = {-1.0, -1.0};
  double t_gemm_us[2] = {-1.0, -1.0};
  double t_best_us[2] = {-1.0, -1.0};
};
enum { DST_M_DEFAULT = 0, DST_M_GEMM = 1, DST_M_TILE = 2 };

// Eigen-scaling parameters for the fused middle pass along the slowest axis.
template <typename T> struct DstScale {
  const T* s_this = nullptr;  // s_t(k), k = 1..n_t   (length n_t)
  const T* s_a = nullptr;     // fastest other axis, length n_a
  const T* s_b = nullptr;     // second other axis (3-D), length n_b, or null
  int na = 1;                 // column decode: col = ia + na * ib (na = row pitch)
  int nva = 1;                // valid ia < nva (columns ia >= nva are row padding)
  T c_ta = 0, c_tb = 0, c_ab = 0;
  T scale = 0;                // sign * prod_a 2/N_a
  // the v-equation's shift by the constant c = beta/alpha (zero otherwise): lambda_L - c mu_M
  // with mu_M = m0 + 2 m1 sum_a cos(theta_a) and cos(theta_a) = 1 + h_a^2 s_a / 2 adds
  // a0 + ka s_a + kb s_b to A and kt to B (lambda = A + B s_this)
  T a0 = 0, ka = 0, kb = 0, kt = 0;
  // symbol of the weighting operator M, mu_M = mc0 + mca s_a + mcb s_b + mct s_this, by
  // which the U-solve's pass with spectral M multiplies the spectrum (m0 + 2 dim m1 and
  // m1 h_a^2 from cos(theta_a) = 1 + h_a^2 s_a / 2)
  T mc0 = 1, mca = 0, mcb = 0, mct = 0;
};

// Optional face sums of a fused pass (one-sided normal combination along the pass axis):
//   mode 1: out[col] = sum_k W(k) w_lo(k), out[plane + col] = sum_k W(k) w_hi(k) over the
//           scaled spectrum W of each column; the pass then stores W itself (forward
//           transform and eigen scaling only, no inverse transform).
template <typename T> struct DstFaces {
  T* out = nullptr;
  const T* w = nullptr;  // w_lo[0..L), w_hi[0..L)
  long long plane = 0;
  long long slab = 0;    // offset of slab o's sums: out + o * slab
  int mode = 0;
};

// Spectral lift of the V-solve (dst_spectral.hip): the slowest-axis pass builds the
// spectrum of the face-layer right-hand side from 2-D face spectra.  Layouts, with
// L = N-1 along the pass axis, side 0 = low face, 1 = high face:
//   lp [side][col]                faces normal to the pass axis (plane pplane)
//   la [side] at ib * arow + (m-1) * apitch   faces normal to the fastest axis a (plane
//                                 aplane; 2-D: ib = 0)
//   lb [side][m-1][ia]            faces normal to the middle axis b, 3-D only (plane
//                                 bplane, row pitch bpitch)
//   wp, wa, wb                    sines of the layer next to each face along the pass axis,
//                                 axis a and axis b: [side][k-1], halves of length L, nwa, nwb
template <typename T> struct DstGen {
  long long pslab = 0, aslab = 0, bslab = 0;  // per-slab offsets of lp, la, lb (outer > 1)
  const T* lp = nullptr;
  long long pplane = 0;
  const T* wp = nullptr;
  const T* la = nullptr;
  long long aplane = 0;
  int apitch = 0;
  int arow = 1;
  const T* wa = nullptr;
  int nwa = 0;
  const T* lb = nullptr;
  long long bplane = 0;
  int bpitch = 0;
  const T* wb = nullptr;
  int nwb = 0;
  // U-solve pass with spectral M: per position m - 1 of the pass axis the 4-tuple
  // (s_this, layer sine wp, face weights w_lo, w_hi), one vector load per position
  const T* ptab = nullptr;
};

template <typename T>
int dst_gen_pass(const DstTables<T>& tb, T* out, long long outer, long long inner, const DstScale<T>& sc,
                 const DstGen<T>& gen, hipStream_t st);
// Persistent variant (dst_pipe.hip); ST_UNSUPPORTED where its layout conditions fail.
template <typename T>
int dst_gen_pipe_pass(const DstTables<T>& tb, T* out, long long outer, long long inner, const DstScale<T>& sc,
                      const DstGen<T>& gen, hipStream_t st);

// Face contractions of a scaled spectrum W stored as planes [o][ky][kx] (row pitch px,
// nx valid columns, ny rows, `planes` planes):
//   fx[side * fx_side + o * fx_plane + ky * fx_row] = sum_kx W[o][ky][kx] wx[side][kx]
//   fy[side][o][kx] = sum_ky W[o][ky][kx] wy[side][ky]        (when fy != null; planes [px],
//                                                              padding columns written as zero)
template <typename T>
int face_reduce(const T* W, long long planes, int ny, int nx, int px, const T* wx, const T* wy, T* fx, T* fy,
                long long fx_side, long long fx_plane, long long fx_row, hipStream_t st);

// One pass of the batched DST-I along an axis of an interior array viewed as
// [outer][L][inner] (L = N-1).  inner == 1 means contiguous pencils: `outer` rows
// of L elements starting `pitch` elements apart.
template <typename T>
int dst_pass(const DstTables<T>& tb, const T* in, T* out, long long outer, long long inner,
             long long pitch, const DstScale<T>* fused, int tile_seqs, hipStream_t st,
             const DstFaces<T>* faces = nullptr);

// Length-specialised kernels (dst_fast.hip) for N in {32, 64, 96, ..., 4096}.
bool dst_fast_supported(int N);
enum { DST_PASS_ROWS = 0, DST_PASS_STRIDED = 1, DST_PASS_FUSED = 2 };
int dst_fast_tile(int N, int elem_bytes, int kind);
int dst_set_tile(int kind, int elem_bytes, int pairs);
template <typename T>
int dst_fast_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long outer,
                  long long inner, long long pitch, const DstScale<T>* fused, int nseq, hipStream_t st,
                  const DstFaces<T>* faces = nullptr);

// Row pass over contiguous pencils with compile-time indexing (dst_rows.hip); in may
// equal out.  ST_UNSUPPORTED where no such kernel applies.
template <typename T>
int dst_rows_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                  hipStream_t st);

// Face layers of the V-solve's lift added to the first (row) pass of a Poisson solve with a
// source (dst_rows.hip): layouts of face_lift (3-D: lx [2][n_y'][n_z'], ly [2][n_z'][px],
// lz [2][n_y'][px]; 2-D per instance b: lx [b][2][n_y'], ly [b][2][px]).
template <typename T> struct RowLift {
  const T* lx = nullptr;
  const T* ly = nullptr;
  const T* lz = nullptr;
  long long xplane = 0, yplane = 0, zplane = 0;  // offset of the high face's array (3-D)
  int dim = 3, ni1 = 0, ni2 = 1, px = 0;
};
// Row pass whose input is in + the lift's face layers (no lift pass); in may equal out.
// dst_rows_lift_supported: whether the pass exists for this length and shape (checked
// before anything is launched).
template <typename T> bool dst_rows_lift_supported(int N, long long nrows, long long pitch);
template <typename T>
int dst_rows_lift_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                       const RowLift<T>& lf, hipStream_t st);

// Row pass plus an addend: out_row = S in_row + add_row (add in the layout of out; in may
// equal out).  ST_UNSUPPORTED where no row kernel exists for N or the shape.
template <typename T>
int dst_rows_add_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, const T* addv, long long nrows,
                      long long pitch, hipStream_t st);

// Two transforms of each row with a pointwise product between them (dst_rows.hip):
// out_row = S (c_row .* (S in_row)), c nodal with the row of interior row
// r = (j - 1) + p ni1 at c + ((p + kofs) nn1 + j) nn0 (position i at offset i); in may
// equal out.  ST_UNSUPPORTED where no such kernel applies.
template <typename T>
int dst_rows_mul_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long nrows, long long pitch,
                      const T* c, int ni1, int kofs, int nn0, int nn1, hipStream_t st);

// Persistent, software-pipelined strided pass (dst_pipe.hip): plain, or (fused with
// faces->mode 1) forward + eigen scaling + face sums; inner must be even.  nseq 0 = the
// kernel's own tile; ST_UNSUPPORTED where no such kernel applies.
template <typename T>
int dst_pipe_pass(int N, const cx<T>* tw, const T* sn, const T* in, T* out, long long outer, long long inner,
                  const DstScale<T>* fused, const DstFaces<T>* faces, int nseq, hipStream_t st);

// The U-solve's slowest-axis pass with the weighting operator in spectral form
// (dst_pipe.hip), in place on buf: forward transform; spectrum times scale mu_M / lambda_L
// (sc, with the mc* fields) plus the spectrum of the face-layer source generated from the
// 2-D face spectra of gen times scale / lambda_L; face sums along the pass axis (faces,
// mode 1); store.  gen's layouts as for dst_gen_pass, except lb: [side][ia][m-1] (row pitch
// bpitch, plane bplane).  gen's y-face array (lb) is turned into its sums and differences
// in place.  ST_UNSUPPORTED where the persistent kernel's layout conditions fail (checked
// before anything is launched).
template <typename T>
int dst_pipe_mpass(int N, const cx<T>* tw, const T* sn, T* buf, long long outer, long long inner,
                   const DstScale<T>& sc, const DstFaces<T>& faces, const DstGen<T>& gen, hipStream_t st);
template <typename T> bool dst_pipe_mpass_ok(int N, long long inner, long long na, const DstGen<T>& gen);

// DST-I of short pencils (even N <= DST_GEMM_MAX_N) as two half-size products with sine
// matrices on the matrix cores (dst_gemm.hip).  Same layouts as dst_pass (plain passes
// only); in may equal out.
constexpr int DST_GEMM_MAX_N = 128;
bool dst_gemm_supported(int N);
int dst_gemm_hp(int N);
template <typename T> int dst_gemm_table(T** S, int N, hipStream_t st, const DevAlloc& al);
template <typename T>
int dst_gemm_pass(const T* S, int N, const T* in, T* out, long long outer, long long inner, long long pitch,
                  hipStream_t st);
// Times the candidate kernels for the plain pass of this shape (buf is overwritten) and
// records the fastest in tb.method / tb.tile (dst_tune.hip); no-op outside automatic
// selection.
template <typename T>
int dst_autotune(DstTables<T>& tb, T* buf, long long outer, long long inner, long long pitch, hipStream_t st);

// Calibration copies of an [nz][ny][nx] FP32 volume (calib.hip): pattern 0 linear, 1 the
// strided passes' tiles along y, 2 along z.
int copy_bandwidth(int pattern, const float* in, float* out, int nx, int ny, int nz, hipStream_t st);

// 0 = automatic (specialised kernels; for plain passes the kernel the setup-time timing
// chose), 1 = generic kernel only, 2 = specialised only, 3 = one-tile specialised kernels,
// 4 = matrix-core pass for every plain pass it supports, 5 = as 0 without setup-time choices
void dst_set_variant(int v);
int dst_get_variant();

// Tables for length N, uploaded on stream st (which is synchronised before returning),
// allocated through `al` (null: hipMalloc).
template <typename T> int dst_tables_init(DstTables<T>& tb, int N, hipStream_t st = nullptr,
                                          const DevAlloc* al = nullptr);
template <typename T> void dst_tables_free(DstTables<T>& tb);
// Only the radix plan of an FFT length (N, ppt, nrad, rad): no device memory.
template <typename T> int dst_plan_only(DstTables<T>& tb, int N);
// Every N in [2, DST_MAX_N] has a pass: radix-2/3/4/8 FFT plans where dst_ppt(N) > 0,
// else the direct sine-sum pass (dst_direct.hip).
constexpr int DST_MAX_N = 8192;
bool dst_supported(int N);
int dst_ppt(int N);
// Direct O(N) per output pass for any length (same layouts and fused scaling as dst_pass;
// `sn2` holds sin(pi j / N), j = 0..2N-1).
template <typename T>
int dst_direct_pass(int N, const T* sn2, const T* in, T* out, long long outer, long long inner, long long pitch,
                    const DstScale<T>* fused, hipStream_t st);
int dst_default_tile(int N, int elem_bytes);

}  // namespace ahoc
