// Device code of the pencil march (paper: algorithm "HDG_Op_3D" in the
// transformed basis; sections "Product factorization of the HDG operator" and
// "Summary of solution method"), shared by the single-problem pencil CG
// kernel (pencil_cg.hip) and the batched persistent solver
// (batch_kernels.hip).
//
// A block owns EPB elements side by side along x1 (one slot each) in one row
// (fixed x2 index) and marches them up x3.  A thread owns the face-node
// column (q1, q2) of its slot's element, so the face between two consecutive
// elements of the march (normal x3) is the same face-node column for the
// same thread: its input is loaded once and carried in a register, and its
// two element contributions are summed in a register and stored once.  Faces
// normal to x1 and x2 keep the two-contribution layout (qa from the element
// below, qb from the element above).
//
// A step of the march first consumes the loaded face values of its element
// (p = z + beta p_old and x += alpha p_old on the faces it owns, the input
// staged in LDS), then issues the loads of the next element into the same
// registers, and then runs the element arithmetic while those loads are in
// flight.  The 1D tables sit in LDS.
#pragma once
#include "elem_unit.hpp"

namespace hdg {

// Two values read together from LDS (one 16-byte access in FP64).
template <typename T>
struct alignas(2 * sizeof(T)) PencilPair {
  T lo, hi;
};

template <typename T, int NP, int EPB>
struct PencilSmem {
  PencilPair<T> face[EPB][2][NP * NP];      // faces normal to x1, x2 (input p), low and high
  T u[EPB][upitch<NP>() * NP * NP + 1];     // the element's u in the eigenspace
  PencilPair<T> bs[NP];                     // B_S[k][0], B_S[k][1]
  T lam[NP];
};

// Face ids of one slot's pencil (element (i, j, k) for the k of the march):
// a face normal to x1 or x2 has id A + B k (its plane does not change along
// the march), a face normal to x3 has id x3A + x3B (pl - 1) on the interior
// plane pl, or one of the two boundary ids at the ends.  A face is free when
// its id is below n_free_faces; a free face on the boundary of the box (a
// Neumann side) has this element alone.  32-bit ids and offsets: the host
// runs this form only when every trace offset fits.
struct PencilRow {
  int A[4];            // faces normal to x1, x2 at k = 0
  int x3A;             // interior x3 face of plane 1 (foff[2] + i + n1 j)
  int x3bot, x3top;    // the boundary x3 faces of the column
  int freem, alonem;   // bits 0..3: faces normal to x1, x2; bits 4, 5: the
                       // boundary x3 faces (used at k = 0 and k = n3 - 1)
};

__device__ inline void pencil_row(const MeshDev& m, int i, int j, PencilRow& R) {
  R.freem = R.alonem = 0;
  const int nff = (int)m.n_free_faces;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int pl0 = i + s;
    if (pl0 >= 1 && pl0 <= m.n1 - 1) {
      R.A[s] = (int)m.foff[0] + (pl0 - 1) + (m.n1 - 1) * j;
      R.freem |= 1 << s;
    } else {
      R.A[s] = (int)m.boff[s] + j;
      if (R.A[s] < nff) R.alonem |= 1 << s;
    }
    const int pl1 = j + s;
    if (pl1 >= 1 && pl1 <= m.n2 - 1) {
      R.A[2 + s] = (int)m.foff[1] + i + m.n1 * (pl1 - 1);
      R.freem |= 4 << s;
    } else {
      R.A[2 + s] = (int)m.boff[2 + s] + i;
      if (R.A[2 + s] < nff) R.alonem |= 4 << s;
    }
  }
  const int ij = i + m.n1 * j;
  R.x3A = (int)m.foff[2] + ij;
  R.x3bot = (int)m.boff[4] + ij;
  R.x3top = (int)m.boff[5] + ij;
  if (R.x3bot < nff) R.alonem |= 16;
  if (R.x3top < nff) R.alonem |= 32;
  R.freem |= R.alonem;
}

// Id of face f of the slot's element at k; *fr: free, *al: alone on it.
// Along the march a face normal to x1 moves by (n1 - 1) n2 ids per element
// when interior and by n2 on a side of the box; normal to x2 by n1 (n2 - 1)
// and n1; normal to x3 by n1 n2.
__device__ inline int pencil_fid(const MeshDev& m, const PencilRow& R, int k, int f, bool* fr,
                                 bool* al) {
  if (f < 4) {
    const bool in = (R.freem >> f) & 1 & ~(R.alonem >> f);
    const int step = f < 2 ? (in ? (m.n1 - 1) * m.n2 : m.n2) : (in ? m.n1 * (m.n2 - 1) : m.n1);
    *fr = (R.freem >> f) & 1;
    *al = (R.alonem >> f) & 1;
    return R.A[f] + step * k;
  }
  const int pl = k + (f & 1);                  // plane of the x3 face
  if (pl >= 1 && pl <= m.n3 - 1) {
    *fr = true;
    *al = false;
    return R.x3A + m.n1 * m.n2 * (pl - 1);
  }
  *fr = (R.freem >> f) & 1;
  *al = *fr;
  return f == 4 ? R.x3bot : R.x3top;
}

// Loads of one element of the march (issued one step ahead of their use).
// Every lane loads from a valid address (faces that are not free, and idle
// lanes, read the first free face) and the values of faces it does not use
// are dropped where they are consumed: no conditional load writes a register
// that an earlier load may still be filling.
template <typename T>
struct PencilLoads {
  T z[6], po[6];      // face 4 (low x3) only at the start of a segment
  T xo[6];            // x on the owned faces (high faces; low faces alone on a Neumann side)
  double d[4], lam;   // metric factors d0..d3 and lambda of the element
};

template <typename T, int NP>
__device__ inline void pencil_load(const MeshDev& m, const T* __restrict__ z,
                                   const T* __restrict__ pin, const T* __restrict__ x,
                                   const PencilRow& R, int k, bool act, int col, int e, bool first,
                                   PencilLoads<T>& L) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    if (f == 4 && !first) {
      L.z[f] = L.po[f] = L.xo[f] = 0;
      continue;
    }
    const bool u = act && fr;
    const int g = (u ? fid * NF : 0) + (act ? col : 0);
    L.z[f] = z[g];
    L.po[f] = pin[g];
    if ((f & 1) || (R.alonem >> f) & 1) L.xo[f] = x[g];
    else L.xo[f] = 0;
  }
  const ElemInfo* ei = m.info + e;      // e is valid for every lane (idle slots clamped)
  L.d[0] = ei->d[0];
  L.d[1] = ei->d[1];
  L.d[2] = ei->d[2];
  L.d[3] = ei->d[3];
  L.lam = m.lam[e];
}

// Element arithmetic on the input p (xf, faces 0..3 staged in LDS by the
// caller before this call): expansion into the element eigenspace, division
// by D_Z, reductions back to the faces, and the face term with the 2 x 2
// matrix H = G + C^T M^-1 C of each axis.  Two barriers per element.
template <typename T, int NP, int EPB>
__device__ inline void pencil_core(PencilSmem<T, NP, EPB>& sm, int sl, int q1, int q2, int col,
                                   bool act, const T* d, const T* xf, T H, T H11, T H01,
                                   T* out) {
  constexpr int P = upitch<NP>();
  __syncthreads();
  T r2lo = 0, r2hi = 0;
  if (act) {
    const PencilPair<T>* f0 = sm.face[sl][0];
    const PencilPair<T>* f1 = sm.face[sl][1];
    const PencilPair<T> b1 = sm.bs[q1], b2 = sm.bs[q2];
    const T c0 = d[1] * b1.lo, c1 = d[1] * b1.hi;
    const T c2 = d[2] * b2.lo, c3 = d[2] * b2.hi;
    const T x2lo = d[3] * xf[4], x2hi = d[3] * xf[5];
    const T dij = d[0] + d[1] * sm.lam[q1] + d[2] * sm.lam[q2];
    T* u = sm.u[sl] + q1 + P * q2;
#pragma unroll 2
    for (int q3 = 0; q3 < NP; ++q3) {
      const PencilPair<T> b = sm.bs[q3];
      const PencilPair<T> a0 = f0[q2 + NP * q3];
      const PencilPair<T> a1 = f1[q1 + NP * q3];
      T F = c0 * a0.lo;
      F += c1 * a0.hi;
      F += c2 * a1.lo;
      F += c3 * a1.hi;
      F += b.lo * x2lo;
      F += b.hi * x2hi;
      const T v = div_fast(F, dij + d[3] * sm.lam[q3]);
      u[P * NP * q3] = v;
      r2lo += b.lo * v;
      r2hi += b.hi * v;
    }
  }
  __syncthreads();
  if (act) {
    T lo = 0, hi = 0;
    const T* ua = sm.u[sl] + P * col;             // axis 0: face node (q2, q3) = col
#pragma unroll 4
    for (int a = 0; a < NP; ++a) {
      const PencilPair<T> b = sm.bs[a];
      lo += b.lo * ua[a];
      hi += b.hi * ua[a];
    }
    out[0] = d[1] * (H * xf[0] + H01 * xf[1] - lo);
    out[1] = d[1] * (H11 * xf[1] + H01 * xf[0] - hi);
    lo = 0;
    hi = 0;
    const T* ub = sm.u[sl] + q1 + P * NP * q2;    // axis 1: face node (q1, q3) = col
#pragma unroll 4
    for (int b = 0; b < NP; ++b) {
      const PencilPair<T> bb = sm.bs[b];
      lo += bb.lo * ub[P * b];
      hi += bb.hi * ub[P * b];
    }
    out[2] = d[2] * (H * xf[2] + H01 * xf[3] - lo);
    out[3] = d[2] * (H11 * xf[3] + H01 * xf[2] - hi);
    out[4] = d[3] * (H * xf[4] + H01 * xf[5] - r2lo);
    out[5] = d[3] * (H11 * xf[5] + H01 * xf[4] - r2hi);
  }
  // no barrier here: the next element stages its faces (read above only
  // before the second barrier) and writes u only after its first barrier,
  // which every wave reaches after finishing these reductions
}

// One element of the march.  In: L holds the loaded values of element k.
// The input p on its faces, p and x on the faces it owns (stored), the input
// staged in LDS; then the loads of element kn into L; then the operator and
// the stores of the contributions.  carry_p / carry_w: p and the
// contribution of the x3 face shared with the previous element of the
// segment (in), and with the next one (out).
template <typename T, int NP, int EPB>
__device__ inline void pencil_step(const T* __restrict__ z, const T* __restrict__ pin,
                                   T* __restrict__ pout, T* __restrict__ x, T* __restrict__ qa,
                                   T* __restrict__ qb, PencilSmem<T, NP, EPB>& sm,
                                   const UnitLane& Ln, bool act, const MeshDev& m,
                                   const PencilRow& R, int k, int kn, int en, PencilLoads<T>& L,
                                   bool first, bool last, T alpha, T beta, T H, T H11, T H01,
                                   T& carry_p, T& carry_w, double* dot) {
  constexpr int NF = NP * NP;
  const int col = Ln.col;
  T xf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    T v = 0;
    if (f == 4 && !first) {
      v = carry_p;
    } else if (act && fr) {
      v = L.z[f] + beta * L.po[f];
      if ((f & 1) || al) {                    // the face is this element's
        pout[fid * NF + col] = v;
        x[fid * NF + col] = L.xo[f] + alpha * L.po[f];
      }
    }
    xf[f] = v;
  }
  if (act) {
    sm.face[Ln.sl][0][col] = PencilPair<T>{xf[0], xf[1]};
    sm.face[Ln.sl][1][col] = PencilPair<T>{xf[2], xf[3]};
  }
  const T d[4] = {(T)(L.d[0] * L.lam), (T)L.d[1], (T)L.d[2], (T)L.d[3]};
  // the next element's loads go out before the arithmetic of this one
  pencil_load<T, NP>(m, z, pin, x, R, kn, act, col, en, false, L);
  T out[6];
  pencil_core<T, NP, EPB>(sm, Ln.sl, Ln.q1, Ln.q2, col, act, d, xf, H, H11, H01, out);
  if (!act) return;
  double acc = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    if (!fr) continue;
    const int g = fid * NF + col;
    acc += (double)(xf[f] * out[f]);
    if (f < 4) {
      if (f & 1) {
        qa[g] = out[f];
        if (al) qb[g] = 0;
      } else {
        qb[g] = out[f];
        if (al) qa[g] = 0;
      }
    } else if (f == 4) {
      if (!first) {
        qa[g] = out[4] + carry_w;             // both contributions, summed here
      } else {
        qb[g] = out[4];                       // the element below is in another segment
        if (al) qa[g] = 0;
      }
    } else if (last) {
      qa[g] = out[5];                         // the element above is in another segment
      if (al) qb[g] = 0;
    }
  }
  carry_p = xf[5];
  carry_w = out[5];
  *dot += acc;
}


// The last x update of a finished solve, x_k = x_{k-1} + alpha_{k-1}
// p_{k-1}, on the faces the block's elements [k0, k1) own.
template <typename T, int NP>
__device__ inline void pencil_final_x(const MeshDev& m, const PencilRow& R, bool act, int col,
                                      int k0, int k1, T alpha, const T* __restrict__ pin,
                                      T* __restrict__ x) {
  if (!act) return;
  constexpr int NF = NP * NP;
  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      bool fr, al;
      const int fid = pencil_fid(m, R, k, f, &fr, &al);
      if (!fr || !((f & 1) || al)) continue;
      const int g = fid * NF + col;
      x[g] = x[g] + alpha * pin[g];
    }
  }
}

}  // namespace hdg
