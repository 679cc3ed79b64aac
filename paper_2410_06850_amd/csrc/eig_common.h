// Device building blocks of the set-up eigensolvers: block-level reductions
// and a parallel cyclic Jacobi eigensolver for small symmetric matrices held
// in LDS.
#pragma once

#include "internal.h"

namespace msmg {

MSMG_DEV int block_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
MSMG_DEV int block_nthr() { return blockDim.x * blockDim.y * blockDim.z; }

// Sum of one value over the block, result returned to every thread.
MSMG_DEV double block_allsum(double v, double* red) {
  const int tid = block_tid(), nw = (block_nthr() + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  __syncthreads();
  return s;
}

MSMG_DEV double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
MSMG_DEV int wave_min_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

MSMG_DEV double block_allmax(double v, double* red) {
  const int tid = block_tid(), nw = (block_nthr() + 63) >> 6;
  v = wave_max(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

MSMG_DEV int block_allmin_int(int v, int* red) {
  const int tid = block_tid(), nw = (block_nthr() + 63) >> 6;
  v = wave_min_int(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  int s = red[0];
  for (int w = 1; w < nw; ++w) s = min(s, red[w]);
  __syncthreads();
  return s;
}

// Sum of NV values per thread over the block; every thread receives the sums.
template <int NV>
MSMG_DEV void block_allsum_vec(double (&v)[NV], double* red) {
  const int tid = block_tid(), nw = (block_nthr() + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if ((tid & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * nw + (tid >> 6)] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[q * nw + w];
    v[q] = s;
  }
  __syncthreads();
}

// Partner of index j in round r of the round-robin pairing of mm (even) indices.
MSMG_DEV int rr_partner(int r, int j, int mm) {
  if (j == mm - 1) return r;
  if (j == r) return mm - 1;
  int p = (2 * r - j) % (mm - 1);
  if (p < 0) p += mm - 1;
  return p;
}

// Rotation (c, s) annihilating A[p][q] (p < q):  tau = (A_qq - A_pp) / (2 A_pq),
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1+t^2), s = t c
// (Golub & Van Loan, symmetric Schur decomposition).
MSMG_DEV void jacobi_rot(const double* A, int m, int p, int q, double& c, double& s) {
  const double apq = A[p * m + q];
  if (fabs(apq) < 1e-300) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// The same parallel cyclic Jacobi method for m = 8, run by one wave with the
// matrix in registers: lane e holds A[e / 8][e % 8] and V[e / 8][e % 8], and
// every operand of a rotation comes from another lane by a shuffle, so the
// sweeps need no barrier.  Same rotations in the same order as block_jacobi;
// eigenvalues ascending (stable in the index on ties) into ev, eigenvectors
// as the columns of Vs.  Only the 64 lanes of one wave may call; the caller
// synchronises before others read ev and Vs.
MSMG_DEV void wave_jacobi8(const double* A, double* Vs, double* ev, int max_sweeps = 16) {
  const int e = threadIdx.x & 63, i = e >> 3, j = e & 7;
  double a = A[e];
  double v = (i == j) ? 1.0 : 0.0;
  auto rot = [](double app, double aqq, double apq, double& c, double& s) {
    if (fabs(apq) < 1e-300) {
      c = 1.0;
      s = 0.0;
      return;
    }
    const double tau = (aqq - app) / (2.0 * apq);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
  };
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      for (int r = 0; r < 7; ++r) {
      // the round's four disjoint rotations: lane e computes the one of its
      // column pair; the row pass takes the rotation of its row pair from lane i
      // (row 0, column i), whose column pair is that row pair
      const int jp = rr_partner(r, j, 8), p = min(j, jp), q = max(j, jp);
      const double app = __shfl(a, p * 9, 64), aqq = __shfl(a, q * 9, 64), apq = __shfl(a, p * 8 + q, 64);
      double c, s;
      rot(app, aqq, apq, c, s);
      // column pass: B = A J, V = V J
      const double aip = __shfl(a, i * 8 + p, 64), aiq = __shfl(a, i * 8 + q, 64);
      const double vip = __shfl(v, i * 8 + p, 64), viq = __shfl(v, i * 8 + q, 64);
      const double b = (j == p) ? c * aip - s * aiq : s * aip + c * aiq;
      v = (j == p) ? c * vip - s * viq : s * vip + c * viq;
      // row pass: A = J^T B
      const int ip = rr_partner(r, i, 8), pr = min(i, ip), qr = max(i, ip);
      const double cr = __shfl(c, i, 64), sr = __shfl(s, i, 64);
      const double bpj = __shfl(b, pr * 8 + j, 64), bqj = __shfl(b, qr * 8 + j, 64);
      a = (i == pr) ? cr * bpj - sr * bqj : sr * bpj + cr * bqj;
    }
    const double a2 = a * a;
    const double off = wave_sum(i != j ? a2 : 0.0), all = wave_sum(a2);
    if (!(off > 1e-32 * all)) break;
  }
  // rank of diagonal entry k among the diagonal (ascending, ties by index)
  const double dj = __shfl(a, j * 9, 64);
  int rank = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double dk = __shfl(a, k * 9, 64);
    rank += (dk < dj || (dk == dj && k < j)) ? 1 : 0;
  }
  Vs[i * 8 + rank] = v;
  if (i == 0) ev[rank] = dj;
}

// Orthonormalising transform of an 8-vector block from its Gram matrix G
// (LDS, 8 x 8), by one wave: the Cholesky factor G = R^T R and C = R^-1
// (upper triangular), so that P C has orthonormal columns.  Lane e holds
// entry (e / 8, e % 8).  Returns false (on every lane) when a pivot is not
// safely positive; C is then not written.  Same result, up to rounding, as
// orthonormalising the columns in order by Gram-Schmidt.
MSMG_DEV bool wave_cholinv8(const double* G, double* C) {
  const int e = threadIdx.x & 63, i = e >> 3, j = e & 7;
  double g = G[e];
  const double g0 = g;
  double r = 0.0;  // R[i][j] once row i is done
  for (int k = 0; k < 8; ++k) {
    // pivots below 1e-14 of the diagonal entry (condition of the block above
    // ~1e7) go to the eigen-decomposition instead
    const double dkk = __shfl(g, k * 9, 64), gkk = __shfl(g0, k * 9, 64);
    if (!(dkk > 1e-14 * gkk) || !(dkk > 1e-300)) return false;
    const double d = sqrt(dkk);
    const double rki = __shfl(g, k * 8 + i, 64) / d, rkj = __shfl(g, k * 8 + j, 64) / d;
    if (i == k) r = (j >= k) ? rkj : 0.0;
    if (i > k && j > k) g -= rki * rkj;
  }
  // X = R^-1 by back substitution, row by row from the bottom
  double x = 0.0;
  for (int ii = 7; ii >= 0; --ii) {
    double acc = (ii == j) ? 1.0 : 0.0;
    for (int k = ii + 1; k < 8; ++k) acc -= __shfl(r, ii * 8 + k, 64) * __shfl(x, k * 8 + j, 64);
    const double rii = __shfl(r, ii * 9, 64);
    if (i == ii) x = (j >= ii) ? acc / rii : 0.0;
  }
  C[e] = x;
  return true;
}

// Eigen-decomposition of the symmetric m x m matrix A (LDS, row-major) by the
// parallel cyclic Jacobi method: rounds of disjoint rotations, each applied as
// a column pass (B = A J, V = V J) and a row pass (A = J^T B).  On return
// ev[k] are the eigenvalues in ascending order and column k of Vs holds the
// matching eigenvector (Vs = V with permuted columns).  Uses threads
// tid < m*m for element work; all threads of the block must call.
// LDS: A, V, B, Vs: m*m; ev: m; perm: m ints; red: >= 2 * nwaves doubles;
// cs: 2 m doubles (the round's rotations, computed once per index).
MSMG_DEV void block_jacobi(double* A, double* V, double* B, double* Vs, double* ev, int* perm, int m,
                           double* red, double* cs, int max_sweeps = 16) {
  const int tid = block_tid(), nthr = block_nthr();
  const int mm = m + (m & 1);
  for (int e = tid; e < m * m; e += nthr) V[e] = (e / m == e % m) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int r = 0; r < mm - 1; ++r) {
      // the rotation of each index's pair (identity for the odd-size dummy);
      // both members of a pair evaluate it from the same entries
      for (int j = tid; j < m; j += nthr) {
        const int jp = rr_partner(r, j, mm);
        double c = 1.0, s = 0.0;
        if (jp < m) jacobi_rot(A, m, min(j, jp), max(j, jp), c, s);
        cs[2 * j] = c;
        cs[2 * j + 1] = s;
      }
      __syncthreads();
      double vnew[4];
      int cnt = 0;
      for (int e = tid; e < m * m; e += nthr, ++cnt) {
        const int i = e / m, j = e % m;
        const int jp = rr_partner(r, j, mm);
        double bv, vv;
        if (jp >= m) {
          bv = A[e];
          vv = V[e];
        } else {
          const double c = cs[2 * j], s = cs[2 * j + 1];
          const int p = min(j, jp), q = max(j, jp);
          if (j == p) {
            bv = c * A[i * m + p] - s * A[i * m + q];
            vv = c * V[i * m + p] - s * V[i * m + q];
          } else {
            bv = s * A[i * m + p] + c * A[i * m + q];
            vv = s * V[i * m + p] + c * V[i * m + q];
          }
        }
        B[e] = bv;
        if (cnt < 4) vnew[cnt] = vv;
      }
      __syncthreads();
      cnt = 0;
      for (int e = tid; e < m * m; e += nthr, ++cnt) {
        if (cnt < 4) V[e] = vnew[cnt];
        const int i = e / m, j = e % m;
        const int ip = rr_partner(r, i, mm);
        double av;
        if (ip >= m) {
          av = B[e];
        } else {
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const int p = min(i, ip), q = max(i, ip);
          av = (i == p) ? (c * B[p * m + j] - s * B[q * m + j]) : (s * B[p * m + j] + c * B[q * m + j]);
        }
        vnew[cnt < 4 ? cnt : 3] = av;
      }
      __syncthreads();
      cnt = 0;
      for (int e = tid; e < m * m; e += nthr, ++cnt) A[e] = vnew[cnt < 4 ? cnt : 3];
      __syncthreads();
    }
    // convergence: off-diagonal mass against the whole
    double off = 0.0, all = 0.0;
    for (int e = tid; e < m * m; e += nthr) {
      const double a2 = A[e] * A[e];
      all += a2;
      if (e / m != e % m) off += a2;
    }
    off = block_allsum(off, red);
    all = block_allsum(all, red);
    if (!(off > 1e-32 * all)) break;
  }
  if (tid == 0) {
    for (int k = 0; k < m; ++k) perm[k] = k;
    for (int k = 1; k < m; ++k) {
      const int pk = perm[k];
      const double v = A[pk * m + pk];
      int j = k - 1;
      while (j >= 0 && A[perm[j] * m + perm[j]] > v) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = pk;
    }
    for (int k = 0; k < m; ++k) ev[k] = A[perm[k] * m + perm[k]];
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += nthr) {
    const int i = e / m, k = e % m;
    Vs[e] = V[i * m + perm[k]];
  }
  __syncthreads();
}

// Stencil weights of the unit-k Q1 operator around one node: w[o] for the
// neighbour offset o = (oz+1)*9 + (oy+1)*3 + (ox+1), given the conductivities
// kk[c] (c = cx + 2cy + 4cz) of the 8 surrounding elements (0 when absent).
MSMG_DEV void stencil27(const Stencil& st, const double kk[8], double w[27]) {
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
      const bool okx = (ox == 0) || (ox > 0 && cx == 1) || (ox < 0 && cx == 0);
      const bool oky = (oy == 0) || (oy > 0 && cy == 1) || (oy < 0 && cy == 0);
      const bool okz = (oz == 0) || (oz > 0 && cz == 1) || (oz < 0 && cz == 0);
      if (okx && oky && okz) s += kk[c];
    }
    const int nd = (ox != 0) + (oy != 0) + (oz != 0);
    double pat;
    if (nd == 0) pat = st.self;
    else if (nd == 3) pat = st.bd;
    else if (nd == 1) pat = st.ax[ox != 0 ? 0 : (oy != 0 ? 1 : 2)];
    else pat = st.fd[ox == 0 ? 0 : (oy == 0 ? 1 : 2)];
    w[o] = pat * s;
  }
}

}  // namespace msmg
