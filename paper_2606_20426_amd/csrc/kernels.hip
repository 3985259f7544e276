// HIP kernels (gfx950, wave64) of one implicit step of a batch of gel pads.
//
// Work is cut into tiles of one pad each (Tile{env, tile}); a launch covers
// the tiles of every pad in the batch, so uneven pads share each launch.
// Per-pad reductions are deterministic: every tile writes one partial, and
// the consumer kernel re-reduces the pad's partials in a fixed order (no
// atomics on floating point anywhere), so a pad's result does not depend on
// which other pads share the batch.
//
// Precision: R = float (mixed mode: element, assembly, SpMV, preconditioner)
// or double (FP64 mode).  Positions, residual, dot products, line-search
// energy and barrier terms are always double.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdint>

#include "../../include/tacauchy.h"
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

// ---------------------------------------------------------------- helpers

// Blocks are handed to the 8 XCDs round-robin by block index; give each XCD
// a contiguous run of tiles so that neighbouring tiles (which gather the same
// vertices) share that XCD's L2.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int t = (b & 7) * (G >> 3) + (b >> 3);
  return t < ntiles ? t : -1;
}

__device__ __forceinline__ bool running(const EnvState* S) {
  return S->phase == PH_RUN && S->status == TC_OK;
}

__device__ __forceinline__ bool initialising(const EnvState* S) {
  return S->phase == PH_INIT && S->status == TC_OK;
}

__device__ __forceinline__ bool at_stage(const EnvState* S, int stage) {
  return running(S) && S->stage == stage;
}

// the CG of this Newton iteration has ended: direction, filter and step
// bound pending
__device__ __forceinline__ bool dir_ready(const EnvState* S) {
  return running(S) && S->stage == ST_CG && S->cg_done;
}

// CG iterations pending (the first product moves the pad from ST_ASM to ST_CG)
__device__ __forceinline__ bool cg_running(const EnvState* S) {
  return running(S) && (S->stage == ST_ASM || S->stage == ST_CG) && !S->cg_done;
}

struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };

// Block-wide reduction, identical result in every thread.  Butterfly within
// each wave (pairs add in both orders -> bitwise equal lanes), then every
// thread folds the per-wave values in wave order.  Must be reached by all
// threads of the block.
template <class Op>
__device__ double block_reduce(double v, Op op, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < nw; ++k) r = op(r, sh[k]);
  return r;
}

template <class Op>
__device__ double reduce_partials(const double* p, int n, Op op, double init, double* sh) {
  double v = init;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v = op(v, p[i]);
  return block_reduce(v, op, sh);
}

template <typename R> __device__ __forceinline__ R rsq(R x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return 1.0f / sqrtf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

// ------------------------------------------------------- 3x3 eigen / SVD

// One cyclic-Jacobi rotation annihilating A[p][q]; Q accumulates the
// eigenvectors (columns).
template <int p, int q, typename R>
__device__ __forceinline__ void jacobi_rot(R A[3][3], R Q[3][3]) {
  const R apq = A[p][q];
  if (apq == R(0)) return;
  const R tau = (A[q][q] - A[p][p]) / (R(2) * apq);
  const R t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + sqrt(R(1) + tau * tau));
  const R c = rsq<R>(R(1) + t * t), s = t * c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R akp = A[k][p], akq = A[k][q];
    A[k][p] = c * akp - s * akq;
    A[k][q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R apk = A[p][k], aqk = A[q][k];
    A[p][k] = c * apk - s * aqk;
    A[q][k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R qkp = Q[k][p], qkq = Q[k][q];
    Q[k][p] = c * qkp - s * qkq;
    Q[k][q] = s * qkp + c * qkq;
  }
}

template <typename R> struct Eps;
template <> struct Eps<float> { static constexpr float v = 1e-7f; static constexpr int sweeps = 6; };
template <> struct Eps<double> { static constexpr double v = 1e-15; static constexpr int sweeps = 10; };

// Symmetric eigen-decomposition: A (destroyed) = Q diag(w) Q^T.
template <typename R>
__device__ void sym_eig3(R A[3][3], R Q[3][3], R w[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? R(1) : R(0);
  for (int sweep = 0; sweep < Eps<R>::sweeps; ++sweep) {
    const R off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const R dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= Eps<R>::v * Eps<R>::v * dia) break;
    jacobi_rot<0, 1>(A, Q);
    jacobi_rot<0, 2>(A, Q);
    jacobi_rot<1, 2>(A, Q);
  }
  w[0] = A[0][0]; w[1] = A[1][1]; w[2] = A[2][2];
}

template <int i, int j, typename R>
__device__ __forceinline__ void sort_pair(R V[3][3], R w[3]) {
  if (w[i] < w[j]) {
    const R t = w[i]; w[i] = w[j]; w[j] = t;
#pragma unroll
    for (int k = 0; k < 3; ++k) { const R a = V[k][i]; V[k][i] = V[k][j]; V[k][j] = a; }
  }
}

template <typename R>
__device__ __forceinline__ R det3(const R M[3][3]) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
       - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
       + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// Rotation-variant SVD F = U diag(s) V^T with U, V in SO(3) and s0 >= s1 >=
// |s2|, s2 < 0 for inverted elements.  V from the eigenvectors of F^T F,
// U by Gram-Schmidt on the columns of F V.
template <typename R>
__device__ void svd3(const R F[3][3], R U[3][3], R s[3], R V[3][3]) {
  R S[3][3], w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
  sym_eig3(S, V, w);
  sort_pair<0, 1>(V, w);
  sort_pair<0, 2>(V, w);
  sort_pair<1, 2>(V, w);
  if (det3(V) < R(0)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k][2] = -V[k][2];
  }
  R B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
  R u0[3] = {B[0][0], B[1][0], B[2][0]};
  R n0 = sqrt(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
  if (n0 > R(1e-30)) { u0[0] /= n0; u0[1] /= n0; u0[2] /= n0; }
  else { u0[0] = 1; u0[1] = 0; u0[2] = 0; n0 = 0; }
  R u1[3] = {B[0][1], B[1][1], B[2][1]};
  const R d01 = u0[0] * u1[0] + u0[1] * u1[1] + u0[2] * u1[2];
  u1[0] -= d01 * u0[0]; u1[1] -= d01 * u0[1]; u1[2] -= d01 * u0[2];
  R n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (n1 > Eps<R>::v * n0 + R(1e-30)) {
    u1[0] /= n1; u1[1] /= n1; u1[2] /= n1;
  } else {  // flattened element: any direction orthogonal to u0
    const R ex = fabs(u0[0]) < R(0.9) ? R(1) : R(0), ey = R(1) - ex;
    u1[0] = u0[1] * R(0) - u0[2] * ey;
    u1[1] = u0[2] * ex - u0[0] * R(0);
    u1[2] = u0[0] * ey - u0[1] * ex;
    const R m = rsq<R>(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    u1[0] *= m; u1[1] *= m; u1[2] *= m;
    n1 = 0;
  }
  const R u2[3] = {u0[1] * u1[2] - u0[2] * u1[1], u0[2] * u1[0] - u0[0] * u1[2],
                   u0[0] * u1[1] - u0[1] * u1[0]};
#pragma unroll
  for (int k = 0; k < 3; ++k) { U[k][0] = u0[k]; U[k][1] = u1[k]; U[k][2] = u2[k]; }
  s[0] = n0;
  s[1] = n1;
  s[2] = u2[0] * B[0][2] + u2[1] * B[1][2] + u2[2] * B[2][2];
}

// K += lam c c^T over the 10 stored blocks of the symmetric 12x12.
template <typename R>
__device__ __forceinline__ void rank1_update(R K[78], const R c[4][3], R lam) {
  int o = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      if (a == b) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = i; k < 3; ++k) K[o++] += lam * c[a][i] * c[a][k];
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = 0; k < 3; ++k) K[o++] += lam * c[a][i] * c[b][k];
      }
    }
}

// ------------------------------------------------ signed distance functions

// Local-frame distance, gradient and (optionally) Hessian of indenter shapes
// (see TC_SPHERE ... in tacauchy.h).
__device__ void sdf_local(int shape, const double* prm, const double y[3], double& phi,
                          double g[3], double H[3][3], bool wantH) {
  if (wantH)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i][j] = 0.0;
  if (shape == TC_SPHERE) {
    const double L = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    phi = L - prm[0];
    if (L > 0) {
      for (int i = 0; i < 3; ++i) g[i] = y[i] / L;
      if (wantH)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) H[i][j] = ((i == j ? 1.0 : 0.0) - g[i] * g[j]) / L;
    } else {
      g[0] = 0; g[1] = 0; g[2] = 1;
    }
    return;
  }
  if (shape == TC_BOX) {
    double q[3], sg[3];
    int npos = 0;
    for (int i = 0; i < 3; ++i) {
      sg[i] = y[i] >= 0 ? 1.0 : -1.0;
      q[i] = fabs(y[i]) - prm[i];
      npos += q[i] > 0;
    }
    if (npos >= 2) {
      double qp[3], L2 = 0;
      for (int i = 0; i < 3; ++i) { qp[i] = q[i] > 0 ? q[i] : 0.0; L2 += qp[i] * qp[i]; }
      const double L = sqrt(L2);
      phi = L;
      for (int i = 0; i < 3; ++i) g[i] = qp[i] * sg[i] / L;
      if (wantH)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            H[i][j] = ((i == j && q[i] > 0) ? 1.0 : 0.0) / L - g[i] * g[j] / L;
    } else {
      int k = 0;
      if (q[1] > q[k]) k = 1;
      if (q[2] > q[k]) k = 2;
      phi = q[k];
      g[0] = g[1] = g[2] = 0;
      g[k] = sg[k];
    }
    return;
  }
  if (shape == TC_TEXTURE) {
    const double A = prm[0], kk = 2.0 * M_PI / prm[1];
    const double c = sqrt(1.0 + (kk * A) * (kk * A));
    const double sx = sin(kk * y[0]), cx = cos(kk * y[0]);
    const double sy = sin(kk * y[1]), cy = cos(kk * y[1]);
    const double eta = A * sx * sy;
    phi = (eta - y[2]) / c;
    g[0] = A * kk * cx * sy / c;
    g[1] = A * kk * sx * cy / c;
    g[2] = -1.0 / c;
    if (wantH) {
      H[0][0] = -kk * kk * eta / c;
      H[1][1] = -kk * kk * eta / c;
      H[0][1] = H[1][0] = A * kk * kk * cx * cy / c;
    }
    return;
  }
  // axisymmetric shapes about local z: cylinder and torus
  const double rho = sqrt(y[0] * y[0] + y[1] * y[1]);
  double er[3] = {1.0, 0.0, 0.0};
  const double irho = rho > 0 ? 1.0 / rho : 1.0;
  if (rho > 0) { er[0] = y[0] * irho; er[1] = y[1] * irho; }
  // Hessian of rho: (I_xy - er er^T) / rho
  auto add_Hrho = [&](double w) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) H[i][j] += w * ((i == j ? 1.0 : 0.0) - er[i] * er[j]) * irho;
  };
  if (shape == TC_CYLINDER) {
    const double r = prm[0], a = prm[1];
    const double sz = y[2] >= 0 ? 1.0 : -1.0;
    const double qx = rho - r, qy = fabs(y[2]) - a;
    if (qx > 0 && qy > 0) {
      const double L = sqrt(qx * qx + qy * qy);
      phi = L;
      const double fr = qx / L, fz = qy / L;
      g[0] = fr * er[0]; g[1] = fr * er[1]; g[2] = fz * sz;
      if (wantH) {
        const double L3 = L * L * L;
        const double prr = qy * qy / L3, pzz = qx * qx / L3, prz = -qx * qy / L3;
        const double ez[3] = {0, 0, sz};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            H[i][j] = prr * er[i] * er[j] + pzz * ez[i] * ez[j] + prz * (er[i] * ez[j] + ez[i] * er[j]);
        add_Hrho(fr);
      }
    } else if (qx > 0 || (qx <= 0 && qy <= 0 && qx >= qy)) {
      phi = (qx > 0) ? qx : fmax(qx, qy);
      g[0] = er[0]; g[1] = er[1]; g[2] = 0;
      if (wantH) add_Hrho(1.0);
    } else {
      phi = (qy > 0) ? qy : fmax(qx, qy);
      g[0] = 0; g[1] = 0; g[2] = sz;
    }
    return;
  }
  // torus: | (rho - Rt, y_z) | - rt
  const double w0 = rho - prm[0], w1 = y[2];
  const double L = sqrt(w0 * w0 + w1 * w1);
  phi = L - prm[1];
  const double fr = w0 / L, fz = w1 / L;
  g[0] = fr * er[0]; g[1] = fr * er[1]; g[2] = fz;
  if (wantH) {
    const double L3 = L * L * L;
    const double prr = w1 * w1 / L3, pzz = w0 * w0 / L3, prz = -w0 * w1 / L3;
    const double ez[3] = {0, 0, 1};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        H[i][j] = prr * er[i] * er[j] + pzz * ez[i] * ez[j] + prz * (er[i] * ez[j] + ez[i] * er[j]);
    add_Hrho(fr);
  }
}

// ------------------------------------------------ rigid triangle meshes

// Closest point on triangle (a, b, c) to y by its Voronoi regions (Ericson,
// Real-Time Collision Detection, 2005, Sec. 5.1.5).  region: 0 face, 1..3
// vertex a, b, c, 4..6 edge ab, bc, ca.
__device__ __forceinline__ int tri_closest(const double* t, const double y[3], double c[3]) {
  const double a[3] = {t[0], t[1], t[2]}, b[3] = {t[3], t[4], t[5]}, q[3] = {t[6], t[7], t[8]};
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i]; ac[i] = q[i] - a[i]; ap[i] = y[i] - a[i]; bp[i] = y[i] - b[i]; cp[i] = y[i] - q[i];
  }
  auto dot = [](const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) { for (int i = 0; i < 3; ++i) c[i] = a[i]; return 1; }
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) { for (int i = 0; i < 3; ++i) c[i] = b[i]; return 2; }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    const double v = d1 / (d1 - d3);
    for (int i = 0; i < 3; ++i) c[i] = a[i] + v * ab[i];
    return 4;
  }
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) { for (int i = 0; i < 3; ++i) c[i] = q[i]; return 3; }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    const double w = d2 / (d2 - d6);
    for (int i = 0; i < 3; ++i) c[i] = a[i] + w * ac[i];
    return 6;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0 && d4 - d3 >= 0 && d5 - d6 >= 0) {
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    for (int i = 0; i < 3; ++i) c[i] = b[i] + w * (q[i] - b[i]);
    return 5;
  }
  const double den = 1.0 / (va + vb + vc);
  const double v = vb * den, w = vc * den;
  for (int i = 0; i < 3; ++i) c[i] = a[i] + v * ab[i] + w * ac[i];
  return 0;
}

// Signed distance to a closed mesh: nearest triangle over the BVH (nearer
// child first, subtrees pruned by box distance), sign from the pseudonormal
// of the closest feature (negative inside); gradient s (y - c) / d, Hessian
// 0 on a face, s (I - t t^T - g g^T) / d on an edge of direction t,
// s (I - g g^T) / d at a vertex.  Only triangles nearer than rmax are
// searched: with none, phi = +inf (callers that need phi only below d_hat
// pass d_hat, which prunes most of the tree for vertices away from the mesh;
// a point inside the mesh deeper than rmax would read as far outside, which
// the feasible start and the step bound rule out for every point they pass).
__device__ void mesh_sdf(const DevMesh& M, const double y[3], double& phi, double g[3], double H[3][3],
                         bool wantH, double rmax) {
  double best = rmax * rmax, cb[3] = {0, 0, 0};
  int bt = -1, br = 0;
  int stack[BVH_STACK];
  int sp = 0;
  stack[sp++] = 0;
  auto box_d2 = [&](const BvhNode& nd) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double v = fmax(fmax(nd.lo[i] - y[i], y[i] - nd.hi[i]), 0.0);
      s += v * v;
    }
    return s;
  };
  while (sp > 0) {
    const BvhNode& nd = M.nodes[stack[--sp]];
    if (box_d2(nd) >= best) continue;
    if (nd.count > 0) {
      for (int t = nd.first; t < nd.first + nd.count; ++t) {
        double c[3];
        const int r = tri_closest(M.tv + 9 * (size_t)t, y, c);
        const double d2 = (y[0] - c[0]) * (y[0] - c[0]) + (y[1] - c[1]) * (y[1] - c[1]) + (y[2] - c[2]) * (y[2] - c[2]);
        if (d2 < best) { best = d2; bt = t; br = r; cb[0] = c[0]; cb[1] = c[1]; cb[2] = c[2]; }
      }
    } else if (sp + 2 <= BVH_STACK) {
      const int l = (int)(&nd - M.nodes) + 1, r = nd.first;
      const double dl = box_d2(M.nodes[l]), dr = box_d2(M.nodes[r]);
      // nearer child on top
      if (dl <= dr) { stack[sp++] = r; stack[sp++] = l; }
      else { stack[sp++] = l; stack[sp++] = r; }
    }
  }
  if (wantH)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i][j] = 0.0;
  if (bt < 0) { phi = INFINITY; g[0] = g[1] = 0.0; g[2] = 1.0; return; }
  const int32_t* id = M.tid + 6 * (size_t)bt;
  const double* N = br == 0 ? M.tn + 3 * (size_t)bt
                  : br <= 3 ? M.vn + 3 * (size_t)id[br - 1]
                  : M.en + 3 * (size_t)id[3 + br - 4];
  const double diff[3] = {y[0] - cb[0], y[1] - cb[1], y[2] - cb[2]};
  const double s = diff[0] * N[0] + diff[1] * N[1] + diff[2] * N[2] >= 0 ? 1.0 : -1.0;
  const double d = sqrt(best);
  const double id_ = d > 0 ? 1.0 / d : 1.0;
  for (int i = 0; i < 3; ++i) g[i] = s * diff[i] * id_;
  phi = s * d;
  if (!wantH || br == 0) return;
  double t[3] = {0, 0, 0};
  if (br >= 4) {
    const double* T = M.tv + 9 * (size_t)bt;
    const int e0 = br - 4, e1 = (br - 4 + 1) % 3;
    for (int i = 0; i < 3; ++i) t[i] = T[3 * e1 + i] - T[3 * e0 + i];
    const double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int i = 0; i < 3; ++i) t[i] /= L;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      H[i][j] = s * id_ * ((i == j ? 1.0 : 0.0) - t[i] * t[j] - g[i] * g[j]);
}

// World frame: y = R^T (x - c), grad = R g, hess = R H R^T.
__device__ void sdf_world(const DevIndenter& ind, const DevMesh* meshes, const double x[3], double& phi,
                          double g[3], double H[3][3], bool wantH, double rmax = INFINITY) {
  const double dx[3] = {x[0] - ind.c[0], x[1] - ind.c[1], x[2] - ind.c[2]};
  double y[3];
  for (int i = 0; i < 3; ++i) y[i] = ind.R[0 * 3 + i] * dx[0] + ind.R[1 * 3 + i] * dx[1] + ind.R[2 * 3 + i] * dx[2];
  double gl[3], Hl[3][3];
  if (ind.shape == TC_MESH)
    mesh_sdf(meshes[ind.reserved], y, phi, gl, Hl, wantH, rmax);
  else
    sdf_local(ind.shape, ind.prm, y, phi, gl, Hl, wantH);
  for (int i = 0; i < 3; ++i) g[i] = ind.R[i * 3 + 0] * gl[0] + ind.R[i * 3 + 1] * gl[1] + ind.R[i * 3 + 2] * gl[2];
  if (wantH) {
    double T[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        T[i][j] = ind.R[i * 3 + 0] * Hl[0][j] + ind.R[i * 3 + 1] * Hl[1][j] + ind.R[i * 3 + 2] * Hl[2][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        H[i][j] = T[i][0] * ind.R[j * 3 + 0] + T[i][1] * ind.R[j * 3 + 1] + T[i][2] * ind.R[j * 3 + 2];
  }
}

__device__ __forceinline__ bool convex_shape(int s) {
  return s == TC_SPHERE || s == TC_CYLINDER || s == TC_BOX;
}

// IPC log barrier b(s) = -(s-1)^2 ln s on (0, 1) and its derivatives.
__device__ __forceinline__ double bar0(double s) {
  return s >= 1.0 ? 0.0 : (s <= 0.0 ? INFINITY : -(s - 1.0) * (s - 1.0) * log(s));
}
__device__ __forceinline__ double bar1(double s) {
  return (s >= 1.0 || s <= 0.0) ? 0.0 : -2.0 * (s - 1.0) * log(s) - (s - 1.0) * (s - 1.0) / s;
}
__device__ __forceinline__ double bar2(double s) {
  return (s >= 1.0 || s <= 0.0) ? 0.0
         : -2.0 * log(s) - 4.0 * (s - 1.0) / s + (s - 1.0) * (s - 1.0) / (s * s);
}

// Barrier of one pad vertex against a rigid mesh summed over its triangles
// nearer than d_hat (mesh_contact 1): per triangle t the unsigned distance
// d_t to the closed triangle, grad d_t = (y - c_t) / d_t and hess d_t as for
// the nearest feature (0 on the face, (I - t t^T - g g^T) / d on an edge,
// (I - g g^T) / d at a vertex).  World-frame results per unit kappa A:
// e = sum d_hat b(s_t), g = sum b'(s_t) grad d_t, H = sum b''(s_t) / d_hat
// grad grad^T + b'(s_t) hess d_t (wantH), Hn its first part; s_t = d_t /
// d_hat.  A vertex on a triangle (d_t = 0) gives e = +inf.
__device__ void mesh_pair_world(const DevIndenter& ind, const DevMesh* meshes, const double x[3], double dhat,
                                bool wantH, double& e, double g[3], double H[3][3], double Hn[3][3]) {
  const DevMesh& M = meshes[ind.reserved];
  double y[3];
  for (int i = 0; i < 3; ++i)
    y[i] = ind.R[0 * 3 + i] * (x[0] - ind.c[0]) + ind.R[1 * 3 + i] * (x[1] - ind.c[1]) +
           ind.R[2 * 3 + i] * (x[2] - ind.c[2]);
  double gl[3] = {0, 0, 0}, Hl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Hnl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  e = 0.0;
  const double r2 = dhat * dhat;
  int stack[BVH_STACK];
  int sp = 0;
  stack[sp++] = 0;
  auto box_d2 = [&](const BvhNode& nd) {
    double s2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double v = fmax(fmax(nd.lo[i] - y[i], y[i] - nd.hi[i]), 0.0);
      s2 += v * v;
    }
    return s2;
  };
  while (sp > 0) {
    const BvhNode& nd = M.nodes[stack[--sp]];
    if (box_d2(nd) >= r2) continue;
    if (nd.count > 0) {
      for (int t = nd.first; t < nd.first + nd.count; ++t) {
        double c[3];
        const double* T = M.tv + 9 * (size_t)t;
        const int r = tri_closest(T, y, c);
        const double df[3] = {y[0] - c[0], y[1] - c[1], y[2] - c[2]};
        const double d2 = df[0] * df[0] + df[1] * df[1] + df[2] * df[2];
        if (!(d2 < r2)) continue;
        const double d = sqrt(d2);
        const double s = d / dhat;
        e += dhat * bar0(s);
        if (!(d > 0.0)) continue;
        const double b1 = bar1(s);
        const double gd[3] = {df[0] / d, df[1] / d, df[2] / d};
        for (int i = 0; i < 3; ++i) gl[i] += b1 * gd[i];
        if (!wantH) continue;
        const double b2 = bar2(s) / dhat;
        double tv[3] = {0, 0, 0};
        if (r >= 4) {
          const int e0 = r - 4, e1 = (r - 4 + 1) % 3;
          for (int i = 0; i < 3; ++i) tv[i] = T[3 * e1 + i] - T[3 * e0 + i];
          const double L = sqrt(tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
          for (int i = 0; i < 3; ++i) tv[i] /= L;
        }
        const double curv = r == 0 ? 0.0 : b1 / d;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            const double nn = b2 * gd[i] * gd[j];
            Hnl[i][j] += nn;
            Hl[i][j] += nn + curv * ((i == j ? 1.0 : 0.0) - tv[i] * tv[j] - gd[i] * gd[j]);
          }
      }
    } else if (sp + 2 <= BVH_STACK) {
      stack[sp++] = nd.first;
      stack[sp++] = (int)(&nd - M.nodes) + 1;
    }
  }
  for (int i = 0; i < 3; ++i) g[i] = ind.R[i * 3 + 0] * gl[0] + ind.R[i * 3 + 1] * gl[1] + ind.R[i * 3 + 2] * gl[2];
  if (!wantH) return;
  auto rot = [&](const double A[3][3], double B[3][3]) {
    double T[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        T[i][j] = ind.R[i * 3 + 0] * A[0][j] + ind.R[i * 3 + 1] * A[1][j] + ind.R[i * 3 + 2] * A[2][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        B[i][j] = T[i][0] * ind.R[j * 3 + 0] + T[i][1] * ind.R[j * 3 + 1] + T[i][2] * ind.R[j * 3 + 2];
  };
  rot(Hl, H);
  rot(Hnl, Hn);
}

__device__ __forceinline__ void load3(const double* p, int i, double v[3]) {
  v[0] = p[3 * i]; v[1] = p[3 * i + 1]; v[2] = p[3 * i + 2];
}

// Step fractions the collision-free bounds cover: the line search may
// double an accepted full step up to this.
constexpr double FILTER_SPAN = 16.0;

// ------------------------------------------------ rigid-mesh pairs (mesh_contact 2)

// IPC's contact primitives between two surfaces are point-triangle and
// edge-edge pairs, both ways (Sec. III-B).  Besides the pad-vertex pairs
// above, mesh_contact 2 takes the two kinds whose pad side is a surface
// triangle or a surface edge:
//   vertex-face: mesh vertex y against pad triangle t, kappa a_y d_hat
//     b(d / d_hat), a_y a third of the area of y's mesh triangles;
//   edge-edge: mesh edge e against pad surface edge f, kappa w d_hat m(c)
//     b(d / d_hat) with w = |e| |f|_0 / 4 and IPC's mollifier m(c) =
//     (2 - c / c0) c / c0 below c0 = 1e-3 |e|^2 |f|_0^2 (1 above), c =
//     |e x f|^2: the term fades out as the edges turn parallel.
// d is the distance between the closed features.  With q = sum_a lam_a x_a
// the pad's closest point and u the unit vector from q to the mesh's
// closest point, dd/dx_a = -lam_a u (envelope theorem); dc/dx_1 = 2 (|e|^2
// f - (e.f) e) = -dc/dx_0.  Hessians are Gauss-Newton, w m b''/d_hat
// (grad d)(grad d)^T, positive semi-definite.
//
// Pad primitives are numbered j < S (surface triangles) and S + f (surface
// edges).  The mesh side is found through the mesh's hierarchy with the
// primitive's box grown by the query radius; a mesh vertex or edge is met
// once, through the leaf triangle that owns it.

// One pair as the kernels use it (world frame).
struct PairTerm {
  double d;         // distance between the features
  double lam[3];    // weights of the pad primitive's vertices at its closest point
  double u[3];      // unit vector from the pad's closest point to the mesh's (0 when d = 0)
  double diff[3];   // the same vector unnormalised
  double wt;        // weight without kappa: a_y, or |e| |f|_0 / 4
  double m, dm;     // mollifier and dm/dc (1 and 0 for vertex-face)
  double dc1[3];    // dc/dx_1 of the pad edge (edge-edge)
  double sep;       // separation along u: min over the mesh feature of w.u - max over the pad
                    // feature's vertices of x_a.u (a lower bound on the distance; 0 when d = 0)
  const double* w0; // the mesh feature in the mesh's frame: the vertex, or the edge's ends
  const double* w1; //   (null for a vertex)
  bool interior;    // both closest points interior to their features
};

// Closest point of triangle (a, b, c) to y by Voronoi regions (Ericson,
// Real-Time Collision Detection, 2005, Sec. 5.1.5), as barycentric weights;
// returns |y - q|^2 and diff = y - q.
__device__ double pt_tri_lam(const double y[3], const double a[3], const double b[3], const double c[3],
                             double lam[3], double diff[3]) {
  double ab[3], ac[3], ap[3], bp[3], cp[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = b[i] - a[i]; ac[i] = c[i] - a[i]; ap[i] = y[i] - a[i]; bp[i] = y[i] - b[i]; cp[i] = y[i] - c[i];
  }
  auto dot = [](const double* p, const double* q) { return p[0] * q[0] + p[1] * q[1] + p[2] * q[2]; };
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
  if (d1 <= 0 && d2 <= 0) {
    lam[0] = 1; lam[1] = 0; lam[2] = 0;
  } else if (d3 >= 0 && d4 <= d3) {
    lam[0] = 0; lam[1] = 1; lam[2] = 0;
  } else if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    const double v = d1 / (d1 - d3);
    lam[0] = 1 - v; lam[1] = v; lam[2] = 0;
  } else if (d6 >= 0 && d5 <= d6) {
    lam[0] = 0; lam[1] = 0; lam[2] = 1;
  } else if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    const double w = d2 / (d2 - d6);
    lam[0] = 1 - w; lam[1] = 0; lam[2] = w;
  } else if (va <= 0 && d4 - d3 >= 0 && d5 - d6 >= 0) {
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    lam[0] = 0; lam[1] = 1 - w; lam[2] = w;
  } else {
    const double den = 1.0 / (va + vb + vc);
    const double v = vb * den, w = vc * den;
    lam[0] = 1 - v - w; lam[1] = v; lam[2] = w;
  }
  double s = 0.0;
  for (int i = 0; i < 3; ++i) {
    diff[i] = y[i] - (lam[0] * a[i] + lam[1] * b[i] + lam[2] * c[i]);
    s += diff[i] * diff[i];
  }
  return s;
}

// Closest points of segments p0 p1 and q0 q1 (Ericson, Sec. 5.1.9): the
// lines' closest point parameter s on the first, clamped to [0, 1], the
// second's t for it, and if t leaves [0, 1] the clamped t with s recomputed.
// Parallel segments (denominator <= 1e-14 |d1|^2 |d2|^2) start from s = 0.
// Returns |p - q|^2 and diff = p - q.
__device__ double seg_seg(const double p0[3], const double p1[3], const double q0[3], const double q1[3],
                          double& s, double& t, double diff[3]) {
  double d1[3], d2[3], r[3];
  for (int i = 0; i < 3; ++i) { d1[i] = p1[i] - p0[i]; d2[i] = q1[i] - q0[i]; r[i] = p0[i] - q0[i]; }
  const double a = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
  const double e = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
  const double f = d2[0] * r[0] + d2[1] * r[1] + d2[2] * r[2];
  const double c = d1[0] * r[0] + d1[1] * r[1] + d1[2] * r[2];
  const double b = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
  const double den = a * e - b * b;
  s = den > 1e-14 * a * e ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
  t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = fmin(fmax(-c / a, 0.0), 1.0);
  } else if (t > 1.0) {
    t = 1.0;
    s = fmin(fmax((b - c) / a, 0.0), 1.0);
  }
  double q = 0.0;
  for (int i = 0; i < 3; ++i) {
    diff[i] = (p0[i] + s * d1[i]) - (q0[i] + t * d2[i]);
    q += diff[i] * diff[i];
  }
  return q;
}

// Leaves of M's hierarchy whose boxes meet [lo, hi]: leaf(s) per triangle
// slot s.
template <typename Leaf>
__device__ void bvh_overlap(const DevMesh& M, const double lo[3], const double hi[3], Leaf&& leaf) {
  int stack[BVH_STACK];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const BvhNode& nd = M.nodes[stack[--sp]];
    if (nd.lo[0] > hi[0] || nd.hi[0] < lo[0] || nd.lo[1] > hi[1] || nd.hi[1] < lo[1] || nd.lo[2] > hi[2] ||
        nd.hi[2] < lo[2])
      continue;
    if (nd.count > 0) {
      for (int s = nd.first; s < nd.first + nd.count; ++s) leaf(s);
    } else if (sp + 2 <= BVH_STACK) {
      stack[sp++] = nd.first;
      stack[sp++] = (int)(&nd - M.nodes) + 1;
    }
  }
}

__device__ __forceinline__ bool pair_active(const EnvDesc& E, const EnvPose* P) {
  return E.n_pt > 0 && P->pairs != 0;
}

// World positions of pad primitive j's vertices (3 for a triangle, 2 for an
// edge) from x; returns the count.
__device__ __forceinline__ int prim_verts(const EnvDesc& E, int j, int vid[3]) {
  if (j < E.S) {
    vid[0] = E.tris[3 * j]; vid[1] = E.tris[3 * j + 1]; vid[2] = E.tris[3 * j + 2];
    return 3;
  }
  const int f = j - E.S;
  vid[0] = E.sedge[2 * f]; vid[1] = E.sedge[2 * f + 1]; vid[2] = -1;
  return 2;
}

// Every pair of pad primitive j (vertices xw, world) with the mesh
// indenters nearer than r[m]: fn(m, PairTerm).
template <typename Fn>
__device__ void visit_pairs(const EnvDesc& E, const EnvPose* P, int j, const double xw[3][3], const double* r,
                            Fn&& fn) {
  const bool tri = j < E.S;
  const int nv = tri ? 3 : 2;
  const double len0 = tri ? 0.0 : E.sedge_len0[j - E.S];
  for (int m = 0; m < P->n_ind; ++m) {
    const DevIndenter& I = P->ind[m];
    if (I.shape != TC_MESH || !(r[m] > 0.0)) continue;
    const DevMesh& M = E.meshes[I.reserved];
    double xl[3][3], lo[3], hi[3];
    for (int k = 0; k < nv; ++k)
      for (int i = 0; i < 3; ++i)
        xl[k][i] = I.R[0 * 3 + i] * (xw[k][0] - I.c[0]) + I.R[1 * 3 + i] * (xw[k][1] - I.c[1]) +
                   I.R[2 * 3 + i] * (xw[k][2] - I.c[2]);
    for (int i = 0; i < 3; ++i) {
      lo[i] = xl[0][i];
      hi[i] = xl[0][i];
      for (int k = 1; k < nv; ++k) { lo[i] = fmin(lo[i], xl[k][i]); hi[i] = fmax(hi[i], xl[k][i]); }
      lo[i] -= r[m];
      hi[i] += r[m];
    }
    const double r2 = r[m] * r[m];
    auto world = [&](const double* l, double* w) {
      for (int i = 0; i < 3; ++i) w[i] = I.R[i * 3 + 0] * l[0] + I.R[i * 3 + 1] * l[1] + I.R[i * 3 + 2] * l[2];
    };
    auto outside = [&](const double* y) {
      return y[0] < lo[0] || y[0] > hi[0] || y[1] < lo[1] || y[1] > hi[1] || y[2] < lo[2] || y[2] > hi[2];
    };
    bvh_overlap(M, lo, hi, [&](int s) {
      const unsigned own = M.own[s];
      const int32_t* id = M.tid + 6 * (size_t)s;
      for (int k = 0; k < 3; ++k) {
        PairTerm pt;
        double dl[3];
        if (tri) {
          if (!((own >> k) & 1u)) continue;
          const int v = id[k];
          const double* y = M.mv + 3 * (size_t)v;
          if (outside(y)) continue;
          const double d2 = pt_tri_lam(y, xl[0], xl[1], xl[2], pt.lam, dl);
          if (!(d2 < r2)) continue;
          pt.d = sqrt(d2);
          pt.wt = M.va[v];
          pt.m = 1.0;
          pt.dm = 0.0;
          pt.dc1[0] = pt.dc1[1] = pt.dc1[2] = 0.0;
          pt.interior = pt.lam[0] > 0 && pt.lam[1] > 0 && pt.lam[2] > 0;
          pt.w0 = y;
          pt.w1 = nullptr;
          pt.sep = 0.0;
          if (pt.d > 0.0) {
            const double iu = 1.0 / pt.d;
            auto pr = [&](const double* q) { return (q[0] * dl[0] + q[1] * dl[1] + q[2] * dl[2]) * iu; };
            pt.sep = pr(y) - fmax(fmax(pr(xl[0]), pr(xl[1])), pr(xl[2]));
          }
        } else {
          if (!((own >> (3 + k)) & 1u)) continue;
          const int e = id[3 + k];
          const double* p0 = M.mv + 3 * (size_t)M.me[2 * e];
          const double* p1 = M.mv + 3 * (size_t)M.me[2 * e + 1];
          if (fmin(p0[0], p1[0]) > hi[0] || fmax(p0[0], p1[0]) < lo[0] || fmin(p0[1], p1[1]) > hi[1] ||
              fmax(p0[1], p1[1]) < lo[1] || fmin(p0[2], p1[2]) > hi[2] || fmax(p0[2], p1[2]) < lo[2])
            continue;
          double sp, tp;
          const double d2 = seg_seg(p0, p1, xl[0], xl[1], sp, tp, dl);
          if (!(d2 < r2)) continue;
          pt.d = sqrt(d2);
          pt.lam[0] = 1.0 - tp; pt.lam[1] = tp; pt.lam[2] = 0.0;
          const double le = M.mel[e];
          pt.wt = 0.25 * le * len0;
          double ev[3], fv[3], cr[3];
          for (int i = 0; i < 3; ++i) { ev[i] = p1[i] - p0[i]; fv[i] = xl[1][i] - xl[0][i]; }
          cr[0] = ev[1] * fv[2] - ev[2] * fv[1];
          cr[1] = ev[2] * fv[0] - ev[0] * fv[2];
          cr[2] = ev[0] * fv[1] - ev[1] * fv[0];
          const double cc = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
          const double c0 = 1e-3 * le * le * len0 * len0;
          const double xq = cc / c0;
          pt.m = xq < 1.0 ? (2.0 - xq) * xq : 1.0;
          pt.dm = xq < 1.0 ? (2.0 - 2.0 * xq) / c0 : 0.0;
          const double ee = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
          const double ef = ev[0] * fv[0] + ev[1] * fv[1] + ev[2] * fv[2];
          double dcl[3];
          for (int i = 0; i < 3; ++i) dcl[i] = 2.0 * (ee * fv[i] - ef * ev[i]);
          world(dcl, pt.dc1);
          pt.interior = sp > 0.0 && sp < 1.0 && tp > 0.0 && tp < 1.0;
          pt.w0 = p0;
          pt.w1 = p1;
          pt.sep = 0.0;
          if (pt.d > 0.0) {
            const double iu = 1.0 / pt.d;
            auto pr = [&](const double* q) { return (q[0] * dl[0] + q[1] * dl[1] + q[2] * dl[2]) * iu; };
            pt.sep = fmin(pr(p0), pr(p1)) - fmax(pr(xl[0]), pr(xl[1]));
          }
        }
        world(dl, pt.diff);
        const double id_ = pt.d > 0.0 ? 1.0 / pt.d : 0.0;
        for (int i = 0; i < 3; ++i) pt.u[i] = pt.diff[i] * id_;
        fn(m, pt);
      }
    });
  }
}

// Loads pad primitive j's vertex positions x (+ al * d when d is given).
template <typename R>
__device__ __forceinline__ int prim_load(const EnvDesc& E, int j, const double* x, const R* d, double al, int vid[3],
                                         double xw[3][3]) {
  const int nv = prim_verts(E, j, vid);
  for (int k = 0; k < nv; ++k)
    for (int c = 0; c < 3; ++c)
      xw[k][c] = x[3 * vid[k] + c] + (d ? al * (double)d[3 * vid[k] + c] : 0.0);
  return nv;
}

// Pair energy of primitive j at positions xw (barrier units: the h^2 factor
// is the caller's); +inf for a touching pair.
__device__ double prim_pair_energy(const EnvDesc& E, const EnvPose* P, int j, const double xw[3][3]) {
  double r[MAX_IND];
  for (int m = 0; m < MAX_IND; ++m) r[m] = E.dhat;
  double e = 0.0;
  visit_pairs(E, P, j, xw, r, [&](int, const PairTerm& pt) {
    if (pt.m > 0.0) e += E.kappa * pt.wt * E.dhat * pt.m * bar0(pt.d / E.dhat);
  });
  return e;
}

// ------------------------------------------------ friction (lagged, smoothed)

// C1 mollifier of the slip y with threshold eps: f0 (potential), f1 = f0'
// as f1 / y (finite at y = 0) and f1'; f1 rises from 0 to 1 on [0, eps].
__device__ __forceinline__ double fr_f0(double y, double eps) {
  return y < eps ? -y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0 : y;
}
__device__ __forceinline__ double fr_f1_over_y(double y, double eps) {
  return y < eps ? 2.0 / eps - y / (eps * eps) : 1.0 / y;
}
__device__ __forceinline__ double fr_f1p(double y, double eps) {
  return y < eps ? 2.0 / eps - 2.0 * y / (eps * eps) : 0.0;
}

__device__ __forceinline__ const double* fr_rec(const EnvDesc& E, int m, int k) {
  return E.fric + ((size_t)m * E.C + k) * FRIC_STRIDE;
}

// Tangential slip over the step against one lagged record:
// u = (I - n n^T)((x - x_t) - w); returns |u|.
__device__ __forceinline__ double fr_slip(const double* f, const double x[3], const double xt[3], double u[3]) {
  double r[3];
  for (int i = 0; i < 3; ++i) r[i] = (x[i] - xt[i]) - f[FRIC_W + i];
  const double rn = r[0] * f[FRIC_N] + r[1] * f[FRIC_N + 1] + r[2] * f[FRIC_N + 2];
  for (int i = 0; i < 3; ++i) u[i] = r[i] - rn * f[FRIC_N + i];
  return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

// Friction part of the step potential per dt^2 at one contact vertex:
// sum_m mu lambda_m f0(|u_m|).
__device__ __forceinline__ double fr_energy(const EnvDesc& E, int n_ind, int k, const double x[3],
                                            const double xt[3]) {
  double e = 0.0;
  for (int m = 0; m < n_ind; ++m) {
    const double* f = fr_rec(E, m, k);
    if (!(f[FRIC_LAM] > 0)) continue;
    double u[3];
    e += E.fr_mu * f[FRIC_LAM] * fr_f0(fr_slip(f, x, xt, u), E.fr_eps);
  }
  return e;
}

// ------------------------------------------------ kinematics (cancellation-free)

// Displacement gradient H = Du Dm^-1 with Du formed from float64 displacement
// differences (u = x - X), so F = I + H carries no O(1) rounding at rest.
template <typename R>
__device__ __forceinline__ void disp_gradient(const double* x, const double* X, const int4 tv,
                                              const R Dm[3][3], R H[3][3]) {
  const int vv[4] = {tv.x, tv.y, tv.z, tv.w};
  double u[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[a][c] = x[3 * vv[a] + c] - X[3 * vv[a] + c];
  R Du[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) Du[i][b] = (R)(u[b + 1][i] - u[0][i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) H[i][j] = Du[i][0] * Dm[0][j] + Du[i][1] * Dm[1][j] + Du[i][2] * Dm[2][j];
}

// cofactor matrix (cof M)_ij = d det M / dM_ij
template <typename R>
__device__ __forceinline__ void cofactor3(const R M[3][3], R C[3][3]) {
  C[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  C[0][1] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  C[0][2] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  C[1][0] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
  C[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
  C[1][2] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
  C[2][0] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  C[2][1] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  C[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
}

// From H: J - 1 = I1 + I2 + I3 (invariants of H) and dC = cof F - I =
// tr(H) I - H^T + cof H, both without cancellation for small H.
template <typename R>
__device__ __forceinline__ R kinematics(const R H[3][3], R dC[3][3]) {
  const R tr = H[0][0] + H[1][1] + H[2][2];
  R trHH = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) trHH += H[i][j] * H[j][i];
  R cH[3][3];
  cofactor3(H, cH);
  const R I3 = H[0][0] * cH[0][0] + H[0][1] * cH[0][1] + H[0][2] * cH[0][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dC[i][j] = (i == j ? tr : R(0)) - H[j][i] + cH[i][j];
  return tr + R(0.5) * (tr * tr - trHH) + I3;
}

// ------------------------------------------------------------ setup (a1)

// Per tet: Dm^-1 and V_e = det(Dm) / 6 from rest positions (float64 math).
template <typename R>
__global__ void k_setup_tets(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const int e = tiles[t].tile * blockDim.x + threadIdx.x;
  if (e >= E.T) return;
  const int4 tv = reinterpret_cast<const int4*>(E.tets)[e];
  double x0[3], x1[3], x2[3], x3[3];
  load3(E.X, tv.x, x0); load3(E.X, tv.y, x1); load3(E.X, tv.z, x2); load3(E.X, tv.w, x3);
  double D[3][3];
  for (int i = 0; i < 3; ++i) { D[i][0] = x1[i] - x0[i]; D[i][1] = x2[i] - x0[i]; D[i][2] = x3[i] - x0[i]; }
  const double det = det3(D);
  double inv[3][3];
  inv[0][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) / det;
  inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
  inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
  inv[1][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) / det;
  inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
  inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
  inv[2][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) / det;
  inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
  inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
  R* Dm = (R*)E.Dminv + 9 * e;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Dm[3 * i + j] = (R)inv[i][j];
  ((R*)E.vol)[e] = (R)(det / 6.0);
}

// Per vertex: lumped mass m_a = sum_e rho_e V_e / 4 gathered over the
// vertex's incident tets (its diagonal contribution list).
template <typename R>
__global__ void k_setup_mass(const Tile* tiles, int ntiles, const EnvDesc* envs, double* mass_out) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const int i = tiles[t].tile * blockDim.x + threadIdx.x;
  if (i >= E.V) return;
  double m = 0.0;
  const size_t it0 = (size_t)i * E.W;
  for (int c = E.cptr[it0]; c < E.cptr[it0 + 1]; ++c) {
    const int e = (int)(E.clist[c] >> 4);
    const int4 tv = reinterpret_cast<const int4*>(E.tets)[e];
    double x0[3], x1[3], x2[3], x3[3];
    load3(E.X, tv.x, x0); load3(E.X, tv.y, x1); load3(E.X, tv.z, x2); load3(E.X, tv.w, x3);
    double D[3][3];
    for (int k = 0; k < 3; ++k) { D[k][0] = x1[k] - x0[k]; D[k][1] = x2[k] - x0[k]; D[k][2] = x3[k] - x0[k]; }
    const int mid = E.mat ? E.mat[e] : 0;
    m += E.rho[mid] * (det3(D) / 6.0) / 4.0;
  }
  mass_out[i] = m;
}

// Per contact vertex: rest barrier weight A_k = 1/3 sum of the areas of its
// triangles (incident contact-face triangles; a side-face vertex: all its
// incident surface triangles).
__global__ void k_setup_cand_area(const Tile* tiles, int ntiles, const EnvDesc* envs, double* area_out) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const int k = tiles[t].tile * blockDim.x + threadIdx.x;
  if (k >= E.C) return;
  double A = 0.0;
  for (int c = E.ctri_ptr[k]; c < E.ctri_ptr[k + 1]; ++c) {
    const int j = E.ctri_idx[c];
    double v0[3], v1[3], v2[3];
    load3(E.X, E.tris[3 * j], v0); load3(E.X, E.tris[3 * j + 1], v1); load3(E.X, E.tris[3 * j + 2], v2);
    const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    A += 0.5 * sqrt(cx * cx + cy * cy + cz * cz) / 3.0;
  }
  area_out[k] = A;
}

// ------------------------------------------------------ predict (a2)

// xhat = x + h v + h^2 g_ext; Newton starts from x (or x + h v on free
// components when init_guess is set).
//
// With friction on, contact vertices also take the friction lag at x_t under
// the previous poses, per indenter m: lambda = -kappa A b'(phi / d_hat),
// n = grad(phi), and the motion over the step of the indenter's material
// point at x_t, w = R R_prev^T (x_t - c_prev) + c - x_t.
__global__ void k_predict(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  if (!initialising(E.st)) return;
  const int i = tiles[t].tile * blockDim.x + threadIdx.x;
  if (i >= E.V) return;
  const double h = E.h;
  const uint8_t fm = E.fixed[i];
  for (int c = 0; c < 3; ++c) {
    const double x = E.x[3 * i + c];
    E.xhat[3 * i + c] = x + h * E.v[3 * i + c] + h * h * E.gravity[c];
    E.xn[3 * i + c] = (E.init_guess && !((fm >> c) & 1)) ? x + h * E.v[3 * i + c] : x;
  }
  const int k = E.cand_of_vert[i];
  if (!(E.fr_mu > 0) || k < 0) return;
  const EnvPose* P = E.pose;
  double xt[3], H[3][3];
  load3(E.x, i, xt);
  const double kA = E.kappa * E.cand_area[k];
  for (int m = 0; m < P->n_ind; ++m) {
    const DevIndenter& A = P->prev[m];
    const DevIndenter& B = P->ind[m];
    double phi, n[3], loc[3], lam;
    if (E.mesh_pairs && A.shape == TC_MESH) {
      // the summed pair force -kappa A sum_t b'(s_t) grad d_t: lambda its
      // length, n its direction
      double gs[3], Hn[3][3];
      mesh_pair_world(A, E.meshes, xt, E.dhat, false, phi, gs, H, Hn);
      const double gm = sqrt(gs[0] * gs[0] + gs[1] * gs[1] + gs[2] * gs[2]);
      lam = kA * gm;
      for (int j = 0; j < 3; ++j) n[j] = gm > 0.0 ? -gs[j] / gm : 0.0;
    } else {
      // lambda n = the barrier force: n the unit normal, lambda the force's
      // length (phi of the texture plate is not a distance, |grad phi| < 1)
      sdf_world(A, E.meshes, xt, phi, n, H, false, E.dhat);
      const double gn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      lam = phi < E.dhat ? -kA * bar1(phi / E.dhat) * gn : 0.0;
      if (gn > 0.0)
        for (int j = 0; j < 3; ++j) n[j] /= gn;
    }
    for (int j = 0; j < 3; ++j)
      loc[j] = A.R[0 * 3 + j] * (xt[0] - A.c[0]) + A.R[1 * 3 + j] * (xt[1] - A.c[1]) + A.R[2 * 3 + j] * (xt[2] - A.c[2]);
    double* f = E.fric + ((size_t)m * E.C + k) * FRIC_STRIDE;
    f[FRIC_LAM] = lam;
    for (int j = 0; j < 3; ++j) {
      f[FRIC_N + j] = n[j];
      f[FRIC_W + j] = B.R[j * 3 + 0] * loc[0] + B.R[j * 3 + 1] * loc[1] + B.R[j * 3 + 2] * loc[2] + B.c[j] - xt[j];
    }
    f[7] = 0.0;
  }
}

// Feasible start: contact vertices closer than 0.1 d_hat to an indenter are
// pushed out along grad(phi) (free components only), at most 8 rounds.
// mode 0: all rounds, then the check phi > 0 (pads without pairs); for pads
// with vertex-face / edge-edge pairs the rounds alternate with the
// primitives' pushes (k_pair_push, k_pair_apply): mode 1 is one round,
// mode 2 the check.
__global__ void k_project(const Tile* tiles, int ntiles, const EnvDesc* envs, int mode) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  EnvState* S = E.st;
  const EnvPose* P = E.pose;
  if (!initialising(S)) return;
  if (pair_active(E, P) != (mode != 0)) return;
  const int k = tiles[t].tile * blockDim.x + threadIdx.x;
  if (k >= E.C) return;
  const int vi = E.cand[k];
  const uint8_t fm = E.fixed[vi];
  double x[3];
  load3(E.xn, vi, x);
  const double dsafe = 0.1 * E.dhat;
  double H[3][3];
  const int rounds = mode == 0 ? 8 : mode == 1 ? 1 : 0;
  for (int round = 0; round < rounds; ++round) {
    bool moved = false;
    for (int m = 0; m < P->n_ind; ++m) {
      double phi, g[3];
      sdf_world(P->ind[m], E.meshes, x, phi, g, H, false);
      if (phi < dsafe * (1.0 - 1e-9)) {
        moved = true;
        for (int c = 0; c < 3; ++c)
          if (!((fm >> c) & 1)) x[c] += (dsafe - phi) * g[c];
      }
    }
    if (!moved) break;
  }
  for (int c = 0; c < 3; ++c) E.xn[3 * vi + c] = x[c];
  if (mode == 1) return;
  double dmin = INFINITY;
  for (int m = 0; m < P->n_ind; ++m) {
    double phi, g[3];
    sdf_world(P->ind[m], E.meshes, x, phi, g, H, false);
    dmin = fmin(dmin, phi);
  }
  if (!(dmin > 0.0)) atomicOr(&S->infeasible, 1);
}

// ------------------------------------------------------ element (a3)

// Per tet: F = Ds Dm^-1, P (Eq. 2 with shift alpha), gradient V_e P G_a^T and
// the PSD-projected element Hessian from the analytic eigensystem of
// d2Psi/dF2 in the SVD frame of F:
//   twist/flip pairs (i,j; k the third index): mu +/- lam (J - alpha) s_k,
//   modes (u_i v_j^T -/+ u_j v_i^T) / sqrt 2;
//   scaling block: mu I + lam cof(S) cof(S)^T + lam (J - alpha) d2J/ds2,
//   a 3x3 symmetric eigenproblem, modes U diag(w) V^T.
// Negative eigenvalues are dropped; K_e = V_e sum lam+ c c^T with
// c = Q G^T (Q the 3x3 mode, G the shape-function gradients).
template <typename R>
__global__ void __launch_bounds__(256) k_element(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  if (!at_stage(E.st, ST_ASM)) return;
  const int e = tiles[t].tile * blockDim.x + threadIdx.x;
  if (e >= E.T) return;
  const int4 tv = reinterpret_cast<const int4*>(E.tets)[e];
  const R* Dmp = (const R*)E.Dminv + 9 * e;
  R Dm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[i][j] = Dmp[3 * i + j];
  R H[3][3];
  disp_gradient(E.xn, E.X, tv, Dm, H);
  const int mid = E.mat ? E.mat[e] : 0;
  const R mu = (R)E.mu[mid], lam = (R)E.lam[mid], csh = (R)E.cshift[mid];
  const R vol = ((const R*)E.vol)[e];
  R dC[3][3];
  const R Jm1 = kinematics(H, dC);
  // lam (J - alpha) = lam (J - 1) - c with c = lam (alpha - 1) (= mu for the
  // rest-stable shift, 0 for alpha = 1)
  const R sJ = lam * Jm1 - csh;
  R F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = H[i][j] + (i == j ? R(1) : R(0));

  R rec[KE_STRIDE];
#pragma unroll
  for (int k = 0; k < KE_STRIDE; ++k) rec[k] = R(0);

  // gradient: vertex a >= 1 gets V P Dm^-T column a-1; vertex 0 minus the sum
  {
    // Eq. 2, P = mu F + lam (J - alpha) cof F, regrouped so every term is
    // O(H): (mu - c + lam (J-1)) I + mu H + (lam (J-1) - c) (cof F - I)
    R P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        P[i][j] = (i == j ? mu - csh + lam * Jm1 : R(0)) + mu * H[i][j] + (lam * Jm1 - csh) * dC[i][j];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R s0 = 0;
#pragma unroll
      for (int a = 1; a < 4; ++a) {
        const R ga = vol * (P[i][0] * Dm[a - 1][0] + P[i][1] * Dm[a - 1][1] + P[i][2] * Dm[a - 1][2]);
        rec[KE_GRAD + 3 * a + i] = ga;
        s0 += ga;
      }
      rec[KE_GRAD + i] = -s0;
    }
  }

  // element eigenvalue filter: 0 clamp, 1 absolute value, 2 clamp until a
  // full Newton step is accepted, then unfiltered (true Hessian)
  const int emode = E.hess_proj & 3;
  const bool unfiltered = emode == 2 && E.st->true_hess;
  R U[3][3], sv[3], V[3][3];
  svd3(F, U, sv, V);
  // h[l][a] = v_l . G_a
  R hh[3][4];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    R s0 = 0;
#pragma unroll
    for (int a = 1; a < 4; ++a) {
      hh[l][a] = V[0][l] * Dm[a - 1][0] + V[1][l] * Dm[a - 1][1] + V[2][l] * Dm[a - 1][2];
      s0 += hh[l][a];
    }
    hh[l][0] = -s0;
  }
  const R isq2 = R(0.70710678118654752440);
  // twist / flip modes
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int i = pr == 2 ? 1 : 0;
    const int j = pr == 0 ? 1 : 2;
    const int k = 3 - i - j;
    R ltw = mu + sJ * sv[k];
    R lfl = mu - sJ * sv[k];
    if (emode == 1) { ltw = fabs(ltw); lfl = fabs(lfl); }
    R c[4][3];
    if (ltw > R(0) || (unfiltered && ltw != R(0))) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int m = 0; m < 3; ++m) c[a][m] = isq2 * (U[m][i] * hh[j][a] - U[m][j] * hh[i][a]);
      rank1_update(rec, c, vol * ltw);
    }
    if (lfl > R(0) || (unfiltered && lfl != R(0))) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int m = 0; m < 3; ++m) c[a][m] = isq2 * (U[m][i] * hh[j][a] + U[m][j] * hh[i][a]);
      rank1_update(rec, c, vol * lfl);
    }
  }
  // scaling block
  {
    const R gh[3] = {sv[1] * sv[2], sv[0] * sv[2], sv[0] * sv[1]};
    R As[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) As[l][m] = lam * gh[l] * gh[m] + (l == m ? mu : R(0));
    As[0][1] += sJ * sv[2]; As[1][0] += sJ * sv[2];
    As[0][2] += sJ * sv[1]; As[2][0] += sJ * sv[1];
    As[1][2] += sJ * sv[0]; As[2][1] += sJ * sv[0];
    R Qs[3][3], ws[3];
    sym_eig3(As, Qs, ws);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (emode == 1) ws[m] = fabs(ws[m]);
      if (ws[m] > R(0) || (unfiltered && ws[m] != R(0))) {
        R c[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int r = 0; r < 3; ++r)
            c[a][r] = Qs[0][m] * hh[0][a] * U[r][0] + Qs[1][m] * hh[1][a] * U[r][1] +
                      Qs[2][m] * hh[2][a] * U[r][2];
        rank1_update(rec, c, vol * ws[m]);
      }
    }
  }
  // scatter the 4 diagonal and 6 edge blocks to their places in the streams
  R* Kd = (R*)E.Ke;
  R* Ko = Kd + (size_t)KC * 4 * E.T;
  const int32_t* cp = E.cpos + 10 * (size_t)e;
  const int vv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    R* o = Kd + (size_t)KC * cp[a];
    const R* p = rec + ke_block_offset(a, a);
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = p[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) o[6 + r] = rec[KE_GRAD + 3 * a + r];
  }
  // edge k = (a, b): block (row min, column max) of the edge, i.e. (a, b) or
  // its transpose (constant a, b per call: no indexed local arrays)
  auto edge_out = [&](int k, int a, int b) {
    R* o = Ko + (size_t)KC * cp[4 + k];
    const R* p = rec + ke_block_offset(a, b);
    if (vv[a] < vv[b]) {
#pragma unroll
      for (int q = 0; q < 9; ++q) o[q] = p[q];
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) o[3 * r + q] = p[3 * q + r];
    }
  };
  edge_out(0, 0, 1); edge_out(1, 0, 2); edge_out(2, 0, 3);
  edge_out(3, 1, 2); edge_out(4, 1, 3); edge_out(5, 2, 3);
}

// ------------------------------------------------------ rigid-mesh pairs (a4, mesh_contact 2)

__device__ __forceinline__ bool extract_ok(const EnvState* S);

template <typename R>
__device__ double prim_pair_bound(const EnvDesc& E, const EnvPose* P, int j, const R* d, double span);

// Per surface primitive (pad triangles, then surface edges) of pads with
// vertex-face / edge-edge pairs:
//   mode 0: records at the Newton iterate (pads running), mode 1: at the
//           extraction positions: gradient and Gauss-Newton blocks of the
//           primitive's pairs within d_hat, flag 0 for a primitive without
//           pairs (its record is then not written);
//   mode 2: pair energy at the line search's trial x + alpha d (pads still
//           searching), mode 4: at the start x (pads being initialised),
//           partial sums after the barrier's in the energy partials;
//   mode 3: the pairs' step bound along the Newton direction, partial
//           minima after the contact vertices' in the filter partials.
// The pair work has its own launches so that its traversal state does not
// raise the register use of the energy and filter kernels.
template <typename R>
__global__ void k_pairs(const Tile* tiles, int ntiles, const EnvDesc* envs, int mode) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  const EnvState* S = E.st;
  const EnvPose* P = E.pose;
  if (!pair_active(E, P)) return;
  const int j = tl.tile * blockDim.x + threadIdx.x;
  if (mode >= 2) {
    // block reductions: every thread of the block takes part
    if (mode == 2 ? (!at_stage(S, ST_LS) || S->ls_done) : mode == 4 ? !initialising(S) : !dir_ready(S)) return;
    const bool in = j < E.S + E.Se;
    if (mode == 3) {
      double a = INFINITY;
      if (in) a = fmin(prim_pair_bound<R>(E, P, j, (const R*)E.d, FILTER_SPAN), FILTER_SPAN);
      a = block_reduce(a, OpMin(), sh);
      if (threadIdx.x == 0) E.part_filt[E.n_ct + tl.tile] = a;
      return;
    }
    double e = 0.0;
    if (in) {
      int vid[3];
      double xw[3][3];
      prim_load<R>(E, j, E.xn, mode == 2 ? (const R*)E.d : nullptr, mode == 2 ? S->ls_alpha : 0.0, vid, xw);
      e = prim_pair_energy(E, P, j, xw);
    }
    e = block_reduce(e, OpSum(), sh);
    if (threadIdx.x == 0) E.part_e[E.n_te + E.n_vt + E.n_ct + tl.tile] = e;
    return;
  }
  if (mode == 0 ? !at_stage(S, ST_ASM) : !extract_ok(S)) return;
  if (j >= E.S + E.Se) return;
  const double* x = (mode == 1 && S->mode == 1) ? E.x : E.xn;
  int vid[3];
  double xw[3][3];
  prim_load<double>(E, j, x, nullptr, 0.0, vid, xw);
  double r[MAX_IND];
  for (int m = 0; m < MAX_IND; ++m) r[m] = E.dhat;
  int n = 0;
  // a primitive has few pairs: each adds straight into the record (cleared
  // at the first), which keeps the 45 sums out of registers
  double* rec = E.prec + (size_t)PREC * j;
  visit_pairs(E, P, j, xw, r, [&](int, const PairTerm& pt) {
    if (n++ == 0)
      for (int q = 0; q < 45; ++q) rec[q] = 0.0;
    const double s = pt.d / E.dhat;
    const double w = E.kappa * pt.wt;
    const double b0 = bar0(s), b1 = bar1(s), b2 = bar2(s);
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 3; ++i) {
        // w d_hat dm b sign(a) dc/dx_1 (edge-edge) + w m b' dd/dx_a
        double ga = -w * pt.m * b1 * pt.lam[a] * pt.u[i];
        if (pt.dm != 0.0 && a < 2) ga += w * E.dhat * pt.dm * b0 * (a == 1 ? 1.0 : -1.0) * pt.dc1[i];
        rec[3 * a + i] += ga;
      }
    // vertex pairs of the blocks (0,0) (1,1) (2,2) (0,1) (1,2) (2,0)
    const double c2 = w * pt.m * b2 / E.dhat;
    const double uu[6] = {pt.u[0] * pt.u[0], pt.u[0] * pt.u[1], pt.u[0] * pt.u[2],
                          pt.u[1] * pt.u[1], pt.u[1] * pt.u[2], pt.u[2] * pt.u[2]};
    const double la[6] = {pt.lam[0] * pt.lam[0], pt.lam[1] * pt.lam[1], pt.lam[2] * pt.lam[2],
                          pt.lam[0] * pt.lam[1], pt.lam[1] * pt.lam[2], pt.lam[2] * pt.lam[0]};
    for (int q = 0; q < 6; ++q)
      for (int c = 0; c < 6; ++c) rec[9 + 6 * q + c] += c2 * la[q] * uu[c];
  });
  E.pflag[j] = n > 0;
}

// Outward direction of pad primitive j at positions x: a triangle's unit
// normal, or for a surface edge the normalised sum of its two triangles'.
__device__ __forceinline__ void prim_outward(const EnvDesc& E, int j, const double* x, double n[3]) {
  auto tri_n = [&](int tj, double* o) {
    const int a = E.tris[3 * tj], b = E.tris[3 * tj + 1], c = E.tris[3 * tj + 2];
    double e1[3], e2[3];
    for (int i = 0; i < 3; ++i) { e1[i] = x[3 * b + i] - x[3 * a + i]; e2[i] = x[3 * c + i] - x[3 * a + i]; }
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double L = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int i = 0; i < 3; ++i) o[i] += cr[i] / L;
  };
  n[0] = n[1] = n[2] = 0.0;
  if (j < E.S) {
    tri_n(j, n);
    return;
  }
  const int f = j - E.S;
  for (int q = 0; q < 2; ++q) {
    const int code = E.sedge_adj[2 * f + q];
    if (code >= 0) tri_n(code >> 3, n);
  }
  const double L = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int i = 0; i < 3; ++i) n[i] /= L;
}

// Feasible start, pads with pairs: a mesh vertex or edge that the
// indenter's jump to its new pose carried through the pad surface shows as
// a pair with both closest points interior and the mesh feature on the
// inner side (sd < 0, the vector between the closest points within 60
// degrees of the primitive's normal line).  mode 0: a primitive whose pairs (within the mesh's travel
// plus d_hat) come below d_safe along its outward direction n asks its
// vertices to move by (sd - d_safe) n for its deepest pair: the push and
// its length go to its record, and k_pair_apply moves each vertex by the
// longest push asked of it.  mode 1 (after the last round): any pair still
// on the inner side makes the start infeasible.
__global__ void k_pair_push(const Tile* tiles, int ntiles, const EnvDesc* envs, int mode) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  EnvState* S = E.st;
  const EnvPose* P = E.pose;
  if (!initialising(S) || !pair_active(E, P)) return;
  const int j = tiles[t].tile * blockDim.x + threadIdx.x;
  if (j >= E.S + E.Se) return;
  int vid[3];
  double xw[3][3];
  prim_load<double>(E, j, E.xn, nullptr, 0.0, vid, xw);
  double r[MAX_IND];
  for (int m = 0; m < MAX_IND; ++m) r[m] = P->travel[m] + E.dhat;
  double n[3];
  prim_outward(E, j, E.xn, n);
  const double dsafe = 0.1 * E.dhat;
  const double below = mode == 0 ? dsafe * (1.0 - 1e-9) : 0.0;
  double sdmin = INFINITY;
  int cnt = 0;
  visit_pairs(E, P, j, xw, r, [&](int, const PairTerm& pt) {
    if (!pt.interior) return;
    const double sd = pt.diff[0] * n[0] + pt.diff[1] * n[1] + pt.diff[2] * n[2];
    // the closest points' vector within 60 degrees of the normal line: next
    // to a pad edge or corner a feature above one surface region can sit
    // behind the plane of a neighbouring one without being inside the pad
    if (!(fabs(sd) >= 0.5 * pt.d) || !(sd < below)) return;
    ++cnt;
    sdmin = fmin(sdmin, sd);
  });
  if (mode == 1) {
    if (cnt) atomicOr(&S->infeasible, 1);
    return;
  }
  E.pflag[j] = cnt > 0;
  if (cnt == 0) return;
  double* rec = E.prec + (size_t)PREC * j;
  for (int i = 0; i < 3; ++i) rec[i] = (sdmin - dsafe) * n[i];
  rec[3] = dsafe - sdmin;
}

// Feasible start, pads with pairs: each contact vertex moves by the
// longest push its surface primitives ask of it (the first primitive in
// order on ties: triangles by index, then edges), free components only.
__global__ void k_pair_apply(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const EnvState* S = E.st;
  if (!initialising(S) || !pair_active(E, E.pose)) return;
  const int k = tiles[t].tile * blockDim.x + threadIdx.x;
  if (k >= E.C) return;
  const double* best = nullptr;
  for (int c = E.vp_ptr[k]; c < E.vp_ptr[k + 1]; ++c) {
    const int j = E.vp_idx[c] >> 2;
    if (!E.pflag[j]) continue;
    const double* rec = E.prec + (size_t)PREC * j;
    if (!best || rec[3] > best[3]) best = rec;
  }
  if (!best) return;
  const double dx[3] = {best[0], best[1], best[2]};
  const int vi = E.cand[k];
  const uint8_t fm = E.fixed[vi];
  for (int i = 0; i < 3; ++i)
    if (!((fm >> i) & 1)) E.xn[3 * vi + i] += dx[i];
}

// Pair gradient (and with H the Gauss-Newton diagonal block) of contact
// vertex k gathered from its primitives' records.
__device__ __forceinline__ void pair_gather(const EnvDesc& E, int k, double g[3], double (*H)[3]) {
  for (int c = E.vp_ptr[k]; c < E.vp_ptr[k + 1]; ++c) {
    const int code = E.vp_idx[c];
    const int j = code >> 2, a = code & 3;
    if (!E.pflag[j]) continue;
    const double* rec = E.prec + (size_t)PREC * j;
    for (int i = 0; i < 3; ++i) g[i] += rec[3 * a + i];
    if (H) {
      const double* b = rec + 9 + 6 * a;
      H[0][0] += b[0]; H[0][1] += b[1]; H[0][2] += b[2];
      H[1][0] += b[1]; H[1][1] += b[3]; H[1][2] += b[4];
      H[2][0] += b[2]; H[2][1] += b[4]; H[2][2] += b[5];
    }
  }
}

// Pair Gauss-Newton block between the ends of unique edge k (symmetric, 6
// values) when it is a surface edge: its two triangles' blocks plus its own
// edge-edge block.  Returns false when there is none.
__device__ __forceinline__ bool pair_edge_block(const EnvDesc& E, int k, double b[6]) {
  const int f = E.edge_sedge[k];
  if (f < 0) return false;
  bool any = false;
  for (int c = 0; c < 6; ++c) b[c] = 0.0;
  for (int q = 0; q < 2; ++q) {
    const int code = E.sedge_adj[2 * f + q];
    if (code < 0 || !E.pflag[code >> 3]) continue;
    const double* r = E.prec + (size_t)PREC * (code >> 3) + 9 + 6 * (code & 7);
    for (int c = 0; c < 6; ++c) b[c] += r[c];
    any = true;
  }
  const int j = E.S + f;
  if (E.pflag[j]) {
    const double* r = E.prec + (size_t)PREC * j + 9 + 6 * 3;
    for (int c = 0; c < 6; ++c) b[c] += r[c];
    any = true;
  }
  return any;
}

// Collision-free step bound of pad primitive j moving by alpha p (p the
// direction at its vertices).  Per pair the larger of two safe bounds:
// conservative advancement (every point of the moving primitive moves at
// most alpha max_a |p_a|, so the pair's distance d(alpha) is Lipschitz with
// that constant, and from a reached alpha the step (d(alpha) - 0.1 d(0)) /
// max_a |p_a| keeps it above 0.1 d(0); advances stop within 0.1 % of that
// floor, after 32 advances, or at FILTER_SPAN), and the separation along
// the pair's unit vector u, which shrinks at most by alpha max_a p_a.u
// (alpha <= 0.9 sep / max_a p_a.u, none when that is <= 0: motion across u
// does not count).  Pairs farther than FILTER_SPAN max |p_a| / 0.9 cannot
// bind.
template <typename R>
__device__ double prim_pair_bound(const EnvDesc& E, const EnvPose* P, int j, const R* d, double span) {
  int vid[3];
  double xw[3][3], pv[3][3];
  const int nv = prim_load<R>(E, j, E.xn, nullptr, 0.0, vid, xw);
  double pm = 0.0;
  for (int k = 0; k < nv; ++k) {
    double q = 0.0;
    for (int c = 0; c < 3; ++c) {
      pv[k][c] = (double)d[3 * vid[k] + c];
      q += pv[k][c] * pv[k][c];
    }
    pm = fmax(pm, sqrt(q));
  }
  if (!(pm > 0.0)) return INFINITY;
  double r[MAX_IND];
  for (int m = 0; m < MAX_IND; ++m) r[m] = span * pm / 0.9;
  double a = INFINITY;
  visit_pairs(E, P, j, xw, r, [&](int m, const PairTerm& pt) {
    const double floor_ = 0.1 * pt.d;
    if (!(pt.d > 0.0)) {
      a = 0.0;
      return;
    }
    // the primitive in the mesh's frame: vertices and directions
    const DevIndenter& I = P->ind[m];
    double xl[3][3], pl[3][3];
    for (int k = 0; k < nv; ++k)
      for (int i = 0; i < 3; ++i) {
        xl[k][i] = I.R[0 * 3 + i] * (xw[k][0] - I.c[0]) + I.R[1 * 3 + i] * (xw[k][1] - I.c[1]) +
                   I.R[2 * 3 + i] * (xw[k][2] - I.c[2]);
        pl[k][i] = I.R[0 * 3 + i] * pv[k][0] + I.R[1 * 3 + i] * pv[k][1] + I.R[2 * 3 + i] * pv[k][2];
      }
    double al = 0.0, dc = pt.d;
    for (int it = 0; it < 32; ++it) {
      al += (dc - floor_) / pm;
      if (al >= span) {
        al = span;
        break;
      }
      double y[3][3], lam[3], df[3], sp, tp;
      for (int k = 0; k < nv; ++k)
        for (int i = 0; i < 3; ++i) y[k][i] = xl[k][i] + al * pl[k][i];
      const double d2 = pt.w1 ? seg_seg(pt.w0, pt.w1, y[0], y[1], sp, tp, df) : pt_tri_lam(pt.w0, y[0], y[1], y[2], lam, df);
      dc = sqrt(d2);
      if (dc - floor_ <= 1e-3 * floor_) break;
    }
    double pu = -INFINITY;
    for (int k = 0; k < nv; ++k) pu = fmax(pu, pv[k][0] * pt.u[0] + pv[k][1] * pt.u[1] + pv[k][2] * pt.u[2]);
    const double b = pt.sep > 0.0 ? (pu > 0.0 ? 0.9 * pt.sep / pu : INFINITY) : 0.0;
    a = fmin(a, fmax(al, b));
  });
  return a;
}

// ------------------------------------------------------ barrier (a4)

__device__ void project_psd3(double H[3][3]) {
  double A[3][3], Q[3][3], w[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (H[i][j] + H[j][i]);
  sym_eig3(A, Q, w);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += Q[i][m] * fmax(w[m], 0.0) * Q[j][m];
      H[i][j] = s;
    }
}

// Per contact vertex: E_b gradient kappa A b'(s) grad(phi) and PSD-projected
// Hessian kappa A [b''(s)/d_hat grad grad^T + b'(s) hess(phi)], summed over
// indenters (float64).
__global__ void k_barrier(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const EnvPose* P = E.pose;
  if (!at_stage(E.st, ST_ASM)) return;
  const int k = tiles[t].tile * blockDim.x + threadIdx.x;
  if (k >= E.C) return;
  const int vi = E.cand[k];
  double x[3];
  load3(E.xn, vi, x);
  const double kA = E.kappa * E.cand_area[k];
  double g[3] = {0, 0, 0}, H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Hn[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int m = 0; m < P->n_ind; ++m) {
    if (E.mesh_pairs && P->ind[m].shape == TC_MESH) {
      double e, gp[3], Hq[3][3], Hnq[3][3];
      mesh_pair_world(P->ind[m], E.meshes, x, E.dhat, true, e, gp, Hq, Hnq);
      for (int i = 0; i < 3; ++i) {
        g[i] += kA * gp[i];
        for (int j = 0; j < 3; ++j) {
          H[i][j] += kA * Hq[i][j];
          Hn[i][j] += kA * Hnq[i][j];
        }
      }
      continue;
    }
    double phi, n[3], Hp[3][3];
    sdf_world(P->ind[m], E.meshes, x, phi, n, Hp, true, E.dhat);
    if (phi < E.dhat) {
      const double s = phi / E.dhat;
      const double b1 = bar1(s), b2 = bar2(s);
      for (int i = 0; i < 3; ++i) {
        g[i] += kA * b1 * n[i];
        for (int j = 0; j < 3; ++j) {
          H[i][j] += kA * (b2 / E.dhat * n[i] * n[j] + b1 * Hp[i][j]);
          Hn[i][j] += kA * b2 / E.dhat * n[i] * n[j];
        }
      }
    }
  }
  // 0 clamp, 1 as is, 2 normal term only, 3 clamp until a full Newton step
  // is accepted, then as is
  int bmode = (E.hess_proj >> 2) & 3;
  if (bmode == 3) bmode = E.st->true_hess ? 1 : 0;
  if (E.st->filt_all) bmode = 0;   // a CG breakdown earlier in this step
  if (bmode == 0) {
    project_psd3(H);
  } else if (bmode == 2) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i][j] = Hn[i][j];
  }
  // vertex-face and edge-edge pairs of the vertex's surface primitives
  // (Gauss-Newton, PSD: added after the filter)
  if (pair_active(E, P)) pair_gather(E, k, g, H);
  // lagged friction (PSD by construction, added after the filter):
  // gradient mu lambda (f1/y) u, Hessian mu lambda [f1/y (P - uh uh^T) +
  // f1' uh uh^T] with P = I - n n^T and uh = u / |u| (u lies in P's range)
  if (E.fr_mu > 0) {
    double xt[3];
    load3(E.x, vi, xt);
    for (int m = 0; m < P->n_ind; ++m) {
      const double* f = fr_rec(E, m, k);
      if (!(f[FRIC_LAM] > 0)) continue;
      double u[3];
      const double y = fr_slip(f, x, xt, u);
      const double c = E.fr_mu * f[FRIC_LAM];
      const double fy = fr_f1_over_y(y, E.fr_eps), fp = fr_f1p(y, E.fr_eps);
      const double iy = y > 0 ? 1.0 / y : 0.0;
      const double uh[3] = {u[0] * iy, u[1] * iy, u[2] * iy};
      for (int i = 0; i < 3; ++i) {
        g[i] += c * fy * u[i];
        for (int j = 0; j < 3; ++j) {
          const double Pij = (i == j ? 1.0 : 0.0) - f[FRIC_N + i] * f[FRIC_N + j];
          H[i][j] += c * (fy * (Pij - uh[i] * uh[j]) + fp * uh[i] * uh[j]);
        }
      }
    }
  }
  for (int i = 0; i < 3; ++i) E.gb[3 * k + i] = g[i];
  double* hb = E.Hb + 6 * k;
  hb[0] = H[0][0]; hb[1] = H[0][1]; hb[2] = H[0][2]; hb[3] = H[1][1]; hb[4] = H[1][2]; hb[5] = H[2][2];
}

// ------------------------------------------------------ assembly

// Diagonal block rows (slot 0): sum of element blocks, inertia, barrier,
// Dirichlet masking, gradient, preconditioner, and CG initialisation
// (d = 0, r = -g, z = P^-1 r, partial r.z and g.g).  A tile is blockDim.x
// rows; groups of ASM_LPR lanes take one row at a time, each lane summing
// every ASM_LPR-th record of the row's contiguous run of diagonal-stream
// records (so a wavefront reads a few long runs instead of 64 scattered
// records), then a shuffle reduction gives the row's sums to its lane 0,
// which finishes the row.
constexpr int ASM_LPR = 8;

template <typename R>
__device__ __forceinline__ void asm_diag_row(const EnvDesc& E, int i, double D[3][3], double gs[3], double& rz,
                                             double& gg, bool warm) {
  D[1][0] = D[0][1]; D[2][0] = D[0][2]; D[2][1] = D[1][2];
  const size_t it0 = (size_t)i * E.W;
  const double h2 = E.h * E.h;
  double xi[3], xh[3];
  load3(E.xn, i, xi);
  load3(E.xhat, i, xh);
  const double m = E.quasi_static ? 0.0 : E.mass[i];
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q) D[r][q] *= h2;
    D[r][r] += m;
    gs[r] = h2 * gs[r] + m * (xi[r] - xh[r]);
  }
  const int k = E.cand_of_vert[i];
  if (k >= 0) {
    const double* hb = E.Hb + 6 * k;
    const double Hk[3][3] = {{hb[0], hb[1], hb[2]}, {hb[1], hb[3], hb[4]}, {hb[2], hb[4], hb[5]}};
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) D[r][q] += h2 * Hk[r][q];
      gs[r] += h2 * E.gb[3 * k + r];
    }
  }
  const uint8_t fm = E.fixed[i];
  for (int r = 0; r < 3; ++r)
    if ((fm >> r) & 1) {
      for (int q = 0; q < 3; ++q) { D[r][q] = 0; D[q][r] = 0; }
      D[r][r] = 1.0;
      gs[r] = 0.0;
    }
  R* A = (R*)E.A + it0 * 9;
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) A[3 * r + q] = (R)D[r][q];
  // preconditioner: inverse of the 3x3 diagonal block, or of its diagonal
  double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  // the block must be positive definite (leading minors) to serve as a CG
  // preconditioner; otherwise fall back to the absolute diagonal
  const bool spd = D[0][0] > 0 && D[0][0] * D[1][1] - D[0][1] * D[1][0] > 0 && det > 0;
  if (E.precond == TC_PRECOND_BLOCK_JACOBI && spd) {
    const double id = 1.0 / det;
    P[0][0] = c00 * id;
    P[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
    P[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
    P[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
    P[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
    P[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
    P[1][0] = P[0][1]; P[2][0] = P[0][2]; P[2][1] = P[1][2];
  } else {
    for (int r = 0; r < 3; ++r) P[r][r] = 1.0 / fmax(fabs(D[r][r]), 1e-300);
  }
  R* Pi = (R*)E.Pinv + 6 * i;
  Pi[0] = (R)P[0][0]; Pi[1] = (R)P[0][1]; Pi[2] = (R)P[0][2];
  Pi[3] = (R)P[1][1]; Pi[4] = (R)P[1][2]; Pi[5] = (R)P[2][2];
  R Pr[3][3] = {{Pi[0], Pi[1], Pi[2]}, {Pi[1], Pi[3], Pi[4]}, {Pi[2], Pi[4], Pi[5]}};
  R* d = (R*)E.d;
  R* z = (R*)E.z;
  R* p1 = (R*)E.p1;
  double rr[3];
  for (int r = 0; r < 3; ++r) {
    E.g[3 * i + r] = gs[r];
    rr[r] = -gs[r];
    E.r[3 * i + r] = rr[r];
    // warm start: the previous Newton direction becomes the search
    // direction of iteration -1 (p_old of parity 0, with z = 0 and beta 1)
    const R dp = warm ? d[3 * i + r] : R(0);
    d[3 * i + r] = R(0);
    p1[3 * i + r] = dp;
    gg += gs[r] * gs[r];
  }
  for (int r = 0; r < 3; ++r) {
    const R zr = Pr[r][0] * (R)rr[0] + Pr[r][1] * (R)rr[1] + Pr[r][2] * (R)rr[2];
    z[3 * i + r] = warm ? R(0) : zr;
    rz += rr[r] * (double)zr;
  }
}

template <typename R>
__global__ void k_asm_diag(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  if (!at_stage(E.st, ST_ASM)) return;
  const int lane = threadIdx.x & (ASM_LPR - 1);
  const int groups = blockDim.x / ASM_LPR;
  const int row0 = tl.tile * blockDim.x + threadIdx.x / ASM_LPR;
  const R* Kd = (const R*)E.Ke;
  const bool warm = E.cg_warm && E.st->warm != 0;
  double rz = 0.0, gg = 0.0;
  for (int k = 0; k < ASM_LPR; ++k) {
    const int i = row0 + k * groups;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // xx xy xz yy yz zz, gradient
    if (i < E.V)
      for (int c = E.dptr[i] + lane; c < E.dptr[i + 1]; c += ASM_LPR) {
        const R* p = Kd + (size_t)KC * c;
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] += (double)p[q];
      }
#pragma unroll
    for (int o = ASM_LPR / 2; o > 0; o >>= 1)
#pragma unroll
      for (int q = 0; q < 9; ++q) v[q] += __shfl_xor(v[q], o, ASM_LPR);
    if (lane == 0 && i < E.V) {
      double D[3][3] = {{v[0], v[1], v[2]}, {0, v[3], v[4]}, {0, 0, v[5]}};
      double gs[3] = {v[6], v[7], v[8]};
      asm_diag_row<R>(E, i, D, gs, rz, gg, warm);
    }
  }
  rz = block_reduce(rz, OpSum(), sh);
  gg = block_reduce(gg, OpSum(), sh);
  if (threadIdx.x == 0) {
    E.part_rz[tl.tile] = rz;
    E.part_g2[tl.tile] = gg;
  }
  if (warm) {
    // r0.d_prev partials over the tile's rows, from r0 and the copy of d_prev
    // just written (the block reductions above ordered those writes); the
    // direction partials are free until k_newton_dir
    const int i = tl.tile * blockDim.x + threadIdx.x;
    double gd = 0.0;
    if (i < E.V) {
      const R* p1 = (const R*)E.p1;
      for (int c = 0; c < 3; ++c) gd += E.r[3 * i + c] * (double)p1[3 * i + c];
    }
    gd = block_reduce(gd, OpSum(), sh);
    if (threadIdx.x == 0) E.part_dir[tl.tile] = gd;
  }
}

// Off-diagonal blocks, one thread per unique edge i < j: sum of the edge
// blocks of every tet sharing it, times h^2, written to (i, slot of j) and
// transposed to (j, slot of i), Dirichlet rows and columns zeroed.
template <typename R>
__global__ void k_asm_off(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  if (!at_stage(E.st, ST_ASM)) return;
  const int k = tiles[t].tile * blockDim.x + threadIdx.x;
  if (k >= E.V_E) return;
  const R* Ko = (const R*)E.Ke + (size_t)KC * 4 * E.T;
  R acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int c = E.eptr[k]; c < E.eptr[k + 1]; ++c) {
    const R* p = Ko + (size_t)KC * c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[r][q] += p[3 * r + q];
  }
  // pair Gauss-Newton block of a surface edge (mesh_contact 2)
  double pb[6];
  if (pair_active(E, E.pose) && pair_edge_block(E, k, pb)) {
    const double B[3][3] = {{pb[0], pb[1], pb[2]}, {pb[1], pb[3], pb[4]}, {pb[2], pb[4], pb[5]}};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[r][q] = (R)((double)acc[r][q] + B[r][q]);
  }
  const int2 it = reinterpret_cast<const int2*>(E.eitem)[k];
  const int i = it.x / E.W, j = it.y / E.W;
  const R h2 = (R)(E.h * E.h);
  const uint8_t fi = E.fixed[i], fj = E.fixed[j];
  R* Aij = (R*)E.A + (size_t)it.x * 9;
  R* Aji = (R*)E.A + (size_t)it.y * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Aij[3 * r + q] = (((fi >> r) & 1) || ((fj >> q) & 1)) ? R(0) : acc[r][q] * h2;
      Aji[3 * q + r] = (((fj >> q) & 1) || ((fi >> r) & 1)) ? R(0) : acc[r][q] * h2;
    }
}

// ------------------------------------------------------ CG (a5)

// Per Newton iteration reset of the CG / line-search flags (one block/pad).
__global__ void k_env_newton_begin(const EnvDesc* envs, int n) {
  if (blockIdx.x >= n || threadIdx.x != 0) return;
  EnvState* S = envs[blockIdx.x].st;
  if (!at_stage(S, ST_START)) return;
  if (S->newton_iters == 0) {
    S->rz0_prev = -1.0;
    S->eta_prev = 0.0;
  } else {
    S->rz0_prev = S->rz0;
    S->eta_prev = sqrt(S->cg_tol2);
  }
  // warm start from the previous Newton direction of this step (still in d)
  S->warm = envs[blockIdx.x].cg_warm && S->newton_iters > 0 && S->apply;
  S->cg_done = 0;
  S->cg_iters = 0;
  S->breakdown = 0;
  S->true_hess = S->true_hess && !S->no_true_hess;
  S->it[0] = -1;
  S->it[1] = S->warm ? -2 : -1;
  S->rzp[0] = S->rzp[1] = 0.0;
  S->dir_conv = 0;
  S->apply = 0;
  S->ls_done = 0;
  S->ls_halv = 0;
  S->ls_expanding = 0;
  S->ls_expand_n = 0;
  S->ls_contracting = 0;
  S->stage = ST_ASM;
}

// Common head of the CG product for one tile: reduce this pad's r.z
// partials, decide whether its CG stops here (r.z <= tol^2 r0.z0, max_cg or a
// breakdown) and publish the iteration's scalars (tile 0).  Every block of the
// pad computes the same decision.  Returns false when the tile has no work;
// else beta for p_new = z + beta p_old.
__device__ __forceinline__ bool cg_go(const EnvDesc& E) {
  EnvState* S = E.st;
  // tile 0 of the pad may set cg_done while this block reads it: one thread
  // reads, the block follows, so that all its waves take the same path
  __shared__ int s_go;
  if (threadIdx.x == 0) s_go = cg_running(S);
  __syncthreads();
  const bool go = s_go != 0;
  __syncthreads();
  return go;
}

// The stop decision on r.z (forcing term at the first iteration); tile 0
// publishes the iteration's scalars.  False: this pad's CG has ended.
__device__ __forceinline__ bool cg_decide(const Tile tl, const EnvDesc& E, int parity, double rz, double* beta,
                                          int* it_out);

__device__ __forceinline__ bool cg_head(const Tile tl, const EnvDesc& E, int parity, double* sh,
                                        double* beta) {
  if (!cg_go(E)) return false;
  const double rz = reduce_partials(E.part_rz, E.n_vt, OpSum(), 0.0, sh);
  int it;
  return cg_decide(tl, E, parity, rz, beta, &it);
}

// Forcing term of a Newton iteration's solve, from its cold-start r0.z0:
// the relative tolerance squared.
__device__ __forceinline__ double cg_tol2_of(const EnvDesc& E, const EnvState* S, double rz) {
  double eta = S->force_tight ? fmin(E.cg_conv_tol, E.cg_rel_tol) : E.cg_rel_tol;
  if (E.cg_forcing && !S->force_tight) {
    if (S->rz0_prev > 0.0) {
      const double r2 = rz / S->rz0_prev;      // (|g_k| / |g_k-1|)^2, preconditioned norms
      if (r2 < 0.25 || E.cg_forcing == 2) {
        eta = 0.9 * r2;                        // Eisenstat-Walker choice 2
        const double safe = 0.9 * S->eta_prev * S->eta_prev;
        if (safe > 0.1) eta = fmax(eta, safe);
      } else {
        eta = 0.25 * S->eta_prev;              // slow progress: solve more accurately
      }
    } else {
      eta = E.cg_eta_max;
    }
    eta = fmin(E.cg_eta_max, fmax(eta, E.cg_rel_tol));
  }
  return eta * eta;
}

__device__ __forceinline__ bool cg_decide(const Tile tl, const EnvDesc& E, int parity, double rz, double* beta,
                                          int* it_out) {
  EnvState* S = E.st;
  const int it = S->it[parity ^ 1] + 1;
  *it_out = it;
  // iteration -1 of a warm start is the product with p = d_prev (z = 0,
  // beta 1); the solve's tolerance is set there, or at iteration 0 of a cold
  // start, from the cold start's r0.z0 (the partials of the assembly)
  const bool first = it < 0 || (it == 0 && !S->warm);
  const double rz0 = first ? rz : S->rz0;
  const double tol2 = first ? cg_tol2_of(E, S, rz) : S->cg_tol2;
  const bool done = it >= 0 && (it >= E.max_cg || !(rz > tol2 * rz0) || S->breakdown);
  double gd = 0.0;
  if (it < 0 && tl.tile == 0) {
    // r0.d_prev from the assembly's partials (block-uniform branch)
    __shared__ double shd[16];
    gd = reduce_partials(E.part_dir, E.n_vt, OpSum(), 0.0, shd);
  }
  if (tl.tile == 0 && threadIdx.x == 0) {
    // the other blocks of this launch read the stage: ST_ASM and ST_CG
    // both let them run
    S->stage = ST_CG;
    if (first) {
      S->cg_tol2 = tol2;
      S->rz0 = rz;
    }
    if (done) {
      S->cg_done = 1;
      S->cg_iters = it;
    } else {
      S->it[parity] = it;
      S->rzp[parity] = it < 0 ? gd : rz;   // the update's alpha = rzp / p.Ap
    }
  }
  if (done) return false;
  *beta = it < 0 ? 1.0 : it == 0 ? 0.0 : rz / S->rzp[parity ^ 1];
  return true;
}

// q = A p_new, one thread per matrix row (tiles of blockDim.x rows); the row
// owner stores p_new.
template <typename R>
__device__ __forceinline__ void cg_spmv_rows_body(const Tile tl, const EnvDesc& E, int parity, R beta, double* sh) {
  const int i = tl.tile * blockDim.x + threadIdx.x;
  const R* z = (const R*)E.z;
  const R* pold = (const R*)(parity ? E.p0 : E.p1);
  R* pnew = (R*)(parity ? E.p1 : E.p0);
  double pq = 0.0;
  if (i < E.V) {
    const R* A = (const R*)E.A;
    R y0 = 0, y1 = 0, y2 = 0;
    R pi0 = 0, pi1 = 0, pi2 = 0;
    for (int s = 0; s < E.W; ++s) {
      const int j = E.col[(size_t)i * E.W + s];
      if (j < 0) break;
      const R pj0 = z[3 * j] + beta * pold[3 * j];
      const R pj1 = z[3 * j + 1] + beta * pold[3 * j + 1];
      const R pj2 = z[3 * j + 2] + beta * pold[3 * j + 2];
      if (s == 0) { pi0 = pj0; pi1 = pj1; pi2 = pj2; }
      const R* As = A + ((size_t)i * E.W + s) * 9;
      y0 += As[0] * pj0 + As[1] * pj1 + As[2] * pj2;
      y1 += As[3] * pj0 + As[4] * pj1 + As[5] * pj2;
      y2 += As[6] * pj0 + As[7] * pj1 + As[8] * pj2;
    }
    pnew[3 * i] = pi0; pnew[3 * i + 1] = pi1; pnew[3 * i + 2] = pi2;
    R* q = (R*)E.q;
    q[3 * i] = y0; q[3 * i + 1] = y1; q[3 * i + 2] = y2;
    pq = (double)pi0 * y0 + (double)pi1 * y1 + (double)pi2 * y2;
  }
  pq = block_reduce(pq, OpSum(), sh);
  if (threadIdx.x == 0) E.part_pq[tl.tile] = pq;
}

// The same product with LPR lanes per matrix row (lane l takes the stored
// 3x3 blocks l, l + LPR, ... of its row, blocks of a row contiguous): every
// lane issues its own independent neighbour gathers, and the row sum is a
// shuffle reduction inside the lane group.  A row's padding slots (col -1)
// come after its blocks, so a lane stops at its first one.  A tile is
// blockDim.x / LPR lane groups x SPMV_ROWS_PER_GROUP rows.
template <typename R, int LPR>
__device__ __forceinline__ void cg_spmv_lanes_body(const Tile tl, const EnvDesc& E, int parity, R beta, double* sh) {
  const int lane = threadIdx.x & (LPR - 1);
  const int groups = blockDim.x / LPR;
  const R* z = (const R*)E.z;
  const R* pold = (const R*)(parity ? E.p0 : E.p1);
  R* pnew = (R*)(parity ? E.p1 : E.p0);
  R* q = (R*)E.q;
  double pq = 0.0;
  const int row0 = tl.tile * groups * SPMV_ROWS_PER_GROUP + threadIdx.x / LPR;
#pragma unroll 2
  for (int k = 0; k < SPMV_ROWS_PER_GROUP; ++k) {
    const int i = row0 + k * groups;
    R y0 = 0, y1 = 0, y2 = 0, pd0 = 0, pd1 = 0, pd2 = 0;
    if (E.W <= LPR) {             // one slot per lane (the common case)
      if (i < E.V && lane < E.W) {
        const size_t item = (size_t)i * E.W + lane;
        const int j = E.col[item];
        if (j >= 0) {
          pd0 = z[3 * j] + beta * pold[3 * j];
          pd1 = z[3 * j + 1] + beta * pold[3 * j + 1];
          pd2 = z[3 * j + 2] + beta * pold[3 * j + 2];
          const R* As = (const R*)E.A + item * 9;
          y0 = As[0] * pd0 + As[1] * pd1 + As[2] * pd2;
          y1 = As[3] * pd0 + As[4] * pd1 + As[5] * pd2;
          y2 = As[6] * pd0 + As[7] * pd1 + As[8] * pd2;
        }
      }
    } else if (i < E.V) {
      for (int sl = lane; sl < E.W; sl += LPR) {
        const size_t item = (size_t)i * E.W + sl;
        const int j = E.col[item];
        if (j < 0) break;
        const R pj0 = z[3 * j] + beta * pold[3 * j];
        const R pj1 = z[3 * j + 1] + beta * pold[3 * j + 1];
        const R pj2 = z[3 * j + 2] + beta * pold[3 * j + 2];
        if (sl == 0) { pd0 = pj0; pd1 = pj1; pd2 = pj2; }
        const R* As = (const R*)E.A + item * 9;
        y0 += As[0] * pj0 + As[1] * pj1 + As[2] * pj2;
        y1 += As[3] * pj0 + As[4] * pj1 + As[5] * pj2;
        y2 += As[6] * pj0 + As[7] * pj1 + As[8] * pj2;
      }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      y0 += __shfl_xor(y0, o, LPR);
      y1 += __shfl_xor(y1, o, LPR);
      y2 += __shfl_xor(y2, o, LPR);
    }
    if (lane == 0 && i < E.V) {   // slot 0 is the diagonal: pd = p_new of row i
      pnew[3 * i] = pd0; pnew[3 * i + 1] = pd1; pnew[3 * i + 2] = pd2;
      q[3 * i] = y0; q[3 * i + 1] = y1; q[3 * i + 2] = y2;
      pq += (double)pd0 * y0 + (double)pd1 * y1 + (double)pd2 * y2;
    }
  }
  pq = block_reduce(pq, OpSum(), sh);
  if (threadIdx.x == 0) E.part_pq[tl.tile] = pq;
}

// The product of one SpMV tile given beta (p_new = z + beta p_old).
template <typename R, int LPR>
__device__ __forceinline__ void cg_spmv_body(const Tile tl, const EnvDesc& E, int parity, R beta, double* sh) {
  if constexpr (LPR == 0) cg_spmv_rows_body<R>(tl, E, parity, beta, sh);
  else cg_spmv_lanes_body<R, LPR>(tl, E, parity, beta, sh);
}

template <typename R, int LPR>
__device__ __forceinline__ void cg_spmv_tile(const Tile tl, const EnvDesc* envs, int parity, double* sh) {
  const EnvDesc& E = envs[tl.env];
  double beta;
  if (!cg_head(tl, E, parity, sh, &beta)) return;
  cg_spmv_body<R, LPR>(tl, E, parity, (R)beta, sh);
}

// alpha = r.z / p.Ap; d += alpha p; r -= alpha Ap (float64); z = P^-1 r;
// partial r.z for the next iteration.
// alpha = r.z / p.Ap from the product's partials (a non-positive p.Ap is a
// breakdown: alpha = 0 and the tile-0 block flags it).
__device__ __forceinline__ double cg_alpha(const Tile tl, const EnvDesc& E, int parity, double* sh) {
  EnvState* S = E.st;
  const double pq = reduce_partials(E.part_pq, E.n_spt, OpSum(), 0.0, sh);
  const double rz = S->rzp[parity];
  double alpha = rz / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    alpha = 0.0;
    // (a warm start along a direction of non-positive curvature is only
    // skipped: the cold start follows)
    if (tl.tile == 0 && threadIdx.x == 0 && S->it[parity] >= 0) S->breakdown = 1;
  }
  return alpha;
}

template <typename R>
__device__ __forceinline__ void cg_update_body(const Tile tl, const EnvDesc& E, int parity, double alpha,
                                               double* sh) {
  const int i = tl.tile * blockDim.x + threadIdx.x;
  double rzn = 0.0;
  if (i < E.V) {
    const R* p = (const R*)(parity ? E.p1 : E.p0);
    const R* q = (const R*)E.q;
    R* d = (R*)E.d;
    R* z = (R*)E.z;
    const R* Pi = (const R*)E.Pinv + 6 * i;
    const R a = (R)alpha;
    double rr[3];
    for (int c = 0; c < 3; ++c) {
      d[3 * i + c] += a * p[3 * i + c];
      rr[c] = E.r[3 * i + c] - alpha * (double)q[3 * i + c];
      E.r[3 * i + c] = rr[c];
    }
    const R r0 = (R)rr[0], r1 = (R)rr[1], r2 = (R)rr[2];
    const R z0 = Pi[0] * r0 + Pi[1] * r1 + Pi[2] * r2;
    const R z1 = Pi[1] * r0 + Pi[3] * r1 + Pi[4] * r2;
    const R z2 = Pi[2] * r0 + Pi[4] * r1 + Pi[5] * r2;
    z[3 * i] = z0; z[3 * i + 1] = z1; z[3 * i + 2] = z2;
    rzn = rr[0] * (double)z0 + rr[1] * (double)z1 + rr[2] * (double)z2;
  }
  rzn = block_reduce(rzn, OpSum(), sh);
  if (threadIdx.x == 0) E.part_rz[tl.tile] = rzn;
}

template <typename R>
__device__ __forceinline__ void cg_update_tile(const Tile tl, const EnvDesc* envs, int parity, double* sh) {
  const EnvDesc& E = envs[tl.env];
  EnvState* S = E.st;
  if (!cg_running(S)) return;
  cg_update_body<R>(tl, E, parity, cg_alpha(tl, E, parity, sh), sh);
}

// Optional self-timing of a launch on the GPU wall clock: every block stores
// its start and end clock in its own pair of cells (plain stores, no
// atomics); the host takes the earliest start and the latest end.
__device__ __forceinline__ void clock_start(unsigned long long* clk) {
  if (threadIdx.x == 0) clk[2 * blockIdx.x] = (unsigned long long)wall_clock64();
}
__device__ __forceinline__ void clock_end(unsigned long long* clk) {
  __syncthreads();
  if (threadIdx.x == 0) clk[2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
}

// TIMED: the self-timing variant, launched only for the sampled launches
// (the plain variant carries no timing code at all).
template <typename R, int LPR, bool TIMED>
__global__ void __launch_bounds__(1024) k_cg_spmv(const Tile* tiles, int ntiles, const EnvDesc* envs, int parity,
                                                  unsigned long long* clk) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  if constexpr (TIMED) clock_start(clk);
  cg_spmv_tile<R, LPR>(tiles[t], envs, parity, sh);
  if constexpr (TIMED) clock_end(clk);
}

template <typename R, bool TIMED>
__global__ void __launch_bounds__(1024) k_cg_update(const Tile* tiles, int ntiles, const EnvDesc* envs, int parity,
                                                    unsigned long long* clk) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  if constexpr (TIMED) clock_start(clk);
  cg_update_tile<R>(tiles[t], envs, parity, sh);
  if constexpr (TIMED) clock_end(clk);
}

// ------------------------------------------------------ Newton direction, filter (a6)

// partials: |d|_inf and g . d
template <typename R>
__global__ void k_newton_dir(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  if (!dir_ready(E.st)) return;
  const int i = tl.tile * blockDim.x + threadIdx.x;
  double dm = 0.0, gd = 0.0;
  if (i < E.V) {
    const R* d = (const R*)E.d;
    for (int c = 0; c < 3; ++c) {
      const double dc = (double)d[3 * i + c];
      dm = fmax(dm, fabs(dc));
      gd += E.g[3 * i + c] * dc;
    }
  }
  dm = block_reduce(dm, OpMax(), sh);
  gd = block_reduce(gd, OpSum(), sh);
  if (threadIdx.x == 0) {
    E.part_dir[2 * tl.tile] = dm;
    E.part_dir[2 * tl.tile + 1] = gd;
  }
}

// Largest safe step per contact vertex.  Convex indenters: phi(x + a p) >=
// phi(x) + a grad(phi).p, so only approach (grad.p < 0) limits the step,
// a <= 0.9 phi / (-grad.p).  The textured plate and the torus have curvature
// bounds K along the step, which give the quadratic lower model
// phi(x + a p) >= phi + a grad.p - K a^2 |p|^2 / 2.  Each keeps
// phi >= 0.1 phi(x).  Steps are bounded for a <= FILTER_SPAN (the line
// search may double an accepted full step up to there).

__device__ __forceinline__ double quadratic_step(double phi, double gp, double K, double pn) {
  const double qa = K * pn * pn;
  return (gp + sqrt(gp * gp + 1.8 * qa * phi)) / qa;
}

template <typename R>
__global__ void k_filter(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  const EnvPose* P = E.pose;
  if (!dir_ready(E.st)) return;
  const int k = tl.tile * blockDim.x + threadIdx.x;
  double amax = INFINITY;
  if (k < E.C) {
    const int vi = E.cand[k];
    double x[3], p[3], H[3][3];
    load3(E.xn, vi, x);
    const R* d = (const R*)E.d;
    for (int c = 0; c < 3; ++c) p[c] = (double)d[3 * vi + c];
    const double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    if (pn > 0) {
      for (int m = 0; m < P->n_ind; ++m) {
        const DevIndenter& I = P->ind[m];
        // a mesh vertex farther than FILTER_SPAN |p| / 0.9 keeps phi >= 0.1
        // phi(x) over the whole span: the query stops at that radius
        double phi, g[3];
        sdf_world(I, E.meshes, x, phi, g, H, false, FILTER_SPAN * pn / 0.9);
        double a = INFINITY;
        const double gp = g[0] * p[0] + g[1] * p[1] + g[2] * p[2];
        if (convex_shape(I.shape) || (I.shape == TC_MESH && E.meshes[I.reserved].convex)) {
          // phi convex along the segment (outside a convex body): it stays
          // above its tangent line, which reaches 0.1 phi(x) at this a
          if (gp < 0) a = 0.9 * phi / (-gp);
        } else if (I.shape == TC_MESH) {
          // conservative advancement: phi is 1-Lipschitz, so phi >= 0.1 phi(x)
          // holds on [a, a + (phi(x + a p) - 0.1 phi(x)) / |p|]; advance until
          // that gap is within 0.1 % of the floor (or the span is covered);
          // the first advance is 0.9 phi(x) / |p|
          const double floor_ = 0.1 * phi;
          a = isinf(phi) ? FILTER_SPAN : (phi > 0.0 ? 0.9 * phi / pn : 0.0);
          for (int it = 1; it < 32 && a < FILTER_SPAN; ++it) {
            const double y[3] = {x[0] + a * p[0], x[1] + a * p[1], x[2] + a * p[2]};
            double ph, gy[3];
            // beyond floor + (span left) |p| the next advance covers the span
            sdf_world(I, E.meshes, y, ph, gy, H, false, floor_ + (FILTER_SPAN - a) * pn);
            const double gap = ph - floor_;
            if (gap <= 1e-3 * floor_) break;
            a += gap / pn;
          }
        } else if (I.shape == TC_TEXTURE) {
          // |hess phi| <= k^2 A / sqrt(1 + (kA)^2) everywhere
          const double A = I.prm[0], kk = 2.0 * M_PI / I.prm[1];
          a = quadratic_step(phi, gp, kk * kk * A / sqrt(1.0 + (kk * A) * (kk * A)), pn);
        } else {
          // torus: outside the tube |hess phi| <= 1/r_t (tube) + 1/rho (ring),
          // rho the distance from the torus axis, at its minimum over the
          // segment a in [0, FILTER_SPAN] (local frame: y = R^T (x - c))
          double y[3], q[3];
          for (int i = 0; i < 3; ++i) {
            y[i] = I.R[0 * 3 + i] * (x[0] - I.c[0]) + I.R[1 * 3 + i] * (x[1] - I.c[1]) + I.R[2 * 3 + i] * (x[2] - I.c[2]);
            q[i] = I.R[0 * 3 + i] * p[0] + I.R[1 * 3 + i] * p[1] + I.R[2 * 3 + i] * p[2];
          }
          const double qq = q[0] * q[0] + q[1] * q[1];
          double as = qq > 0.0 ? -(y[0] * q[0] + y[1] * q[1]) / qq : 0.0;
          as = fmin(fmax(as, 0.0), FILTER_SPAN);
          const double rho = sqrt((y[0] + as * q[0]) * (y[0] + as * q[0]) + (y[1] + as * q[1]) * (y[1] + as * q[1]));
          const double K = 1.0 / I.prm[1] + 1.0 / fmax(rho, 1e-9);
          a = quadratic_step(phi, gp, K, pn);
        }
        a = fmin(a, FILTER_SPAN);
        amax = fmin(amax, a);
      }
    }
  }
  amax = block_reduce(amax, OpMin(), sh);
  if (threadIdx.x == 0) E.part_filt[tl.tile] = amax;
}

// One block per pad: reduce |d|_inf, g.d, the step bound; decide
// convergence (|d|_inf <= tol * bbox diagonal -> take the filtered step and
// stop) or start the line search at min(1, bound).
__global__ void k_env_dir(const EnvDesc* envs, int n) {
  __shared__ double sh[16];
  if (blockIdx.x >= n) return;
  const EnvDesc& E = envs[blockIdx.x];
  EnvState* S = E.st;
  if (!dir_ready(S)) return;
  double dm = -INFINITY, gd = 0.0, am = INFINITY;
  for (int k = threadIdx.x; k < E.n_vt; k += blockDim.x) {
    dm = fmax(dm, E.part_dir[2 * k]);
    gd += E.part_dir[2 * k + 1];
  }
  // the pairs' partial minima follow when the pad has pairs this step
  const int nf = E.n_ct + (pair_active(E, E.pose) ? E.n_pt : 0);
  for (int k = threadIdx.x; k < nf; k += blockDim.x) am = fmin(am, E.part_filt[k]);
  dm = block_reduce(dm, OpMax(), sh);
  gd = block_reduce(gd, OpSum(), sh);
  am = block_reduce(am, OpMin(), sh);
  if (threadIdx.x == 0) {
    S->final_step_inf = dm;
    S->gTd = gd;
    S->alpha_max = am;
    S->ls_alpha = fmin(1.0, am);
    // a direction from a loose CG solve can be short only because the soft
    // modes are unresolved: convergence is judged on a floor-tolerance solve
    const bool tight = S->cg_tol2 <= E.cg_conv_tol * E.cg_conv_tol * (1.0 + 1e-12) || S->cg_iters >= E.max_cg;
    if (S->breakdown) {
      // negative curvature met (an unfiltered element or barrier Hessian):
      // keep the CG iterate (a descent direction) but judge nothing on it,
      // and filter the element Hessians for the rest of the step.  The
      // barrier Hessians too once the iterate is zero (a breakdown at the
      // first iteration) or at the second breakdown of the step: the
      // unfiltered ones would give the same breakdown again
      S->no_true_hess = 1;
      S->true_hess = 0;
      if (!(dm > 0.0) || ++S->n_breakdown >= 2) S->filt_all = 1;
      S->dir_conv = 0;
    } else {
      S->dir_conv = dm <= E.tol_abs && tight;
      // once a loose direction has looked converged, every further direction
      // of this step is solved to the floor tolerance (no loose/tight
      // alternation while the iterates creep towards the tolerance)
      if (dm <= E.tol_abs && !tight) S->force_tight = 1;
    }
    S->ls_done = S->dir_conv;
    S->apply = S->dir_conv;
    S->cg_total += S->cg_iters + S->warm;   // (a warm start's product counts as an iteration)
    S->stage = S->ls_done ? ST_UPD : ST_LS;
  }
}

// ------------------------------------------------------ energy / line search (a6)

// Incremental potential at y = x + alpha d (float64 throughout): tet tiles
// give sum V_e Psi(F_e), vertex tiles the inertia term, candidate tiles the
// barrier (+inf on contact) and friction.  mode 0: E(x) of pads being initialised (d is
// not read); mode 1: trial step of pads still searching.
template <typename R>
__global__ void k_energy(const Tile* tiles, int ntiles, const EnvDesc* envs, int mode) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  const EnvState* S = E.st;
  const EnvPose* P = E.pose;
  if (mode == 0 ? !initialising(S) : (!at_stage(S, ST_LS) || S->ls_done)) return;
  const double al = mode == 0 ? 0.0 : S->ls_alpha;
  const R* d = (const R*)E.d;
  double acc = 0.0;
  int tt = tl.tile;
  if (tt < E.n_te) {
    const int e = tt * blockDim.x + threadIdx.x;
    if (e < E.T) {
      const int4 tv = reinterpret_cast<const int4*>(E.tets)[e];
      const int vv[4] = {tv.x, tv.y, tv.z, tv.w};
      double u[4][3];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c)
          u[a][c] = E.xn[3 * vv[a] + c] + (mode ? al * (double)d[3 * vv[a] + c] : 0.0) - E.X[3 * vv[a] + c];
      const R* Dmp = (const R*)E.Dminv + 9 * e;
      double H[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          H[i][j] = (u[1][i] - u[0][i]) * (double)Dmp[j] + (u[2][i] - u[0][i]) * (double)Dmp[3 + j] +
                    (u[3][i] - u[0][i]) * (double)Dmp[6 + j];
      const int mid = E.mat ? E.mat[e] : 0;
      double dC[3][3];
      const double Jm1 = kinematics(H, dC);
      double hh = 0, tr = H[0][0] + H[1][1] + H[2][2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) hh += H[i][j] * H[i][j];
      // Psi = mu/2 (tr F^T F - 3) + lam/2 (J - alpha)^2 with F = I + H
      const double sJ = Jm1 - E.cshift[mid] / E.lam[mid];
      const double psi = 0.5 * E.mu[mid] * (2.0 * tr + hh) + 0.5 * E.lam[mid] * sJ * sJ;
      acc = (double)((const R*)E.vol)[e] * psi;
    }
  } else if ((tt -= E.n_te) < E.n_vt) {
    const int i = tt * blockDim.x + threadIdx.x;
    if (i < E.V && !E.quasi_static) {
      double s = 0;
      for (int c = 0; c < 3; ++c) {
        const double dy = E.xn[3 * i + c] + (mode ? al * (double)d[3 * i + c] : 0.0) - E.xhat[3 * i + c];
        s += dy * dy;
      }
      acc = 0.5 * E.mass[i] * s;
    }
  } else {
    tt -= E.n_vt;
    const int k = tt * blockDim.x + threadIdx.x;
    if (k < E.C) {
      const int vi = E.cand[k];
      double y[3], g[3], H[3][3];
      for (int c = 0; c < 3; ++c) y[c] = E.xn[3 * vi + c] + (mode ? al * (double)d[3 * vi + c] : 0.0);
      for (int m = 0; m < P->n_ind; ++m) {
        double phi;
        if (E.mesh_pairs && P->ind[m].shape == TC_MESH) {
          double Hn[3][3];
          mesh_pair_world(P->ind[m], E.meshes, y, E.dhat, false, phi, g, H, Hn);
          acc += E.kappa * E.cand_area[k] * phi;
          continue;
        }
        sdf_world(P->ind[m], E.meshes, y, phi, g, H, false, E.dhat);
        if (phi < E.dhat) acc += E.kappa * E.cand_area[k] * E.dhat * bar0(phi / E.dhat);
      }
      if (E.fr_mu > 0) {
        double xt[3];
        load3(E.x, vi, xt);
        acc += fr_energy(E, P->n_ind, k, y, xt);
      }
    }
  }
  acc = block_reduce(acc, OpSum(), sh);
  if (threadIdx.x == 0) E.part_e[tl.tile] = acc;
}

// One block per pad: E = inertia + h^2 (elastic + barrier + friction).  mode 0 stores
// E(x).  mode 1: Armijo test E(x + a d) <= E(x) + 1e-4 a g.d + noise |E(x)|,
// accept or halve a.
// After a full step passes Armijo with much less decrease than the model
// predicts: the quadratic through E(0), E'(0) = g.d and E(1) has its
// minimum at alpha* = -g.d / (2 (E(1) - E(0) - g.d)).  With the CG
// direction's own curvature (d.Hd = -g.d) the model's minimum is at 1; a
// minimum below 0.7 means the energy curves up along d at least 1.4 times
// as fast as the model (the full step overshoots, and Newton stalls on
// the component it keeps overshooting).  Then alpha* (at least 0.1) is
// tried next, and kept if it lowers the energy below E(1).
__device__ __forceinline__ bool ls_try_contract(EnvState* S, double E1) {
  const double gd = S->gTd;
  const double c = E1 - S->E_cur - gd;
  if (!(gd < 0.0) || !(c > 0.0)) return false;
  const double as = -gd / (2.0 * c);
  if (!(as < 0.7)) return false;
  S->ls_contracting = 1;
  S->ls_best_alpha = 1.0;
  S->ls_best_E = E1;
  S->ls_alpha = fmax(as, 0.1);
  return true;
}

__global__ void k_env_ls(const EnvDesc* envs, int n, int mode) {
  __shared__ double sh[16];
  if (blockIdx.x >= n) return;
  const EnvDesc& E = envs[blockIdx.x];
  EnvState* S = E.st;
  if (mode == 0 ? !initialising(S) : (!at_stage(S, ST_LS) || S->ls_done)) return;
  double el = 0, in = 0, ba = 0;
  for (int k = threadIdx.x; k < E.n_te; k += blockDim.x) el += E.part_e[k];
  for (int k = threadIdx.x; k < E.n_vt; k += blockDim.x) in += E.part_e[E.n_te + k];
  const int nb = E.n_ct + (pair_active(E, E.pose) ? E.n_pt : 0);   // the pairs' partial sums follow
  for (int k = threadIdx.x; k < nb; k += blockDim.x) ba += E.part_e[E.n_te + E.n_vt + k];
  el = block_reduce(el, OpSum(), sh);
  in = block_reduce(in, OpSum(), sh);
  ba = block_reduce(ba, OpSum(), sh);
  if (threadIdx.x != 0) return;
  const double Etot = in + E.h * E.h * (el + ba);
  if (mode == 0) {
    S->E_cur = Etot;
    if (S->infeasible) {
      S->status = TC_E_INFEASIBLE;
      S->phase = PH_FINISH;
    } else {
      S->phase = PH_RUN;
    }
    return;
  }
  const double a = S->ls_alpha;
  const bool armijo = Etot <= S->E_cur + 1e-4 * a * S->gTd + E.noise * fabs(S->E_cur);
  if (S->ls_contracting) {
    if (Etot < S->ls_best_E) {
      S->ls_best_alpha = a;
      S->ls_best_E = Etot;
    }
    S->ls_alpha = S->ls_best_alpha;
    S->E_next = S->ls_best_E;
    S->ls_done = 1;
    S->apply = 1;
    S->stage = ST_UPD;
    return;
  }
  if (S->ls_expanding) {
    // doubling an accepted full step: keep the larger step while it lowers
    // the energy further (and still passes Armijo)
    if (armijo && Etot < S->ls_best_E) {
      S->ls_best_alpha = a;
      S->ls_best_E = Etot;
      S->ls_expand_n += 1;
      if (S->ls_expand_n < E.ls_expand && 2.0 * a <= S->alpha_max) {
        S->ls_alpha = 2.0 * a;
        return;
      }
    }
    S->ls_alpha = S->ls_best_alpha;
    S->E_next = S->ls_best_E;
    S->ls_done = 1;
    S->apply = 1;
    S->stage = ST_UPD;
    return;
  }
  if (armijo) {
    if (S->ls_halv == 0 && a == 1.0 && ls_try_contract(S, Etot)) return;
    if (E.ls_expand > 0 && S->ls_halv == 0 && a == 1.0 && 2.0 <= S->alpha_max) {
      S->ls_expanding = 1;
      S->ls_best_alpha = a;
      S->ls_best_E = Etot;
      S->ls_alpha = 2.0;
      return;
    }
    S->ls_done = 1;
    S->apply = 1;
    S->E_next = Etot;
    S->stage = ST_UPD;
  } else {
    S->ls_alpha = 0.5 * a;
    S->ls_halv += 1;
    if (S->ls_halv > E.max_halvings) {
      S->status = TC_E_LINESEARCH;
      S->phase = PH_FINISH;
    }
  }
}

// x += alpha d for pads whose step was accepted.
template <typename R>
__global__ void k_update(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  EnvState* S = E.st;
  if (!at_stage(S, ST_UPD)) return;
  const int i = tl.tile * blockDim.x + threadIdx.x;
  if (S->apply && i < E.V) {
    const R* d = (const R*)E.d;
    const double a = S->ls_alpha;
    for (int c = 0; c < 3; ++c) E.xn[3 * i + c] += a * (double)d[3 * i + c];
  }
}

// One block per pad, after k_update (which must see the pad at its update
// stage in every block): Newton counters and the end-of-solve transition.
__global__ void k_env_update(const EnvDesc* envs, int n) {
  if (blockIdx.x >= n || threadIdx.x != 0) return;
  const EnvDesc& E = envs[blockIdx.x];
  EnvState* S = E.st;
  if (!at_stage(S, ST_UPD)) return;
  S->newton_iters += 1;
  S->ls_total += S->ls_halv;
  const bool adaptive = (E.hess_proj & 3) == 2 || ((E.hess_proj >> 2) & 3) == 3;
  if (adaptive && S->apply && S->ls_alpha >= 1.0 && !S->no_true_hess) S->true_hess = 1;
  if (!S->dir_conv) S->E_cur = S->E_next;
  if (S->dir_conv) {
    S->newton_done = 1;
    S->phase = PH_FINISH;
  } else if (S->newton_iters >= E.max_newton) {
    S->status = TC_E_NOT_CONVERGED;
    S->phase = PH_FINISH;
  } else {
    S->stage = ST_START;
  }
}

// ------------------------------------------------------ extraction (a8-a10)

__device__ __forceinline__ bool extract_ok(const EnvState* S) {
  return S->phase == PH_FINISH && S->status == TC_OK;
}

// Eq. 4 per tet: sigma = (mu / J) F F^T + lam (J - alpha) I, Voigt order
// (xx, yy, zz, yz, xz, xy).
template <typename R>
__global__ void k_sigma(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  EnvState* S = E.st;
  if (!extract_ok(S)) return;
  // the pad's extraction is under way: k_env_extract may finish it (a pad
  // that ended its Newton solve while other pads' extraction was launched
  // waits for its own)
  if (tiles[t].tile == 0 && threadIdx.x == 0) S->extracting = 1;
  const int e = tiles[t].tile * blockDim.x + threadIdx.x;
  if (e >= E.T) return;
  const double* x = S->mode == 1 ? E.x : E.xn;
  const int4 tv = reinterpret_cast<const int4*>(E.tets)[e];
  const R* Dmp = (const R*)E.Dminv + 9 * e;
  R Dm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[i][j] = Dmp[3 * i + j];
  R H[3][3], dC[3][3];
  disp_gradient(x, E.X, tv, Dm, H);
  const R Jm1 = kinematics(H, dC);
  const int mid = E.mat ? E.mat[e] : 0;
  const R mu = (R)E.mu[mid], lam = (R)E.lam[mid], csh = (R)E.cshift[mid];
  const R J = R(1) + Jm1;
  // Eq. 4 with F = I + H: (mu/J)(H + H^T + H H^T) + [mu - c - mu (J-1)/J + lam (J-1)] I
  const R muJ = mu / J, vol = (mu - csh) - mu * Jm1 / J + lam * Jm1;
  R b[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      b[i][j] = H[i][j] + H[j][i] + H[i][0] * H[j][0] + H[i][1] * H[j][1] + H[i][2] * H[j][2];
  R* s = (R*)E.sigma + 6 * e;
  s[0] = muJ * b[0][0] + vol;
  s[1] = muJ * b[1][1] + vol;
  s[2] = muJ * b[2][2] + vol;
  s[3] = muJ * b[1][2];
  s[4] = muJ * b[0][2];
  s[5] = muJ * b[0][1];
}

// Alg. 1 per surface triangle (current positions): n = e1 x e2 / |e1 x e2|,
// t = sigma_parent n, p_n = t . n, t_tau = t - p_n n; partial sum of t * area
// over contact-face triangles.
template <typename R>
__global__ void k_traction(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  const EnvState* S = E.st;
  if (!extract_ok(S)) return;
  const double* x = S->mode == 1 ? E.x : E.xn;
  const int j = tl.tile * blockDim.x + threadIdx.x;
  double ts[3] = {0, 0, 0};
  if (j < E.S) {
    double v0[3], v1[3], v2[3];
    load3(x, E.tris[3 * j], v0); load3(x, E.tris[3 * j + 1], v1); load3(x, E.tris[3 * j + 2], v2);
    const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    const double L = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int c = 0; c < 3; ++c) E.tri_cross[3 * j + c] = cr[c];
    const R n[3] = {(R)(cr[0] / L), (R)(cr[1] / L), (R)(cr[2] / L)};
    const R* s6 = (const R*)E.sigma + 6 * E.parent[j];
    const R sg[3][3] = {{s6[0], s6[5], s6[4]}, {s6[5], s6[1], s6[3]}, {s6[4], s6[3], s6[2]}};
    R tr[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) tr[r] = sg[r][0] * n[0] + sg[r][1] * n[1] + sg[r][2] * n[2];
    const R pn = tr[0] * n[0] + tr[1] * n[1] + tr[2] * n[2];
    R* to = (R*)E.traction + 3 * j;
    R* tt = (R*)E.tangential + 3 * j;
    R* no = (R*)E.tri_normal + 3 * j;
    for (int c = 0; c < 3; ++c) {
      to[c] = tr[c];
      tt[c] = tr[c] - pn * n[c];
      no[c] = n[c];
    }
    ((R*)E.pressure)[j] = pn;
    const R area = (R)(0.5 * L);
    ((R*)E.tri_area)[j] = area;
    if (E.is_top[j])
      for (int c = 0; c < 3; ++c) ts[c] = (double)tr[c] * (double)area;
  }
  for (int c = 0; c < 3; ++c) {
    const double v = block_reduce(ts[c], OpSum(), sh);
    if (threadIdx.x == 0) E.part_s3[3 * tl.tile + c] = v;
  }
}

// Alg. 2 contact path per contact vertex: f = -dE_b/dx (plus the friction
// force after a step with friction on; float64), vertex
// normal = normalised sum of e1 x e2 over the vertex's triangles (contact
// face, else its side faces), A = 1/3 their area, f_n = (f.n) n, f_tau = f - f_n, p = |f| / A; partial sum of f.
__global__ void k_contact(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  __shared__ double sh[16];
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const Tile tl = tiles[t];
  const EnvDesc& E = envs[tl.env];
  const EnvState* S = E.st;
  const EnvPose* P = E.pose;
  if (!extract_ok(S)) return;
  const double* x = S->mode == 1 ? E.x : E.xn;
  const int k = tl.tile * blockDim.x + threadIdx.x;
  double fs[3] = {0, 0, 0};
  if (k < E.C) {
    const int vi = E.cand[k];
    double xv[3], H[3][3];
    load3(x, vi, xv);
    const double kA = E.kappa * E.cand_area[k];
    double f[3] = {0, 0, 0};
    for (int m = 0; m < P->n_ind; ++m) {
      double phi, g[3];
      if (E.mesh_pairs && P->ind[m].shape == TC_MESH) {
        double Hn[3][3];
        mesh_pair_world(P->ind[m], E.meshes, xv, E.dhat, false, phi, g, H, Hn);
        for (int c = 0; c < 3; ++c) f[c] -= kA * g[c];
        continue;
      }
      sdf_world(P->ind[m], E.meshes, xv, phi, g, H, false, E.dhat);
      if (phi < E.dhat) {
        const double b1 = bar1(phi / E.dhat);
        for (int c = 0; c < 3; ++c) f[c] -= kA * b1 * g[c];
      }
    }
    // vertex-face and edge-edge pairs of the vertex's surface primitives
    if (pair_active(E, P)) {
      double gp[3] = {0, 0, 0};
      pair_gather(E, k, gp, nullptr);
      for (int c = 0; c < 3; ++c) f[c] -= gp[c];
    }
    // friction force of the step, -mu lambda (f1/y) u (extraction after a
    // step only: the lag belongs to that step's start state)
    if (S->mode == 0 && E.fr_mu > 0) {
      double xt[3];
      load3(E.x, vi, xt);
      for (int m = 0; m < P->n_ind; ++m) {
        const double* fr = fr_rec(E, m, k);
        if (!(fr[FRIC_LAM] > 0)) continue;
        double u[3];
        const double y = fr_slip(fr, xv, xt, u);
        const double c = E.fr_mu * fr[FRIC_LAM] * fr_f1_over_y(y, E.fr_eps);
        for (int q = 0; q < 3; ++q) f[q] -= c * u[q];
      }
    }
    double nn[3] = {0, 0, 0}, A = 0;
    for (int c = E.ctri_ptr[k]; c < E.ctri_ptr[k + 1]; ++c) {
      const int j = E.ctri_idx[c];
      const double* cr = E.tri_cross + 3 * j;
      for (int q = 0; q < 3; ++q) nn[q] += cr[q];
      A += 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / 3.0;
    }
    const double L = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int q = 0; q < 3; ++q) nn[q] /= L;
    const double fn = f[0] * nn[0] + f[1] * nn[1] + f[2] * nn[2];
    const double fm = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int q = 0; q < 3; ++q) {
      E.c_force[3 * k + q] = f[q];
      E.c_normal[3 * k + q] = nn[q];
      E.c_fn[3 * k + q] = fn * nn[q];
      E.c_ft[3 * k + q] = f[q] - fn * nn[q];
      fs[q] = f[q];
    }
    E.c_area[k] = A;
    E.c_press[k] = fm / A;
  }
  for (int c = 0; c < 3; ++c) {
    const double v = block_reduce(fs[c], OpSum(), sh);
    if (threadIdx.x == 0) E.part_c3[3 * tl.tile + c] = v;
  }
}

// One block per pad: reaction = -sum f_k, contact-face traction integral.
__global__ void k_env_extract(const EnvDesc* envs, int n) {
  __shared__ double sh[16];
  if (blockIdx.x >= n) return;
  const EnvDesc& E = envs[blockIdx.x];
  EnvState* S = E.st;
  if (S->phase != PH_FINISH) return;
  if (S->status != TC_OK) {
    if (threadIdx.x == 0) S->phase = PH_DONE;
    return;
  }
  if (!S->extracting) return;
  for (int c = 0; c < 3; ++c) {
    double f = 0, s = 0;
    for (int k = threadIdx.x; k < E.n_ct; k += blockDim.x) f += E.part_c3[3 * k + c];
    for (int k = threadIdx.x; k < E.n_st; k += blockDim.x) s += E.part_s3[3 * k + c];
    f = block_reduce(f, OpSum(), sh);
    s = block_reduce(s, OpSum(), sh);
    if (threadIdx.x == 0) {
      E.reaction[c] = -f;
      E.traction_sum[c] = s;
      S->reaction[c] = -f;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S->phase = PH_DONE;
}

// Commit: v = (x_new - x) / h, x = x_new.
__global__ void k_commit(const Tile* tiles, int ntiles, const EnvDesc* envs) {
  const int t = xcd_tile(ntiles);
  if (t < 0) return;
  const EnvDesc& E = envs[tiles[t].env];
  const EnvState* S = E.st;
  if (S->mode != 0 || S->phase != PH_FINISH || S->status != TC_OK) return;
  const int i = tiles[t].tile * blockDim.x + threadIdx.x;
  if (i >= E.V) return;
  for (int c = 0; c < 3; ++c) {
    const double xn = E.xn[3 * i + c];
    E.v[3 * i + c] = (xn - E.x[3 * i + c]) / E.h;
    E.x[3 * i + c] = xn;
  }
}

// ------------------------------------------------------------ launchers

static inline unsigned grid8(int ntiles) { return (unsigned)(((ntiles + 7) / 8) * 8); }

// With timing events the dispatch itself carries them (its own start and end
// timestamps, no separate marker packets around it).
#define TC_GO(kern, grid, block, stream, ...)                                                       \
  do {                                                                                              \
    if (a.ev0)                                                                                      \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, a.ev0, a.ev1, 0, __VA_ARGS__); \
    else                                                                                            \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);                   \
  } while (0)

#define TC_LAUNCH(kern, ntiles, block, stream, ...)                   \
  do {                                                                \
    if ((ntiles) > 0) TC_GO(kern, grid8(ntiles), block, stream, __VA_ARGS__); \
  } while (0)

template <typename R>
hipError_t launch_typed(KernelId id, const LaunchArgs& a) {
  hipError_t err = hipSuccess;
  switch (id) {
    case KernelId::setup_tets: TC_LAUNCH(k_setup_tets<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::setup_mass: TC_LAUNCH(k_setup_mass<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.out); break;
    case KernelId::setup_area: TC_LAUNCH(k_setup_cand_area, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.out); break;
    case KernelId::predict: TC_LAUNCH(k_predict, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::project: TC_LAUNCH(k_project, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.mode); break;
    case KernelId::element: TC_LAUNCH(k_element<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::barrier: TC_LAUNCH(k_barrier, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::asm_diag: TC_LAUNCH(k_asm_diag<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::asm_off: TC_LAUNCH(k_asm_off<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::newton_begin:
      if (a.n_env > 0) TC_GO(k_env_newton_begin, a.n_env, 64, a.stream, a.envs, a.n_env);
      break;
    case KernelId::cg_spmv:
      if (a.clock) {
        if (a.lpr == 16) TC_LAUNCH((k_cg_spmv<R, 16, true>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, a.clock);
        else if (a.lpr == 32) TC_LAUNCH((k_cg_spmv<R, 32, true>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, a.clock);
        else TC_LAUNCH((k_cg_spmv<R, 0, true>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, a.clock);
      } else {
        if (a.lpr == 16) TC_LAUNCH((k_cg_spmv<R, 16, false>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, nullptr);
        else if (a.lpr == 32) TC_LAUNCH((k_cg_spmv<R, 32, false>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, nullptr);
        else TC_LAUNCH((k_cg_spmv<R, 0, false>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, nullptr);
      }
      break;
    case KernelId::cg_update:
      if (a.clock) TC_LAUNCH((k_cg_update<R, true>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, a.clock);
      else TC_LAUNCH((k_cg_update<R, false>), a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.parity, nullptr);
      break;
    case KernelId::newton_dir: TC_LAUNCH(k_newton_dir<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::filter: TC_LAUNCH(k_filter<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::env_dir:
      if (a.n_env > 0) TC_GO(k_env_dir, a.n_env, 256, a.stream, a.envs, a.n_env);
      break;
    case KernelId::energy: TC_LAUNCH(k_energy<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.mode); break;
    case KernelId::env_ls:
      if (a.n_env > 0) TC_GO(k_env_ls, a.n_env, 256, a.stream, a.envs, a.n_env, a.mode);
      break;
    case KernelId::update: TC_LAUNCH(k_update<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::env_update:
      if (a.n_env > 0) TC_GO(k_env_update, a.n_env, 64, a.stream, a.envs, a.n_env);
      break;
    case KernelId::sigma: TC_LAUNCH(k_sigma<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::traction: TC_LAUNCH(k_traction<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::contact: TC_LAUNCH(k_contact, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::env_extract:
      if (a.n_env > 0) TC_GO(k_env_extract, a.n_env, 256, a.stream, a.envs, a.n_env);
      break;
    case KernelId::commit: TC_LAUNCH(k_commit, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    case KernelId::pairs: TC_LAUNCH(k_pairs<R>, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.mode); break;
    case KernelId::pair_push:
      TC_LAUNCH(k_pair_push, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs, a.mode);
      break;
    case KernelId::pair_apply: TC_LAUNCH(k_pair_apply, a.ntiles, a.block, a.stream, a.tiles, a.ntiles, a.envs); break;
    default: break;
  }
  return err;
}

hipError_t launch_kernel(KernelId id, bool fp64, const LaunchArgs& a) {
  return fp64 ? launch_typed<double>(id, a) : launch_typed<float>(id, a);
}

}  // namespace tc
