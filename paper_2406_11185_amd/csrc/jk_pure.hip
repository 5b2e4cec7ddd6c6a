// Change of basis between Cartesian and pure (spherical) d functions for the
// matrices of jk_build: densities go from the pure basis to the Cartesian one
// before a build, and J, K and dE/dD come back.  The paper's workloads use bases
// of pure functions ("Benchmarks"); the integral kernels work on Cartesian
// shells, so a pure d shell enters as its six Cartesian components and leaves as
// its five pure functions.
//
// With T the block-diagonal [n_cart][n_pure] matrix (identity for s and p shells,
// the table below for d shells), a pure function is phi_f = sum_c T[c][f] chi_c,
// so for a pure density P the Cartesian density is T P T^T and the pure J and K
// are T^T J T and T^T K T (every integral over pure functions is the same
// combination of Cartesian ones).  Both directions are one kernel,
//   out[i][j] = sum_p sum_q w_ip w_jq in[r_ip][r_jq],
// where output index i lists its (at most three) input indices r_ip with their
// weights w_ip.  HBM-bound: each output element is written once and its input
// rows are shared by the whole row of outputs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "jk.h"

namespace {

// The five pure d functions over the Cartesian components (xx, xy, xz, yy, yz,
// zz), in the order m = -2, -1, 0, 1, 2: the real solid harmonics of degree 2,
//   m=-2: sqrt3 xy,  m=-1: sqrt3 yz,  m=0: zz - (xx + yy)/2,  m=1: sqrt3 xz,
//   m=2: sqrt3/2 (xx - yy),
// each with the norm of xx and free of the s-type combination xx + yy + zz.
struct PureTerm {
  int cart;
  double w;
};
struct PureFun {
  int n;
  PureTerm t[3];
};
PureFun pure_fun(int m) {
  const double r3 = std::sqrt(3.0);
  switch (m) {
    case 0: return {1, {{1, r3}, {0, 0.0}, {0, 0.0}}};
    case 1: return {1, {{4, r3}, {0, 0.0}, {0, 0.0}}};
    case 2: return {3, {{5, 1.0}, {0, -0.5}, {3, -0.5}}};
    case 3: return {1, {{2, r3}, {0, 0.0}, {0, 0.0}}};
    default: return {2, {{0, 0.5 * r3}, {3, -0.5 * r3}, {0, 0.0}}};
  }
}

// Row map of one direction: output index i reads input indices idx[i].x..
// (idx[i].w of them) with weights wt[i].
struct RowMap {
  std::vector<int4> idx;
  std::vector<double4> wt;
};

// to_cart = true: output Cartesian, input pure (rows of T); false: output pure,
// input Cartesian (columns of T).
RowMap row_map(const jk_basis* b, bool to_cart, int* n_in, int* n_out) {
  RowMap r;
  int cart0 = 0, pure0 = 0;
  for (int s = 0; s < b->n_shells; ++s) {
    const int l = b->shell_l[s];
    const int nc = (l + 1) * (l + 2) / 2;
    if (l < 2) {   // s, p: the same functions in both bases
      for (int k = 0; k < nc; ++k) {
        r.idx.push_back(make_int4(to_cart ? pure0 + k : cart0 + k, 0, 0, 1));
        r.wt.push_back(make_double4(1.0, 0.0, 0.0, 0.0));
      }
      cart0 += nc;
      pure0 += nc;
      continue;
    }
    if (to_cart) {
      // Cartesian component c = sum over the pure functions that contain it
      for (int c = 0; c < 6; ++c) {
        int in[3] = {0, 0, 0}, n = 0;
        double w[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < 5; ++m) {
          const PureFun f = pure_fun(m);
          for (int t = 0; t < f.n; ++t)
            if (f.t[t].cart == c) { in[n] = pure0 + m; w[n] = f.t[t].w; ++n; }
        }
        r.idx.push_back(make_int4(in[0], in[1], in[2], n));
        r.wt.push_back(make_double4(w[0], w[1], w[2], 0.0));
      }
    } else {
      for (int m = 0; m < 5; ++m) {
        const PureFun f = pure_fun(m);
        r.idx.push_back(make_int4(cart0 + f.t[0].cart, cart0 + f.t[1].cart, cart0 + f.t[2].cart, f.n));
        r.wt.push_back(make_double4(f.t[0].w, f.t[1].w, f.t[2].w, 0.0));
      }
    }
    cart0 += 6;
    pure0 += 5;
  }
  *n_in = to_cart ? pure0 : cart0;
  *n_out = to_cart ? cart0 : pure0;
  return r;
}

constexpr int kRowThreads = 256;

// One thread per output element out[m][i][j]; block (x: j tile, y: i, z: m).
__global__ __launch_bounds__(kRowThreads) void basis_change_kernel(
    const double* __restrict__ in, double* __restrict__ out, int n_in, int n_out,
    const int4* __restrict__ idx, const double4* __restrict__ wt) {
  const int j = blockIdx.x * kRowThreads + threadIdx.x;
  const int i = blockIdx.y;
  const int m = blockIdx.z;
  if (j >= n_out) return;
  const int4 ri = idx[i];
  const double4 wi = wt[i];
  const int4 rj = idx[j];
  const double4 wj = wt[j];
  const double* X = in + static_cast<size_t>(m) * n_in * n_in;
  const int ri_[3] = {ri.x, ri.y, ri.z}, rj_[3] = {rj.x, rj.y, rj.z};
  const double wi_[3] = {wi.x, wi.y, wi.z}, wj_[3] = {wj.x, wj.y, wj.z};
  double s = 0.0;
  for (int p = 0; p < ri.w; ++p) {
    const double* row = X + static_cast<size_t>(ri_[p]) * n_in;
    double t = 0.0;
    for (int q = 0; q < rj.w; ++q) t += wj_[q] * row[rj_[q]];
    s += wi_[p] * t;
  }
  out[(static_cast<size_t>(m) * n_out + i) * n_out + j] = s;
}

int change_basis(const jk_basis* b, int32_t n_dm, const double* in, double* out, void* stream,
                 bool to_cart) {
  int32_t n_cart = 0;
  const int rc = jk_validate_basis(b, &n_cart);
  if (rc != JK_OK) return rc;
  if (!in || !out || n_dm < 1 || n_dm > JK_MAX_NDM) return JK_EINVAL;
  int n_in = 0, n_out = 0;
  const RowMap r = row_map(b, to_cart, &n_in, &n_out);
  if (n_out > 65535) return JK_EUNSUPPORTED;   // one grid row per output row
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t ib = r.idx.size() * sizeof(int4), wb = r.wt.size() * sizeof(double4);
  void* tab = nullptr;
  if (hipMallocAsync(&tab, ib + wb, s) != hipSuccess) return JK_ENOMEM;
  int4* d_idx = static_cast<int4*>(tab);
  double4* d_wt = reinterpret_cast<double4*>(static_cast<char*>(tab) + ib);
  bool ok = hipMemcpyAsync(d_idx, r.idx.data(), ib, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(d_wt, r.wt.data(), wb, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;   // the host tables go out of scope
  if (ok) {
    const dim3 grid((n_out + kRowThreads - 1) / kRowThreads, n_out, n_dm);
    hipLaunchKernelGGL(basis_change_kernel, grid, dim3(kRowThreads), 0, s, in, out, n_in, n_out,
                       d_idx, d_wt);
    ok = hipGetLastError() == hipSuccess;
  }
  const bool freed = hipFreeAsync(tab, s) == hipSuccess;
  return ok && freed ? JK_OK : JK_EHIP;
}

}  // namespace

extern "C" {

int jk_pure_count(const jk_basis* basis, int32_t* n_pure_out) {
  int32_t n = 0;
  const int rc = jk_validate_basis(basis, &n);
  if (rc != JK_OK) return rc;
  int32_t np = 0;
  for (int s = 0; s < basis->n_shells; ++s) np += 2 * basis->shell_l[s] + 1;
  if (n_pure_out) *n_pure_out = np;
  return JK_OK;
}

int jk_pure_to_cart(const jk_basis* basis, int32_t n_dm, const double* X_pure, double* X_cart,
                    void* hip_stream) {
  return change_basis(basis, n_dm, X_pure, X_cart, hip_stream, true);
}

int jk_cart_to_pure(const jk_basis* basis, int32_t n_dm, const double* X_cart, double* X_pure,
                    void* hip_stream) {
  return change_basis(basis, n_dm, X_cart, X_pure, hip_stream, false);
}

}  // extern "C"
