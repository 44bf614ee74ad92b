// A client of the C ABI with no Python: builds the 2D convection-diffusion
// matrix -Lap(u) + (1, 0.5).grad(u) on a g x g grid (central differences,
// h^2-scaled, Dirichlet boundary eliminated, x fastest), k right-hand sides
// b = A x* with x*[i, c] = sin(i + 7 c), solves with the library on the GPU
// and writes the problem and the solution to a file: int32 n, k, nnz; row_ptr
// (n + 1 int32), col_idx (nnz int32), values (nnz double), b and x (n x k
// doubles each, row-major).
//
// usage: c_abi_client <g> <k> <variant> <formulation> <precond> <out-file>
// prints one line "iters=... status=... relres=... err=..." and exits 0 when
// every column converged; also checks that invalid arguments are rejected.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "bicgstab.h"

#define HIP_OK(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      return 2;                                                          \
    }                                                                    \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s g k variant formulation precond out-file\n", argv[0]);
    return 2;
  }
  const int g = std::atoi(argv[1]), k = std::atoi(argv[2]);
  const int variant = std::atoi(argv[3]), formulation = std::atoi(argv[4]), precond = std::atoi(argv[5]);
  const int n = g * g;
  const double h = 1.0 / (g + 1), bx = 1.0, by = 0.5;
  std::vector<int32_t> rp(n + 1, 0), col;
  std::vector<double> val;
  for (int i = 0; i < n; ++i) {
    const int x = i % g, y = i / g;
    // entries in increasing column order: south, west, centre, east, north
    if (y > 0) { col.push_back(i - g); val.push_back(-1.0 - by * h / 2); }
    if (x > 0) { col.push_back(i - 1); val.push_back(-1.0 - bx * h / 2); }
    col.push_back(i); val.push_back(4.0);
    if (x < g - 1) { col.push_back(i + 1); val.push_back(-1.0 + bx * h / 2); }
    if (y < g - 1) { col.push_back(i + g); val.push_back(-1.0 + by * h / 2); }
    rp[i + 1] = (int32_t)col.size();
  }
  const int nnz = (int)col.size();
  std::vector<double> xs((size_t)n * k), b((size_t)n * k, 0.0);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < k; ++c) xs[(size_t)i * k + c] = std::sin((double)i + 7.0 * c);
  for (int i = 0; i < n; ++i)
    for (int e = rp[i]; e < rp[i + 1]; ++e)
      for (int c = 0; c < k; ++c) b[(size_t)i * k + c] += val[e] * xs[(size_t)col[e] * k + c];

  int32_t *d_rp = nullptr, *d_col = nullptr;
  double *d_val = nullptr, *d_b = nullptr, *d_x = nullptr;
  HIP_OK(hipMalloc((void**)&d_rp, (n + 1) * sizeof(int32_t)));
  HIP_OK(hipMalloc((void**)&d_col, nnz * sizeof(int32_t)));
  HIP_OK(hipMalloc((void**)&d_val, nnz * sizeof(double)));
  HIP_OK(hipMalloc((void**)&d_b, (size_t)n * k * sizeof(double)));
  HIP_OK(hipMalloc((void**)&d_x, (size_t)n * k * sizeof(double)));
  HIP_OK(hipMemcpy(d_rp, rp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_col, col.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_val, val.data(), nnz * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_b, b.data(), (size_t)n * k * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemset(d_x, 0, (size_t)n * k * sizeof(double)));

  bicgstab_csr A;
  A.n = n;
  A.nnz = nnz;
  A.d_row_ptr = d_rp;
  A.d_col_idx = d_col;
  A.d_values = d_val;

  // invalid arguments are errors with a message, not crashes
  bicgstab_t bad = nullptr;
  const int rc_bad = bicgstab_create(&A, n, 0, variant, formulation, precond, BICGSTAB_FP64, nullptr, &bad);
  if (rc_bad != BICGSTAB_EINVAL || std::strlen(bicgstab_last_error()) == 0) {
    std::fprintf(stderr, "k = 0 was not rejected (code %d)\n", rc_bad);
    return 1;
  }

  bicgstab_t s = nullptr;
  int rc = bicgstab_create(&A, n, k, variant, formulation, precond, BICGSTAB_FP64, nullptr, &s);
  if (rc != BICGSTAB_OK) {
    std::fprintf(stderr, "bicgstab_create: %s (%s)\n", bicgstab_strerror(rc), bicgstab_last_error());
    return 1;
  }
  size_t ws = 0;
  void* d_ws = nullptr;
  if (bicgstab_workspace_bytes(s, &ws) != BICGSTAB_OK) return 1;
  HIP_OK(hipMalloc(&d_ws, ws));
  if (bicgstab_set_workspace(s, d_ws, ws) != BICGSTAB_OK) return 1;

  std::vector<int32_t> iters(k), status(k);
  std::vector<double> rt(k), rr(k);
  bicgstab_info info;
  info.iters = iters.data();
  info.status = status.data();
  info.relres_true = rt.data();
  info.relres_recursive = rr.data();
  rc = bicgstab_solve(s, d_b, d_x, 1e-10, 2000, &info);
  if (rc != BICGSTAB_OK) {
    std::fprintf(stderr, "bicgstab_solve: %s (%s)\n", bicgstab_strerror(rc), bicgstab_last_error());
    return 1;
  }
  std::vector<double> x((size_t)n * k);
  HIP_OK(hipMemcpy(x.data(), d_x, x.size() * sizeof(double), hipMemcpyDeviceToHost));
  FILE* f = std::fopen(argv[6], "wb");
  if (!f) return 2;
  const int32_t head[3] = {n, k, nnz};
  bool wrote = std::fwrite(head, sizeof(int32_t), 3, f) == 3;
  wrote = wrote && std::fwrite(rp.data(), sizeof(int32_t), rp.size(), f) == rp.size();
  wrote = wrote && std::fwrite(col.data(), sizeof(int32_t), col.size(), f) == col.size();
  wrote = wrote && std::fwrite(val.data(), sizeof(double), val.size(), f) == val.size();
  wrote = wrote && std::fwrite(b.data(), sizeof(double), b.size(), f) == b.size();
  wrote = wrote && std::fwrite(x.data(), sizeof(double), x.size(), f) == x.size();
  std::fclose(f);
  if (!wrote) return 2;

  bool ok = true;
  std::printf("iters=");
  for (int c = 0; c < k; ++c) std::printf("%s%d", c ? "," : "", iters[c]);
  std::printf(" status=");
  for (int c = 0; c < k; ++c) {
    std::printf("%s%d", c ? "," : "", status[c]);
    ok = ok && status[c] == BICGSTAB_COL_CONVERGED;
  }
  double worst_rt = 0.0, worst_err = 0.0;
  for (int c = 0; c < k; ++c) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
      const double d = x[(size_t)i * k + c] - xs[(size_t)i * k + c];
      num += d * d;
      den += xs[(size_t)i * k + c] * xs[(size_t)i * k + c];
    }
    worst_err = std::fmax(worst_err, std::sqrt(num / den));
    worst_rt = std::fmax(worst_rt, rt[c]);
  }
  std::printf(" relres=%.3e err=%.3e\n", worst_rt, worst_err);
  bicgstab_destroy(s);
  for (void* p : {d_ws, (void*)d_rp, (void*)d_col, (void*)d_val, (void*)d_b, (void*)d_x}) HIP_OK(hipFree(p));
  return ok && worst_rt < 1e-9 ? 0 : 1;
}
