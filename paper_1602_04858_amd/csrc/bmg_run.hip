// bmg_run: command-line driver of libbmg.so with no Python or PyTorch in the process.
//
// It sets up one handle, assembles the right-hand sides on the host, solves them on
// the device and prints one line per solve, so that profilers that preload their own
// HIP/HSA runtime (hardware-counter collection) see a process with exactly one copy
// of each.  A plain device copy of known size (--copy-mib) serves to calibrate memory
// counters: its kernel moves exactly 2 * MiB bytes.
//
//   bmg_run --kappa FILE [--sources FILE] --n0 2 --levels 10 --k 2 --mu 0.01 --sigma 12
//           --bc 0,0,1,1 --prec 2 --nrhs 16 --restart 7 --rtol 1e-10 --maxit 200
//           --solves 1 [--cycle 1] [--m-fine 2] [--dense-coarse-max 16384] [--colouring 0]
//   bmg_run --copy-mib 2048
//
// kappa FILE: N*N float64 values (cell (cx, cy) at cy*N + cx), N = n0 << levels.
// sources FILE: text, one line per right-hand side with `modes` groups of five numbers
// (amplitude, direction angle, kx, ky, phase): f(x, y) = sum a sin(2 pi (kx x + ky y) +
// phase) (cos angle, sin angle).  Without it every column uses f = (1, 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bmg.h"

namespace {

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

[[noreturn]] void die(const char* what) {
  std::fprintf(stderr, "bmg_run: %s\n", what);
  std::exit(2);
}

void hipok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::fprintf(stderr, "bmg_run: %s: %s\n", what, hipGetErrorString(e));
    std::exit(3);
  }
}

int copy_calibration(int64_t mib) {
  const int64_t bytes = mib << 20, n = bytes / 16;
  void *a = nullptr, *b = nullptr;
  hipok(hipMalloc(&a, bytes), "hipMalloc");
  hipok(hipMalloc(&b, bytes), "hipMalloc");
  hipok(hipMemset(a, 0, bytes), "hipMemset");
  hipEvent_t e0, e1;
  hipok(hipEventCreate(&e0), "event");
  hipok(hipEventCreate(&e1), "event");
  const int grid = 256 * 32;
  for (int it = 0; it < 6; ++it) {
    hipok(hipEventRecord(e0, nullptr), "record");
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, nullptr, (const float4*)a, (float4*)b, n);
    hipok(hipGetLastError(), "launch");
    hipok(hipEventRecord(e1, nullptr), "record");
    hipok(hipEventSynchronize(e1), "sync");
    float ms = 0.f;
    hipok(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    std::printf("copy %lld MiB: %.3f ms, %.0f GB/s (read + write)\n", (long long)mib, ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
  }
  hipok(hipFree(a), "hipFree");
  hipok(hipFree(b), "hipFree");
  return 0;
}

struct Mode {
  double a, th, kx, ky, ph;
};

}  // namespace

int main(int argc, char** argv) {
  bmg_params p{};
  p.n0 = 2;
  p.levels = 3;
  p.k = 1;
  p.mu = 1e-2;
  p.sigma = -1.0;
  p.bc[0] = p.bc[1] = BMG_BC_DIRICHLET;
  p.bc[2] = p.bc[3] = BMG_BC_OPEN;
  p.cycle = BMG_CYCLE_VARIABLE;
  p.m_fine = 2;
  p.precond_prec = BMG_P_FP64;
  p.restart = 60;
  p.dense_coarse_max = 16384;
  p.n_rhs = 1;
  std::string kfile, sfile;
  double rtol = 1e-10;
  int maxit = 200, solves = 1;
  for (int i = 1; i < argc; ++i) {
    const std::string a = argv[i];
    auto val = [&]() -> const char* {
      if (i + 1 >= argc) die(("missing value after " + a).c_str());
      return argv[++i];
    };
    if (a == "--copy-mib") return copy_calibration(std::atoll(val()));
    else if (a == "--kappa") kfile = val();
    else if (a == "--sources") sfile = val();
    else if (a == "--n0") p.n0 = std::atoi(val());
    else if (a == "--levels") p.levels = std::atoi(val());
    else if (a == "--k") p.k = std::atoi(val());
    else if (a == "--mu") p.mu = std::atof(val());
    else if (a == "--sigma") p.sigma = std::atof(val());
    else if (a == "--bc") {
      if (std::sscanf(val(), "%d,%d,%d,%d", &p.bc[0], &p.bc[1], &p.bc[2], &p.bc[3]) != 4) die("--bc wants a,b,c,d");
    } else if (a == "--prec") p.precond_prec = std::atoi(val());
    else if (a == "--nrhs") p.n_rhs = std::atoi(val());
    else if (a == "--restart") p.restart = std::atoi(val());
    else if (a == "--cycle") p.cycle = std::atoi(val());
    else if (a == "--m-fine") p.m_fine = std::atoi(val());
    else if (a == "--dense-coarse-max") p.dense_coarse_max = std::atoi(val());
    else if (a == "--colouring") p.colouring = std::atoi(val());
    else if (a == "--rtol") rtol = std::atof(val());
    else if (a == "--maxit") maxit = std::atoi(val());
    else if (a == "--solves") solves = std::atoi(val());
    else die(("unknown argument " + a).c_str());
  }
  if (p.sigma < 0) p.sigma = (p.k + 1.0) * (p.k + 2.0);
  const int N = p.n0 << p.levels, R = p.n_rhs < 1 ? 1 : p.n_rhs;
  if (kfile.empty()) die("--kappa FILE is required");
  std::vector<double> kappa((size_t)N * N);
  {
    std::ifstream f(kfile, std::ios::binary);
    if (!f.read(reinterpret_cast<char*>(kappa.data()), (std::streamsize)(kappa.size() * sizeof(double))))
      die("kappa file shorter than N*N doubles");
  }
  std::vector<std::vector<Mode>> src(R);
  if (!sfile.empty()) {
    std::ifstream f(sfile);
    std::string line;
    for (int r = 0; r < R; ++r) {
      if (!std::getline(f, line)) die("sources file has fewer lines than right-hand sides");
      std::istringstream is(line);
      Mode m;
      while (is >> m.a >> m.th >> m.kx >> m.ky >> m.ph) src[r].push_back(m);
    }
  }
  size_t ws = 0;
  if (bmg_plan(&p, &ws) != BMG_OK) die("bmg_plan rejected the parameters");
  std::printf("N=%d levels=%d k=%d nrhs=%d prec=%d workspace %.1f GiB\n", N, p.levels, p.k, R, p.precond_prec,
              ws / 1073741824.0);
  std::fflush(stdout);

  // right-hand sides on the host, one column per thread
  const int q = p.k + 2;
  const size_t ncq = (size_t)N * N * q * q;
  std::vector<double> cell_xy(ncq * 2), face_xy((size_t)4 * N * q * 2);
  if (bmg_quad_points(&p, cell_xy.data(), face_xy.data()) != BMG_OK) die("bmg_quad_points failed");
  hipStream_t stream;
  hipok(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "stream");
  double t0 = now();
  bmg_handle h = nullptr;
  const bmg_status st = bmg_setup(&p, kappa.data(), nullptr, 0, stream, &h);
  if (st != BMG_OK) {
    std::fprintf(stderr, "bmg_setup: %s (%s)\n", bmg_status_string(st), bmg_last_error(nullptr));
    return 4;
  }
  hipok(hipStreamSynchronize(stream), "setup sync");
  std::printf("setup %.1f s\n", now() - t0);
  std::fflush(stdout);
  int32_t Nf = 0;
  int64_t nu = 0, np = 0;
  if (bmg_sizes(h, p.levels, &Nf, &nu, &np) != BMG_OK) die("bmg_sizes failed");
  const size_t ndof = (size_t)(nu + np);
  double *bd = nullptr, *xd = nullptr;
  hipok(hipMalloc((void**)&bd, ndof * R * sizeof(double)), "hipMalloc b");
  hipok(hipMalloc((void**)&xd, ndof * R * sizeof(double)), "hipMalloc x");
  {
    const int nthr = std::min(R, 16);
    std::vector<std::thread> th;
    std::vector<int> bad(R, 0);
    for (int t = 0; t < nthr; ++t)
      th.emplace_back([&, t]() {
        std::vector<double> f(ncq * 2), b(ndof);
        for (int r = t; r < R; r += nthr) {
          for (size_t i = 0; i < ncq; ++i) {
            const double x = cell_xy[2 * i], y = cell_xy[2 * i + 1];
            double fx = src[r].empty() ? 1.0 : 0.0, fy = 0.0;
            for (const Mode& m : src[r]) {
              const double s = m.a * std::sin(2.0 * M_PI * (m.kx * x + m.ky * y) + m.ph);
              fx += std::cos(m.th) * s;
              fy += std::sin(m.th) * s;
            }
            f[2 * i] = fx;
            f[2 * i + 1] = fy;
          }
          if (bmg_assemble_rhs(&p, f.data(), nullptr, nullptr, b.data()) != BMG_OK) bad[r] = 1;
          else if (hipMemcpy(bd + (size_t)r * ndof, b.data(), ndof * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            bad[r] = 1;
        }
      });
    for (auto& t : th) t.join();
    for (int r = 0; r < R; ++r)
      if (bad[r]) die("right-hand side assembly or upload failed");
  }
  std::printf("right-hand sides ready (%zu unknowns each)\n", ndof);
  std::fflush(stdout);
  std::vector<bmg_solve_info> info(R);
  for (int s = 0; s < solves; ++s) {
    t0 = now();
    const bmg_status ss = bmg_solve(h, bd, xd, rtol, maxit, nullptr, info.data());
    hipok(hipStreamSynchronize(stream), "solve sync");
    const double dt = now() - t0;
    int imin = 1 << 30, imax = 0;
    double worst = 0.0;
    for (int r = 0; r < R; ++r) {
      imin = std::min(imin, info[r].iterations);
      imax = std::max(imax, info[r].iterations);
      worst = std::max(worst, info[r].rel_residual_true);
    }
    std::printf("solve %d: %s, %.3f s, %.3f right-hand sides/s, iterations %d..%d, worst true residual %.2e\n", s,
                bmg_status_string(ss), dt, R / dt, imin, imax, worst);
    std::fflush(stdout);
    if (ss != BMG_OK && ss != BMG_E_NOT_CONVERGED) return 5;
  }
  bmg_destroy(h);
  hipok(hipFree(bd), "hipFree");
  hipok(hipFree(xd), "hipFree");
  hipok(hipStreamDestroy(stream), "stream destroy");
  return 0;
}
