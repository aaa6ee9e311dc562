// Host-emulation driver (test infrastructure): factors one CSR problem
// written by tests/test_host_emulation.py, optionally solves, and prints the
// results.  Every device buffer sits between large inaccessible regions so
// an access that leaves it traps.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/mman.h>
#include <vector>

// Device buffers live between huge PROT_NONE guard regions, so an access
// that leaves a buffer (as it would leave the GPU allocation) traps.
static void* guarded(size_t bytes) {
  const size_t G = size_t(64) << 30;
  const size_t pg = 4096, body = (bytes + pg - 1) / pg * pg;
  char* base = static_cast<char*>(mmap(nullptr, body + 2 * G, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0));
  if (base == MAP_FAILED) std::abort();
  if (mprotect(base + G, body, PROT_READ | PROT_WRITE)) std::abort();
  char* end = base + G + body;
  return end - (bytes + 255) / 256 * 256;
}
template <typename X>
static X* to_guarded(const std::vector<X>& v) {
  X* p = static_cast<X*>(guarded(v.size() * sizeof(X) + 1));
  std::memcpy(p, v.data(), v.size() * sizeof(X));
  return p;
}
#include <string>
#include <vector>

#include "spalu.h"

template <typename X>
std::vector<X> load(const std::string& p) {
  FILE* f = std::fopen(p.c_str(), "rb");
  if (!f) return {};
  std::fseek(f, 0, SEEK_END);
  long n = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<X> v(size_t(n) / sizeof(X));
  if (std::fread(v.data(), sizeof(X), v.size(), f) != v.size()) std::abort();
  std::fclose(f);
  return v;
}

int main(int argc, char** argv) {
  if (argc < 5) {
    std::fprintf(stderr, "usage: emu_run dir prec(64|32) model(0|1) eps [nrhs tol]\n");
    return 2;
  }
  const std::string d = argv[1];
  const int prec = std::atoi(argv[2]);
  const int model = std::atoi(argv[3]);
  const double eps = std::atof(argv[4]);
  const int nrhs = argc > 5 ? std::atoi(argv[5]) : 0;
  const double tol = argc > 6 ? std::atof(argv[6]) : 0.0;
  const unsigned seed = argc > 7 ? unsigned(std::atoi(argv[7])) : 1234u;
  const int restart = argc > 8 ? std::atoi(argv[8]) : 0;
  auto dims = load<int32_t>(d + "/dims.bin");
  auto rp = load<int64_t>(d + "/rowptr.bin");
  auto ci = load<int32_t>(d + "/colind.bin");
  auto va = load<double>(d + "/vals.bin");
  auto pm = load<float>(d + "/params.bin");
  const int dim = int(dims.size());
  spalu_nd_t* nd = nullptr;
  int rc = spalu_nd_order(dim, dims.data(), nullptr, &nd);
  if (rc) {
    std::printf("nd rc %d %s\n", rc, spalu_last_error());
    return 1;
  }
  spalu_factor_opts o;
  spalu_factor_opts_default(&o);
  o.eps = eps;
  o.seed = seed;
  o.precision = prec == 32 ? SPALU_FP32 : SPALU_FP64;
  if (model) o.rank_model = to_guarded(pm);
  if (const char* h0 = std::getenv("EMU_H0")) o.h0 = std::atoi(h0);
  if (const char* sy = std::getenv("EMU_SYM")) o.symmetric = std::atoi(sy);
  if (const char* tu = std::getenv("EMU_TUNING")) {
    // nine comma-separated spalu_tuning fields
    spalu_tuning t;
    int32_t* f = &t.id_lds_a;
    for (int i = 0; i < 9; ++i) f[i] = std::atoi(tu), tu = std::strchr(tu, ',') ? std::strchr(tu, ',') + 1 : tu;
    if (spalu_tuning_set(&t)) {
      std::printf("tuning refused: %s\n", spalu_last_error());
      return 1;
    }
  }
  size_t wb = 0;
  rc = spalu_factor_workspace(nd, &o, &wb);
  std::printf("workspace %zu bytes rc %d\n", wb, rc);
  void* ws = guarded(wb);
  {
    const char* gf = std::getenv("EMU_FILL");
    const int fill = gf ? std::atoi(gf) : 0x5A;
    std::memset(ws, fill, wb);
  }
  spalu_factor_t* F = nullptr;
  spalu_factor_info info{};
  const int64_t n = int64_t(rp.size()) - 1;
  int64_t* grp = to_guarded(rp);
  int32_t* gci = to_guarded(ci);
  double* gva = to_guarded(va);
  rc = spalu_factor(nd, n, grp, gci, gva, &o, ws, wb, nullptr, &F, &info);
  std::printf("factor rc %d (%s): sparsified %lld passes %lld resampled %lld max_front %lld\n", rc,
              rc ? spalu_last_error() : "ok", (long long)info.sparsified, (long long)info.sample_passes,
              (long long)info.resampled, (long long)info.max_front);
  if (rc) return 1;
  {
    // largest skeleton over the levels (row passes of the separator kernels)
    int64_t nn = 0, nnodes = 0, nsegs = 0;
    int32_t L = 0;
    spalu_nd_info(nd, &nn, &L, &nnodes, &nsegs);
    std::vector<int64_t> base(size_t(L) + 2);
    spalu_factor_seg_base(nd, base.data());
    const size_t ns = size_t(base[size_t(L) + 1]);
    std::vector<int32_t> nb(ns), rk(ns), hh(ns), ps(ns);
    int kmax = 0;
    if (spalu_factor_ranks(F, nb.data(), rk.data(), hh.data(), ps.data()) == 0)
      for (size_t i = 0; i < ns; ++i) kmax = std::max(kmax, int(rk[i]));
    std::printf("max_rank %d\n", kmax);
  }
  if (nrhs > 0) {
    std::vector<double> Bv(size_t(n) * nrhs);
    srand(7);
    for (auto& b : Bv) b = double(rand()) / RAND_MAX * 2.0 - 1.0;
    double* B = to_guarded(Bv);
    double* X = to_guarded(Bv);
    size_t sb = 0;
    spalu_solve_opts so{tol, 30, 1, restart};
    spalu_solve_workspace(F, nrhs, &so, &sb);
    void* sw = guarded(sb);
    {
      // NaN bytes by default: a value read before it is written, even one
      // multiplied by zero, poisons the result
      const char* gf = std::getenv("EMU_SOLVE_FILL");
      const int fill = gf ? std::atoi(gf) : 0xFF;
      std::memset(sw, fill, sb);
    }
    spalu_solve_info si{};
    rc = spalu_solve(F, nrhs, B, n, X, n, &so, sw, sb, nullptr, nullptr, &si);
    std::printf("solve rc %d (%s) iters %d first %.3e final %.3e\n", rc, rc ? spalu_last_error() : "ok",
                si.iterations, si.first_rel_residual, si.max_rel_residual);
  }
  spalu_factor_free(F);
  spalu_nd_free(nd);
  return 0;
}
