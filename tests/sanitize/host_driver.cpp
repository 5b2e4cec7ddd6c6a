// Host-side checks of libjk's C entry points that need no GPU: option
// defaults, basis validation (every rejection rule and the accepted case),
// NULL and invalid handles, and context creation on a machine without a
// usable device.  Compiled with the host library's translation unit
// (csrc/jk_host.hip, host pass only) under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  The per-class
// launch tables are stubs here: nothing below reaches a kernel launch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "jk.h"
#include "jk_grad_device.hpp"

namespace jk {
[[noreturn]] static void unreachable(const char* f) {
  std::fprintf(stderr, "host driver: %s called without a device\n", f);
  std::abort();
}
void launch_eri(int, int, const EriLaunch&, hipStream_t) { unreachable("launch_eri"); }
void launch_grad(int, int, const GradLaunch&, hipStream_t) { unreachable("launch_grad"); }
void launch_schwarz(int, const EriLaunch&, double*, hipStream_t) { unreachable("launch_schwarz"); }
size_t split_ws_bytes(int, int, int) { unreachable("split_ws_bytes"); }
size_t split_schwarz_ws_bytes(int) { unreachable("split_schwarz_ws_bytes"); }
int class_lanes(int, int) { unreachable("class_lanes"); }
int class_lane_mask(int, int) { unreachable("class_lane_mask"); }
double class_cost(int, int) { unreachable("class_cost"); }
int grad_ws_elems(int) { unreachable("grad_ws_elems"); }
int grad_lanes(int) { unreachable("grad_lanes"); }
int grad_lane_mask(int) { unreachable("grad_lane_mask"); }
}  // namespace jk

static int failures = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "host driver: FAILED %s\n", what);
    ++failures;
  }
}

struct Basis {
  std::vector<double> xyz{0.0, 0.0, 0.0, 1.2, -0.4, 0.9};
  std::vector<int32_t> atom{0, 0, 1, 1}, l{0, 2, 1, 0}, nprim{3, 1, 2, 8}, prim0{0, 3, 4, 6};
  std::vector<double> exps, coefs;
  Basis() {
    for (int p = 0; p < 14; ++p) {
      exps.push_back(0.3 * (p + 1));
      coefs.push_back(0.5 + 0.01 * p);
    }
  }
  jk_basis view() {
    jk_basis b{};
    b.n_atoms = static_cast<int32_t>(xyz.size() / 3);
    b.xyz = xyz.data();
    b.n_shells = static_cast<int32_t>(atom.size());
    b.shell_atom = atom.data();
    b.shell_l = l.data();
    b.shell_nprim = nprim.data();
    b.shell_prim0 = prim0.data();
    b.exps = exps.data();
    b.coefs = coefs.data();
    return b;
  }
};

int main() {
  jk_opts o;
  expect(jk_opts_default(&o) == JK_OK && o.precision == JK_FP64 && o.n_dm == 1 &&
             o.deterministic == 0 && o.energy == nullptr && o.dEdD == nullptr,
         "jk_opts_default");
  expect(jk_opts_default(nullptr) == JK_EINVAL, "jk_opts_default(NULL)");

  int32_t nbf = -1;
  {
    Basis B;
    jk_basis b = B.view();
    expect(jk_validate_basis(&b, &nbf) == JK_OK && nbf == 1 + 6 + 3 + 1, "valid basis");
    expect(jk_validate_basis(&b, nullptr) == JK_OK, "valid basis, no count");
  }
  expect(jk_validate_basis(nullptr, &nbf) == JK_EINVAL, "NULL basis");
  struct Case {
    const char* what;
    int want;
    void (*edit)(Basis&, jk_basis&);
  };
  const Case cases[] = {
      {"no atoms", JK_EINVAL, [](Basis&, jk_basis& b) { b.n_atoms = 0; }},
      {"no shells", JK_EINVAL, [](Basis&, jk_basis& b) { b.n_shells = 0; }},
      {"NULL xyz", JK_EINVAL, [](Basis&, jk_basis& b) { b.xyz = nullptr; }},
      {"NULL exps", JK_EINVAL, [](Basis&, jk_basis& b) { b.exps = nullptr; }},
      {"NULL coefs", JK_EINVAL, [](Basis&, jk_basis& b) { b.coefs = nullptr; }},
      {"NaN coordinate", JK_EINVAL, [](Basis& B, jk_basis&) { B.xyz[4] = std::nan(""); }},
      {"atom index", JK_EINVAL, [](Basis& B, jk_basis&) { B.atom[2] = 2; }},
      {"negative atom", JK_EINVAL, [](Basis& B, jk_basis&) { B.atom[0] = -1; }},
      {"negative l", JK_EINVAL, [](Basis& B, jk_basis&) { B.l[1] = -1; }},
      {"f shell", JK_EUNSUPPORTED, [](Basis& B, jk_basis&) { B.l[1] = 3; }},
      {"no primitives", JK_EINVAL, [](Basis& B, jk_basis&) { B.nprim[0] = 0; }},
      {"nine primitives", JK_EUNSUPPORTED, [](Basis& B, jk_basis&) { B.nprim[3] = 9; }},
      {"negative prim0", JK_EINVAL, [](Basis& B, jk_basis&) { B.prim0[2] = -1; }},
      {"zero exponent", JK_EINVAL, [](Basis& B, jk_basis&) { B.exps[5] = 0.0; }},
      {"infinite coefficient", JK_EINVAL, [](Basis& B, jk_basis&) { B.coefs[7] = INFINITY; }},
  };
  for (const Case& c : cases) {
    Basis B;
    jk_basis b = B.view();
    c.edit(B, b);
    nbf = -1;
    expect(jk_validate_basis(&b, &nbf) == c.want && nbf == -1, c.what);
  }
  {  // more than 32768 functions: 5462 d shells on one atom
    Basis B;
    B.atom.assign(5462, 0);
    B.l.assign(5462, 2);
    B.nprim.assign(5462, 1);
    B.prim0.assign(5462, 0);
    jk_basis b = B.view();
    expect(jk_validate_basis(&b, &nbf) == JK_EUNSUPPORTED, "too many functions");
  }

  // NULL handles and out-of-range devices fail cleanly
  expect(jk_ctx_create(nullptr, 0) == JK_EINVAL, "jk_ctx_create(NULL)");
  jk_ctx* c = reinterpret_cast<jk_ctx*>(0x1);
  const int rc = jk_ctx_create(&c, 1 << 20);
  expect(rc != JK_OK && c == nullptr, "jk_ctx_create on a missing device");
  expect(jk_last_error(nullptr) != nullptr, "jk_last_error(NULL)");
  expect(jk_ctx_destroy(nullptr) == JK_OK, "jk_ctx_destroy(NULL)");
  {
    Basis B;
    jk_basis b = B.view();
    double dummy = 0.0;
    expect(jk_build(nullptr, &b, &dummy, &dummy, &dummy, 0.0, nullptr, nullptr) == JK_EINVAL,
           "jk_build(NULL ctx)");
    expect(jk_grad(nullptr, &b, &dummy, &dummy, 0.0, nullptr, nullptr) == JK_EINVAL,
           "jk_grad(NULL ctx)");
    jk_stats st;
    expect(jk_get_stats(nullptr, &st) == JK_EINVAL, "jk_get_stats(NULL ctx)");
  }
  if (failures) return 1;
  std::printf("host driver ok\n");
  return 0;
}
