// Sanitizer driver for the CPU oracle (test infrastructure only): built
// together with lsb_oracle.cpp and refine_oracle.cpp under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py, it runs a
// small moving-interface case on every velocity set (refill, reinitialisation,
// walls of each kind, gravity with the gas baseline, the cumulant gas, several
// bubbles), the dual-number tangent, a refill on a crafted state, decision
// record and replay, and a two-level refinement with a sensor and a re-mesh.
// Exit status 0 and no sanitizer report is a pass.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

namespace orc {
struct Params {  // the oracle's parameter block (same layout, lsb_oracle.cpp)
  int lattice, storage, nx, ny, nz;
  int bc[6];
  double wall_u[6][3];
  double rho_phys[2], tau[2];
  double accel[2][3];
  double sigma;
  double band;
  int n_ext;
  double ext_dtau;
  int reinit_every, n_reinit;
  double reinit_dtau;
  double heaviside_eps;
  int use_pb;
  double pb0;
  int init_hydrostatic;
  int fp16_scale_log2;
  int collision[2];
};
}  // namespace orc

extern "C" {
void* orc_create(const orc::Params* p);
void orc_destroy(void* h);
int orc_init(void* h, const double* phi0, const double* rho0, const double* u0);
int orc_step(void* h, int n);
int orc_get_pop(void* h, double* out);
int orc_get_integrals(void* h, double* out);
int orc_set_decisions(void* h, int mode, void* src);
int orc_replay_failed(void* h);
int orc_lattice(int lattice, int* D, int* Q, int* c, double* w, int* opp);
int orc_refill(const orc::Params* p, const double* phi_new, const unsigned char* old_gas, double* pop, double* rho,
               double* u, double* S, double pb);
void* orc_tan_create(const orc::Params* p);
void orc_tan_destroy(void* h);
int orc_tan_init(void* h, const double* phi0, const double* dphi0, double dsigma, const double* rho0, const double* u0);
int orc_tan_step(void* h, int n);
int orc_tan_centroid(void* h, int axis, double* value, double* tangent);
void* orc_ref_create(int lattice, const int* n, const int* patch, double tau_c, double tau_f);
void orc_ref_destroy(void* h);
int orc_ref_init(void* h, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f);
int orc_ref_step(void* h, int n);
int orc_ref_sensor(void* h, const double* phi, double d_ref, int margin, int* out);  // 1 if any node is tagged
int orc_ref_remesh(void* h, const int* patch);
int orc_ref_get(void* h, double* fc, double* ff);
}

static int fails = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) { std::printf("FAILED: %s (line %d)\n", #cond, __LINE__); ++fails; } \
  } while (0)

static orc::Params params(int lat, int nx, int ny, int nz) {
  orc::Params p;
  std::memset(&p, 0, sizeof(p));
  p.lattice = lat; p.nx = nx; p.ny = ny; p.nz = nz;
  p.rho_phys[0] = 1.0; p.rho_phys[1] = 0.1; p.tau[0] = 0.7; p.tau[1] = 0.9;
  p.sigma = 3e-3; p.band = 6.0; p.n_ext = 8; p.ext_dtau = 0.5;
  p.reinit_every = 4; p.n_reinit = 2; p.reinit_dtau = 0.3; p.heaviside_eps = 1.5;
  p.fp16_scale_log2 = 12;
  return p;
}

// a bubble in a shear flow with walls of each kind and gravity
static void moving_bubble(int lat, int use_pb, int cum) {
  const bool d2 = lat == 0;
  const int nx = d2 ? 23 : 13, ny = d2 ? 21 : 12, nz = d2 ? 1 : 11;
  orc::Params p = params(lat, nx, ny, nz);
  p.bc[2] = p.bc[3] = 1;                 // no-slip y (moving +y face)
  p.wall_u[3][0] = 0.01;
  if (!d2) p.bc[4] = p.bc[5] = 2;        // free-slip z
  else { p.bc[0] = p.bc[1] = 2; }        // free-slip x in 2D
  const double g = 1e-4;
  p.accel[0][1] = p.accel[1][1] = -g;
  p.use_pb = use_pb;
  p.init_hydrostatic = 1;
  if (cum) p.collision[1] = 1;
  const long N = (long)nx * ny * nz;
  std::vector<double> phi(N), u(3 * N, 0.0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long c = ((long)z * ny + y) * nx + x;
        const double X = x + 0.5 - nx / 2.0, Y = y + 0.5 - ny / 2.0, Z = d2 ? 0.0 : z + 0.5 - nz / 2.0;
        double d = 3.5 - std::sqrt(X * X + Y * Y + Z * Z);
        if (use_pb == 2) d = std::max(d, 2.5 - std::sqrt((X - 5) * (X - 5) + (Y + 5) * (Y + 5) + Z * Z));
        phi[c] = d;
        u[3 * c] = 0.02 * std::sin(2 * M_PI * (y + 0.5) / ny);
        u[3 * c + 1] = 0.01 * std::cos(2 * M_PI * (x + 0.5) / nx);
      }
  p.pb0 = p.sigma / 3.5 * (d2 ? 1.0 : 2.0);
  void* h = orc_create(&p);
  CHECK(h != nullptr);
  if (!h) return;
  CHECK(orc_set_decisions(h, 1, nullptr) == 0);
  CHECK(orc_init(h, phi.data(), nullptr, u.data()) == 0);
  CHECK(orc_step(h, 20) == 0);
  double I[16];
  orc_get_integrals(h, I);
  CHECK(std::isfinite(I[0]) && std::isfinite(I[2]));
  // replay of the recorded decisions on a perturbed sigma
  orc::Params q = p;
  q.sigma *= 1.0 + 1e-6;
  void* r = orc_create(&q);
  CHECK(orc_set_decisions(r, 2, h) == 0);
  CHECK(orc_init(r, phi.data(), nullptr, u.data()) == 0);
  CHECK(orc_step(r, 20) == 0);
  CHECK(orc_replay_failed(r) == 0);
  orc_destroy(r);
  orc_destroy(h);
  if (use_pb != 2) {  // the tangent
    void* t = orc_tan_create(&p);
    CHECK(t != nullptr);
    CHECK(orc_tan_init(t, phi.data(), nullptr, 1.0, nullptr, u.data()) == 0);
    CHECK(orc_tan_step(t, 6) == 0);
    double v = 0, dv = 0;
    orc_tan_centroid(t, 1, &v, &dv);
    CHECK(std::isfinite(v) && std::isfinite(dv));
    orc_tan_destroy(t);
  }
}

static void refill_probe() {
  orc::Params p = params(0, 12, 12, 1);
  const long N = 144;
  int D, Q, c[81], opp[27];
  double w[27];
  orc_lattice(0, &D, &Q, c, w, opp);
  std::vector<double> phi(N), pop((size_t)Q * N), rho(N, 1.0), u(3 * N, 0.0), S(6 * N, 0.0);
  std::vector<unsigned char> old(N);
  for (long k = 0; k < N; ++k) {
    const double y = (double)(k / 12) + 0.5;
    phi[k] = y - 6.3;
    old[k] = (y - 5.4) >= 0.0;
    for (int i = 0; i < Q; ++i) pop[(size_t)i * N + k] = w[i];
  }
  CHECK(orc_refill(&p, phi.data(), old.data(), pop.data(), rho.data(), u.data(), S.data(), 0.0) == 0);
}

static void refinement() {
  const int n[3] = {30, 28, 1}, patch[6] = {8, 20, 7, 19, 0, 0};
  void* h = orc_ref_create(0, n, patch, 0.7, -1.0);
  CHECK(h != nullptr);
  if (!h) return;
  const int nc = 30 * 28, nf = 25 * 25;
  std::vector<double> rc(nc, 1.0), uc(2 * nc, 0.0), rf(nf, 1.0), uf(2 * nf, 0.0);
  for (int k = 0; k < nc; ++k) uc[2 * k] = 0.01 * std::sin(2 * M_PI * (k / 30) / 28.0);
  for (int k = 0; k < nf; ++k) uf[2 * k] = 0.01 * std::sin(2 * M_PI * (7 + 0.5 * (k / 25)) / 28.0);
  CHECK(orc_ref_init(h, rc.data(), uc.data(), rf.data(), uf.data()) == 0);
  CHECK(orc_ref_step(h, 5) == 0);
  std::vector<double> phi(nc);
  for (int k = 0; k < nc; ++k) phi[k] = 4.0 - std::hypot(k % 30 - 15.0, k / 30 - 14.0);
  int box[6];
  CHECK(orc_ref_sensor(h, phi.data(), 1.0, 2, box) == 1);  // nodes tagged
  CHECK(orc_ref_remesh(h, box) == 0);
  CHECK(orc_ref_step(h, 3) == 0);
  orc_ref_destroy(h);
}

int main() {
  for (int lat = 0; lat < 3; ++lat) moving_bubble(lat, 1, 0);
  moving_bubble(2, 1, 1);  // cumulant gas
  moving_bubble(0, 2, 0);  // two bubbles, one baseline each
  refill_probe();
  refinement();
  std::printf("%s\n", fails ? "sanitize: FAILED" : "sanitize: ok");
  return fails ? 1 : 0;
}
