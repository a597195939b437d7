// yq_eval_potential_noalloc: the off-surface potential (eq. intrep) with every
// scratch buffer in one file-scope device array, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// The kernels are those of yq_eval_potential (post.hip): the chunk partial sums
// [M x chunks] and the oversampled panel rule (points, weighted normals and the
// interpolated density, 5 x panels x pot_oversample x 16 doubles) live in the
// array below instead of the problem's own buffers.  The oversampled points are
// rebuilt on every call, since the array is shared by every problem on the
// device.
#include <mutex>

#include "common.h"
#include "problem.h"

namespace yq {

// Largest scratch of one call.  Each device the library runs on holds the array
// for the life of the process.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of the scratch array (looked up once
// per device; the array's name is only a host-side stand-in).
void* scratch_on(int dev) {
  YQ_REQUIRE(dev >= 0 && dev < kMaxDevices, YQ_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    YQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    YQ_REQUIRE(p != nullptr, YQ_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

// Bytes of scratch one call needs (partials, then the five oversampled arrays).
size_t noalloc_potential_bytes(int64_t M, int64_t npan, int nsub) {
  const PotPlan pp = pot_plan(M, npan);
  const size_t nf = (size_t)npan * nsub * Q;
  return round256((size_t)pp.chunks * M * sizeof(double)) + 5 * round256(nf * sizeof(double));
}

}  // namespace yq

using namespace yq;

extern "C" int yq_eval_potential_noalloc(yq_problem* pb, const double* sigma, int64_t M,
                                         const double* tx, const double* ty, double* u) {
  try {
    YQ_REQUIRE(pb != nullptr, YQ_EINVAL, "null problem");
    YQ_REQUIRE(pb->ready, YQ_ESTATE, "yq_set_particles has not been called");
    YQ_REQUIRE(M >= 0, YQ_EINVAL, "M < 0");
    if (M == 0) return YQ_OK;
    YQ_REQUIRE(sigma && tx && ty && u, YQ_EINVAL, "null argument");
    const int64_t npan = pb->npan;
    const int nsub = pb->prm.pot_oversample;
    const size_t need = noalloc_potential_bytes(M, npan, nsub);
    YQ_REQUIRE(need <= kNoAllocScratchBytes, YQ_EINVAL,
               "yq_eval_potential_noalloc: " + std::to_string(need) + " bytes of scratch needed, " +
                   std::to_string(kNoAllocScratchBytes) + " available (fewer targets or panels)");
    int dev = 0;
    YQ_HIP(hipGetDevice(&dev));
    unsigned char* base = static_cast<unsigned char*>(scratch_on(dev));
    const PotPlan pp = pot_plan(M, npan);
    const size_t nf = (size_t)npan * nsub * Q;
    double* partial = reinterpret_cast<double*>(base);
    size_t off = round256((size_t)pp.chunks * M * sizeof(double));
    double* arr[5];
    for (auto& a : arr) {
      a = reinterpret_cast<double*>(base + off);
      off += round256(nf * sizeof(double));
    }
    PotFine pf{nsub, arr[0], arr[1], arr[2], arr[3], arr[4]};
    const GeomView g = pb->view();
    // every slot read later is written first in stream order: the oversampled
    // points here, the interpolated density and each (target, chunk) partial
    // by the launches of launch_potential, so nothing needs clearing
    launch_pot_fine(g, pb->consts, nsub, pf, pb->stream);
    launch_potential(g, pf, pb->Lpot.p, pb->prm.pot_beta, sigma, M, tx, ty, pp, partial, u,
                     pb->stream);
    return YQ_OK;
  } catch (const Error& e) {
    if (pb) pb->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (pb) pb->err = e.what();
    return YQ_EDEVICE;
  } catch (...) {
    return YQ_EDEVICE;
  }
}
