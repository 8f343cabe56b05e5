// Host allocation failure at the C ABI (no GPU needed): this program replaces
// the global operator new so that, while `g_fail` is set, every allocation
// throws std::bad_alloc, and checks that the library's entry points turn the
// exception into MG_ENOMEM (with *out cleared) instead of letting it cross
// the ABI.  Only calls that allocate on the host before their first HIP call
// can be reached without a GPU: mg_batch_setup (its batch object) and
// mg_setup (its context, by a non-throwing new that yields null).
#include <cstdio>
#include <cstdlib>
#include <new>

#include "mgkkt.h"

static bool g_fail = false;

void* operator new(std::size_t n) {
  if (g_fail) throw std::bad_alloc();
  void* p = std::malloc(n ? n : 1);
  if (!p) throw std::bad_alloc();
  return p;
}
void operator delete(void* p) noexcept { std::free(p); }
void operator delete(void* p, std::size_t) noexcept { std::free(p); }

int main() {
  int levels[2] = {7, 8};
  double alphas[2] = {1.0, 1e-4};
  mg_batch* b = reinterpret_cast<mg_batch*>(0x1);
  g_fail = true;
  const int sb = mg_batch_setup(2, levels, alphas, MG_POISSON, nullptr, &b);
  mg_ctx* c = reinterpret_cast<mg_ctx*>(0x1);
  const int sc = mg_setup(6, 1e-2, MG_POISSON, nullptr, &c);
  g_fail = false;
  std::printf("mg_batch_setup %d (out %p), mg_setup %d (out %p)\n", sb, (void*)b, sc, (void*)c);
  if (sb != MG_ENOMEM || b != nullptr || sc != MG_ENOMEM || c != nullptr) return 1;
  std::printf("ok\n");
  return 0;
}
