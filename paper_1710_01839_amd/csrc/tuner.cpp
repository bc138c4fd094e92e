// Tuning table of the context (filled by the tuner).
#include "capi_internal.hpp"

bool mpg_table_lookup(mpg_ctx* c, int precision, int64_t m, int64_t n, int64_t l, int* algo,
                      mpg_tile* tile) {
  auto it = c->table.find(std::make_tuple(precision, m, n, l));
  if (it == c->table.end()) return false;
  *algo = it->second.first;
  *tile = it->second.second;
  return true;
}

void mpg_destroy_cached(mpg_ctx*) {}
