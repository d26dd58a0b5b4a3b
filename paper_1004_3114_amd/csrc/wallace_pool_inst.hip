// Instantiates the pool-resident pass kernels for one (n, reduction mode);
// compiled once per pair with -DWALLACE_POOL_N=<4|16> -DWALLACE_POOL_RM=<0|1|2>.
#include "wallace_pool.hpp"

#ifndef WALLACE_POOL_N
#error "WALLACE_POOL_N must be defined"
#endif
#ifndef WALLACE_POOL_RM
#error "WALLACE_POOL_RM must be defined"
#endif

#define WALLACE_CAT3(a, b, c) a##b##_##c
#define WALLACE_TABLE(n, rm) WALLACE_CAT3(pool_table_, n, rm)
#define WALLACE_TABLE_LEN(n, rm) WALLACE_CAT3(pool_table_len_, n, rm)

#define WALLACE_SHAPES_OF(n) WALLACE_SHAPES_OF_I(n)
#define WALLACE_SHAPES_OF_I(n) WALLACE_POOL_SHAPES_##n

namespace wallace {
namespace pool {

#define WALLACE_ENTRY(NC, T, L, NST)                                                     \
    {NC, T, L, NST, reinterpret_cast<const void *>(&k_pool<NC, T, L, WALLACE_POOL_RM, NST>), \
     Cfg<NC, T, L, WALLACE_POOL_RM, NST>::LDS_BYTES, Cfg<NC, T, L, WALLACE_POOL_RM, NST>::BLOCK},

extern const PoolEntry WALLACE_TABLE(WALLACE_POOL_N, WALLACE_POOL_RM)[] = {
    WALLACE_SHAPES_OF(WALLACE_POOL_N)(WALLACE_ENTRY)};
extern const int WALLACE_TABLE_LEN(WALLACE_POOL_N, WALLACE_POOL_RM) =
    (int)(sizeof(WALLACE_TABLE(WALLACE_POOL_N, WALLACE_POOL_RM)) / sizeof(PoolEntry));

}  // namespace pool
}  // namespace wallace
