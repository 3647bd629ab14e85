// Compile-time state walk for TSC with H' = 8, gamma = 3.
#include "k_states_tree.hpp"

namespace prosper {
PROSPER_TREE_INSTANCE(true, 8, 3)
}  // namespace prosper
