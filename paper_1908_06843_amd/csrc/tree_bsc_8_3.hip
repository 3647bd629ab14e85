// Compile-time state walk for BSC with H' = 8, gamma = 3.
#include "k_states_tree.hpp"

namespace prosper {
PROSPER_TREE_INSTANCE(false, 8, 3)
}  // namespace prosper
