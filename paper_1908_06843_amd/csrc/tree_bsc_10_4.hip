// Compile-time state walk for BSC with H' = 10, gamma = 4.
#include "k_states_tree.hpp"

namespace prosper {
PROSPER_TREE_INSTANCE(false, 10, 4)
}  // namespace prosper
