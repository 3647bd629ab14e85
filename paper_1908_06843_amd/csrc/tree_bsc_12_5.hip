// Compile-time state walk for BSC with H' = 12, gamma = 5.
#include "k_states_tree.hpp"

namespace prosper {
PROSPER_TREE_INSTANCE(false, 12, 5)
}  // namespace prosper
