"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This package only *draws* inputs: Hamiltonian coefficients in sum-of-products
form, tree topologies, bond-dimension shapes, product-state occupations and
random tensors.  It holds none of the eigensolver's arithmetic (no operator
matrices, no TTNO construction, no contraction, no decomposition), so the
oracle and the HIP path can both read it without sharing any of the method.
"""
from .hamiltonians import (SOPModel, make_config_model, coupled_oscillators, quartic_force_field, paper_64d_model,
                           ensemble_members)
from .trees import Tree, mps_tree, binary_tree, fork_tree, t_tree, leaf_only_12, full_t3ns_12, paper_topology, bond_dims
from .states import (node_shape, lowest_product_states, initial_block, random_block, random_tensor,
                     sketch_matrices)
