"""MI355X-native staggered Dslash, even-odd CG and fermion force (binding placeholder)."""
