"""MI355X-native dynamic-bonding Langevin MD hot path (HIP library + binding)."""
