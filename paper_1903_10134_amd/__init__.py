"""MI355X-native many-body DPD timestep (placeholder while the binding is written)."""
