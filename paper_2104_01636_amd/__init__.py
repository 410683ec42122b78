"""MI355X-native variable-density pressure-Poisson solver."""
