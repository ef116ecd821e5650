"""MI355X-native fast mean-curvature estimator (package stub; binding added below)."""
