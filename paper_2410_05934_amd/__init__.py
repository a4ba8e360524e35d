"""MI355X-native negacyclic NTT library (placeholder; binding added next)."""
