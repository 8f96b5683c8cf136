"""MI355X-native SG-WLS filtering (placeholder; the binding is added with the library)."""
