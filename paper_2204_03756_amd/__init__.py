"""MI355X-native mass-transfer particle tracking (placeholder; binding follows)."""
