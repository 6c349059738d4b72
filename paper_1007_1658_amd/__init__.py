"""MI355X-native direct Lomb-Scargle periodogram (placeholder binding)."""
