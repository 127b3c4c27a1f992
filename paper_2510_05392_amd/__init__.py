"""MI355X-native leading-order matrix elements for g g -> t tbar + n gluons."""
